"""GPU parity: the HIP path (through the C ABI) against the CPU oracle, element by element.

Floating-point bar.  The residual of the split form is a sum of flux differences whose terms
are far larger than the result (at Ma 0.1 the pressure p0 = 71.4 and total enthalpy ~250
cancel to O(0.1-1) rates), so any two FP64 evaluations that round differently disagree by
the rounding level of that sum.  That level is measured, per test, as the difference between
the oracle's double build and its long-double build on the same input (e64).  The GPU result
must lie within max(1e-12 |R|, GATE e64) of the long-double oracle, per conserved variable,
with GATE = 2 (tests/helpers.py): the GPU path rounds at most twice as badly as a plain FP64
evaluation.  The relative error against the double
oracle is printed as well.
"""
import math
import sys

import numpy as np
import pytest

from helpers import to_conservative, GATE, gate_ok, parity_log, FP32_TOL as FP32_TOLS
from paper_2206_09733_amd import synth

pytestmark = pytest.mark.gpu

TWO_PI = 2 * math.pi


@pytest.fixture(scope="module")
def dg():
    from paper_2206_09733_amd import dgsem
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    dgsem.lib()
    return dgsem


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def cfg(**kw):
    base = dict(ex=3, N=3, deform=False, Ma=0.3, Re=0.0, vol="ec", surf="roe")
    base.update(kw)
    return base


def oracle_pair(orc, c, U):
    o64 = orc.OracleSolver(**c)
    o64.set_state(U)
    o80 = orc.OracleSolver(**c, precision="fp80")
    o80.set_state(U)
    return o64.residual(), o80.residual()


def per_var(A, nvar=5, E=None, nn=None):
    return np.asarray(A).reshape(E, nvar, nn)


def assert_parity(name, Rg, R64, R80, E, nn, factor=GATE):
    G, A, B = (x.reshape(E, 5, nn) for x in (Rg, R64, R80))
    scale = np.abs(B).max(axis=(0, 2))
    e64 = np.abs(A - B).max(axis=(0, 2))
    eg = np.abs(G - B).max(axis=(0, 2))
    rel64 = np.abs(G - A).max(axis=(0, 2)) / np.maximum(np.abs(A).max(axis=(0, 2)), 1e-300)
    tol = np.maximum(1e-12 * scale, factor * e64)
    glob = np.abs(G - B).max() / np.abs(B).max()
    log(f"[{name}] |R|={np.array2string(scale, precision=2)} gpu-vs-fp80={np.array2string(eg, precision=2)} "
        f"fp64-vs-fp80={np.array2string(e64, precision=2)} rel-vs-fp64={np.array2string(rel64, precision=2)} "
        f"global rel vs fp80 {glob:.2e}")
    parity_log(name + " global", gpu_global_rel=float(glob), fp64_global_rel=float(np.abs(A - B).max() / np.abs(B).max()))
    assert gate_ok(name, eg, e64, scale) and np.all(eg <= tol), (name, eg, tol)
    return rel64


def perturbed_state(orc, c, seed, amp=(0.02, 0.05, 0.02)):
    """Oracle TGV state with seeded random primitive perturbations (exercises every branch)."""
    o = orc.OracleSolver(**c)
    o.set_ic("tgv")
    nn = (c["N"] + 1) ** 3
    U0 = o.state().reshape(o.E, 5, nn)
    drho, dv, dp = synth.primitive_perturbation(o.nodes, seed, amp)
    rho = U0[:, 0].reshape(-1)
    v = (U0[:, 1:4] / U0[:, :1]).transpose(0, 2, 1).reshape(-1, 3)
    p = 0.4 * (U0[:, 4].reshape(-1) - 0.5 * rho * (v * v).sum(1))
    U = to_conservative(rho * (1 + drho), v + dv.T, p * (1 + dp))
    return U.reshape(o.E, nn, 5).transpose(0, 2, 1).reshape(-1)


# ------------------------------------------------------------------ geometry and initial state
@pytest.mark.parametrize("N", [1, 2, 3, 4, 5, 6, 7])
def test_geometry_parity(dg, orc, N):
    """FP64 geometry kernel: node coordinates, curl-form metric terms and Jacobian against the
    oracle's long-double build, within GATE = 2 times the double build's own rounding (the metric terms are
    sums of O(N^2) products, so their rounding grows with N)."""
    log(f"geometry N={N}")
    c = dict(ex=3, ey=2, ez=4, N=N, deform=True)
    o = orc.OracleSolver(**c)
    o80 = orc.OracleSolver(**c, precision="fp80")
    g = dg.Solver(**c)
    Xg, Jag, Jg = g.geometry()
    Xo = o.coords()
    assert np.abs(Xg - Xo).max() < 1e-14
    for name, a, b, b80 in (("Ja", Jag, *o.metrics()[:1], o80.metrics()[0]),
                            ("J", Jg, o.metrics()[1], o80.metrics()[1])):
        eg, e64 = np.abs(a - b80).max(), np.abs(b - b80).max()
        log(f"[geometry N={N} {name}] gpu-vs-fp80 {eg:.2e} fp64-vs-fp80 {e64:.2e} scale {np.abs(b80).max():.2e}")
        assert gate_ok("test_geometry_parity", eg, e64, np.abs(b80).max(), 1e-14), "parity gate"


@pytest.mark.parametrize("ic,params", [("tgv", None), ("uniform", [1.2, 0.3, -0.1, 0.2, 3.0]),
                                       ("density_wave", [0.2, 1.0, 0.5, 0.0, 1.0, 1.0, 1.0, 0.0, 0.3]),
                                       ("vortex", [5.0, 0.5, -0.3, 0.4, 0.4])])
def test_initial_condition_parity(dg, orc, ic, params):
    log(f"ic {ic}")
    c = dict(ex=4, N=4, deform=True, Ma=0.1)
    o = orc.OracleSolver(**c)
    g = dg.Solver(**c)
    o.set_ic(ic, params)
    g.set_ic(ic, params)
    Uo, Ug = o.state(), g.state()
    assert np.abs(Ug - Uo).max() <= 1e-14 * np.abs(Uo).max()


# ------------------------------------------------------------------ residual
def test_residual_c1_tgv(dg, orc):
    """The 4^3, N=3 Euler Taylor-Green case at Ma 0.1 (EC volume, Roe faces)."""
    c = dict(ex=4, N=3, Ma=0.1)
    o = orc.OracleSolver(**c)
    o.set_ic("tgv")
    U = o.state()
    R64, R80 = oracle_pair(orc, c, U)
    g = dg.Solver(**c)
    g.set_state(U)
    Rg = g.residual()
    assert_parity("C1 TGV", Rg, R64, R80, o.E, 64)
    glob = np.abs(Rg - R80).max() / np.abs(R80).max()
    log(f"[C1 TGV] global relative Linf vs the long-double oracle {glob:.2e}")
    assert glob < 1e-12


@pytest.mark.parametrize("N", [1, 2, 3, 4, 5, 6, 7])
@pytest.mark.parametrize("surf", ["roe", "llf", "ec", "central"])
def test_residual_orders_and_fluxes(dg, orc, N, surf):
    c = cfg(ex=3, ey=2, ez=2, N=N, deform=True, surf=surf, Ma=0.3)
    log(f"residual N={N} surf={surf}")
    U = perturbed_state(orc, c, seed=100 + N)
    R64, R80 = oracle_pair(orc, c, U)
    g = dg.Solver(**c)
    g.set_state(U)
    assert_parity(f"N={N} {surf}", g.residual(), R64, R80, 12, (N + 1) ** 3)


@pytest.mark.parametrize("N", [2, 3, 4, 5, 7])
@pytest.mark.parametrize("vol,surf,Re", [("ir", "ir", 0.0), ("ec", "es", 0.0), ("ir", "es", 100.0),
                                         ("ec", "ir", 100.0)])
def test_residual_ismail_roe_and_entropy_stable(dg, orc, N, vol, surf, Re):
    """Ismail-Roe volume/surface fluxes and the entropy-stable surface flux (FP64)."""
    c = cfg(ex=3, ey=2, ez=2, N=N, deform=True, vol=vol, surf=surf, Re=Re, Ma=0.3)
    log(f"residual N={N} vol={vol} surf={surf} Re={Re}")
    U = perturbed_state(orc, c, seed=300 + N)
    R64, R80 = oracle_pair(orc, c, U)
    g = dg.Solver(**c)
    g.set_state(U)
    assert_parity(f"N={N} {vol}/{surf} Re={Re}", g.residual(), R64, R80, 12, (N + 1) ** 3)


@pytest.mark.parametrize("N", [2, 3, 4, 5, 7])
@pytest.mark.parametrize("vol,surf,Re", [("kg", "roe", 0.0), ("pirozzoli", "llf", 100.0), ("ducros", "ec", 0.0),
                                         ("morinishi", "central", 100.0), ("ec", "es_matrix", 0.0),
                                         ("ir", "es_matrix", 100.0), ("ec", "ld_roe", 100.0),
                                         ("pirozzoli", "es_matrix", 0.0), ("morinishi", "ld_roe", 100.0),
                                         ("kg", "ld_roe", 0.0), ("ec", "lf_global", 0.0),
                                         ("pirozzoli", "lf_global", 100.0)])
def test_residual_kep_and_dissipative_surface_fluxes(dg, orc, N, vol, surf, Re):
    """Kinetic-energy-preserving volume fluxes (Kennedy-Gruber, Pirozzoli, Ducros, Morinishi),
    the matrix-dissipation entropy-stable flux and the low-dissipation Roe flux, alone and
    combined (FP64)."""
    c = cfg(ex=3, ey=2, ez=2, N=N, deform=True, vol=vol, surf=surf, Re=Re, Ma=0.3)
    log(f"residual N={N} vol={vol} surf={surf} Re={Re}")
    U = perturbed_state(orc, c, seed=500 + N)
    R64, R80 = oracle_pair(orc, c, U)
    g = dg.Solver(**c)
    g.set_state(U)
    assert_parity(f"N={N} {vol}/{surf} Re={Re}", g.residual(), R64, R80, 12, (N + 1) ** 3)


def test_global_lax_friedrichs_trajectory(dg, orc):
    """The global wave speed is reduced on the device before every stage: three RK3 steps of a
    perturbed state against the oracle, which takes it from each stage's state as well."""
    c = cfg(ex=3, N=4, deform=True, Ma=0.3, surf="lf_global")
    U = perturbed_state(orc, c, seed=91, amp=(0.02, 0.05, 0.02))
    o, o80 = orc.OracleSolver(**c), orc.OracleSolver(**c, precision="fp80")
    o.set_state(U)
    o80.set_state(U)
    dt = o.suggest_dt(0.5)
    o.rk3(dt, 3)
    o80.rk3(dt, 3)
    g = dg.Solver(**c)
    g.set_state(U)
    g.rk_step(dt, 3)
    Ug, Uo, U80 = g.state(), o.state(), o80.state()
    d = lambda a, b: np.abs(a - b).reshape(27, 5, 125).max(axis=(0, 2))
    sc = np.abs(U80).reshape(27, 5, 125).max(axis=(0, 2))
    log(f"[lf_global RK] gpu-vs-fp80 {d(Ug, U80) / sc} fp64-vs-fp80 {d(Uo, U80) / sc}")
    assert gate_ok("test_global_lax_friedrichs_trajectory", d(Ug, U80), d(Uo, U80), sc, 1e-14), "parity gate"


def test_gpu_entropy_matrix_dissipation(dg, orc):
    """On the GPU path, entropy decays with the matrix-dissipation faces (EC volume flux), and
    the rate lies within rounding of the oracle's."""
    c = cfg(ex=3, N=3, deform=True, Ma=0.4, surf="es_matrix")
    U = perturbed_state(orc, c, seed=13, amp=(0.05, 0.1, 0.05))
    o = orc.OracleSolver(**c)
    o.set_state(U)
    g = dg.Solver(**c)
    g.set_state(U)
    R = g.residual()
    ref = abs(o.entropy_production(np.abs(R)))
    eg, eo = o.entropy_production(R), o.entropy_production(o.residual())
    log(f"entropy production es_matrix GPU {eg:.6e} oracle {eo:.6e} scale {ref:.3e}")
    assert eg < -1e-6 * ref
    assert abs(eg - eo) < 1e-11 * ref


def test_gpu_entropy_ismail_roe_and_stable(dg, orc):
    """On the GPU path: the Ismail-Roe split form with Ismail-Roe faces conserves entropy; with
    the entropy-stable faces entropy decays; FP32-bulk refuses these fluxes."""
    c = cfg(ex=3, N=3, deform=True, Ma=0.4)
    U = perturbed_state(orc, c, seed=12, amp=(0.05, 0.1, 0.05))
    o = orc.OracleSolver(**c)
    o.set_state(U)
    g = dg.Solver(**dict(c, vol="ir", surf="ir"))
    g.set_state(U)
    R = g.residual()
    ref = abs(o.entropy_production(np.abs(R)))
    assert abs(o.entropy_production(R)) < 1e-11 * ref
    g2 = dg.Solver(**dict(c, surf="es"))
    g2.set_state(U)
    assert o.entropy_production(g2.residual()) < -1e-6 * ref
    with pytest.raises(dg.DgError) as ei:
        dg.Solver(**dict(c, surf="es"), precision="fp32_bulk", bind=False)
    assert ei.value.code == dg.DG_EUNSUPPORTED


def test_residual_central_volume_flux(dg, orc):
    c = cfg(ex=2, ey=3, ez=2, N=4, deform=True, vol="central", surf="llf")
    U = perturbed_state(orc, c, seed=7)
    R64, R80 = oracle_pair(orc, c, U)
    g = dg.Solver(**c)
    g.set_state(U)
    assert_parity("central volume", g.residual(), R64, R80, 12, 125)


@pytest.mark.parametrize("N", [1, 2, 3, 4, 5, 6, 7])
def test_residual_navier_stokes(dg, orc, N):
    c = cfg(ex=3, ey=2, ez=3, N=N, deform=True, Re=100.0, Ma=0.3)
    log(f"NS residual N={N}")
    U = perturbed_state(orc, c, seed=200 + N)
    R64, R80 = oracle_pair(orc, c, U)
    g = dg.Solver(**c)
    g.set_state(U)
    assert_parity(f"NS N={N}", g.residual(), R64, R80, 18, (N + 1) ** 3)


@pytest.mark.parametrize("N", [1, 2, 3, 4, 5, 6, 7])
@pytest.mark.parametrize("visc,eta", [("br2", 0.0), ("ip", 0.0), ("br2", 4.0), ("ip", 3.0)])
def test_residual_viscous_face_schemes(dg, orc, N, visc, eta):
    """BR2 and symmetric interior-penalty face viscous fluxes on a perturbed state (the traces
    jump across every face), curvilinear mesh, FP64."""
    c = cfg(ex=3, ey=2, ez=3, N=N, deform=True, Re=100.0, Ma=0.3)
    log(f"NS residual N={N} {visc} eta={eta}")
    U = perturbed_state(orc, c, seed=700 + N)
    o64 = orc.OracleSolver(**c, visc=visc, visc_eta=eta)
    o64.set_state(U)
    o80 = orc.OracleSolver(**c, precision="fp80", visc=visc, visc_eta=eta)
    o80.set_state(U)
    g = dg.Solver(**c, visc=visc, visc_eta=eta)
    g.set_state(U)
    assert_parity(f"NS N={N} {visc} eta={eta}", g.residual(), o64.residual(), o80.residual(), 18, (N + 1) ** 3)


@pytest.mark.parametrize("visc", ["br2", "ip"])
def test_viscous_face_schemes_trajectory_and_fp32(dg, orc, visc):
    """Three RK3 steps of a perturbed Navier-Stokes state against the oracle (FP64), and the
    FP32-bulk residual within the stated tolerance."""
    c = cfg(ex=3, N=4, deform=True, Re=400.0, Ma=0.2)
    U = perturbed_state(orc, c, seed=77, amp=(0.01, 0.02, 0.01))
    o, o80 = orc.OracleSolver(**c, visc=visc), orc.OracleSolver(**c, visc=visc, precision="fp80")
    o.set_state(U)
    o80.set_state(U)
    dt = o.suggest_dt(0.5)
    o.rk3(dt, 3)
    o80.rk3(dt, 3)
    g = dg.Solver(**c, visc=visc)
    g.set_state(U)
    g.rk_step(dt, 3)
    Ug, Uo, U80 = g.state(), o.state(), o80.state()
    d = lambda a, b: np.abs(a - b).reshape(27, 5, 125).max(axis=(0, 2))
    sc = np.abs(U80).reshape(27, 5, 125).max(axis=(0, 2))
    log(f"[{visc} RK] gpu-vs-fp80 {d(Ug, U80) / sc} fp64-vs-fp80 {d(Uo, U80) / sc}")
    assert gate_ok("test_viscous_face_schemes_trajectory_and_fp32", d(Ug, U80), d(Uo, U80), sc, 1e-14), "parity gate"
    c8 = dict(ex=8, N=4, deform=True, Ma=0.1, Re=1600.0)
    U8 = perturbed_state(orc, dict(c8, vol="ec", surf="roe"), seed=78, amp=(1e-3, 1e-3, 1e-3))
    o8 = orc.OracleSolver(**c8, visc=visc)
    o8.set_state(U8)
    Ro = o8.residual()
    g32 = dg.Solver(**c8, visc=visc, precision="fp32_bulk")
    g32.set_state(U8)
    Rg = g32.residual()
    err = np.abs(Rg - Ro).reshape(512, 5, 125).max(axis=(0, 2)) / np.abs(Ro).reshape(512, 5, 125).max(axis=(0, 2))
    log(f"[FP32-bulk {visc}] rel err per var {err}")
    assert np.all(err < FP32_TOL), err


def test_residual_edge_meshes(dg, orc):
    """One element across a direction (a face is its own periodic neighbour), element counts
    that are not multiples of 8 (plain workgroup order), a non-cubic box."""
    for c in (cfg(ex=1, ey=1, ez=1, N=3), cfg(ex=1, ey=3, ez=2, N=4, deform=True, Re=50.0),
              cfg(ex=5, ey=3, ez=1, N=2, hi=(1.0, 2.0, 0.5), surf="llf")):
        log(f"edge mesh {c}")
        E = c["ex"] * c["ey"] * c["ez"]
        U = perturbed_state(orc, c, seed=E)
        R64, R80 = oracle_pair(orc, c, U)
        g = dg.Solver(**c)
        g.set_state(U)
        assert_parity(f"edge {c['ex']}x{c['ey']}x{c['ez']}", g.residual(), R64, R80, E, (c["N"] + 1) ** 3)


# ------------------------------------------------------------------ invariants on the GPU path
def test_gpu_freestream_and_conservation(dg, orc):
    c = cfg(ex=4, N=4, deform=True, Re=200.0, Ma=0.3)
    g = dg.Solver(**c)
    p = 1 / (1.4 * 0.09)
    g.set_ic("uniform", [1.0, 0.3, -0.2, 0.1, p])
    R = g.residual()
    _, Ja, J = g.geometry()
    scale = (p / 0.4 + p) * np.abs(Ja).max() / J.min() * 10
    assert np.abs(R).max() < 1e-13 * scale
    g.set_ic("tgv")
    R = g.residual().reshape(g.E, 5, 125)
    _, w, _ = orc.gll(4)
    wq = (w[:, None, None] * w[None, :, None] * w[None, None, :]).reshape(-1)[None, :] * J.reshape(g.E, 125)
    tot = np.einsum("en,evn->v", wq, R)
    mag = np.einsum("en,evn->v", wq, np.abs(R))
    assert np.all(np.abs(tot) < 1e-12 * mag.max()), tot


def test_gpu_entropy_conservation(dg, orc):
    c = cfg(ex=3, N=3, deform=True, surf="ec", Ma=0.4)
    U = perturbed_state(orc, c, seed=11, amp=(0.05, 0.1, 0.05))
    g = dg.Solver(**c)
    g.set_state(U)
    R = g.residual()
    o = orc.OracleSolver(**c)
    o.set_state(U)
    ent = o.entropy_production(R)  # sum w J w(U).R with the GPU's R
    ent_ref = abs(o.entropy_production(np.abs(R)))
    assert abs(ent) < 1e-11 * ent_ref


# ------------------------------------------------------------------ time integration
def test_rk3_trajectory_c1(dg, orc):
    """The full 4^3, N=3 Euler TGV configuration: 10 low-storage RK3 steps at CFL 0.5."""
    c = dict(ex=4, N=3, Ma=0.1)
    o = orc.OracleSolver(**c)
    o.set_ic("tgv")
    U0 = o.state()
    dt = o.suggest_dt(0.5)
    o.rk3(dt, 10)
    o80 = orc.OracleSolver(**c, precision="fp80")
    o80.set_state(U0)
    o80.rk3(dt, 10)
    g = dg.Solver(**c)
    g.set_ic("tgv")
    assert abs(g.suggest_dt(0.5) - dt) < 1e-13 * dt
    g.set_state(U0)
    g.rk_step(dt, 10)
    Ug, Uo, U80 = g.state(), o.state(), o80.state()
    d = lambda a, b: np.abs(a - b).reshape(64, 5, 64).max(axis=(0, 2))
    sc = np.abs(U80).reshape(64, 5, 64).max(axis=(0, 2))
    log(f"[C1 RK] gpu-vs-fp80 {d(Ug, U80) / sc} fp64-vs-fp80 {d(Uo, U80) / sc}")
    assert gate_ok("test_rk3_trajectory_c1", d(Ug, U80), d(Uo, U80), sc, 1e-14), "parity gate"


def test_rk3_trajectory_navier_stokes(dg, orc):
    c = dict(ex=3, N=4, deform=True, Ma=0.1, Re=1600.0)
    o = orc.OracleSolver(**c)
    o.set_ic("tgv")
    U0 = o.state()
    dt = o.suggest_dt(0.5)
    o.rk3(dt, 5)
    o80 = orc.OracleSolver(**c, precision="fp80")
    o80.set_state(U0)
    o80.rk3(dt, 5)
    g = dg.Solver(**c)
    g.set_state(U0)
    g.rk_step(dt, 5)
    Ug, Uo, U80 = g.state(), o.state(), o80.state()
    d = lambda a, b: np.abs(a - b).reshape(27, 5, 125).max(axis=(0, 2))
    sc = np.abs(U80).reshape(27, 5, 125).max(axis=(0, 2))
    log(f"[NS RK] gpu-vs-fp80 {d(Ug, U80) / sc} fp64-vs-fp80 {d(Uo, U80) / sc}")
    assert gate_ok("test_rk3_trajectory_navier_stokes", d(Ug, U80), d(Uo, U80), sc, 1e-14), "parity gate"


@pytest.mark.parametrize("case", ["c1_euler", "navier_stokes"])
def test_rk4_trajectory(dg, orc, case):
    """Carpenter-Kennedy RK4 (the paper's RK4 option): GPU trajectory against the oracle's double
    and long-double builds, with graph replay, and against eager launches bitwise."""
    c = dict(ex=4, N=3, Ma=0.1) if case == "c1_euler" else dict(ex=3, N=4, deform=True, Ma=0.1, Re=1600.0)
    steps = 10 if case == "c1_euler" else 5
    o = orc.OracleSolver(**c)
    o.set_ic("tgv")
    U0 = o.state()
    dt = o.suggest_dt(0.8)
    o.rk(dt, steps, "rk4")
    o80 = orc.OracleSolver(**c, precision="fp80")
    o80.set_state(U0)
    o80.rk(dt, steps, "rk4")
    g = dg.Solver(**c)
    g.set_scheme("rk4")
    g.set_state(U0)
    g.rk_step(dt, steps)
    ge = dg.Solver(**c)
    ge.set_scheme("rk4")
    ge.use_graphs(False)
    ge.set_state(U0)
    for _ in range(steps):
        ge.rk_step(dt, 1)
    Ug, Uo, U80 = g.state(), o.state(), o80.state()
    assert np.array_equal(Ug, ge.state())
    E, nn = o.E, (c["N"] + 1) ** 3
    d = lambda a, b: np.abs(a - b).reshape(E, 5, nn).max(axis=(0, 2))
    dG, d64, d80 = Ug - U0, Uo - U0, U80 - U0
    sc = np.abs(d80).reshape(E, 5, nn).max(axis=(0, 2))
    log(f"[RK4 {case}] increment error: gpu-vs-fp80 {d(dG, d80) / sc} fp64-vs-fp80 {d(d64, d80) / sc}")
    assert gate_ok("test_rk4_trajectory", d(dG, d80), d(d64, d80), sc, 1e-12), "parity gate"
    # not the RK3 trajectory
    g3 = dg.Solver(**c)
    g3.set_state(U0)
    g3.rk_step(dt, steps)
    assert np.abs(g3.state() - Ug).max() > 1e3 * np.abs(Ug - U80).max()


def test_gpu_vortex_spectral_convergence(dg, orc):
    """The GPU path converges spectrally to the exact solution of the isentropic vortex (a
    translation of the initial state): 16 x 16 x 1 elements on [-10, 10]^3, Mach 0.5 free stream
    along the diagonal, RK4 to t = 0.5 at CFL 0.5; the L-infinity error falls by at least 2x per
    order and by more than 200x from N = 2 to N = 6 (the oracle gives 0.37 -> 5.8e-4)."""
    import math
    U = 0.5 * math.sqrt(0.7)
    T = 0.5
    errs = []
    for N in (2, 3, 4, 5, 6):
        c = dict(ex=16, ey=16, ez=1, N=N, Ma=0.5, lo=(-10.0,) * 3, hi=(10.0,) * 3)
        g = dg.Solver(**c)
        g.set_scheme("rk4")
        g.set_ic("vortex", [5.0, 0.0, 0.0, U, U])
        dt = g.suggest_dt(0.5)
        m = int(math.ceil(T / dt))
        g.rk_step(T / m, m)
        ex = dg.Solver(**c)
        ex.set_ic("vortex", [5.0, U * T, U * T, U, U])
        errs.append(np.abs(g.state() - ex.state()).max())
        g.close()
        ex.close()
    log(f"[vortex convergence N=2..6] {errs}")
    assert all(b < a / 2 for a, b in zip(errs, errs[1:])), errs
    assert errs[-1] < errs[0] / 200


def test_diagnostics_parity(dg, orc):
    c = dict(ex=4, N=4, deform=True, Ma=0.1, Re=1600.0)
    o = orc.OracleSolver(**c)
    o.set_ic("tgv")
    g = dg.Solver(**c)
    g.set_state(o.state())
    do, dgd = o.diagnostics(), g.diagnostics()
    keys = {"mass_rho": "mass_rho", "mass_rhoE": "mass_rhoE", "entropy": "entropy",
            "entropy_paper": "entropy_paper", "ke": "ke", "enstrophy": "enstrophy",
            "lambda_max": "lambda_max", "rho_min": "rho_min", "p_min": "p_min", "volume": "volume"}
    for ko, kg in keys.items():
        assert abs(dgd[kg] - do[ko]) <= 1e-12 * abs(do[ko]), (ko, dgd[kg], do[ko])
    for k in ("mass_rhou", "mass_rhov", "mass_rhow"):
        assert abs(dgd[k] - do[k]) <= 1e-12 * do["mass_rho"]
    assert dgd["nonfinite"] == 0
    # bitwise reproducible reductions
    assert g.diagnostics() == dgd


def test_set_state_rejects_bad_input(dg, orc):
    g = dg.Solver(ex=2, N=2)
    g.set_ic("tgv")
    U = g.state()
    bad = U.copy()
    bad[7] = np.nan
    with pytest.raises(dg.DgError) as ei:
        g.set_state(bad)
    assert ei.value.code == dg.DG_ENONFINITE
    bad = U.copy()
    bad[0] = -1.0
    with pytest.raises(dg.DgError):
        g.set_state(bad)
    assert np.array_equal(g.state(), U)


# ------------------------------------------------------------------ FP32-bulk
# Stated tolerance of the FP32-bulk path (FP32 flux and derivative arithmetic in deviation form
# about the state's mean density and pressure; mass flux, metric terms, RK state and reductions
# in FP64): relative L-infinity per conserved variable against the FP64 oracle, FP32_TOL in
# tests/helpers.py ("small" for these meshes, "c2" for the 32^3 benchmark mesh).
FP32_TOL = FP32_TOLS["small"]


@pytest.mark.parametrize("Re", [0.0, 1600.0])
def test_fp32_bulk_error(dg, orc, Re):
    c = dict(ex=8, N=4, deform=True, Ma=0.1, Re=Re)
    o = orc.OracleSolver(**c)
    o.set_ic("tgv")
    U = o.state()
    Ro = o.residual()
    g = dg.Solver(**c, precision="fp32_bulk")
    g.set_state(U)
    Rg = g.residual()
    E = 512
    err = np.abs(Rg - Ro).reshape(E, 5, 125).max(axis=(0, 2)) / np.abs(Ro).reshape(E, 5, 125).max(axis=(0, 2))
    glob = np.abs(Rg - Ro).max() / np.abs(Ro).max()
    log(f"[FP32-bulk Re={Re}] rel err per var {err} global {glob:.2e}")
    assert np.all(err < FP32_TOL), err


@pytest.mark.parametrize("N", [1, 2, 3, 5, 6, 7])
@pytest.mark.parametrize("surf", ["roe", "llf", "ec", "central"])
def test_fp32_bulk_orders_and_fluxes(dg, orc, N, surf):
    """FP32-bulk at every compiled order and surface flux (Navier-Stokes, deformed 4^3 mesh,
    Ma 0.1 TGV): relative error per conserved variable against the FP64 oracle within the stated
    tolerance."""
    c = dict(ex=4, N=N, deform=True, Ma=0.1, Re=1600.0, surf=surf)
    o = orc.OracleSolver(**c)
    o.set_ic("tgv")
    U = o.state()
    Ro = o.residual()
    g = dg.Solver(**c, precision="fp32_bulk")
    g.set_state(U)
    Rg = g.residual()
    E, nn = 64, (N + 1) ** 3
    err = np.abs(Rg - Ro).reshape(E, 5, nn).max(axis=(0, 2)) / np.abs(Ro).reshape(E, 5, nn).max(axis=(0, 2))
    log(f"[FP32-bulk N={N} {surf}] rel err per var {err}")
    assert np.all(err < FP32_TOL), err


def test_fp32_bulk_conservation_drift(dg, orc):
    """20 RK3 steps of the 8^3, N=4 Navier-Stokes TGV in FP32-bulk and in FP64: the conserved
    totals drift only by rounding, and the FP32-bulk state stays close to the FP64 one."""
    c = dict(ex=8, N=4, deform=True, Ma=0.1, Re=1600.0)
    g64 = dg.Solver(**c)
    g32 = dg.Solver(**c, precision="fp32_bulk")
    g64.set_ic("tgv")
    g32.set_ic("tgv")
    d0 = g64.diagnostics()
    dt = g64.suggest_dt(0.5)
    g64.rk_step(dt, 20)
    g32.rk_step(dt, 20)
    d64, d32 = g64.diagnostics(), g32.diagnostics()
    V = d0["volume"]
    drift = {k: abs(d32[k] - d0[k]) / V for k in ("mass_rho", "mass_rhou", "mass_rhov", "mass_rhow", "mass_rhoE")}
    drift64 = {k: abs(d64[k] - d0[k]) / V for k in drift}
    log(f"[FP32-bulk drift per unit volume after 20 steps] fp32: {drift} fp64: {drift64}")
    assert drift["mass_rho"] < 1e-13
    assert all(drift[k] < 1e-7 for k in ("mass_rhou", "mass_rhov", "mass_rhow"))
    assert drift["mass_rhoE"] < 1e-9 * d0["mass_rhoE"] / V
    U64, U32 = g64.state(), g32.state()
    du = np.abs(U32 - U64).reshape(512, 5, 125).max(axis=(0, 2)) / np.abs(U64).reshape(512, 5, 125).max(axis=(0, 2))
    log(f"[FP32-bulk vs FP64 state after 20 steps] rel diff per var {du}")
    assert du.max() < 1e-4
    assert abs(d32["ke"] - d64["ke"]) < 1e-6 * d64["ke"]


def test_fp32_bulk_full_size(dg, orc):
    """The benchmark configuration (32^3, N=4, Navier-Stokes TGV) in FP32-bulk: residual error
    per conserved variable against the FP64 oracle."""
    c = dict(ex=32, N=4, deform=True, Ma=0.1, Re=1600.0)
    o = orc.OracleSolver(**c)
    o.set_ic("tgv")
    U = o.state()
    Ro = o.residual()
    g = dg.Solver(**c, precision="fp32_bulk")
    g.set_state(U)
    Rg = g.residual()
    E = 32768
    err = np.abs(Rg - Ro).reshape(E, 5, 125).max(axis=(0, 2)) / np.abs(Ro).reshape(E, 5, 125).max(axis=(0, 2))
    glob = np.abs(Rg - Ro).max() / np.abs(Ro).max()
    log(f"[FP32-bulk 32^3] rel err per var {err} global {glob:.2e}")
    assert np.all(err < FP32_TOLS["c2"]), err


# ------------------------------------------------------------------ full size
def test_full_size_c2_residual_and_step(dg, orc):
    """32^3 elements, N=4, deformed, Navier-Stokes TGV Re 1600 Ma 0.1 -- the benchmark
    configuration, in the launch configuration the benchmark times: every node's residual and
    the increment of one RK3 step against the oracle (double and long-double builds)."""
    c = dict(ex=32, N=4, deform=True, Ma=0.1, Re=1600.0)
    E, nn = 32768, 125
    log("C2 full size: oracle fp64")
    o = orc.OracleSolver(**c)
    o.set_ic("tgv")
    U = o.state()
    R64 = o.residual()
    log("C2 full size: oracle fp80")
    o80 = orc.OracleSolver(**c, precision="fp80")
    o80.set_state(U)
    R80 = o80.residual()
    log("C2 full size: gpu")
    g = dg.Solver(**c)
    g.set_ic("tgv")
    assert np.abs(g.state() - U).max() <= 1e-14 * np.abs(U).max()
    g.set_state(U)
    Rg = g.residual()
    assert_parity("C2 full size", Rg, R64, R80, E, nn)
    glob = np.abs(Rg - R80).max() / np.abs(R80).max()
    log(f"[C2] global relative Linf vs the long-double oracle {glob:.2e}")
    dt = o.suggest_dt(0.5)
    o.rk3(dt, 1)
    o80.rk3(dt, 1)
    g.rk_step(dt, 1)
    dG, d64, d80 = g.state() - U, o.state() - U, o80.state() - U
    sc = np.abs(d80).reshape(E, 5, nn).max(axis=(0, 2))
    eg = np.abs(dG - d80).reshape(E, 5, nn).max(axis=(0, 2))
    e64 = np.abs(d64 - d80).reshape(E, 5, nn).max(axis=(0, 2))
    log(f"[C2] one RK3 step, increment error: gpu-vs-fp80 {eg / sc} fp64-vs-fp80 {e64 / sc}")
    assert gate_ok("test_full_size_c2_residual_and_step", eg, e64, sc, 1e-12), "parity gate"
