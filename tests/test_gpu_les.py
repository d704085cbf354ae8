"""Explicit LES closures on the GPU (turbulence models: Smagorinsky, WALE, Vreman and
SVV-Smagorinsky) against the oracle: the model's eddy viscosity joins the artificial viscosity of
the SVV term node by node.

- Residuals of perturbed states on deformed meshes for orders 1..7: SVV-Smagorinsky (Maday kernel)
  on Euler, the plain Smagorinsky, WALE and Vreman models (every mode kept) on Navier-Stokes, and
  the closure added to a constant artificial viscosity, to the parity bar (within GATE times the FP64 oracle's
  distance to the long-double oracle, or 1e-12 relative); with the density sensor marking some
  elements.
- The closure's term alone (GPU residual with it minus without) against the oracle's term.
- RK3 trajectories against the oracle; graph replay agrees bitwise with eager steps.
"""
import sys

import numpy as np
import pytest

from helpers import GATE, gate_ok
from paper_2206_09733_amd import synth

pytestmark = pytest.mark.gpu


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


def perturbed(orc, c, seed, amp=(0.03, 0.05, 0.03)):
    o = orc.OracleSolver(**c)
    o.set_ic("tgv")
    nn = (c["N"] + 1) ** 3
    U0 = o.state().reshape(o.E, 5, nn).transpose(0, 2, 1).reshape(-1, 5)
    drho, dv, dp = synth.primitive_perturbation(o.nodes, seed, amp)
    rho = U0[:, 0] * (1 + drho)
    v = U0[:, 1:4] / U0[:, :1] + dv.T
    p = 0.4 * (U0[:, 4] - 0.5 * (U0[:, 1:4] ** 2).sum(1) / U0[:, 0]) * (1 + dp)
    U = np.concatenate([rho[:, None], rho[:, None] * v, (p / 0.4 + 0.5 * rho * (v * v).sum(1))[:, None]], 1)
    return U.reshape(o.E, nn, 5).transpose(0, 2, 1).reshape(-1)


def parity(name, G, A, B, E, nn, factor=GATE):
    G, A, B = (x.reshape(E, 5, nn) for x in (G, A, B))
    scale = np.abs(B).max(axis=(0, 2))
    e64 = np.abs(A - B).max(axis=(0, 2))
    eg = np.abs(G - B).max(axis=(0, 2))
    tol = np.maximum(1e-12 * scale, factor * e64)
    log(f"[{name}] gpu-vs-fp80={np.array2string(eg, precision=2)} fp64-vs-fp80={np.array2string(e64, precision=2)}")
    assert gate_ok(name, eg, e64, scale) and np.all(eg <= tol), (name, eg, tol)


def oracles(orc, c, U, les):
    out = []
    for prec in ("fp64", "fp80"):
        o = orc.OracleSolver(**c, precision=prec)
        o.set_state(U)
        o.set_les(les["cs"], les.get("model", "smagorinsky"))
        o.set_svv(les["mu"], les["kernel"], les["cutoff"], les.get("sensor", -1.0))
        out.append(o)
    return out


def gpu_solver(dg, c, les):
    return dg.Solver(**c, svv_mu=les["mu"], svv_kernel=les["kernel"], svv_cutoff=les["cutoff"],
                     svv_sensor=les.get("sensor", -1.0), les_cs=les["cs"],
                     les_model=les.get("model", "smagorinsky"))


# (kernel, cutoff, Re, constant artificial viscosity, LES model): SVV-Smagorinsky, the plain
# Smagorinsky, WALE and Vreman models, SVV-Smagorinsky on top of a constant viscosity
MODELS = {"svv_smagorinsky": ("maday", None, 0.0, 0.0, "smagorinsky"),
          "smagorinsky": ("tadmor", -1, 200.0, 0.0, "smagorinsky"),
          "wale": ("tadmor", -1, 200.0, 0.0, "wale"), "vreman": ("tadmor", -1, 200.0, 0.0, "vreman"),
          "svv_plus_smagorinsky": ("maday", None, 0.0, 0.01, "smagorinsky")}
# the models' usual constants: C_s, C_w (Nicoud and Ducros), c = 2.5 C_s^2 (Vreman)
CONST = {"smagorinsky": 0.17, "wale": 0.5, "vreman": 0.07}
CASES = [(N, m) for N in range(1, 8) for m in MODELS]


def les_args(model, N):
    kernel, cut, Re, mu, lm = MODELS[model]
    return Re, dict(cs=CONST[lm], mu=mu, kernel=kernel, cutoff=N // 2 if cut is None else cut, model=lm)


@pytest.mark.parametrize("N,model", CASES)
def test_les_residual_parity(dg, orc, N, model):
    Re, les = les_args(model, N)
    c = dict(ex=3, ey=2, ez=3, N=N, deform=True, Ma=0.3, Re=Re)
    log(f"les residual N={N} {model}")
    U = perturbed(orc, c, seed=1500 + N)
    o64, o80 = oracles(orc, c, U, les)
    g = gpu_solver(dg, c, les)
    g.set_state(U)
    parity(f"les N={N} {model}", g.residual(), o64.residual(), o80.residual(), 18, (N + 1) ** 3)
    g.close()


@pytest.mark.parametrize("N,model", [(N, m) for N in (2, 4, 6) for m in MODELS])
def test_les_part_alone(dg, orc, N, model):
    """The closure's term by itself (a few percent of the residual): the GPU's residual with the
    term minus its residual without, against the oracle's term.  The difference carries the
    rounding of the two full residuals: on Euler (the term added by its own kernels after the
    stage kernel) the bar is the parity gate or 1e-15 of the full residual, whichever is larger;
    on Navier-Stokes the term is folded into the stage kernel's viscous flux, so the two full
    residuals round apart and the bar is the sum of their two parity gates."""
    Re, les = les_args(model, N)
    c = dict(ex=3, ey=2, ez=3, N=N, deform=True, Ma=0.3, Re=Re)
    U = perturbed(orc, c, seed=1700 + N)
    o64, o80 = oracles(orc, c, U, les)
    a64, a80 = o64.svv_residual()[0], o80.svv_residual()[0]
    g, p = gpu_solver(dg, c, les), dg.Solver(**c)
    for s in (g, p):
        s.set_state(U)
    Rg = g.residual()
    part = Rg - p.residual()
    nn, E = (N + 1) ** 3, 18
    B, A, G = (x.reshape(E, 5, nn) for x in (a80, a64, part))
    sc = np.abs(B).max(axis=(0, 2))
    e64, eg = np.abs(A - B).max(axis=(0, 2)), np.abs(G - B).max(axis=(0, 2))
    floor = 1e-15 * np.abs(Rg.reshape(E, 5, nn)).max(axis=(0, 2))
    if Re > 0:  # folded: the gates of the full residual with the term and of the one without
        p64, p80 = orc.OracleSolver(**c), orc.OracleSolver(**c, precision="fp80")
        for o in (p64, p80):
            o.set_state(U)
        err = lambda a, b: np.abs(a - b).reshape(E, 5, nn).max(axis=(0, 2))  # noqa: E731
        floor = np.maximum(floor, GATE * (err(o64.residual(), o80.residual()) + err(p64.residual(), p80.residual())))
    log(f"[les part N={N} {model}] |part|/|R| {sc[1:] / np.abs(Rg.reshape(E, 5, nn)).max(axis=(0, 2))[1:]} "
        f"gpu-vs-fp80 {eg[1:] / sc[1:]} fp64-vs-fp80 {e64[1:] / sc[1:]}")
    assert np.all(B[:, 0] == 0) and np.all(np.abs(G[:, 0]) <= floor[0])
    assert np.all(eg[1:] <= np.maximum(GATE * e64[1:], floor[1:])), (eg, e64, floor)
    g.close()
    p.close()


@pytest.mark.parametrize("N", [3, 5])
def test_les_with_sensor_marking_some_elements(dg, orc, N):
    c = dict(ex=3, ey=3, ez=2, N=N, deform=True, Ma=0.3)
    U = perturbed(orc, c, seed=1600 + N, amp=(0.08, 0.05, 0.05))
    o = orc.OracleSolver(**c)
    o.set_state(U)
    s = np.sort(o.svv_sensor())
    lo, hi = len(s) // 4, 3 * len(s) // 4
    k = lo + int(np.argmax(np.diff(s[lo:hi + 1])))
    thr = 0.5 * (s[k] + s[k + 1])
    assert (s[k + 1] - s[k]) > 1e-6 * s[k + 1]
    les = dict(cs=0.15, mu=0.0, kernel="maday", cutoff=N // 2, sensor=thr)
    log(f"les sensor N={N}: threshold {thr:.6g}, {len(s) - k - 1} troubled")
    o64, o80 = oracles(orc, c, U, les)
    g = gpu_solver(dg, c, les)
    g.set_state(U)
    parity(f"les sensor N={N}", g.residual(), o64.residual(), o80.residual(), 18, (N + 1) ** 3)
    g.close()


@pytest.mark.parametrize("model", ["svv_smagorinsky", "smagorinsky", "wale", "vreman"])
def test_les_trajectory(dg, orc, model):
    Re, les = les_args(model, 4)
    c = dict(ex=3, N=4, deform=True, Ma=0.3, Re=Re)
    U0 = perturbed(orc, c, seed=51, amp=(0.02, 0.03, 0.02))
    o, o80 = oracles(orc, c, U0, les)
    dt = o.suggest_dt(0.4)
    o.rk(dt, 5, "rk3")
    o80.rk(dt, 5, "rk3")
    g = gpu_solver(dg, c, les)
    g.set_state(U0)
    g.rk_step(dt, 5)
    Ug, Uo, U80 = g.state(), o.state(), o80.state()
    d = lambda a, b: np.abs(a - b).reshape(27, 5, 125).max(axis=(0, 2))
    sc = np.abs(U80).reshape(27, 5, 125).max(axis=(0, 2))
    log(f"[les {model}] gpu-vs-fp80 {d(Ug, U80) / sc} fp64-vs-fp80 {d(Uo, U80) / sc}")
    assert gate_ok(f"test_les_trajectory {model}", d(Ug, U80), d(Uo, U80), sc, 1e-14), "parity gate"
    g.close()


@pytest.mark.parametrize("model", ["smagorinsky", "wale", "vreman"])
def test_les_graph_replay_equals_eager(dg, model):
    c = dict(ex=3, ey=3, ez=2, N=4, deform=True, Ma=0.3, Re=400.0, svv_kernel="maday", svv_cutoff=2,
             les_cs=CONST[model], les_model=model)
    eager, graph = dg.Solver(**c), dg.Solver(**c)
    for s in (eager, graph):
        s.set_ic("tgv")
    eager.use_graphs(False)
    dt = eager.suggest_dt(0.5)
    eager.rk_step(dt, 10)
    graph.rk_step(dt, 10)
    assert np.array_equal(graph.state(), eager.state())
    eager.close()
    graph.close()
