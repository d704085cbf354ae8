"""Adaptive step size chosen on the device (dg_rk_step_adaptive).

- A step equals dg_rk_step with dg_suggest_dt of the same state, bit for bit, for uniform
  orders (Euler and Navier-Stokes, RK3 and RK4, FP32-bulk, the interior-penalty viscous flux,
  an extended flux family) and mixed orders, with graph replay on and off, and the time advanced
  is the sum of those step sizes.
- Against the oracle: the oracle takes its own suggested step before every step; the GPU
  trajectory lies within the parity bar of the long-double oracle's.
- A state that blows up is reported (DG_ENONFINITE) instead of being advanced further.
"""
import sys

import numpy as np

from helpers import GATE, gate_ok
import pytest

from paper_2206_09733_amd import synth

pytestmark = pytest.mark.gpu

VORTEX = [5.0, 0.0, 0.0, 0.4, 0.4]


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


CASES = {
    "euler_n3": (dict(ex=3, ey=2, ez=4, N=3, Ma=0.3, deform=True), "tgv", None),
    "ns_n4": (dict(ex=3, N=4, Ma=0.2, Re=400.0, deform=True), "tgv", None),
    "ns_n4_rk4": (dict(ex=3, N=4, Ma=0.2, Re=400.0, deform=True), "tgv", "rk4"),
    "ns_n4_fp32_bulk": (dict(ex=3, N=4, Ma=0.2, Re=400.0, deform=True, precision="fp32_bulk"), "tgv", None),
    "ns_n3_ip": (dict(ex=3, N=3, Ma=0.2, Re=400.0, deform=True, visc="ip"), "tgv", None),
    "euler_n4_kep_esm": (dict(ex=3, N=4, Ma=0.3, deform=True, vol="pirozzoli", surf="es_matrix"), "tgv", None),
    "mixed": (dict(ex=3, ey=3, ez=2, orders=synth.mixed_orders(18, seed=4), Ma=0.5, lo=(-10.0,) * 3,
                   hi=(10.0,) * 3), "vortex", None),
}


def make(dg, c, ic, scheme, graphs=True):
    s = dg.Solver(**c)
    s.set_ic(ic, VORTEX if ic == "vortex" else None)
    if scheme:
        s.set_scheme(scheme)
    s.use_graphs(graphs)
    return s


@pytest.mark.parametrize("case", list(CASES))
def test_adaptive_equals_suggested_fixed_steps(dg, case):
    c, ic, scheme = CASES[case]
    cfl, steps = 0.6, 6
    log(f"adaptive {case}")
    ref = make(dg, c, ic, scheme)
    dts = []
    for _ in range(steps):
        dts.append(ref.suggest_dt(cfl))
        ref.rk_step(dts[-1], 1)
    t_ref = 0.0
    for d in dts:
        t_ref += d
    Ur = ref.state()
    for graphs in (True, False):
        a = make(dg, c, ic, scheme, graphs)
        t = a.rk_step_adaptive(cfl, steps)
        Ua = a.state()
        log(f"[{case} graphs={graphs}] t={t!r} sum(dt)={t_ref!r} max|dU|={np.abs(Ua - Ur).max():.3e}")
        assert t == t_ref
        assert np.array_equal(Ua, Ur)
        # split calls continue where the first stopped (the graph of the other parity, a fresh time)
        b = make(dg, c, ic, scheme, graphs)
        t1 = b.rk_step_adaptive(cfl, 2)
        t2 = b.rk_step_adaptive(cfl, steps - 2)
        assert t1 == dts[0] + dts[1]
        assert np.array_equal(b.state(), Ur)
        assert t2 > 0
        a.close()
        b.close()
    ref.close()


def test_adaptive_against_oracle(dg, orc):
    """The oracle takes its own suggested step before each of 5 steps (FP64 and long double);
    the GPU's adaptive trajectory lies within GATE (2) times the FP64 oracle's distance to the long-double
    one, as every fixed-step trajectory does."""
    c = dict(ex=3, N=4, deform=True, Ma=0.1, Re=1600.0)
    o, o80 = orc.OracleSolver(**c), orc.OracleSolver(**c, precision="fp80")
    o.set_ic("tgv")
    U0 = o.state()
    o80.set_state(U0)
    for s in (o, o80):
        for _ in range(5):
            s.rk3(s.suggest_dt(0.5), 1)
    g = dg.Solver(**c)
    g.set_state(U0)
    g.rk_step_adaptive(0.5, 5)
    Ug, Uo, U80 = g.state(), o.state(), o80.state()
    d = lambda a, b: np.abs(a - b).reshape(27, 5, 125).max(axis=(0, 2))
    sc = np.abs(U80).reshape(27, 5, 125).max(axis=(0, 2))
    log(f"[adaptive NS] gpu-vs-fp80 {d(Ug, U80) / sc} fp64-vs-fp80 {d(Uo, U80) / sc}")
    assert gate_ok("test_adaptive_against_oracle", d(Ug, U80), d(Uo, U80), sc, 1e-14), "parity gate"


def test_adaptive_reports_blow_up_and_bad_arguments(dg):
    """At CFL 30 the explicit scheme is far outside its stability region and the state leaves the
    physical range within a few steps; the call reports it.  Non-positive CFL numbers and negative
    step counts are refused."""
    s = dg.Solver(ex=2, N=3, Ma=0.3)
    s.set_ic("tgv")
    for bad in (0.0, -1.0, float("nan")):
        with pytest.raises(dg.DgError) as ei:
            s.rk_step_adaptive(bad, 1)
        assert ei.value.code == dg.DG_EINVAL
    with pytest.raises(dg.DgError) as ei:
        s.rk_step_adaptive(0.5, -1)
    assert ei.value.code == dg.DG_EINVAL
    assert s.rk_step_adaptive(0.5, 0) == 0.0
    with pytest.raises(dg.DgError) as ei:
        s.rk_step_adaptive(30.0, 40)
    assert ei.value.code == dg.DG_ENONFINITE
    log(f"blow-up reported: {ei.value}")
    s.close()
