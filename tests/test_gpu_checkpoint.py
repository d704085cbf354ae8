"""Checkpoint / resume through the C ABI: a run that stops, saves its state with dg_get_state,
and continues in a fresh solver from dg_set_state reproduces the uninterrupted run bit for bit
(FP64: uniform Navier-Stokes with RK3 and RK4, a mixed-order Euler mesh, graph replay on both
sides).  In FP32-bulk the deviation form's reference state (mean density and pressure) is
recomputed from the state handed to dg_set_state, so a resumed run matches to rounding only:
both runs lie within the FP32-bulk tolerance of the FP64 result, so they are checked against each
other within twice that tolerance, relative to the increment."""
import numpy as np
import pytest

from helpers import FP32_TOL
from paper_2206_09733_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dg():
    from paper_2206_09733_amd import dgsem
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    dgsem.lib()
    return dgsem


CASES = {
    "ns_rk3": (dict(ex=4, N=4, deform=True, Ma=0.1, Re=1600.0), "rk3", "tgv", None),
    "ns_rk4": (dict(ex=3, N=5, deform=True, Ma=0.3, Re=800.0), "rk4", "tgv", None),
    "mixed_euler": (dict(ex=4, orders=synth.mixed_orders(64, seed=6), Ma=0.5, lo=(-10.0,) * 3, hi=(10.0,) * 3),
                    "rk3", "vortex", [5.0, 0.0, 0.0, 0.4, 0.4]),
}


@pytest.mark.parametrize("case", list(CASES))
def test_resume_is_bitwise(dg, case):
    c, scheme, ic, params = CASES[case]
    print(f"[checkpoint] {case}", flush=True)
    ref = dg.Solver(**c)
    ref.set_scheme(scheme)
    ref.set_ic(ic, params)
    dt = ref.suggest_dt(0.4)
    ref.rk_step(dt, 11)          # 8-step graph + 3 single steps
    saved = ref.state()
    ref.rk_step(dt, 9)
    U_ref = ref.state()
    ref.close()
    res = dg.Solver(**c)
    res.set_scheme(scheme)
    res.set_state(saved)
    res.rk_step(dt, 9)
    assert np.array_equal(res.state(), U_ref), np.abs(res.state() - U_ref).max()
    res.close()


def test_resume_fp32_bulk_within_tolerance(dg):
    c = dict(ex=4, N=4, deform=True, Ma=0.1, Re=1600.0, precision="fp32_bulk")
    ref = dg.Solver(**c)
    ref.set_ic("tgv")
    dt = ref.suggest_dt(0.5)
    ref.rk_step(dt, 6)
    saved = ref.state()
    ref.rk_step(dt, 6)
    U_ref = ref.state()
    ref.close()
    res = dg.Solver(**c)
    res.set_state(saved)
    res.rk_step(dt, 6)
    U = res.state()
    res.close()
    E, nn = 64, 125
    d_ref = (U_ref - saved).reshape(E, 5, nn)
    err = np.abs(U.reshape(E, 5, nn) - U_ref.reshape(E, 5, nn)).max(axis=(0, 2)) / np.abs(d_ref).max(axis=(0, 2))
    print(f"[checkpoint fp32-bulk] resumed vs uninterrupted, relative to the increment {err}", flush=True)
    assert np.all(err < 2 * FP32_TOL["small"]), err
