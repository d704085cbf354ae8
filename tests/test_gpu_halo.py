"""Halo boxes on the GPU: the box run as one block of a split domain, its periodic neighbours reached
through ghost elements that a halo exchange (pack, transfer, unpack) fills before every stage.

Every comparison is bitwise against the same box with direct periodic neighbours: the ghosts hold
exact copies of the neighbours' face values, so each kernel sees the same operands in the same
order.  Residuals, RK3 steps (graph replay and eager), the adaptive step and the diagnostics;
Euler and Navier-Stokes (BR1, BR2, the interior penalty), FP64 and FP32-bulk, the extended flux
family, the global Lax-Friedrichs flux, spectral vanishing viscosity on its folded and unfolded
routes and an LES closure, one element across a direction, and the real share of a split 64^3
N=5 run (a 32^3 block).  A batch refuses a halo box.
"""
import sys

import numpy as np
import pytest

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


CASES = {
    "euler_fp64": dict(ex=3, ey=2, ez=4, N=3, Ma=0.3),
    "ns_br1_deformed": dict(ex=4, ey=3, ez=2, N=4, deform=True, Ma=0.3, Re=200.0),
    "ns_br2": dict(ex=2, ey=2, ez=3, N=2, Ma=0.3, Re=200.0, visc="br2"),
    "ns_fp32_bulk": dict(ex=3, ey=3, ez=3, N=4, deform=True, Ma=0.2, Re=400.0, precision="fp32_bulk"),
    "kg_es_matrix": dict(ex=2, ey=3, ez=2, N=3, Ma=0.3, Re=300.0, vol="kg", surf="es_matrix"),
    "lf_global": dict(ex=3, ey=2, ez=2, N=3, Ma=0.3, surf="lf_global"),
    "one_element_ns": dict(ex=1, ey=1, ez=1, N=3, Ma=0.3, Re=100.0),
    "thin_box": dict(ex=5, ey=1, ez=2, N=2, Ma=0.3, Re=100.0, hi=(1.0, 0.5, 2.0)),
    # the interior penalty reads the neighbour's J on the face: the ghosts' faces hold it
    "ns_ip": dict(ex=3, ey=2, ez=2, N=3, deform=True, Ma=0.3, Re=200.0, visc="ip"),
    # spectral vanishing viscosity: the filtered flux's face components are exchanged too
    "svv_ns_br1": dict(ex=3, ey=3, ez=2, N=4, deform=True, Ma=0.3, Re=200.0, svv_mu=0.02, svv_kernel="maday",
                       svv_cutoff=2),
    "svv_ns_br2_fp32_bulk": dict(ex=2, ey=3, ez=2, N=4, Ma=0.2, Re=300.0, visc="br2", svv_mu=0.02,
                                 svv_kernel="tadmor", svv_cutoff=2, precision="fp32_bulk"),
    "svv_euler": dict(ex=3, ey=2, ez=3, N=3, Ma=0.3, svv_mu=0.02, svv_kernel="maday", svv_cutoff=1),
    "svv_kg_es_matrix": dict(ex=2, ey=2, ez=3, N=3, Ma=0.3, Re=300.0, vol="kg", surf="es_matrix", svv_mu=0.02,
                             svv_kernel="maday", svv_cutoff=1),
    "les_wale": dict(ex=3, ey=2, ez=2, N=4, deform=True, Ma=0.3, Re=200.0, les_cs=0.5, les_model="wale",
                     svv_kernel="tadmor", svv_cutoff=-1),
    "svv_one_element_across": dict(ex=1, ey=3, ez=2, N=3, Ma=0.3, Re=100.0, svv_mu=0.02, svv_cutoff=1),
}


@pytest.mark.parametrize("name", list(CASES))
def test_halo_equals_direct_bitwise(dg, name):
    c = CASES[name]
    log(f"halo {name}")
    a, h = dg.Solver(**c), dg.Solver(**c, halo=True)
    for s in (a, h):
        s.set_ic("tgv")
    assert np.array_equal(a.residual(), h.residual())
    dt = a.suggest_dt(0.5)
    for s in (a, h):
        s.rk_step(dt, 3)
    assert np.array_equal(a.state(), h.state())
    for s in (a, h):  # eager launches, then graph replay again
        s.use_graphs(False)
        s.rk_step(dt, 1)
        s.use_graphs(True)
        s.rk_step(dt, 2)
    assert np.array_equal(a.state(), h.state())
    da, dh = a.diagnostics(), h.diagnostics()
    assert all(da[k] == dh[k] for k in da), (da, dh)
    a.close()
    h.close()


def test_halo_adaptive_step_equals_direct(dg):
    c = dict(ex=3, ey=3, ez=2, N=4, deform=True, Ma=0.3, Re=300.0)
    a, h = dg.Solver(**c), dg.Solver(**c, halo=True)
    for s in (a, h):
        s.set_ic("tgv")
    ta, th = a.rk_step_adaptive(0.5, 4), h.rk_step_adaptive(0.5, 4)
    assert ta == th
    assert np.array_equal(a.state(), h.state())
    a.close()
    h.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32_bulk"])
def test_halo_real_share_of_a_split_run(dg, precision):
    """A 32^3 block of order 5 (one GPU's share of the 64^3 N=5 Navier-Stokes TGV split in eight):
    residual and one RK3 step equal the direct box bitwise."""
    c = dict(ex=32, N=5, deform=True, Ma=0.1, Re=1600.0, precision=precision)
    a, h = dg.Solver(**c), dg.Solver(**c, halo=True)
    for s in (a, h):
        s.set_ic("tgv")
    assert np.array_equal(a.residual(), h.residual())
    dt = a.suggest_dt(0.5)
    for s in (a, h):
        s.rk_step(dt, 1)
    assert np.array_equal(a.state(), h.state())
    log(f"halo 32^3 N=5 {precision}: bitwise equal")
    a.close()
    h.close()


def test_batch_refuses_a_halo_box(dg):
    h = dg.Solver(ex=2, N=3, halo=True)
    p = dg.Solver(ex=2, N=3)
    with pytest.raises(dg.DgError) as ei:
        dg.Batch([p, h])
    assert ei.value.code == dg.DG_EUNSUPPORTED
    h.close()
    p.close()
