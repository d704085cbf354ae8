"""Edge meshes on the newer paths, against the oracle: one element across a direction (the element
is its own periodic neighbour on that face), element counts that are not multiples of 8, a
non-cubic box.

- Gauss-Legendre points with BR1, BR2 and the interior penalty (the face factors of the penalty
  and of BR2's lift formed once after the geometry; both sides of a face are then one element).
- Spectral vanishing viscosity on all three routes: Navier-Stokes with BR1 (the gradient pass and
  the filtered flux in one launch, folded into the stage kernel), Navier-Stokes with BR2 (the
  flux kernel alone, folded), Euler (the correction after the stage kernel); and an explicit LES
  closure (WALE).
The bar is the parity gate (GATE times the FP64 oracle's distance to the long-double oracle, or
1e-12 relative).
"""
import sys

import numpy as np
import pytest

from helpers import GATE, gate_ok
from paper_2206_09733_amd import synth

pytestmark = pytest.mark.gpu

MESHES = [dict(ex=1, ey=1, ez=1, N=3), dict(ex=1, ey=3, ez=2, N=4, deform=True),
          dict(ex=5, ey=3, ez=1, N=2, hi=(1.0, 2.0, 0.5))]


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


def parity(name, G, A, B, E, nn):
    G, A, B = (x.reshape(E, 5, nn) for x in (G, A, B))
    scale = np.abs(B).max(axis=(0, 2))
    e64 = np.abs(A - B).max(axis=(0, 2))
    eg = np.abs(G - B).max(axis=(0, 2))
    tol = np.maximum(1e-12 * scale, GATE * e64)
    log(f"[{name}] gpu-vs-fp80={np.array2string(eg, precision=2)} fp64-vs-fp80={np.array2string(e64, precision=2)}")
    assert gate_ok(name, eg, e64, scale) and np.all(eg <= tol), (name, eg, tol)


def run_case(dg, orc, name, c, gpu_kw, setup, seed):
    E = c["ex"] * c["ey"] * c["ez"]
    log(f"edge {name} {c}")
    U = perturbed(orc, c, seed)
    res = []
    for prec in ("fp64", "fp80"):
        o = orc.OracleSolver(**c, precision=prec)
        o.set_state(U)
        setup(o)
        res.append(o.residual())
    g = dg.Solver(**c, **gpu_kw)
    g.set_state(U)
    parity(f"edge {name} {c['ex']}x{c['ey']}x{c['ez']}", g.residual(), res[0], res[1], E, (c["N"] + 1) ** 3)
    g.close()


@pytest.mark.parametrize("mesh", range(len(MESHES)))
@pytest.mark.parametrize("visc", ["br1", "br2", "ip"])
def test_gauss_edge_meshes(dg, orc, mesh, visc):
    c = dict(MESHES[mesh], Ma=0.3, Re=80.0, vol="central", surf="roe", nodes="gauss", visc=visc)
    run_case(dg, orc, f"gauss {visc}", c, {}, lambda o: None, seed=3000 + mesh)


SVV_ROUTES = {"ns_br1": dict(Re=150.0), "ns_br2": dict(Re=150.0, visc="br2"), "euler": dict(Re=0.0)}


@pytest.mark.parametrize("mesh", range(len(MESHES)))
@pytest.mark.parametrize("route", list(SVV_ROUTES))
def test_svv_edge_meshes(dg, orc, mesh, route):
    c = dict(MESHES[mesh], Ma=0.3, **SVV_ROUTES[route])
    cut = c["N"] // 2
    run_case(dg, orc, f"svv {route}", c, dict(svv_mu=0.02, svv_kernel="maday", svv_cutoff=cut),
             lambda o: o.set_svv(0.02, "maday", cut, -1.0), seed=3100 + mesh)


@pytest.mark.parametrize("mesh", range(len(MESHES)))
def test_les_edge_meshes(dg, orc, mesh):
    c = dict(MESHES[mesh], Ma=0.3, Re=200.0)

    def setup(o):
        o.set_les(0.5, "wale")
        o.set_svv(0.0, "tadmor", -1, -1.0)

    run_case(dg, orc, "les wale", c, dict(svv_kernel="tadmor", svv_cutoff=-1, les_cs=0.5, les_model="wale"),
             setup, seed=3200 + mesh)
