"""Pins of the oracle's Gauss-Legendre path on the deformed (curvilinear) box.

Reading: on Gauss-Legendre points the map and its metric terms are those of the Lobatto grid of
the same order (the isoparametric map there, metric terms in the conservative curl form there),
evaluated as the polynomials they are at the Gauss points; J is the determinant of that map's
Jacobian at the Gauss points.  The paper leaves the geometry of curvilinear elements to its
cited free-stream rules; this is the route that keeps a uniform state steady.

- The Gauss solver's coordinates and metric terms equal the Lobatto solver's (same mesh, same
  order) interpolated to the Gauss points by numpy's barycentric Lagrange interpolation; its J
  is positive and gives each element's volume within the quadrature error of the Lobatto
  solver's.
- A uniform state stays steady at orders 1-7, Euler and Navier-Stokes, for several surface fluxes
  (the metric computed by the curl form at the Gauss points instead leaves 1e-5..1e-3).
- Totals sum w J dU/dt vanish on the deformed mesh (single-valued face metrics and fluxes).
- Spectral convergence of a density wave on the deformed mesh.
"""
import math

import numpy as np
import pytest

from helpers import quad_weights_uniform


def lagrange_matrix(xs, ys):
    """M[g][l]: the Lagrange polynomial of node l over xs at point ys[g] (barycentric form)."""
    xs, ys = np.asarray(xs, float), np.asarray(ys, float)
    n = len(xs)
    wb = np.array([1.0 / np.prod([xs[l] - xs[m] for m in range(n) if m != l]) for l in range(n)])
    M = np.zeros((len(ys), n))
    for g, y in enumerate(ys):
        diff = y - xs
        if np.any(diff == 0):
            M[g, np.argmin(np.abs(diff))] = 1.0
            continue
        t = wb / diff
        M[g] = t / t.sum()
    return M


def interp3(M, f, n):
    """Tensor-product interpolation of nodal fields f[..., k, j, i] (n^3 values) by M."""
    f = f.reshape(f.shape[:-1] + (n, n, n))
    f = np.einsum("gl,...kjl->...kjg", M, f)
    f = np.einsum("gl,...klj->...kgj", M, f)
    f = np.einsum("gl,...lkj->...gkj", M, f)
    return f.reshape(f.shape[:-3] + (n ** 3,))


@pytest.mark.parametrize("N", [1, 2, 3, 4, 5, 7])
def test_gauss_geometry_is_the_lobatto_geometry_at_the_gauss_points(orc, N):
    n = N + 1
    c = dict(ex=3, ey=2, ez=3, N=N, deform=True, Ma=0.3, vol="central", surf="roe")
    g, l = orc.OracleSolver(**c, nodes="gauss"), orc.OracleSolver(**c)
    xg, _, _, _ = orc.gl(N)
    xl, wl, _ = orc.gll(N)
    M = lagrange_matrix(xl, xg)
    Xg, Xl = g.coords().reshape(g.E, 3, -1), l.coords().reshape(l.E, 3, -1)
    (Jag, Jg), (Jal, Jl) = g.metrics(), l.metrics()
    Jag, Jal = Jag.reshape(g.E, 9, -1), Jal.reshape(l.E, 9, -1)
    assert np.abs(Xg - interp3(M, Xl, n)).max() < 1e-13
    scale = np.abs(Jal).max()
    assert np.abs(Jag - interp3(M, Jal, n)).max() < 1e-13 * scale, np.abs(Jag - interp3(M, Jal, n)).max() / scale
    # J: the element volumes by each node set's quadrature.  J is a polynomial of degree 3N per
    # direction, which neither rule integrates exactly, so the two volumes agree to the
    # quadrature error, which the deformation's smoothness keeps small.
    _, wg, _, _ = orc.gl(N)
    vg = (quad_weights_uniform(np.asarray(wg), g.E) * Jg).reshape(g.E, -1).sum(1)
    vl = (quad_weights_uniform(np.asarray(wl), l.E) * Jl).reshape(l.E, -1).sum(1)
    assert np.all(Jg > 0)
    assert np.abs(vg - vl).max() < (1e-3 if N < 3 else 1e-6) * vl.max()


@pytest.mark.parametrize("N", range(1, 8))
@pytest.mark.parametrize("Re,surf", [(0.0, "roe"), (0.0, "llf"), (0.0, "es"), (200.0, "roe")])
def test_gauss_freestream_on_the_deformed_box(orc, N, Re, surf):
    o = orc.OracleSolver(3, 2, 3, N=N, deform=True, Ma=0.3, Re=Re, vol="central", surf=surf, nodes="gauss")
    o.set_ic("uniform", [1.2, 0.3, -0.2, 0.1, 0.9, 0, 0, 0, 0])
    assert np.abs(o.residual()).max() < 1e-11


@pytest.mark.parametrize("N,Re", [(3, 0.0), (4, 150.0), (6, 0.0)])
def test_gauss_conservation_on_the_deformed_box(orc, N, Re):
    s = orc.OracleSolver(3, 2, 3, N=N, deform=True, Ma=0.4, Re=Re, vol="central", surf="roe", nodes="gauss")
    s.set_ic("tgv")
    rng = np.random.default_rng(N)
    U = s.state().reshape(s.E, 5, -1)
    U[:, 0] *= 1 + 0.05 * rng.standard_normal(U[:, 0].shape)
    U[:, 4] *= 1 + 0.05 * rng.standard_normal(U[:, 4].shape)
    s.set_state(U.reshape(-1))
    R = s.residual()
    _, w, _, _ = orc.gl(N)
    _, J = s.metrics()
    wq = (quad_weights_uniform(np.asarray(w), s.E) * J).reshape(s.E, -1)
    Rv = R.reshape(s.E, 5, -1)
    tot = np.einsum("en,evn->v", wq, Rv)
    mag = np.einsum("en,evn->v", wq, np.abs(Rv))
    assert np.all(np.abs(tot) < 1e-12 * mag.max()), (tot, mag)


def test_gauss_density_wave_converges_spectrally_on_the_deformed_box(orc):
    """rho = 1 + 0.2 sin(x + y) in a uniform stream (0.7, 0.4, 0), p = 1, advected to t = 0.5 with
    RK4 at a small step on the deformed 3^3 box: the error falls spectrally with N, and below the
    Lobatto points' at every N (the paper's accuracy statement, here on curvilinear elements)."""
    T = 0.5
    errs = {"gauss": [], "lobatto": []}
    for N in (2, 3, 4, 5):
        for nodes in ("gauss", "lobatto"):
            kw = dict(vol="central", surf="roe", deform=True, Ma=0.5)
            if nodes == "gauss":
                kw["nodes"] = "gauss"
            s = orc.OracleSolver(3, N=N, **kw)
            s.set_ic("density_wave", [0.2, 0.7, 0.4, 0.0, 1.0, 1.0, 1.0, 0.0, 0.0])
            dt = s.suggest_dt(0.05)
            steps = int(math.ceil(T / dt))
            s.rk(T / steps, steps, "rk4")
            ex = orc.OracleSolver(3, N=N, **kw)
            ex.set_ic("density_wave", [0.2, 0.7, 0.4, 0.0, 1.0, 1.0, 1.0, 0.0, -(0.7 + 0.4) * T])
            errs[nodes].append(np.abs(s.state() - ex.state()).reshape(s.E, 5, -1)[:, 0].max())
    g, l = np.array(errs["gauss"]), np.array(errs["lobatto"])
    assert np.all(g[:-1] / g[1:] > 4), g
    assert np.all(g < l), (g, l)
