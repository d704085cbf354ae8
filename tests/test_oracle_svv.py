"""Pins of the oracle's spectral vanishing viscosity (section "Shock capturing").

- The modal filter: a product of Legendre polynomials is an eigenfunction with the kernel's value
  (numpy's Legendre series, not the oracle's, builds the modes); the filter is symmetric positive
  semi-definite in the nodal quadrature, and Tadmor's step kernel is a projection.
- The factorisation B = L^T D L: the unfiltered flux from entropy-variable gradients equals the
  Navier-Stokes viscous flux with the artificial viscosity, both gradients taken by central
  differences of the same smooth field.
- The discrete entropy identity: the entropy production of the SVV residual equals minus
  sum_m <y_m, F* y_m>, so it is never positive; totals of momentum and energy are conserved;
  a uniform state and a filter that passes nothing give a zero term.
- The sensor: the closed-form integral of J |grad_xi rho|^2 for a sine density wave; troubled
  elements take the unfiltered flux, which equals a filter that passes every mode.
"""
import math
import os

import numpy as np
import numpy.polynomial.legendre as npleg
import pytest

GAMMA = 1.4


def lobatto_nodes(orc, N):
    xi, w, D = orc.gll(N)
    return xi, w


def sigma(N, kernel, M, k):
    if k <= M:
        return 0.0
    if kernel == "tadmor":
        return 1.0
    return math.exp(-(((k - N) / (k - M)) ** 2))


@pytest.mark.parametrize("N", [2, 3, 4, 5, 7])
@pytest.mark.parametrize("kernel,M", [("maday", None), ("tadmor", None), ("maday", 0), ("tadmor", -1)])
def test_filter_multiplies_each_legendre_mode_by_the_kernel(orc, N, kernel, M):
    M = N // 2 if M is None else M
    xi, _ = lobatto_nodes(orc, N)
    Pm = [npleg.legval(xi, np.eye(N + 1)[a]) for a in range(N + 1)]
    rng = np.random.default_rng(N)
    for _ in range(6):
        a, b, c = rng.integers(0, N + 1, 3)
        f = np.einsum("k,j,i->kji", Pm[c], Pm[b], Pm[a]).reshape(-1)
        out = orc.svv_filter(N, f, kernel, M)
        s = 1 - (1 - sigma(N, kernel, M, a)) * (1 - sigma(N, kernel, M, b)) * (1 - sigma(N, kernel, M, c))
        assert np.abs(out - s * f).max() < 1e-12, (a, b, c, s)


@pytest.mark.parametrize("N", [3, 5, 6])
def test_filter_is_symmetric_semidefinite_and_tadmor_projects(orc, N):
    xi, w = lobatto_nodes(orc, N)
    W = np.einsum("k,j,i->kji", w, w, w).reshape(-1)
    rng = np.random.default_rng(7)
    f, g = rng.standard_normal((2, (N + 1) ** 3))
    for kernel in ("maday", "tadmor"):
        Ff, Fg = orc.svv_filter(N, f, kernel), orc.svv_filter(N, g, kernel)
        assert abs(np.sum(W * g * Ff) - np.sum(W * f * Fg)) < 1e-12 * np.sum(W * f * f)
        assert np.sum(W * f * Ff) > 0
    Tf = orc.svv_filter(N, f, "tadmor")
    assert np.abs(orc.svv_filter(N, Tf, "tadmor") - Tf).max() < 1e-12


def _prim(u):
    rho = u[0]
    v = u[1:4] / rho
    p = (GAMMA - 1) * (u[4] - 0.5 * rho * v @ v)
    return rho, v, p


@pytest.mark.parametrize("seed", range(4))
def test_unfiltered_flux_is_the_navier_stokes_viscous_flux(orc, seed):
    """L^T D L G with G = grad w equals F_v(mu_a) of grad(v, p/rho) of the same field."""
    rng = np.random.default_rng(seed)
    rho0, v0, p0 = 0.8 + 0.4 * rng.random(), rng.standard_normal(3) * 0.5, 0.7 + 0.6 * rng.random()
    du = rng.standard_normal((3, 5)) * 0.1  # the field's derivative along x, y, z

    def state(x):
        rho = rho0 + du[:, 0] @ x
        v = v0 + du[:, 1:4].T @ x
        p = p0 + du[:, 4] @ x
        return np.array([rho, *(rho * v), p / (GAMMA - 1) + 0.5 * rho * v @ v])

    h = 1e-5
    Gw, Gg = np.zeros(15), np.zeros(12)
    for x in range(3):
        e = np.zeros(3)
        e[x] = h
        up, um = state(e), state(-e)
        dw = (orc.entropy_vars(up) - orc.entropy_vars(um)) / (2 * h)
        rp, vp, pp = _prim(up)
        rm, vm, pm = _prim(um)
        dg = np.concatenate([(vp - vm), [pp / rp - pm / rm]]) / (2 * h)
        for c in range(5):
            Gw[3 * c + x] = dw[c]
        for c in range(4):
            Gg[3 * c + x] = dg[c]
    mu = 0.037
    u0 = state(np.zeros(3))
    Fa = orc.svv_flux(u0, Gw, mu)
    Fv = orc.viscous_flux(u0, Gg, GAMMA, 0.71, 1.0 / mu)
    assert np.abs(Fa - Fv).max() < 1e-8 * np.abs(Fv).max(), (Fa, Fv)
    assert np.all(Fa[:, 0] == 0)


def _perturbed(orc, c, seed):
    o = orc.OracleSolver(**c)
    o.set_ic("tgv")
    rng = np.random.default_rng(seed)
    U = o.state().reshape(o.E, 5, -1)
    U[:, 0] *= 1 + 0.05 * rng.standard_normal(U[:, 0].shape)
    U[:, 4] *= 1 + 0.05 * rng.standard_normal(U[:, 4].shape)
    o.set_state(U.reshape(-1))
    return o


@pytest.mark.parametrize("N,kernel,deform,Re", [(3, "maday", True, 0.0), (4, "tadmor", True, 100.0),
                                                (5, "maday", False, 0.0), (2, "tadmor", True, 0.0)])
def test_entropy_production_equals_minus_the_filtered_form(orc, N, kernel, deform, Re):
    o = _perturbed(orc, dict(ex=3, ey=2, ez=3, N=N, deform=deform, Ma=0.3, Re=Re), seed=N)
    o.set_svv(0.02, kernel)
    Ra, form = o.svv_residual()
    ep = o.entropy_production(Ra)
    assert form > 0
    assert abs(ep + form) < 1e-11 * form, (ep, form)
    # with an entropy-conserving baseline the whole residual dissipates exactly the SVV form
    if Re == 0.0:
        c = dict(ex=3, ey=2, ez=3, N=N, deform=deform, Ma=0.3, vol="ec", surf="ec")
        b = orc.OracleSolver(**c)
        b.set_state(o.state())
        b.set_svv(0.02, kernel)
        assert abs(b.entropy_production(b.residual()) + form) < 1e-9 * form


@pytest.mark.parametrize("N", [3, 4])
def test_svv_conserves_momentum_and_energy(orc, N):
    o = _perturbed(orc, dict(ex=2, ey=3, ez=2, N=N, deform=True, Ma=0.3), seed=11)
    o.set_svv(0.05)
    Ra, _ = o.svv_residual()
    Ja, J = o.metrics()
    _, w = lobatto_nodes(orc, N)
    W = np.einsum("k,j,i->kji", w, w, w).reshape(-1)
    R = Ra.reshape(o.E, 5, -1)
    Jn = J.reshape(o.E, -1)
    tot = np.einsum("evn,en,n->v", R, Jn, W)
    scale = np.einsum("evn,en,n->v", np.abs(R), Jn, W)
    assert np.all(R[:, 0] == 0)
    assert np.all(np.abs(tot[1:]) < 1e-13 * scale[1:].max()), tot


def test_uniform_state_and_a_filter_that_passes_nothing(orc):
    o = orc.OracleSolver(2, N=4, deform=True, Ma=0.3)
    o.set_ic("uniform", [1.2, 0.3, -0.2, 0.1, 0.9, 0, 0, 0, 0])
    o.set_svv(0.1)
    Ra, form = o.svv_residual()
    assert np.abs(Ra).max() < 1e-12 and abs(form) < 1e-20
    p = _perturbed(orc, dict(ex=2, N=4, deform=True, Ma=0.3), seed=3)
    p.set_svv(0.1, "tadmor", cutoff=4)  # every mode k <= M = N: the kernel is zero
    Ra, form = p.svv_residual()
    assert np.all(Ra == 0) and form == 0


def test_sensor_closed_form_for_a_sine_density_wave(orc):
    """rho = 1 + a sin x on an undeformed box: J |grad_xi rho|^2 integrates to
    (h_x/2)^2 a^2 h_y h_z int cos^2 x dx over the element."""
    ex, ey, ez, a = 3, 2, 2, 0.3
    o = orc.OracleSolver(ex, ey, ez, N=7, Ma=0.3)
    o.set_ic("density_wave", [a, 0.0, 0.0, 0.0, 1.0, 1.0, 0.0, 0.0, 0.0])
    s = o.svv_sensor()
    h = 2 * math.pi / np.array([ex, ey, ez])
    for e in range(o.E):
        i = e % ex
        x0, x1 = i * h[0], (i + 1) * h[0]
        icos2 = 0.5 * (x1 - x0) + 0.25 * (math.sin(2 * x1) - math.sin(2 * x0))
        ref = (h[0] / 2) ** 2 * a * a * h[1] * h[2] * icos2
        assert abs(s[e] - ref) < 1e-9 * ref, (e, s[e], ref)


def test_troubled_elements_take_the_unfiltered_flux(orc):
    c = dict(ex=2, ey=2, ez=3, N=4, deform=True, Ma=0.3)
    o = _perturbed(orc, c, seed=5)
    sens = o.svv_sensor()
    o.set_svv(0.03, "maday", sensor=0.0)  # every element troubled
    R_all, _ = o.svv_residual()
    o.set_svv(0.03, "tadmor", cutoff=-1)  # a filter that passes every mode
    R_id, _ = o.svv_residual()
    assert np.abs(R_all - R_id).max() < 1e-13 * np.abs(R_id).max()
    o.set_svv(0.03, "maday", sensor=2 * sens.max())  # none troubled
    R_none, _ = o.svv_residual()
    o.set_svv(0.03, "maday")
    R_off, _ = o.svv_residual()
    assert np.array_equal(R_none, R_off)
    thr = float(np.median(sens))
    o.set_svv(0.03, "maday", sensor=thr)  # some troubled, some not
    R_mix, _ = o.svv_residual()
    assert not np.array_equal(R_mix, R_off) and not np.array_equal(R_mix, R_id)


def test_svv_rejects_what_it_does_not_cover(orc):
    g = orc.OracleSolver(2, N=3, Ma=0.3, vol="central", nodes="gauss")
    with pytest.raises(ValueError):
        g.set_svv(0.1)
    o = orc.OracleSolver(2, N=3, Ma=0.3)
    for bad in (dict(mu_a=-1.0), dict(mu_a=0.1, cutoff=4), dict(mu_a=0.1, cutoff=-2)):
        with pytest.raises(ValueError):
            o.set_svv(**bad)


def test_entropy_form_does_not_depend_on_the_thread_count():
    """The oracle's entropy form and SVV residual are the same, bit for bit, with 1 and 4 OpenMP
    threads (its per-element terms are summed in element order)."""
    import subprocess
    import sys
    code = ("import numpy as np, oracle\n"
            "o = oracle.OracleSolver(ex=3, ey=2, ez=3, N=3, deform=True, Ma=0.3)\n"
            "o.set_ic('tgv')\n"
            "U = o.state().reshape(o.E, 5, -1)\n"
            "U[:, 0] *= 1 + 0.05 * np.random.default_rng(3).standard_normal(U[:, 0].shape)\n"
            "o.set_state(U.reshape(-1))\n"
            "o.set_svv(0.02, 'maday')\n"
            "R, f = o.svv_residual()\n"
            "print(float(f).hex(), __import__('hashlib').sha1(R.tobytes()).hexdigest())\n")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    out = []
    for t in ("1", "4"):
        env = dict(os.environ, OMP_NUM_THREADS=t)
        r = subprocess.run([sys.executable, "-c", code], cwd=root, env=env, capture_output=True, text=True,
                           timeout=120)
        assert r.returncode == 0, r.stderr
        out.append(r.stdout.strip())
    assert out[0] == out[1], out
