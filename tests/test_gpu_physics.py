"""A physical check of the Navier-Stokes path on the GPU, independent of the oracle: the kinetic
energy budget of the compressible Taylor-Green vortex at Ma 0.1, Re 1600 (periodic box, an
undeformed 16^3 mesh of order 4).

For the compressible equations the volume mean K of rho|v|^2/2 changes at
    dK/dt = <p div v> - <tau : grad v>,   tau = mu (grad v + grad v^T - 2/3 (div v) I),
and only the pressure fluctuation does work on a periodic box.  The scheme's own rate follows
from a residual R = dU/dt by the chain rule, dK/dt = <v . R_m - |v|^2/2 R_rho>; its viscous part
is the rate of the Navier-Stokes residual minus that of an Euler solver given the same state.
The two volume terms are formed on the host from the state (element-local derivatives of the
nodal polynomials, Lobatto quadrature).  Checked at t = 0.05, 1 and 2:
  - the viscous part of the rate equals <tau : grad v> (the discrete viscous flux dissipates
    kinetic energy as the stress tensor does);
  - the time difference of the reported kinetic energy over two RK3 steps equals the residual's
    rate in the middle;
  - early on (t <= 1) the whole budget closes, pressure work included; later the pressure work is
    a small difference of element-local products and is only bounded;
  - at t = 0.05, where the flow is still nearly solenoidal, the rate equals twice nu times the
    reported enstrophy (<tau : grad v> = mu <|curl v|^2> for a solenoidal periodic field).

And the decay on the benchmark mesh itself (32^3 deformed hexahedra of order 4) up to t = 9.5,
through the transition: the kinetic energy falls monotonically, its dissipation rate rises to a
single peak near t = 9 of about 0.0125 (the flow's well-known behaviour at Re 1600: the vortex
sheets roll up and break down there), the enstrophy peaks there too, and at the peak the rate
exceeds 2 nu times the enstrophy by the scheme's own dissipation at this resolution.
"""
import numpy as np
import pytest
from numpy.polynomial import legendre as leg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dg():
    from paper_2206_09733_amd import dgsem
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    dgsem.lib()
    return dgsem


def lobatto(N):
    """Lobatto nodes on [-1, 1], their quadrature weights and the nodal differentiation matrix
    (from the barycentric weights)."""
    c = np.zeros(N + 1)
    c[N] = 1.0
    x = np.concatenate([[-1.0], np.sort(leg.legroots(leg.legder(c))), [1.0]])
    w = 2.0 / (N * (N + 1) * leg.legval(x, c) ** 2)
    bw = np.array([1.0 / np.prod([x[j] - x[m] for m in range(N + 1) if m != j]) for j in range(N + 1)])
    D = np.zeros((N + 1, N + 1))
    for i in range(N + 1):
        for j in range(N + 1):
            if i != j:
                D[i, j] = bw[j] / bw[i] / (x[i] - x[j])
        D[i, i] = -D[i].sum()
    return x, w, D


def energy_terms(U, E, N, h, mu, gamma=1.4):
    """Volume means of tau : grad v and of p div v for a state on an undeformed box of cubes of
    side h (layout: element, variable, node with i fastest)."""
    _, w, D = lobatto(N)
    n = N + 1
    U = U.reshape(E, 5, n, n, n)  # axes: element, variable, k, j, i
    rho = U[:, 0]
    v = U[:, 1:4] / rho[:, None]
    p = (gamma - 1) * (U[:, 4] - 0.5 * rho * (v * v).sum(1))
    s = 2.0 / h
    g = np.empty((3, 3) + rho.shape)  # g[a, b] = d v_b / d x_a
    for b in range(3):
        g[0, b] = s * np.einsum("ai,eKJi->eKJa", D, v[:, b])
        g[1, b] = s * np.einsum("aj,eKjI->eKaI", D, v[:, b])
        g[2, b] = s * np.einsum("ak,ekJI->eaJI", D, v[:, b])
    div = g[0, 0] + g[1, 1] + g[2, 2]
    S = 0.5 * (g + g.transpose(1, 0, 2, 3, 4, 5))
    diss = mu * (2.0 * (S * S).sum((0, 1)) - 2.0 / 3.0 * div * div)
    W = w[None, :, None, None] * w[None, None, :, None] * w[None, None, None, :]
    mean = lambda f: float((f * W).sum() / (W.sum() * E))
    # the mean pressure does no work on a periodic box; with element-local derivatives its
    # product with div v would not vanish (it would weigh the small jumps of v.n across faces by
    # the large p_0 = 1/(gamma Ma^2)), so only the fluctuation enters
    return mean(diss), mean((p - mean(p)) * div)


def ke_rate(U, R, E, N):
    """dK/dt = <v . R_m - |v|^2/2 R_rho> for a residual R of the state U."""
    _, w, _ = lobatto(N)
    n = N + 1
    U, R = U.reshape(E, 5, n, n, n), R.reshape(E, 5, n, n, n)
    v = U[:, 1:4] / U[:, :1]
    f = (v * R[:, 1:4]).sum(1) - 0.5 * (v * v).sum(1) * R[:, 0]
    W = w[None, :, None, None] * w[None, None, :, None] * w[None, None, None, :]
    return float((f * W).sum() / (W.sum() * E))


@pytest.mark.parametrize("precision", ["fp64", "fp32_bulk"])
def test_kinetic_energy_budget(dg, precision):
    Re, N, ex = 1600.0, 4, 16
    mu, h = 1.0 / Re, 2 * np.pi / ex
    E = ex ** 3
    s = dg.Solver(ex, N=N, Ma=0.1, Re=Re, precision=precision)
    eu = dg.Solver(ex, N=N, Ma=0.1, Re=0.0, precision=precision)
    s.set_ic("tgv")
    diss0, pdil0 = energy_terms(s.state(), E, N, h, mu)
    # the initial field: <tau : grad v> = mu <|curl v|^2> = 3 mu / 4, and div v = 0
    assert abs(diss0 / (0.75 * mu) - 1) < 1e-6 and abs(pdil0) < 1e-12, (diss0, pdil0)
    dt = s.suggest_dt(0.3)
    t = 0.0
    for t_target in (0.05, 1.0, 2.0):
        n_adv = max(0, int(round((t_target - t) / dt)) - 1)
        if n_adv:
            s.rk_step(dt, n_adv)
            t += n_adv * dt
        k0 = s.diagnostics()["ke"]
        s.rk_step(dt, 1)
        t += dt
        ens = 2 * mu * s.diagnostics()["enstrophy"]
        U = s.state()
        eu.set_state(U)
        full = -ke_rate(U, s.residual(), E, N)
        inviscid = -ke_rate(U, eu.residual(), E, N)
        diss, pdil = energy_terms(U, E, N, h, mu)
        s.rk_step(dt, 1)
        k2 = s.diagnostics()["ke"]
        t += dt
        stepped = -(k2 - k0) / (2 * dt)
        print(f"[physics {precision}] t={t - dt:.3f} -dK/dt: stepped={stepped:.6e} residual={full:.6e} "
              f"viscous={full - inviscid:.6e} inviscid={inviscid:.3e}; <tau:grad v>={diss:.6e} "
              f"-<p' div v>={-pdil:.3e} 2 nu enstrophy={ens:.6e}", flush=True)
        assert abs((full - inviscid) / diss - 1) < 1e-3
        assert abs(stepped / full - 1) < 1e-3
        if t_target <= 1.0:
            assert abs(full / (diss - pdil) - 1) < 1e-3
        assert abs(inviscid) < 0.1 * diss and abs(pdil) < 0.1 * diss  # 4.9% at t = 1
        if t_target < 0.1:
            assert abs(full / ens - 1) < 5e-3
    s.close()
    eu.close()


def test_taylor_green_decay_on_the_benchmark_mesh(dg):
    Re = 1600.0
    s = dg.Solver(32, N=4, deform=True, Ma=0.1, Re=Re)
    s.set_ic("tgv")
    dt = s.suggest_dt(0.5)
    chunk = max(1, int(round(0.05 / dt)))
    t, ts, ke, ens = 0.0, [0.0], [s.diagnostics()["ke"]], [s.diagnostics()["enstrophy"]]
    while t < 9.5:
        s.rk_step(dt, chunk)
        t += chunk * dt
        d = s.diagnostics()
        assert d["nonfinite"] == 0, t
        ts.append(t)
        ke.append(d["ke"])
        ens.append(d["enstrophy"])
        if len(ts) % 40 == 0:
            print(f"[tgv decay] t={t:.2f} ke={d['ke']:.6f} enstrophy={d['enstrophy']:.4f}", flush=True)
    ts, ke, ens = map(np.array, (ts, ke, ens))
    eps = -np.gradient(ke, ts)
    i, j = int(np.argmax(eps)), int(np.argmax(ens))
    print(f"[tgv decay] peak -dK/dt {eps[i]:.5f} at t={ts[i]:.2f} (2 nu enstrophy there {2 / Re * ens[i]:.5f}); "
          f"enstrophy peak {ens[j]:.3f} at t={ts[j]:.2f}", flush=True)
    assert np.all(np.diff(ke) < 0)
    assert 8.0 <= ts[i] <= 9.5 and 0.011 <= eps[i] <= 0.014, (ts[i], eps[i])
    assert 8.0 <= ts[j] <= 9.5 and 7.0 <= ens[j] <= 11.0, (ts[j], ens[j])
    assert eps[i] > 2 / Re * ens[i]
    s.close()
