"""Pins of the oracle's BR2 and interior-penalty viscous fluxes on Gauss-Legendre points (box of
viscous fluxes in section "Spatial discretisation", with its Gauss quadrature).

Reading: Gauss quadrature integrates the weak derivative exactly (degree 2N-1), so the BR1
gradient splits into the element's broken (strong) gradient and, per face, the lift of
g* - g(+-1), with g(+-1) the trace of the element's interpolant of g = (v, T).  BR2 takes on a
face the trace of the broken gradient plus eta times the trace of that face's lift; the interior
penalty takes the trace of the broken gradient and adds sigma F_v(v_mean, [g] n^) . S with
sigma = eta (N+1)^2 / h, h = 2 min(J_L, J_R)/|S| from the two traces of J.

- The decomposition itself: broken gradient + the six face lifts = the BR1 gradient, to rounding,
  on the deformed box (a wrong lift weight, sign or trace fails it).
- A field with constant density and linear velocity and temperature (g = (v, T) linear, in the
  element space): on the faces away from the periodic wrap, where the field jumps, BR2 and the
  interior penalty give the exact viscous flux (each face's gradient sees only its own jump;
  BR1's sees every face's lift along the line, the wrap's included).
- A velocity step across the x faces (v_y = a in one element, b in the other): closed forms of
  all three face fluxes from the Gauss sums K = sum_i l_i(1)^2 / w_i and K' = sum_i
  l_i(1) l_i(-1) / w_i, computed here with numpy's Gauss-Legendre rule (BR1 (K - K')(b-a)/h_x,
  BR2 eta K (b-a)/h_x, interior penalty eta (N+1)^2 (b-a)/h_x as d v_y / d x at the face).
- Face fluxes are single-valued and the residual conserves every variable on the deformed box.
"""
import numpy as np
import pytest

from helpers import quad_weights_uniform

GAMMA = 1.4


def lagrange_at(xs, y):
    """The Lagrange polynomials of the nodes xs evaluated at the point y."""
    xs = np.asarray(xs, float)
    return np.array([np.prod([(y - xs[m]) / (xs[l] - xs[m]) for m in range(len(xs)) if m != l])
                     for l in range(len(xs))])


def gauss_sums(N):
    x, w = np.polynomial.legendre.leggauss(N + 1)
    lp, lm = lagrange_at(x, 1.0), lagrange_at(x, -1.0)
    return float(np.sum(lp * lp / w)), float(np.sum(lp * lm / w))


def perturbed(s, seed):
    s.set_ic("tgv")
    rng = np.random.default_rng(seed)
    U = s.state().reshape(s.E, 5, -1)
    U[:, 0] *= 1 + 0.05 * rng.standard_normal(U[:, 0].shape)
    U[:, 4] *= 1 + 0.05 * rng.standard_normal(U[:, 4].shape)
    s.set_state(U.reshape(-1))
    return U.reshape(-1)


@pytest.mark.parametrize("N", [1, 2, 3, 5])
def test_broken_gradient_plus_face_lifts_is_the_br1_gradient(orc, N):
    s = orc.OracleSolver(3, 2, 3, N=N, deform=True, Ma=0.3, Re=100.0, vol="central", nodes="gauss")
    perturbed(s, N)
    G = s.gradients()
    Gb, Gl = s.gauss_gradient_parts()
    sc = np.abs(G).max()
    assert np.abs(Gl).max() > 0.05 * sc  # the lifts carry a real part of the gradient
    assert np.abs(Gb + Gl - G).max() < 1e-13 * sc, np.abs(Gb + Gl - G).max() / sc


def linear_state(s, grad_v, grad_T, rho=1.2, v0=(0.3, -0.1, 0.2), T0=0.8):
    """rho constant, v and T = p/rho linear in x: g = (v, T) is linear, U is quadratic."""
    X = s.coords().reshape(s.E, 3, -1)
    v = np.asarray(v0)[None, :, None] + np.einsum("kx,exn->ekn", grad_v, X)
    T = T0 + np.einsum("x,exn->en", grad_T, X)
    p = rho * T
    U = np.zeros((s.E, 5, X.shape[2]))
    U[:, 0] = rho
    U[:, 1:4] = rho * v
    U[:, 4] = p / (GAMMA - 1) + 0.5 * rho * (v * v).sum(1)
    return U.reshape(-1)


@pytest.mark.parametrize("N", [2, 4])
def test_br2_and_ip_give_the_exact_flux_of_a_continuous_linear_field(orc, N):
    grad_v = np.array([[0.02, -0.03, 0.01], [0.015, 0.01, -0.02], [-0.01, 0.025, 0.005]])
    grad_T = np.array([0.01, -0.005, 0.008])
    Re = 50.0
    F = {}
    for visc in ("br2", "ip"):
        s = orc.OracleSolver(3, 3, 3, N=N, Ma=0.3, Re=Re, vol="central", nodes="gauss", visc=visc)
        U = linear_state(s, grad_v, grad_T)
        s.set_state(U)
        F[visc] = s.gauss_face_viscous()
    n = N + 1
    x, _ = np.polynomial.legendre.leggauss(n)
    # interior faces: the +x, +y, +z faces of the elements that are not last along that direction
    hbox = 2 * np.pi / 3
    grad = np.zeros(12)
    for k in range(3):
        grad[3 * k:3 * k + 3] = grad_v[k]
    grad[9:12] = grad_T
    checked = 0
    for e in range(s.E):
        idx = (e % 3, (e // 3) % 3, e // 9)
        for d in range(3):
            if idx[d] == 2:
                continue
            f = 2 * d + 1
            ta, tb = [c for c in range(3) if c != d]
            for r in range(n):
                for p in range(n):
                    pos = np.zeros(3)
                    pos[d] = (idx[d] + 1) * hbox
                    pos[ta] = (idx[ta] + 0.5 * (1 + x[p])) * hbox
                    pos[tb] = (idx[tb] + 0.5 * (1 + x[r])) * hbox
                    v = np.array([0.3, -0.1, 0.2]) + grad_v @ pos
                    T = 0.8 + grad_T @ pos
                    u = np.concatenate([[1.2], 1.2 * v, [1.2 * T / (GAMMA - 1) + 0.6 * v @ v]])
                    Fv = orc.viscous_flux(u, grad, GAMMA, 0.71, Re)
                    S = np.zeros(3)
                    S[d] = hbox * hbox / 4
                    ref = S @ Fv
                    for visc in F:
                        got = F[visc][e, f, :, p + n * r]
                        assert np.allclose(got, ref, rtol=0, atol=1e-11 * np.abs(ref).max()), (visc, e, f, got, ref)
                    checked += 1
    assert checked == 3 * 18 * n * n


@pytest.mark.parametrize("N", [1, 2, 3, 4, 6])
def test_velocity_step_closed_forms(orc, N):
    a, b, Re, rho, T = 0.3, -0.2, 40.0, 1.1, 0.9
    mu = 1 / Re
    out = {}
    for visc, eta in (("br1", 0.0), ("br2", 1.5), ("ip", 2.5)):
        s = orc.OracleSolver(2, 1, 1, N=N, Ma=0.3, Re=Re, vol="central", nodes="gauss", visc=visc, visc_eta=eta)
        nn = (N + 1) ** 3
        U = np.zeros((2, 5, nn))
        for e, vy in ((0, a), (1, b)):
            U[e, 0], U[e, 2] = rho, rho * vy
            U[e, 4] = rho * T / (GAMMA - 1) + 0.5 * rho * vy * vy
        s.set_state(U.reshape(-1))
        out[visc] = (eta, s.gauss_face_viscous())
    hx = np.pi  # two elements across 2 pi
    area = (2 * np.pi) ** 2 / 4
    K, Kp = gauss_sums(N)
    Gx = {"br1": (K - Kp) * (b - a) / hx, "br2": 1.5 * K * (b - a) / hx, "ip": 2.5 * (N + 1) ** 2 * (b - a) / hx}
    for visc, (eta, F) in out.items():
        # element 0: its +x face (L = 0, R = 1) and its -x face (L = 1, R = 0: the step reversed)
        for f, sgn in ((1, 1.0), (0, -1.0)):
            g = sgn * Gx[visc]
            ref = np.array([0.0, 0.0, mu * g * area, 0.0, 0.5 * (a + b) * mu * g * area])
            got = F[0, f]
            assert np.allclose(got, ref[:, None], rtol=0, atol=1e-13 * np.abs(ref).max()), (visc, f, got[:, 0], ref)
            assert np.array_equal(F[1, f ^ 1], got)  # the same face seen from element 1
        if visc != "br1":  # y and z faces: no jump and no broken gradient
            assert np.all(np.abs(F[:, 2:]) < 1e-14), (visc, np.abs(F[:, 2:]).max())


@pytest.mark.parametrize("visc,N", [("br2", 3), ("ip", 3), ("br2", 5), ("ip", 4)])
def test_face_flux_single_valued_and_conservation_on_the_deformed_box(orc, visc, N):
    s = orc.OracleSolver(3, 2, 3, N=N, deform=True, Ma=0.3, Re=80.0, vol="central", nodes="gauss", visc=visc)
    perturbed(s, 10 + N)
    F = s.gauss_face_viscous()
    dims = (3, 2, 3)  # element e = i + 3 (j + 2 k)
    for e in range(s.E):
        idx = [e % 3, (e // 3) % 2, e // 6]
        for d in range(3):
            j = list(idx)
            j[d] = (j[d] + 1) % dims[d]
            ne = j[0] + 3 * (j[1] + 2 * j[2])
            assert np.array_equal(F[e, 2 * d + 1], F[ne, 2 * d]), (e, d)
    R = s.residual()
    _, w, _, _ = orc.gl(N)
    _, J = s.metrics()
    wq = (quad_weights_uniform(np.asarray(w), s.E) * J).reshape(s.E, -1)
    Rv = R.reshape(s.E, 5, -1)
    tot = np.einsum("en,evn->v", wq, Rv)
    mag = np.einsum("en,evn->v", wq, np.abs(Rv))
    assert np.all(np.abs(tot) < 1e-12 * mag.max()), (tot, mag)
    # and the scheme matters: BR1's residual differs
    b1 = orc.OracleSolver(3, 2, 3, N=N, deform=True, Ma=0.3, Re=80.0, vol="central", nodes="gauss")
    b1.set_state(s.state())
    assert np.abs(b1.residual() - R).max() > 1e-6 * np.abs(R).max()


@pytest.mark.parametrize("N", [2, 4])
def test_penalty_on_the_deformed_box(orc, N):
    """A velocity step on the deformed box: each element's state is constant, so the broken
    gradients vanish and the interior penalty's face flux is its penalty alone, with h from the
    traces of J (interpolated here with numpy's Lagrange weights from the oracle's metric terms)
    and S the owner's interpolated metric.  The box's map is smooth, so J is continuous across
    faces and the two traces agree: taking the smaller of them is not pinned by this case."""
    a, b, Re, rho, T, eta = 0.3, -0.2, 40.0, 1.1, 0.9, 1.7
    s = orc.OracleSolver(2, 2, 2, N=N, deform=True, Ma=0.3, Re=Re, vol="central", nodes="gauss", visc="ip",
                         visc_eta=eta)
    n, nn = N + 1, (N + 1) ** 3
    U = np.zeros((8, 5, nn))
    for e in range(8):  # element e = i + 2 (j + 2 k): the step is across x
        vy = a if e % 2 == 0 else b
        U[e, 0], U[e, 2] = rho, rho * vy
        U[e, 4] = rho * T / (GAMMA - 1) + 0.5 * rho * vy * vy
    s.set_state(U.reshape(-1))
    F = s.gauss_face_viscous()
    Ja, J = s.metrics()
    Ja, J = Ja.reshape(8, 9, nn), J.reshape(8, nn)
    x, _ = np.polynomial.legendre.leggauss(n)
    lp, lm = lagrange_at(x, 1.0), lagrange_at(x, -1.0)
    ratios = []  # tangential parts of S
    for L, R, f, jump in ((0, 1, 1, b - a), (1, 0, 0, a - b)):  # element 0's +x face, then its -x face
        for r in range(n):
            for p in range(n):
                line = np.arange(n) + n * p + n * n * r  # nodes i of the x line through (p, r)
                S = np.array([lp @ Ja[L, c, line] for c in range(3)])
                JL, JR = lp @ J[L, line], lm @ J[R, line]
                area = np.sqrt(S @ S)
                sigma = eta * n * n / (2 * min(JL, JR) / area)
                grad = np.zeros(12)
                grad[3:6] = sigma * jump * S / area  # d v_y / d x_k
                um = np.array([1.0, 0.0, 0.5 * (a + b), 0.0, 2.0])
                ref = S @ orc.viscous_flux(um, grad, GAMMA, 0.71, Re)
                got = F[0, f, :, p + n * r]
                assert np.allclose(got, ref, rtol=0, atol=1e-12 * np.abs(ref).max()), (f, p, r, got, ref)
                ratios.append(abs(S[1]) + abs(S[2]))
    assert max(ratios) > 1e-3 * area  # the face is curved: S is not along x
