"""ctypes binding of the plain CPU oracle (test infrastructure only).

Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may import this module.
It never touches the HIP library; the HIP path never imports it.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))

VOL = {"ec": 0, "central": 1, "ir": 2, "kg": 3, "pirozzoli": 4, "ducros": 5, "morinishi": 6}
SURF = {"roe": 0, "llf": 1, "ec": 2, "central": 3, "es": 4, "ir": 5, "es_matrix": 6, "ld_roe": 7,
        "lf_global": 8}
VISC = {"br1": 0, "br2": 1, "ip": 2}
SVV_KERNEL = {"tadmor": 0, "maday": 1}
IC = {"uniform": 0, "tgv": 1, "vortex": 2, "density_wave": 3}
DIAG_KEYS = ["mass_rho", "mass_rhou", "mass_rhov", "mass_rhow", "mass_rhoE", "entropy_paper",
             "entropy", "ke", "enstrophy", "lambda_max", "rho_min", "p_min", "nonfinite", "volume"]

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)
_libs = {}


def _lib(precision="fp64"):
    name = {"fp64": "liborc64.so", "fp80": "liborc80.so"}[precision]
    if name not in _libs:
        # ORACLE_LIB_DIR: another build of the same source (the sanitizer test's instrumented one)
        path = os.path.join(os.environ.get("ORACLE_LIB_DIR", HERE), name)
        if not os.path.exists(path):
            from . import build as _b
            _b.build()
        L = ctypes.CDLL(path)
        L.orc_create.restype = ctypes.c_void_p
        L.orc_create.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, _dp, _dp, ctypes.c_int,
                                 ctypes.c_double, ctypes.c_int, _ip, ctypes.c_double,
                                 ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                 ctypes.c_int]
        L.orc_destroy.argtypes = [ctypes.c_void_p]
        L.orc_set_viscous_flux.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_double]
        L.orc_num_nodes.restype = ctypes.c_long
        L.orc_num_nodes.argtypes = [ctypes.c_void_p]
        L.orc_num_elements.argtypes = [ctypes.c_void_p]
        L.orc_elem_info.argtypes = [ctypes.c_void_p, ctypes.c_int, _ip,
                                    ctypes.POINTER(ctypes.c_long)]
        for fn in ("orc_get_coords", "orc_set_state", "orc_get_state", "orc_residual",
                   "orc_gradients", "orc_diagnostics"):
            getattr(L, fn).argtypes = [ctypes.c_void_p, _dp]
        L.orc_get_metrics.argtypes = [ctypes.c_void_p, _dp, _dp]
        L.orc_gauss_gradient_parts.argtypes = [ctypes.c_void_p, _dp, _dp]
        L.orc_gauss_face_viscous.argtypes = [ctypes.c_void_p, _dp]
        L.orc_set_ic.argtypes = [ctypes.c_void_p, ctypes.c_int, _dp]
        L.orc_rk3.argtypes = [ctypes.c_void_p, ctypes.c_double, ctypes.c_int]
        L.orc_rk.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_int]
        L.orc_suggest_dt.restype = ctypes.c_double
        L.orc_suggest_dt.argtypes = [ctypes.c_void_p, ctypes.c_double]
        L.orc_entropy_production.restype = ctypes.c_double
        L.orc_entropy_production.argtypes = [ctypes.c_void_p, _dp]
        L.orc_set_threads.argtypes = [ctypes.c_int]
        L.orc_gll.argtypes = [ctypes.c_int, _dp, _dp, _dp]
        L.orc_gl.argtypes = [ctypes.c_int, _dp, _dp, _dp, _dp]
        L.orc_create_gauss.restype = ctypes.c_void_p
        L.orc_create_gauss.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, _dp, _dp, ctypes.c_int,
                                       ctypes.c_double, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_double, ctypes.c_double, ctypes.c_int]
        L.orc_mortar_matrices.argtypes = [ctypes.c_int, ctypes.c_int, _dp, _dp]
        L.orc_euler_flux.argtypes = [_dp, _dp, ctypes.c_double, _dp]
        L.orc_two_point_ec.argtypes = [_dp, _dp, _dp, ctypes.c_double, _dp]
        L.orc_two_point_central.argtypes = [_dp, _dp, _dp, ctypes.c_double, _dp]
        L.orc_two_point_ir.argtypes = [_dp, _dp, _dp, ctypes.c_double, _dp]
        L.orc_two_point.argtypes = [ctypes.c_int, _dp, _dp, _dp, ctypes.c_double, _dp]
        L.orc_riemann.argtypes = [ctypes.c_int, _dp, _dp, _dp, ctypes.c_double, _dp]
        L.orc_lax_friedrichs.argtypes = [_dp, _dp, _dp, ctypes.c_double, ctypes.c_double, _dp]
        L.orc_roe_waves.argtypes = [_dp, _dp, _dp, ctypes.c_double, ctypes.c_int, _dp]
        L.orc_entropy_vars.argtypes = [_dp, ctypes.c_double, _dp]
        L.orc_entropy.restype = ctypes.c_double
        L.orc_entropy.argtypes = [_dp, ctypes.c_double]
        L.orc_logmean.restype = ctypes.c_double
        L.orc_logmean.argtypes = [ctypes.c_double, ctypes.c_double]
        L.orc_viscous_flux.argtypes = [_dp, _dp, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_double, _dp]
        L.orc_set_svv.argtypes = [ctypes.c_void_p, ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_double]
        L.orc_svv_residual.argtypes = [ctypes.c_void_p, _dp, _dp]
        L.orc_svv_sensor.argtypes = [ctypes.c_void_p, _dp]
        L.orc_svv_filter.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, _dp, _dp]
        L.orc_svv_flux.argtypes = [_dp, _dp, ctypes.c_double, ctypes.c_double, ctypes.c_double, _dp]
        L.orc_set_les.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_double]
        L.orc_les_viscosity.argtypes = [_dp, _dp, ctypes.c_double, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                        ctypes.c_int, _dp]
        L.orc_les_flux.argtypes = [_dp, _dp, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                   ctypes.c_double, ctypes.c_double, ctypes.c_int, _dp]
        _libs[name] = L
    return _libs[name]


def _ptr(a):
    return a.ctypes.data_as(_dp)


def _f64(a, n=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if n is not None:
        assert a.size == n, (a.size, n)
    return a


def set_threads(n, precision="fp64"):
    _lib(precision).orc_set_threads(int(n))


# ---------------------------------------------------------------------------- point functions
def gll(N, precision="fp64"):
    xi, w, D = np.zeros(N + 1), np.zeros(N + 1), np.zeros((N + 1) * (N + 1))
    rc = _lib(precision).orc_gll(N, _ptr(xi), _ptr(w), _ptr(D))
    if rc:
        raise ValueError(f"orc_gll({N}) failed")
    return xi, w, D.reshape(N + 1, N + 1)


def gl(N, precision="fp64"):
    """Gauss-Legendre points, weights, derivative matrix and the Lagrange basis at -1 and +1."""
    xi, w, D, lb = np.zeros(N + 1), np.zeros(N + 1), np.zeros((N + 1) * (N + 1)), np.zeros(2 * (N + 1))
    rc = _lib(precision).orc_gl(N, _ptr(xi), _ptr(w), _ptr(D), _ptr(lb))
    if rc:
        raise ValueError(f"orc_gl({N}) failed")
    return xi, w, D.reshape(N + 1, N + 1), lb.reshape(2, N + 1)


def mortar_matrices(N, M, precision="fp64"):
    I, P = np.zeros((M + 1) * (N + 1)), np.zeros((N + 1) * (M + 1))
    if _lib(precision).orc_mortar_matrices(N, M, _ptr(I), _ptr(P)):
        raise ValueError(f"orc_mortar_matrices({N},{M}) failed")
    return I.reshape(M + 1, N + 1), P.reshape(N + 1, M + 1)


def _point(fn, *arrays, out=5, scalars=(), precision="fp64"):
    res = np.zeros(out)
    args = [_ptr(_f64(a)) for a in arrays] + list(scalars) + [_ptr(res)]
    getattr(_lib(precision), fn)(*args)
    return res


def euler_flux(U, n, gamma=1.4, precision="fp64"):
    return _point("orc_euler_flux", U, n, scalars=(ctypes.c_double(gamma),), precision=precision)


def two_point_ec(UL, UR, n, gamma=1.4, precision="fp64"):
    return _point("orc_two_point_ec", UL, UR, n, scalars=(ctypes.c_double(gamma),),
                  precision=precision)


def two_point_central(UL, UR, n, gamma=1.4, precision="fp64"):
    return _point("orc_two_point_central", UL, UR, n, scalars=(ctypes.c_double(gamma),),
                  precision=precision)


def two_point_ir(UL, UR, n, gamma=1.4, precision="fp64"):
    return _point("orc_two_point_ir", UL, UR, n, scalars=(ctypes.c_double(gamma),),
                  precision=precision)


def two_point(kind, UL, UR, n, gamma=1.4, precision="fp64"):
    """Any volume two-point flux by name (see VOL)."""
    res = np.zeros(5)
    _lib(precision).orc_two_point(VOL[kind], _ptr(_f64(UL)), _ptr(_f64(UR)), _ptr(_f64(n)),
                                  gamma, _ptr(res))
    return res


def riemann(kind, UL, UR, S, gamma=1.4, precision="fp64"):
    res = np.zeros(5)
    _lib(precision).orc_riemann(SURF[kind], _ptr(_f64(UL)), _ptr(_f64(UR)), _ptr(_f64(S)),
                                gamma, _ptr(res))
    return res


def lax_friedrichs(UL, UR, S, lam, gamma=1.4, precision="fp64"):
    res = np.zeros(5)
    _lib(precision).orc_lax_friedrichs(_ptr(_f64(UL)), _ptr(_f64(UR)), _ptr(_f64(S)), gamma, float(lam),
                                       _ptr(res))
    return res


def roe_waves(UL, UR, nhat, gamma=1.4, absval=True, precision="fp64"):
    res = np.zeros(5)
    _lib(precision).orc_roe_waves(_ptr(_f64(UL)), _ptr(_f64(UR)), _ptr(_f64(nhat)), gamma,
                                  int(absval), _ptr(res))
    return res


def entropy_vars(U, gamma=1.4, precision="fp64"):
    res = np.zeros(5)
    _lib(precision).orc_entropy_vars(_ptr(_f64(U)), gamma, _ptr(res))
    return res


def entropy(U, gamma=1.4, precision="fp64"):
    return _lib(precision).orc_entropy(_ptr(_f64(U)), gamma)


def logmean(a, b, precision="fp64"):
    return _lib(precision).orc_logmean(a, b)


def viscous_flux(U, grad, gamma=1.4, Pr=0.71, Re=1600.0, precision="fp64"):
    res = np.zeros(15)
    _lib(precision).orc_viscous_flux(_ptr(_f64(U)), _ptr(_f64(grad)), gamma, Pr, Re, _ptr(res))
    return res.reshape(3, 5)


def svv_filter(N, f, kernel="maday", cutoff=None, precision="fp64"):
    """The modal SVV filter of one nodal field of an order-N element (f[k][j][i])."""
    cutoff = N // 2 if cutoff is None else cutoff
    out = np.zeros((N + 1) ** 3)
    if _lib(precision).orc_svv_filter(int(N), SVV_KERNEL[kernel], int(cutoff), _ptr(_f64(f, (N + 1) ** 3)),
                                      _ptr(out)):
        raise ValueError("orc_svv_filter rejected the arguments")
    return out


def svv_flux(U, Gw, mu_a, gamma=1.4, Pr=0.71, precision="fp64"):
    """Unfiltered artificial flux L^T D L G at one state; Gw[3c+x] = d w_c / d x_x; rows = directions."""
    res = np.zeros(15)
    _lib(precision).orc_svv_flux(_ptr(_f64(U, 5)), _ptr(_f64(Gw, 15)), gamma, Pr, float(mu_a), _ptr(res))
    return res.reshape(3, 5)


LES_MODEL = {"smagorinsky": 0, "wale": 1, "vreman": 2}


def les_viscosity(U, Gw, cs, J, n, model="smagorinsky", gamma=1.4, precision="fp64"):
    """The eddy viscosity rho nu_t of the explicit LES closure at one state (Smagorinsky, WALE or
    Vreman with constant cs): Gw[3c+x] = d w_c / d x_x, J the Jacobian, n the element's node
    count."""
    out = np.zeros(1)
    if _lib(precision).orc_les_viscosity(_ptr(_f64(U, 5)), _ptr(_f64(Gw, 15)), gamma, LES_MODEL[model], float(cs),
                                         float(J), int(n), _ptr(out)):
        raise ValueError("orc_les_viscosity rejected the arguments")
    return float(out[0])


def les_flux(U, Gw, cs, J, n, mu_a=0.0, model="smagorinsky", gamma=1.4, Pr=0.71, precision="fp64"):
    """Unfiltered artificial flux at one state with the model's eddy viscosity added (rows =
    directions), the factors the solver's filtered flux uses."""
    res = np.zeros(15)
    if _lib(precision).orc_les_flux(_ptr(_f64(U, 5)), _ptr(_f64(Gw, 15)), gamma, Pr, float(mu_a), LES_MODEL[model],
                                    float(cs), float(J), int(n), _ptr(res)):
        raise ValueError("orc_les_flux rejected the arguments")
    return res.reshape(3, 5)


# ---------------------------------------------------------------------------- solver
class OracleSolver:
    """Periodic-box DGSEM solver on the CPU (plain loops, fp64 or fp80)."""

    def __init__(self, ex, ey=None, ez=None, lo=(0.0, 0.0, 0.0), hi=None, deform=False,
                 amp=0.05, N=3, orders=None, gamma=1.4, Pr=0.71, Ma=0.1, Re=0.0, vol="ec",
                 surf="roe", precision="fp64", visc="br1", visc_eta=0.0, nodes="lobatto"):
        ey = ex if ey is None else ey
        ez = ex if ez is None else ez
        self.N = int(N)
        if hi is None:
            hi = (2 * np.pi,) * 3
        self.L = _lib(precision)
        self.shape = (ex, ey, ez)
        self.gamma, self.Pr, self.Ma, self.Re = gamma, Pr, Ma, Re
        lo = _f64(lo, 3)
        hi = _f64(hi, 3)
        optr = None
        if orders is not None:
            self._orders = np.ascontiguousarray(orders, dtype=np.int32).reshape(-1)
            assert self._orders.size == 3 * ex * ey * ez
            optr = self._orders.ctypes.data_as(_ip)
        if nodes == "gauss":  # uniform order, plain weak form
            if orders is not None or vol != "central":
                raise ValueError("Gauss-Legendre nodes: uniform-order boxes, central volume form")
            self.h = self.L.orc_create_gauss(ex, ey, ez, _ptr(lo), _ptr(hi), int(bool(deform)), amp, int(N), gamma,
                                             Pr, Ma, Re, SURF[surf])
        else:
            self.h = self.L.orc_create(ex, ey, ez, _ptr(lo), _ptr(hi), int(bool(deform)), amp, int(N),
                                       optr, gamma, Pr, Ma, Re, VOL[vol], SURF[surf])
        if not self.h:
            raise ValueError("orc_create rejected the configuration")
        if self.L.orc_set_viscous_flux(self.h, VISC[visc], float(visc_eta)) != 0:
            raise ValueError("orc_set_viscous_flux rejected the configuration")
        self.nodes = self.L.orc_num_nodes(self.h)
        self.E = self.L.orc_num_elements(self.h)

    def close(self):
        if self.h:
            self.L.orc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def elem(self, e):
        n3 = (ctypes.c_int * 3)()
        off = ctypes.c_long()
        self.L.orc_elem_info(self.h, e, n3, ctypes.byref(off))
        return tuple(n3), off.value

    def coords(self):
        X = np.zeros(3 * self.nodes)
        self.L.orc_get_coords(self.h, _ptr(X))
        return X

    def metrics(self):
        Ja, J = np.zeros(9 * self.nodes), np.zeros(self.nodes)
        self.L.orc_get_metrics(self.h, _ptr(Ja), _ptr(J))
        return Ja, J

    def set_ic(self, ic, params=None):
        p = _f64(params if params is not None else np.zeros(9))
        if self.L.orc_set_ic(self.h, IC[ic], _ptr(p)):
            raise ValueError("orc_set_ic failed")

    def set_state(self, U):
        U = _f64(U, 5 * self.nodes)
        self.L.orc_set_state(self.h, _ptr(U))

    def state(self):
        U = np.zeros(5 * self.nodes)
        self.L.orc_get_state(self.h, _ptr(U))
        return U

    def residual(self):
        R = np.zeros(5 * self.nodes)
        self.L.orc_residual(self.h, _ptr(R))
        return R

    def gradients(self):
        G = np.zeros(12 * self.nodes)
        self.L.orc_gradients(self.h, _ptr(G))
        return G

    def gauss_gradient_parts(self):
        """Gauss-Legendre meshes: (broken gradient, sum of the six face lifts) of g = (v, T) at
        every node, in the layout of gradients(); their sum is the BR1 gradient."""
        Gb, Gl = np.zeros(12 * self.nodes), np.zeros(12 * self.nodes)
        if self.L.orc_gauss_gradient_parts(self.h, _ptr(Gb), _ptr(Gl)):
            raise ValueError("not a Gauss-Legendre solver")
        return Gb, Gl

    def gauss_face_viscous(self):
        """Gauss-Legendre Navier-Stokes meshes: the face viscous flux of the current state,
        [E][6 faces][5][nf], f = 2 d + side, face point p + n r."""
        n = self.N + 1
        F = np.zeros(self.E * 6 * 5 * n * n)
        if self.L.orc_gauss_face_viscous(self.h, _ptr(F)):
            raise ValueError("not a Gauss-Legendre Navier-Stokes solver")
        return F.reshape(self.E, 6, 5, n * n)

    def rk3(self, dt, nsteps):
        self.L.orc_rk3(self.h, float(dt), int(nsteps))

    def rk(self, dt, nsteps, scheme="rk3"):
        """scheme "rk3" (Williamson) or "rk4" (Carpenter-Kennedy, five stages)."""
        rc = self.L.orc_rk(self.h, {"rk3": 0, "rk4": 1}[scheme], float(dt), int(nsteps))
        assert rc == 0

    def suggest_dt(self, cfl):
        return self.L.orc_suggest_dt(self.h, float(cfl))

    def diagnostics(self):
        out = np.zeros(14)
        self.L.orc_diagnostics(self.h, _ptr(out))
        return dict(zip(DIAG_KEYS, out.tolist()))

    def entropy_production(self, R):
        return self.L.orc_entropy_production(self.h, _ptr(_f64(R, 5 * self.nodes)))

    def set_svv(self, mu_a, kernel="maday", cutoff=None, sensor=-1.0):
        """Spectral vanishing viscosity: artificial viscosity mu_a, filter kernel and cutoff mode
        (default N // 2 of the element orders' minimum), troubled-element sensor threshold
        (< 0: none)."""
        if cutoff is None:
            cutoff = min(self.elem(e)[0][d] for e in range(self.E) for d in range(3)) // 2
        if self.L.orc_set_svv(self.h, float(mu_a), SVV_KERNEL[kernel], int(cutoff), float(sensor)):
            raise ValueError("orc_set_svv rejected the configuration")

    def set_les(self, cs, model="smagorinsky"):
        """Explicit LES closure: the model's eddy viscosity (Smagorinsky, WALE or Vreman, constant
        cs) joins the artificial viscosity of the SVV term (then filtered by its kernel:
        SVV-Smagorinsky; Tadmor's kernel with cutoff -1 keeps every mode: the plain model).
        Call before set_svv."""
        if self.L.orc_set_les(self.h, LES_MODEL[model], float(cs)):
            raise ValueError("orc_set_les rejected the configuration")

    def svv_residual(self):
        """The artificial-viscosity part of the residual, and the entropy form sum <y, F* y>."""
        R = np.zeros(5 * self.nodes)
        form = ctypes.c_double()
        if self.L.orc_svv_residual(self.h, _ptr(R), ctypes.byref(form)):
            raise ValueError("SVV is not set")
        return R, form.value

    def svv_sensor(self):
        out = np.zeros(self.E)
        self.L.orc_svv_sensor(self.h, _ptr(out))
        return out
