"""Python binding of libdgsem.so (argument marshalling only; every step runs in HIP kernels).

The names follow the C ABI of include/dgsem.h.  Device memory comes from PyTorch (one uint8
tensor per solver) and the work is enqueued on the current PyTorch stream.  There is no CPU
fallback: without the compiled library every call raises.
"""
import ctypes
import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdgsem.so")

DG_OK, DG_EINVAL, DG_ENOMEM, DG_EHIP, DG_ENONFINITE, DG_EUNSUPPORTED, DG_ESTATE = 0, -1, -2, -3, -4, -5, -6
VOL = {"ec": 0, "central": 1, "ir": 2, "kg": 3, "pirozzoli": 4, "ducros": 5, "morinishi": 6}
SURF = {"roe": 0, "llf": 1, "ec": 2, "central": 3, "es": 4, "ir": 5, "es_matrix": 6, "ld_roe": 7,
        "lf_global": 8}
VISC = {"br1": 0, "br2": 1, "ip": 2}
SVV_KERNEL = {"tadmor": 0, "maday": 1}
LES_MODEL = {"smagorinsky": 0, "wale": 1, "vreman": 2}
PRECISION = {"fp64": 0, "fp32_bulk": 1}
IC = {"uniform": 0, "tgv": 1, "vortex": 2, "density_wave": 3}
SCHEME = {"rk3": 0, "rk4": 1}
IC_NPARAMS = {"uniform": 5, "tgv": 0, "vortex": 5, "density_wave": 9}

_c = ctypes
_dp = _c.POINTER(_c.c_double)


class BoxDesc(_c.Structure):
    _fields_ = [("ex", _c.c_int), ("ey", _c.c_int), ("ez", _c.c_int), ("lo", _c.c_double * 3),
                ("hi", _c.c_double * 3), ("deform", _c.c_int), ("deform_amp", _c.c_double),
                ("n_uniform", _c.c_int), ("orders", _c.POINTER(_c.c_int)), ("nodes", _c.c_int),
                ("halo", _c.c_int)]


class Physics(_c.Structure):
    _fields_ = [("gamma", _c.c_double), ("Pr", _c.c_double), ("Ma", _c.c_double),
                ("Re", _c.c_double), ("vol_flux", _c.c_int), ("surf_flux", _c.c_int),
                ("precision", _c.c_int), ("visc_flux", _c.c_int), ("visc_eta", _c.c_double),
                ("svv_mu", _c.c_double), ("svv_kernel", _c.c_int), ("svv_cutoff", _c.c_int),
                ("svv_sensor", _c.c_double), ("les_cs", _c.c_double), ("les_model", _c.c_int)]


class Diag(_c.Structure):
    _fields_ = [("mass", _c.c_double * 5), ("entropy_paper", _c.c_double),
                ("entropy", _c.c_double), ("ke", _c.c_double), ("enstrophy", _c.c_double),
                ("lambda_max", _c.c_double), ("rho_min", _c.c_double), ("p_min", _c.c_double),
                ("volume", _c.c_double), ("nonfinite", _c.c_longlong)]


class Profile(_c.Structure):
    _fields_ = [("ms", _c.c_double * 4), ("launches", _c.c_longlong * 4)]


KERNEL_CLASSES = ["gradient", "stage", "diagnostics", "other"]

EXPORTS = ["dg_last_error", "dg_mesh_create_box", "dg_mesh_destroy", "dg_mesh_info",
           "dg_solver_create", "dg_solver_required_bytes", "dg_solver_bind",
           "dg_set_initial_condition", "dg_set_state", "dg_get_state", "dg_residual", "dg_rk_step",
           "dg_rk_step_adaptive",
           "dg_diagnostics", "dg_suggest_dt", "dg_get_geometry", "dg_device_pointers",
           "dg_synchronize", "dg_solver_destroy", "dg_profile_begin", "dg_profile_end",
           "dg_solver_use_graphs", "dg_autotune", "dg_solver_set_tiles", "dg_batch_create",
           "dg_batch_rk_step", "dg_batch_use_graphs", "dg_batch_launches", "dg_batch_destroy",
           "dg_solver_set_scheme", "dg_diagnostics_noalloc"]

_lib = None


class DgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libdgsem error {code}: {msg}")
        self.code = code


def lib():
    """Load libdgsem.so (built by paper_2206_09733_amd.build / __graft_entry__.build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2206_09733_amd.build`"
                           " (there is no CPU fallback)")
    # PyTorch ships its own HIP runtime under the same soname: load it first, so that the
    # library binds to it and the process holds one runtime (torch's device pointers and
    # streams are then valid in the library)
    import torch  # noqa: F401
    L = _c.CDLL(LIB_PATH)
    vp = _c.c_void_p
    L.dg_last_error.restype = _c.c_char_p
    L.dg_mesh_create_box.argtypes = [_c.POINTER(BoxDesc), _c.POINTER(vp)]
    L.dg_mesh_destroy.argtypes = [vp]
    L.dg_mesh_destroy.restype = None
    L.dg_mesh_info.argtypes = [vp, _c.POINTER(_c.c_longlong), _c.POINTER(_c.c_longlong), _c.POINTER(_c.c_int)]
    L.dg_solver_create.argtypes = [vp, _c.POINTER(Physics), _c.POINTER(vp)]
    L.dg_solver_required_bytes.argtypes = [vp, _c.POINTER(_c.c_size_t)]
    L.dg_solver_bind.argtypes = [vp, vp, _c.c_size_t, vp]
    L.dg_set_initial_condition.argtypes = [vp, _c.c_int, _dp]
    L.dg_set_state.argtypes = [vp, _dp, _c.c_size_t]
    L.dg_get_state.argtypes = [vp, _dp, _c.c_size_t]
    L.dg_residual.argtypes = [vp, _dp, _c.c_size_t]
    L.dg_rk_step.argtypes = [vp, _c.c_double, _c.c_int]
    L.dg_rk_step_adaptive.argtypes = [vp, _c.c_double, _c.c_int, _dp]
    L.dg_diagnostics.argtypes = [vp, _c.POINTER(Diag)]
    L.dg_diagnostics_noalloc.argtypes = [vp, vp]
    L.dg_suggest_dt.argtypes = [vp, _c.c_double, _dp]
    L.dg_get_geometry.argtypes = [vp, _dp, _dp, _dp]
    L.dg_device_pointers.argtypes = [vp, _c.POINTER(vp), _c.POINTER(vp)]
    L.dg_synchronize.argtypes = [vp]
    L.dg_profile_begin.argtypes = [vp]
    L.dg_profile_end.argtypes = [vp, _c.POINTER(Profile)]
    L.dg_solver_destroy.argtypes = [vp]
    L.dg_solver_destroy.restype = None
    L.dg_solver_use_graphs.argtypes = [vp, _c.c_int]
    L.dg_autotune.argtypes = [vp, _c.POINTER(_c.c_int), _dp]
    L.dg_solver_set_tiles.argtypes = [vp, _c.c_int]
    L.dg_batch_create.argtypes = [_c.POINTER(vp), _c.c_int, vp, _c.POINTER(vp)]
    L.dg_batch_rk_step.argtypes = [vp, _dp, _c.c_int]
    L.dg_batch_use_graphs.argtypes = [vp, _c.c_int]
    L.dg_batch_launches.argtypes = [vp, _c.POINTER(_c.c_int)]
    L.dg_batch_destroy.argtypes = [vp]
    L.dg_batch_destroy.restype = None
    L.dg_solver_set_scheme.argtypes = [vp, _c.c_int]
    _lib = L
    return L


def check(rc):
    if rc != DG_OK:
        raise DgError(rc, lib().dg_last_error().decode())
    return rc


def _ptr(a):
    return a.ctypes.data_as(_dp)


NODES = {"lobatto": 0, "gauss": 1}


def box_desc(ex, ey, ez, lo, hi, deform, amp, N, orders=None, nodes="lobatto", halo=False):
    d = BoxDesc()
    d.nodes = NODES[nodes]
    d.halo = 1 if halo else 0
    d.ex, d.ey, d.ez = ex, ey, ez
    d.lo[:] = list(lo)
    d.hi[:] = list(hi)
    d.deform = 1 if deform else 0
    d.deform_amp = amp
    d.n_uniform = N
    keep = None
    if orders is not None:
        keep = np.ascontiguousarray(orders, dtype=np.int32).reshape(-1)
        d.orders = keep.ctypes.data_as(_c.POINTER(_c.c_int))
    return d, keep


def physics(gamma=1.4, Pr=0.71, Ma=0.1, Re=0.0, vol="ec", surf="roe", precision="fp64", visc="br1",
            visc_eta=0.0, svv_mu=0.0, svv_kernel="maday", svv_cutoff=0, svv_sensor=-1.0, les_cs=0.0,
            les_model="smagorinsky"):
    p = Physics()
    p.gamma, p.Pr, p.Ma, p.Re = gamma, Pr, Ma, Re
    p.vol_flux, p.surf_flux, p.precision = VOL[vol], SURF[surf], PRECISION[precision]
    p.visc_flux, p.visc_eta = VISC[visc], float(visc_eta)
    p.svv_mu, p.svv_kernel = float(svv_mu), SVV_KERNEL[svv_kernel]
    p.svv_cutoff, p.svv_sensor = int(svv_cutoff), float(svv_sensor)
    p.les_cs, p.les_model = float(les_cs), LES_MODEL[les_model]
    return p


class Solver:
    """One DGSEM solve on a periodic box, resident in device memory.

    `orders` (optional, shape (E, 3) or 3 E integers) gives every element its own order per
    direction; otherwise all elements take order N.  `svv_mu` > 0 adds spectral vanishing
    viscosity (kernel "maday" or "tadmor", cutoff mode `svv_cutoff`, default N // 2, and the
    troubled-element threshold `svv_sensor` of the density sensor, < 0 for none).  `les_cs` > 0
    adds the eddy viscosity of `les_model` ("smagorinsky", "wale" or "vreman") with that constant
    to the artificial viscosity, node by node (filtered by the SVV kernel: SVV-Smagorinsky; kernel
    "tadmor" with cutoff -1 keeps every mode: the plain model).  `halo=True` runs the box as one
    block of a split domain: faces on the box boundary read ghost elements that a halo exchange
    (pack, transfer, unpack) fills before every stage; results equal the direct periodic box.
    """

    def __init__(self, ex, ey=None, ez=None, lo=(0.0, 0.0, 0.0), hi=None, deform=False, amp=0.05,
                 N=3, gamma=1.4, Pr=0.71, Ma=0.1, Re=0.0, vol="ec", surf="roe", precision="fp64",
                 device="cuda", bind=True, orders=None, visc="br1", visc_eta=0.0, nodes="lobatto",
                 svv_mu=0.0, svv_kernel="maday", svv_cutoff=None, svv_sensor=-1.0, les_cs=0.0,
                 les_model="smagorinsky", halo=False):
        L = lib()
        ey = ex if ey is None else ey
        ez = ex if ez is None else ez
        hi = (2 * math.pi,) * 3 if hi is None else hi
        self.shape = (ex, ey, ez)
        self.N = N
        self.gamma, self.Pr, self.Ma, self.Re = gamma, Pr, Ma, Re
        self.h = None
        self.buf = None
        d, _keep = box_desc(ex, ey, ez, lo, hi, deform, amp, N, orders, nodes, halo)
        mesh = _c.c_void_p()
        check(L.dg_mesh_create_box(_c.byref(d), _c.byref(mesh)))
        try:
            ne, nn, nmax = _c.c_longlong(), _c.c_longlong(), _c.c_int()
            check(L.dg_mesh_info(mesh, _c.byref(ne), _c.byref(nn), _c.byref(nmax)))
            self.E, self.nodes, self.nmax = ne.value, nn.value, nmax.value
            h = _c.c_void_p()
            cut = N // 2 if svv_cutoff is None else svv_cutoff
            ph = physics(gamma, Pr, Ma, Re, vol, surf, precision, visc, visc_eta, svv_mu, svv_kernel, cut,
                         svv_sensor, les_cs, les_model)
            check(L.dg_solver_create(mesh, _c.byref(ph), _c.byref(h)))
            self.h = h
        finally:
            L.dg_mesh_destroy(mesh)
        nb = _c.c_size_t()
        check(L.dg_solver_required_bytes(self.h, _c.byref(nb)))
        self.required_bytes = nb.value
        if bind:
            self.bind(device)

    def bind(self, device="cuda", stream=None):
        import torch
        self.buf = torch.empty(self.required_bytes + 256, dtype=torch.uint8, device=device)
        base = self.buf.data_ptr()
        ptr = (base + 255) & ~255
        if stream is None:
            stream = torch.cuda.current_stream(self.buf.device)
        self.stream = stream
        check(lib().dg_solver_bind(self.h, _c.c_void_p(ptr), self.required_bytes,
                                   _c.c_void_p(stream.cuda_stream)))

    # -- state
    def set_ic(self, ic, params=None):
        n = IC_NPARAMS[ic]
        p = np.zeros(9)
        if n:
            p[:n] = np.asarray(params, dtype=np.float64)[:n]
        check(lib().dg_set_initial_condition(self.h, IC[ic], _ptr(p)))

    def set_state(self, U):
        U = np.ascontiguousarray(U, dtype=np.float64).reshape(-1)
        check(lib().dg_set_state(self.h, _ptr(U), U.size))

    def state(self):
        U = np.empty(5 * self.nodes)
        check(lib().dg_get_state(self.h, _ptr(U), U.size))
        return U

    def residual(self, to_host=True):
        if not to_host:
            check(lib().dg_residual(self.h, None, 0))
            return None
        R = np.empty(5 * self.nodes)
        check(lib().dg_residual(self.h, _ptr(R), R.size))
        return R

    def rk_step(self, dt, nsteps=1):
        check(lib().dg_rk_step(self.h, float(dt), int(nsteps)))

    def rk_step_adaptive(self, cfl, nsteps=1):
        """nsteps steps with the step size chosen on the device before each step; returns the
        simulated time advanced."""
        t = _c.c_double(0.0)
        check(lib().dg_rk_step_adaptive(self.h, float(cfl), int(nsteps), _c.byref(t)))
        return t.value

    def diagnostics(self):
        d = Diag()
        check(lib().dg_diagnostics(self.h, _c.byref(d)))
        out = {f"mass_{k}": d.mass[i] for i, k in enumerate(["rho", "rhou", "rhov", "rhow", "rhoE"])}
        for k in ("entropy_paper", "entropy", "ke", "enstrophy", "lambda_max", "rho_min", "p_min",
                  "volume"):
            out[k] = getattr(d, k)
        out["nonfinite"] = d.nonfinite
        return out

    def diagnostics_noalloc(self, dev_out):
        """Enqueue the diagnostics into the device memory at address dev_out (a dg_diag record;
        e.g. the data_ptr of a 112-byte uint8 tensor); no allocation, no synchronisation."""
        check(lib().dg_diagnostics_noalloc(self.h, _c.c_void_p(dev_out)))

    @staticmethod
    def diag_record(raw):
        """The dg_diag record in the bytes `raw` (112 bytes, as written by diagnostics_noalloc) as
        the dict of diagnostics()."""
        d = Diag.from_buffer_copy(bytes(raw))
        out = {f"mass_{k}": d.mass[i] for i, k in enumerate(["rho", "rhou", "rhov", "rhow", "rhoE"])}
        for k in ("entropy_paper", "entropy", "ke", "enstrophy", "lambda_max", "rho_min", "p_min",
                  "volume"):
            out[k] = getattr(d, k)
        out["nonfinite"] = d.nonfinite
        return out

    def suggest_dt(self, cfl):
        dt = _c.c_double()
        check(lib().dg_suggest_dt(self.h, float(cfl), _c.byref(dt)))
        return dt.value

    def geometry(self, want_X=True, want_Ja=True, want_J=True):
        """(X, Ja, J) as host arrays; the ones not wanted are None (not copied)."""
        X = np.empty(3 * self.nodes) if want_X else None
        Ja = np.empty(9 * self.nodes) if want_Ja else None
        J = np.empty(self.nodes) if want_J else None
        check(lib().dg_get_geometry(self.h, _ptr(X) if want_X else None, _ptr(Ja) if want_Ja else None,
                                    _ptr(J) if want_J else None))
        return X, Ja, J

    def device_pointers(self):
        u, r = _c.c_void_p(), _c.c_void_p()
        check(lib().dg_device_pointers(self.h, _c.byref(u), _c.byref(r)))
        return u.value, r.value

    def profile_begin(self):
        check(lib().dg_profile_begin(self.h))

    def profile_end(self):
        p = Profile()
        check(lib().dg_profile_end(self.h, _c.byref(p)))
        return {k: {"ms": p.ms[i], "launches": p.launches[i]} for i, k in enumerate(KERNEL_CLASSES)}

    def use_graphs(self, enable=True):
        check(lib().dg_solver_use_graphs(self.h, 1 if enable else 0))

    def set_scheme(self, scheme):
        """"rk3" (Williamson, the default) or "rk4" (Carpenter-Kennedy, five stages)."""
        check(lib().dg_solver_set_scheme(self.h, SCHEME[scheme]))

    def autotune(self):
        """Pick the faster launch shape of every node-count bucket (mixed-order meshes); returns
        (tile mask, summed launch time in microseconds)."""
        b, us = _c.c_int(), _c.c_double()
        check(lib().dg_autotune(self.h, _c.byref(b), _c.byref(us)))
        return b.value, us.value

    def set_tiles(self, tiles):
        check(lib().dg_solver_set_tiles(self.h, int(tiles)))

    def synchronize(self):
        check(lib().dg_synchronize(self.h))

    def close(self):
        if self.h:
            lib().dg_solver_destroy(self.h)
            self.h = None
        self.buf = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Solvers advanced together on one stream (one launch per order/precision group).

    `stream` (a torch.cuda.Stream) defaults to the first member's stream.  Work the members
    have pending on other streams must be complete (or ordered before) the batch's steps.
    """

    def __init__(self, solvers, stream=None):
        self.h = None
        self.solvers = list(solvers)
        self.stream = self.solvers[0].stream if stream is None else stream
        arr = (_c.c_void_p * len(self.solvers))(*[s.h for s in self.solvers])
        h = _c.c_void_p()
        check(lib().dg_batch_create(arr, len(self.solvers), _c.c_void_p(self.stream.cuda_stream),
                                    _c.byref(h)))
        self.h = h

    def rk_step(self, dts, nsteps=1):
        d = np.ascontiguousarray(dts, dtype=np.float64).reshape(-1)
        if d.size != len(self.solvers):
            raise ValueError("one dt per member")
        check(lib().dg_batch_rk_step(self.h, _ptr(d), int(nsteps)))

    def use_graphs(self, enable=True):
        check(lib().dg_batch_use_graphs(self.h, 1 if enable else 0))

    def launches_per_stage(self):
        k = _c.c_int()
        check(lib().dg_batch_launches(self.h, _c.byref(k)))
        return k.value

    def close(self):
        if self.h:
            lib().dg_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
