"""The C-ABI library loads, exports every entry point that include/dgsem.h declares, and its
host-side argument checks answer with the documented codes -- without touching a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    src = open(os.path.join(ROOT, "include", "dgsem.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|void|const char\s*\*)\s*(dg_\w+)\s*\(", src, flags=re.M)))


@pytest.fixture(scope="module")
def dg():
    from paper_2206_09733_amd import dgsem
    if not os.path.exists(dgsem.LIB_PATH):
        from paper_2206_09733_amd import build
        build.build()
    return dgsem


def test_library_exports_every_declared_symbol(dg):
    names = _header_functions()
    assert len(names) >= 18, names
    L = dg.lib()
    for n in names:
        assert hasattr(L, n), n
    assert set(dg.EXPORTS) <= set(names)


def test_mesh_argument_errors(dg):
    L = dg.lib()
    m = ctypes.c_void_p()
    d, _ = dg.box_desc(0, 2, 2, (0, 0, 0), (1, 1, 1), False, 0.0, 3)
    assert L.dg_mesh_create_box(ctypes.byref(d), ctypes.byref(m)) == dg.DG_EINVAL
    assert b"element" in L.dg_last_error()
    d, _ = dg.box_desc(2, 2, 2, (0, 0, 0), (1, -1, 1), False, 0.0, 3)
    assert L.dg_mesh_create_box(ctypes.byref(d), ctypes.byref(m)) == dg.DG_EINVAL
    d, _ = dg.box_desc(2, 2, 2, (0, 0, 0), (1, 1, 1), False, 0.0, 8)
    assert L.dg_mesh_create_box(ctypes.byref(d), ctypes.byref(m)) == dg.DG_EINVAL
    # mixed orders are taken up to 6; an order 7 element in a mixed mesh is refused
    d, _ = dg.box_desc(2, 1, 1, (0, 0, 0), (1, 1, 1), False, 0.0, 3, orders=[3, 3, 3, 7, 3, 3])
    assert L.dg_mesh_create_box(ctypes.byref(d), ctypes.byref(m)) == dg.DG_EUNSUPPORTED
    d, _ = dg.box_desc(2, 1, 1, (0, 0, 0), (1, 1, 1), False, 0.0, 3, orders=[3, 3, 3, 0, 3, 3])
    assert L.dg_mesh_create_box(ctypes.byref(d), ctypes.byref(m)) == dg.DG_EINVAL
    # all-equal orders make a uniform mesh, even at order 7
    d, _ = dg.box_desc(2, 1, 1, (0, 0, 0), (1, 1, 1), False, 0.0, 3, orders=[7] * 6)
    assert L.dg_mesh_create_box(ctypes.byref(d), ctypes.byref(m)) == dg.DG_OK
    L.dg_mesh_destroy(m)
    d, _ = dg.box_desc(2, 3, 4, (0, 0, 0), (1, 1, 1), True, 0.05, 4)
    assert L.dg_mesh_create_box(ctypes.byref(d), ctypes.byref(m)) == dg.DG_OK
    ne, nn, nmax = ctypes.c_longlong(), ctypes.c_longlong(), ctypes.c_int()
    assert L.dg_mesh_info(m, ctypes.byref(ne), ctypes.byref(nn), ctypes.byref(nmax)) == 0
    assert (ne.value, nn.value, nmax.value) == (24, 24 * 125, 4)
    L.dg_mesh_destroy(m)


def _mesh(dg, ex=2, N=3):
    L = dg.lib()
    m = ctypes.c_void_p()
    d, _ = dg.box_desc(ex, ex, ex, (0, 0, 0), (1, 1, 1), False, 0.0, N)
    dg.check(L.dg_mesh_create_box(ctypes.byref(d), ctypes.byref(m)))
    return m


def test_gauss_legendre_limits(dg):
    """Gauss-Legendre nodes: uniform-order boxes (undeformed or deformed), FP64, central volume
    form, BR1."""
    L = dg.lib()
    m = ctypes.c_void_p()
    d, _ = dg.box_desc(2, 2, 2, (0, 0, 0), (1, 1, 1), True, 0.05, 3, nodes="gauss")
    dg.check(L.dg_mesh_create_box(ctypes.byref(d), ctypes.byref(m)))
    L.dg_mesh_destroy(m)
    d, _k = dg.box_desc(2, 2, 2, (0, 0, 0), (1, 1, 1), False, 0.0, 3, orders=[2, 3, 3] * 8, nodes="gauss")
    assert L.dg_mesh_create_box(ctypes.byref(d), ctypes.byref(m)) == dg.DG_EUNSUPPORTED
    d, _ = dg.box_desc(2, 2, 2, (0, 0, 0), (1, 1, 1), False, 0.0, 3)
    d.nodes = 2
    assert L.dg_mesh_create_box(ctypes.byref(d), ctypes.byref(m)) == dg.DG_EINVAL
    d, _ = dg.box_desc(2, 2, 2, (0, 0, 0), (1, 1, 1), False, 0.0, 3, nodes="gauss")
    dg.check(L.dg_mesh_create_box(ctypes.byref(d), ctypes.byref(m)))
    s = ctypes.c_void_p()
    for bad in (dict(vol="ec"), dict(vol="central", precision="fp32_bulk")):
        p = dg.physics(**bad)
        assert L.dg_solver_create(m, ctypes.byref(p), ctypes.byref(s)) == dg.DG_EUNSUPPORTED, bad
    for visc in ("br1", "br2", "ip"):
        p = dg.physics(vol="central", Re=100.0, visc=visc)
        dg.check(L.dg_solver_create(m, ctypes.byref(p), ctypes.byref(s)))
        L.dg_solver_destroy(s)
    for surf in dg.SURF:
        p = dg.physics(vol="central", surf=surf, Re=100.0 if surf == "roe" else 0.0)
        assert L.dg_solver_create(m, ctypes.byref(p), ctypes.byref(s)) == dg.DG_OK
        L.dg_solver_destroy(s)
    L.dg_mesh_destroy(m)


def test_solver_argument_errors_and_sizes(dg):
    L = dg.lib()
    m = _mesh(dg, 2, 3)
    s = ctypes.c_void_p()
    for bad in (dict(gamma=1.0), dict(vol="ec", surf="roe", precision="fp64", Ma=-1.0)):
        p = dg.physics(**bad)
        assert L.dg_solver_create(m, ctypes.byref(p), ctypes.byref(s)) == dg.DG_EINVAL
    for vol, surf in ((7, 0), (0, 9), (-1, 0), (0, -1)):
        p = dg.physics()
        p.vol_flux, p.surf_flux = vol, surf
        assert L.dg_solver_create(m, ctypes.byref(p), ctypes.byref(s)) == dg.DG_EINVAL
    for vf, eta in ((3, 0.0), (-1, 0.0), (1, -1.0), (2, float("nan"))):
        p = dg.physics(Re=100.0)
        p.visc_flux, p.visc_eta = vf, eta
        assert L.dg_solver_create(m, ctypes.byref(p), ctypes.byref(s)) == dg.DG_EINVAL
    # FP32-bulk covers the EC / central volume fluxes and the first four surface fluxes only
    for vol, surf in (("ir", "roe"), ("kg", "roe"), ("morinishi", "llf"), ("ec", "es"),
                      ("ec", "es_matrix"), ("central", "ld_roe")):
        p = dg.physics(vol=vol, surf=surf, precision="fp32_bulk")
        assert L.dg_solver_create(m, ctypes.byref(p), ctypes.byref(s)) == dg.DG_EUNSUPPORTED
    for vol in dg.VOL:
        for surf in dg.SURF:
            p = dg.physics(vol=vol, surf=surf)
            assert L.dg_solver_create(m, ctypes.byref(p), ctypes.byref(s)) == dg.DG_OK, (vol, surf)
            L.dg_solver_destroy(s)
    p = dg.physics(Re=100.0)
    assert L.dg_solver_create(m, ctypes.byref(p), ctypes.byref(s)) == dg.DG_OK
    nb = ctypes.c_size_t()
    assert L.dg_solver_required_bytes(s, ctypes.byref(nb)) == 0
    nodes = 8 * 64
    assert nb.value >= 8 * nodes * (5 * 4 + 3 + 9 + 2)
    assert L.dg_solver_set_scheme(s, 2) == dg.DG_EINVAL
    assert L.dg_solver_set_scheme(s, 1) == dg.DG_OK
    # a too-small buffer is refused before any device work
    assert L.dg_solver_bind(s, ctypes.c_void_p(256), nb.value - 1, None) == dg.DG_ENOMEM
    assert b"smaller" in L.dg_last_error()
    assert L.dg_solver_bind(s, None, nb.value, None) == dg.DG_EINVAL
    # calls that need device memory refuse an unbound solver
    assert L.dg_rk_step(s, ctypes.c_double(1e-3), 1) == dg.DG_ESTATE
    assert L.dg_rk_step_adaptive(s, ctypes.c_double(0.5), 1, None) == dg.DG_ESTATE
    assert L.dg_residual(s, None, 0) == dg.DG_ESTATE
    L.dg_solver_destroy(s)
    L.dg_mesh_destroy(m)


def test_required_bytes_c2_fits_one_gpu(dg):
    """32^3 elements, N = 4, Navier-Stokes: ~1.3 GB, far below 288 GB of HBM."""
    L = dg.lib()
    m = ctypes.c_void_p()
    d, _ = dg.box_desc(32, 32, 32, (0, 0, 0), (6.283185307179586,) * 3, True, 0.05, 4)
    dg.check(L.dg_mesh_create_box(ctypes.byref(d), ctypes.byref(m)))
    s = ctypes.c_void_p()
    p = dg.physics(Re=1600.0)
    dg.check(L.dg_solver_create(m, ctypes.byref(p), ctypes.byref(s)))
    nb = ctypes.c_size_t()
    dg.check(L.dg_solver_required_bytes(s, ctypes.byref(nb)))
    assert 1.0e9 < nb.value < 2.0e9
    L.dg_solver_destroy(s)
    L.dg_mesh_destroy(m)


def test_mixed_order_mesh_info_and_solver_limits(dg):
    L = dg.lib()
    m = ctypes.c_void_p()
    orders = [1, 2, 3, 6, 5, 4, 2, 2, 2]
    d, _keep = dg.box_desc(3, 1, 1, (0, 0, 0), (1, 1, 1), False, 0.0, 3, orders=orders)
    dg.check(L.dg_mesh_create_box(ctypes.byref(d), ctypes.byref(m)))
    ne, nn, nmax = ctypes.c_longlong(), ctypes.c_longlong(), ctypes.c_int()
    dg.check(L.dg_mesh_info(m, ctypes.byref(ne), ctypes.byref(nn), ctypes.byref(nmax)))
    assert (ne.value, nn.value, nmax.value) == (3, 2 * 3 * 4 + 7 * 6 * 5 + 27, 6)
    s = ctypes.c_void_p()
    p = dg.physics(Re=100.0)
    assert L.dg_solver_create(m, ctypes.byref(p), ctypes.byref(s)) == dg.DG_EUNSUPPORTED
    assert b"mixed" in L.dg_last_error()
    p = dg.physics(Ma=0.5, precision="fp32_bulk")
    dg.check(L.dg_solver_create(m, ctypes.byref(p), ctypes.byref(s)))
    assert L.dg_solver_set_tiles(s, 64) == dg.DG_EINVAL
    assert L.dg_solver_set_tiles(s, 0b100101) == dg.DG_OK
    L.dg_solver_destroy(s)
    p = dg.physics(Ma=0.5)
    dg.check(L.dg_solver_create(m, ctypes.byref(p), ctypes.byref(s)))
    nb = ctypes.c_size_t()
    dg.check(L.dg_solver_required_bytes(s, ctypes.byref(nb)))
    assert nb.value >= 8 * nn.value * (5 * 4 + 3 + 9 + 2)
    # unbound: graph switch is host state, autotuning needs the device
    assert L.dg_solver_use_graphs(s, 0) == dg.DG_OK
    assert L.dg_autotune(s, None, None) == dg.DG_ESTATE
    L.dg_solver_destroy(s)
    L.dg_mesh_destroy(m)


def test_spectral_vanishing_viscosity_limits(dg):
    """SVV: uniform-order Lobatto meshes, either precision (not Gauss-Legendre); kernel, cutoff and
    viscosity checked; the workspace grows by the filtered-flux buffer (12 doubles per node) and
    the filter table."""
    L = dg.lib()
    m, s = ctypes.c_void_p(), ctypes.c_void_p()
    d, _ = dg.box_desc(2, 2, 2, (0, 0, 0), (1, 1, 1), True, 0.05, 3)
    dg.check(L.dg_mesh_create_box(ctypes.byref(d), ctypes.byref(m)))
    sizes = []
    for svv in (0.0, 0.05):
        p = dg.physics(svv_mu=svv, svv_cutoff=1)
        dg.check(L.dg_solver_create(m, ctypes.byref(p), ctypes.byref(s)))
        nb = ctypes.c_size_t()
        dg.check(L.dg_solver_required_bytes(s, ctypes.byref(nb)))
        sizes.append(nb.value)
        L.dg_solver_destroy(s)
    assert sizes[1] - sizes[0] >= 12 * 8 * 8 * 64 + 16 * 8
    for bad in (dict(svv_mu=-1.0), dict(svv_mu=float("nan")), dict(svv_mu=0.1, svv_cutoff=4),
                dict(svv_mu=0.1, svv_cutoff=-2), dict(svv_mu=0.1, svv_sensor=float("nan")),
                dict(svv_mu=0.1, Pr=0.0)):
        p = dg.physics(**bad)
        assert L.dg_solver_create(m, ctypes.byref(p), ctypes.byref(s)) == dg.DG_EINVAL, bad
    p = dg.physics(svv_mu=0.1)
    p.svv_kernel = 2
    assert L.dg_solver_create(m, ctypes.byref(p), ctypes.byref(s)) == dg.DG_EINVAL
    # FP32-bulk solvers take the term too (formed in FP64 after their stage): same buffers
    for prec in ("fp32_bulk",):
        nb2 = []
        for svv in (0.0, 0.05):
            p = dg.physics(svv_mu=svv, svv_cutoff=1, precision=prec)
            dg.check(L.dg_solver_create(m, ctypes.byref(p), ctypes.byref(s)))
            nb = ctypes.c_size_t()
            dg.check(L.dg_solver_required_bytes(s, ctypes.byref(nb)))
            nb2.append(nb.value)
            L.dg_solver_destroy(s)
        assert nb2[1] - nb2[0] == sizes[1] - sizes[0]
    dg_gauss, _ = dg.box_desc(2, 2, 2, (0, 0, 0), (1, 1, 1), False, 0.0, 3, nodes="gauss")
    mg = ctypes.c_void_p()
    dg.check(L.dg_mesh_create_box(ctypes.byref(dg_gauss), ctypes.byref(mg)))
    p = dg.physics(svv_mu=0.1, vol="central")
    assert L.dg_solver_create(mg, ctypes.byref(p), ctypes.byref(s)) == dg.DG_EUNSUPPORTED
    L.dg_mesh_destroy(mg)
    for kernel, cut in (("tadmor", -1), ("maday", 3), ("tadmor", 0)):
        p = dg.physics(svv_mu=0.1, svv_kernel=kernel, svv_cutoff=cut, Re=100.0)
        assert L.dg_solver_create(m, ctypes.byref(p), ctypes.byref(s)) == dg.DG_OK
        L.dg_solver_destroy(s)
    # the explicit LES closure alone switches the term on (same buffers, same checks)
    p = dg.physics(les_cs=0.17, svv_cutoff=1)
    dg.check(L.dg_solver_create(m, ctypes.byref(p), ctypes.byref(s)))
    nb = ctypes.c_size_t()
    dg.check(L.dg_solver_required_bytes(s, ctypes.byref(nb)))
    assert nb.value == sizes[1]
    L.dg_solver_destroy(s)
    for bad in (dict(les_cs=-0.1), dict(les_cs=float("nan")), dict(les_cs=float("inf")),
                dict(les_cs=0.1, svv_cutoff=4)):
        p = dg.physics(**bad)
        assert L.dg_solver_create(m, ctypes.byref(p), ctypes.byref(s)) == dg.DG_EINVAL, bad
    for model in ("wale", "vreman"):
        p = dg.physics(les_cs=0.3, les_model=model, svv_cutoff=1)
        dg.check(L.dg_solver_create(m, ctypes.byref(p), ctypes.byref(s)))
        L.dg_solver_destroy(s)
    p = dg.physics(les_cs=0.1, svv_cutoff=1)
    p.les_model = 3
    assert L.dg_solver_create(m, ctypes.byref(p), ctypes.byref(s)) == dg.DG_EINVAL
    p.les_cs = 0.0  # the model code is read only with the closure on
    dg.check(L.dg_solver_create(m, ctypes.byref(p), ctypes.byref(s)))
    L.dg_solver_destroy(s)
    p = dg.physics(les_cs=0.1, precision="fp32_bulk")
    dg.check(L.dg_solver_create(m, ctypes.byref(p), ctypes.byref(s)))
    L.dg_solver_destroy(s)
    L.dg_mesh_destroy(m)
    for kw in (dict(orders=[2, 3, 3] * 8), dict(nodes="gauss")):
        d, _k = dg.box_desc(2, 2, 2, (0, 0, 0), (1, 1, 1), False, 0.0, 3, **kw)
        dg.check(L.dg_mesh_create_box(ctypes.byref(d), ctypes.byref(m)))
        p = dg.physics(svv_mu=0.1, vol="central", svv_cutoff=1)
        assert L.dg_solver_create(m, ctypes.byref(p), ctypes.byref(s)) == dg.DG_EUNSUPPORTED, kw
        p = dg.physics(les_cs=0.1, vol="central", svv_cutoff=1)
        assert L.dg_solver_create(m, ctypes.byref(p), ctypes.byref(s)) == dg.DG_EUNSUPPORTED, kw
        L.dg_mesh_destroy(m)


def test_halo_box_limits_and_sizes(dg):
    """Halo boxes (the box as one block of a split domain): uniform-order Gauss-Lobatto only; the
    buffer grows by the ghost elements' state (two copies), Jacobian, face viscous fluxes and (with
    spectral vanishing viscosity) filtered flux, the map and the send / receive buffers."""
    L = dg.lib()
    m = ctypes.c_void_p()
    d, _ = dg.box_desc(3, 2, 4, (0, 0, 0), (1, 1, 1), False, 0.0, 3)
    d.halo = 2
    assert L.dg_mesh_create_box(ctypes.byref(d), ctypes.byref(m)) == dg.DG_EINVAL
    for kw in (dict(orders=[2, 3, 3] * 24), dict(nodes="gauss")):
        d, _k = dg.box_desc(3, 2, 4, (0, 0, 0), (1, 1, 1), False, 0.0, 3, halo=True, **kw)
        assert L.dg_mesh_create_box(ctypes.byref(d), ctypes.byref(m)) == dg.DG_EUNSUPPORTED, kw
    sizes = {}
    for halo in (False, True):
        d, _ = dg.box_desc(3, 2, 4, (0, 0, 0), (1, 1, 1), False, 0.0, 3, halo=halo)
        dg.check(L.dg_mesh_create_box(ctypes.byref(d), ctypes.byref(m)))
        s = ctypes.c_void_p()
        cases = ((0.0, "br1", "fp64", 0.0), (100.0, "br1", "fp64", 0.0), (100.0, "br2", "fp32_bulk", 0.0),
                 (100.0, "ip", "fp64", 0.0), (100.0, "br1", "fp64", 0.1), (0.0, "br1", "fp64", 0.1))
        for Re, visc, prec, svv in cases:
            p = dg.physics(Re=Re, visc=visc, precision=prec, svv_mu=svv, svv_cutoff=1)
            dg.check(L.dg_solver_create(m, ctypes.byref(p), ctypes.byref(s)))
            nb = ctypes.c_size_t()
            dg.check(L.dg_solver_required_bytes(s, ctypes.byref(nb)))
            sizes[(halo, Re, visc, svv)] = nb.value
            L.dg_solver_destroy(s)
        L.dg_mesh_destroy(m)
    K, nn, nf = 2 * (2 * 4 + 3 * 4 + 3 * 2), 64, 16
    for Re, visc, _, svv in cases:
        extra = sizes[(True, Re, visc, svv)] - sizes[(False, Re, visc, svv)]
        least = 8 * (2 * 5 * K * nn + K * nn + 2 * 5 * K * nf) + 16 * K
        if Re > 0:
            least += 8 * (K * 6 * 4 * nf + 2 * 4 * K * nf)
        if svv > 0:
            least += 8 * 12 * K * nn
        assert least <= extra <= least + 256 * 8, (Re, visc, svv, extra, least)
