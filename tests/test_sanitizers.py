"""AddressSanitizer / UndefinedBehaviorSanitizer builds of the CPU-side code (CPU only, no GPU):

- the oracle (plain C), built with gcc -fsanitize=address,undefined, runs residuals of every
  configuration family (Euler and Navier-Stokes on a deformed mesh, mixed orders, Gauss-Legendre
  points, spectral vanishing viscosity), RK steps, diagnostics and the point functions;
- the library's host code (argument checks, mesh and memory plan, Gauss-Lobatto tables), whose
  two host translation units are rebuilt with the sanitizers on their host pass only, runs the
  entry points that need no GPU, on valid and invalid input.

Each runs in a child process with the sanitizer runtime preloaded; any report fails the test."""
import os
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
REPORT_MARKERS = ("ERROR: AddressSanitizer", "runtime error:", "ERROR: LeakSanitizer")


def _run_child(code, env_extra):
    env = dict(os.environ)
    env.update(env_extra)
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    for m in REPORT_MARKERS:
        assert m not in out, out[-4000:]
    return r.stdout


def test_oracle_under_asan_ubsan(tmp_path):
    src = os.path.join(ROOT, "oracle", "dgsem_oracle.c")
    for name, extra in (("liborc64.so", []), ("liborc80.so", ["-DORC_LONG_DOUBLE"])):
        subprocess.run(["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                        "-fno-sanitize-recover=undefined", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
                        "-std=c11", *extra, "-o", str(tmp_path / name), src, "-lm"], check=True)
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    ubsan = subprocess.run(["gcc", "-print-file-name=libubsan.so"], capture_output=True, text=True).stdout.strip()
    code = textwrap.dedent(f"""
        import sys, numpy as np
        sys.path.insert(0, {ROOT!r})
        import oracle
        from paper_2206_09733_amd import synth
        oracle.set_threads(2)
        cases = [dict(ex=2, N=3, deform=True, Ma=0.3),
                 dict(ex=2, N=4, deform=True, Ma=0.1, Re=1600.0),
                 dict(ex=2, N=3, Ma=0.3, Re=400.0, visc="br2"),
                 dict(ex=2, N=3, Ma=0.3, Re=400.0, visc="ip", vol="kg", surf="es_matrix"),
                 dict(ex=2, orders=synth.mixed_orders(8, seed=1), Ma=0.5, lo=(-10.0,) * 3, hi=(10.0,) * 3),
                 dict(ex=2, N=4, Ma=0.3, vol="central", surf="roe", nodes="gauss", Re=800.0)]
        for c in cases:
            for prec in ("fp64", "fp80"):
                o = oracle.OracleSolver(**c, precision=prec)
                if "orders" in c:
                    o.set_ic("vortex", [5.0, 0.0, 0.0, 0.4, 0.4])
                else:
                    o.set_ic("tgv")
                R = o.residual()
                assert np.isfinite(R).all()
                o.rk(o.suggest_dt(0.5), 1, "rk3")
                o.rk(o.suggest_dt(0.5), 1, "rk4")
                d = o.diagnostics()
                assert d["nonfinite"] == 0
                o.close()
        o = oracle.OracleSolver(ex=2, N=4, deform=True, Ma=0.3)
        o.set_ic("tgv")
        o.set_svv(0.02, "maday", 2, 1e-3)
        R, form = o.svv_residual()
        assert np.isfinite(R).all()
        o.svv_sensor()
        g = synth.state_pairs(4, 0)
        for a, b in zip(g[0], g[1]):
            UL = np.r_[a[0], a[0] * a[1:4], a[4] / 0.4 + 0.5 * a[0] * (a[1:4] ** 2).sum()]
            UR = np.r_[b[0], b[0] * b[1:4], b[4] / 0.4 + 0.5 * b[0] * (b[1:4] ** 2).sum()]
            for k in oracle.SURF:
                oracle.riemann(k, UL, UR, np.array([0.3, -0.2, 0.9]))
            for k in oracle.VOL:
                oracle.two_point(k, UL, UR, np.array([0.3, -0.2, 0.9]))
        for N in range(1, 8):
            oracle.gll(N); oracle.gl(N)
            oracle.svv_filter(N, np.ones((N + 1) ** 3), "tadmor", N // 2)
        print("ORACLE OK", flush=True)
    """)
    out = _run_child(code, {"LD_PRELOAD": f"{asan}:{ubsan}", "ORACLE_LIB_DIR": str(tmp_path)})
    assert "ORACLE OK" in out


def test_library_host_code_under_asan_ubsan(tmp_path):
    from paper_2206_09733_amd import build
    if not os.path.isdir(build.OBJ) or not all(os.path.exists(os.path.join(build.OBJ, s + ".o"))
                                                for s in build.SOURCES):
        build.build()
    host_sources = ["api.cpp", "gll_host.cpp"]
    objs = [os.path.join(build.OBJ, s + ".o") for s in build.SOURCES if s not in host_sources]
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]
    for s in host_sources:
        out = str(tmp_path / (s + ".o"))
        subprocess.run([build.HIPCC, *build.FLAGS, "-g", *san, "-x", "hip", "-c", os.path.join(build.CSRC, s),
                        "-o", out], check=True, capture_output=True)
        objs.append(out)
    lib = str(tmp_path / "libdgsem_san.so")
    subprocess.run([build.HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *san, "-o", lib, *objs], check=True,
                   capture_output=True)
    rt = subprocess.run([os.path.join(os.path.dirname(build.HIPCC), "..", "llvm", "bin", "clang"),
                         "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True).stdout.strip()
    if not os.path.exists(rt):
        pytest.skip("clang's AddressSanitizer runtime is not installed")
    code = textwrap.dedent(f"""
        import ctypes, sys
        sys.path.insert(0, {ROOT!r})
        import numpy as np
        from paper_2206_09733_amd import dgsem, synth
        L = ctypes.CDLL({lib!r})
        vp = ctypes.c_void_p
        L.dg_last_error.restype = ctypes.c_char_p
        def mesh(*a, **k):
            d, keep = dgsem.box_desc(*a, **k)
            m = vp()
            rc = L.dg_mesh_create_box(ctypes.byref(d), ctypes.byref(m))
            return rc, m, keep
        # invalid meshes
        for a in ((0, 2, 2, (0, 0, 0), (1, 1, 1), False, 0.0, 3), (2, 2, 2, (0, 0, 0), (1, -1, 1), False, 0.0, 3),
                  (2, 2, 2, (0, 0, 0), (1, 1, 1), False, 0.0, 9)):
            rc, m, _ = mesh(*a)
            assert rc != 0 and L.dg_last_error()
        rc, m, _ = mesh(2, 1, 1, (0, 0, 0), (1, 1, 1), False, 0.0, 3, orders=[3, 3, 3, 7, 3, 3])
        assert rc == dgsem.DG_EUNSUPPORTED
        rc, m, _ = mesh(2, 2, 2, (0, 0, 0), (1, 1, 1), False, 0.0, 3, orders=[2, 3, 3] * 8, nodes="gauss")
        assert rc == dgsem.DG_EUNSUPPORTED
        rc, m, _ = mesh(2, 2, 2, (0, 0, 0), (1, 1, 1), False, 0.0, 3, nodes="gauss", halo=True)
        assert rc == dgsem.DG_EUNSUPPORTED
        # valid meshes and solvers of every option family, their memory plans, then destroy
        specs = [((3, 2, 4, (0, 0, 0), (1, 1, 1), True, 0.05, 4), {{}}),
                 ((3, 3, 3, (-1, -1, -1), (1, 1, 1), False, 0.0, 3), dict(orders=synth.mixed_orders(27, seed=3))),
                 ((2, 2, 2, (0, 0, 0), (1, 1, 1), False, 0.0, 5), dict(nodes="gauss")),
                 ((2, 3, 2, (0, 0, 0), (1, 1, 1), True, 0.05, 4), dict(nodes="gauss")),
                 ((1, 3, 2, (0, 0, 0), (1, 1, 1), True, 0.05, 3), dict(halo=True))]
        phys = [dgsem.physics(Ma=0.1), dgsem.physics(Ma=0.1, Re=1600.0, precision="fp32_bulk"),
                dgsem.physics(Ma=0.3, Re=400.0, visc="ip", vol="kg", surf="es_matrix"),
                dgsem.physics(Ma=0.3, svv_mu=0.01, svv_kernel="tadmor", svv_cutoff=2),
                dgsem.physics(Ma=0.3, vol="central"), dgsem.physics(Ma=0.0), dgsem.physics(Ma=0.1, vol="morinishi", surf="lf_global")]
        phys[-1].vol_flux = 99
        n_ok = 0
        for a, k in specs:
            rc, m, keep = mesh(*a, **k)
            assert rc == 0, L.dg_last_error()
            ne, nn, nmax = ctypes.c_longlong(), ctypes.c_longlong(), ctypes.c_int()
            assert L.dg_mesh_info(m, ctypes.byref(ne), ctypes.byref(nn), ctypes.byref(nmax)) == 0
            for p in phys:
                s = vp()
                rc = L.dg_solver_create(m, ctypes.byref(p), ctypes.byref(s))
                if rc == 0:
                    nb = ctypes.c_size_t()
                    assert L.dg_solver_required_bytes(s, ctypes.byref(nb)) == 0 and nb.value > 0
                    # calls that need a bound solver answer DG_ESTATE without touching a GPU
                    assert L.dg_rk_step(s, ctypes.c_double(1e-3), 1) == dgsem.DG_ESTATE
                    L.dg_solver_destroy(s)
                    n_ok += 1
                else:
                    assert L.dg_last_error()
            L.dg_mesh_destroy(m)
        assert n_ok >= 6, n_ok
        print("LIBRARY OK", flush=True)
    """)
    out = _run_child(code, {"LD_PRELOAD": rt})
    assert "LIBRARY OK" in out
