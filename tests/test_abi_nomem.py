"""No exception crosses the C ABI: a host allocation that fails inside an entry point is
reported as DG_ENOMEM with a message, and the process goes on (CPU only, no GPU needed).

The failure is forced in a child process whose address space is capped (RLIMIT_AS) after the
library is loaded; dg_solver_create of a 1024^3-element mesh then cannot allocate its 8 GiB
element offset table."""
import os
import subprocess
import sys
import textwrap

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = textwrap.dedent("""
    import ctypes, resource, sys
    sys.path.insert(0, {root!r})
    from paper_2206_09733_amd import dgsem
    L = dgsem.lib()
    m = ctypes.c_void_p()
    d, _ = dgsem.box_desc(1024, 1024, 1024, (0, 0, 0), (1, 1, 1), False, 0.0, 3)
    dgsem.check(L.dg_mesh_create_box(ctypes.byref(d), ctypes.byref(m)))
    vm = 0
    for line in open("/proc/self/status"):
        if line.startswith("VmSize:"):
            vm = int(line.split()[1]) * 1024
    cap = vm + (1 << 30)
    resource.setrlimit(resource.RLIMIT_AS, (cap, resource.RLIM_INFINITY))
    ph = dgsem.physics(Ma=0.1)
    s = ctypes.c_void_p(123)
    rc = L.dg_solver_create(m, ctypes.byref(ph), ctypes.byref(s))
    msg = L.dg_last_error().decode()
    print("RC", rc, "HANDLE", s.value, "MSG", msg, flush=True)
    # the library still answers afterwards
    n = ctypes.c_longlong()
    rc2 = L.dg_mesh_info(m, None, ctypes.byref(n), None)
    print("INFO", rc2, n.value, flush=True)
    L.dg_mesh_destroy(m)
""")


def test_host_allocation_failure_is_reported_not_thrown():
    from paper_2206_09733_amd import dgsem
    if not os.path.exists(dgsem.LIB_PATH):
        from paper_2206_09733_amd import build
        build.build()
    r = subprocess.run([sys.executable, "-c", CHILD.format(root=ROOT)], capture_output=True, text=True,
                       timeout=300)
    out = r.stdout
    assert r.returncode == 0, (r.returncode, out, r.stderr[-2000:])
    line = next(l for l in out.splitlines() if l.startswith("RC "))
    parts = line.split()
    assert int(parts[1]) == dgsem.DG_ENOMEM, line
    assert parts[3] in ("None", "0"), line          # no handle on failure
    assert "allocation" in line, line
    info = next(l for l in out.splitlines() if l.startswith("INFO ")).split()
    assert int(info[1]) == dgsem.DG_OK and int(info[2]) == 1024 ** 3 * 64
