"""dg_diagnostics_noalloc (the entry point for callers that cannot allocate: its scratch is a
static device array of the library) against dg_diagnostics, through the C ABI: bitwise equal
on two calls in a row, the second on a smaller mesh, then a mixed-order mesh; a mesh above the
scratch's 32768 elements is refused."""
import numpy as np
import pytest

from paper_2206_09733_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dg():
    from paper_2206_09733_amd import dgsem
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    dgsem.lib()
    return dgsem


def _noalloc(dg, s):
    import torch
    out = torch.full((112,), 255, dtype=torch.uint8, device="cuda")
    s.diagnostics_noalloc(out.data_ptr())
    s.synchronize()
    return dg.Solver.diag_record(out.cpu().numpy().tobytes())


def _same(a, b):
    for k in a:
        assert (a[k] == b[k]) or (np.isnan(a[k]) and np.isnan(b[k])), (k, a[k], b[k])


def test_noalloc_diagnostics_equal_dg_diagnostics(dg):
    cases = [dict(ex=8, N=4, deform=True, Ma=0.1, Re=1600.0),      # 512 elements
             dict(ex=3, N=3, Ma=0.3),                               # 27 elements, after a larger one
             dict(ex=3, orders=synth.mixed_orders(27, seed=4), Ma=0.5, lo=(-10.0,) * 3, hi=(10.0,) * 3)]
    for c in cases:
        print(f"[noalloc] case {c.get('ex')} N={c.get('N')} mixed={'orders' in c}", flush=True)
        s = dg.Solver(**c)
        if "orders" in c:
            s.set_ic("vortex", [5.0, 0.0, 0.0, 0.4, 0.4])
        else:
            s.set_ic("tgv")
        s.rk_step(s.suggest_dt(0.5), 2)
        ref = s.diagnostics()
        got = _noalloc(dg, s)
        _same(ref, got)
        assert got["nonfinite"] == 0 and got["volume"] > 0
        s.close()


def test_noalloc_diagnostics_rejects_large_mesh(dg):
    import torch
    s = dg.Solver(ex=33, N=1, Ma=0.3)  # 35937 elements > 32768
    s.set_ic("tgv")
    out = torch.zeros(112, dtype=torch.uint8, device="cuda")
    with pytest.raises(dg.DgError) as ei:
        s.diagnostics_noalloc(out.data_ptr())
    assert ei.value.code == dg.DG_EUNSUPPORTED
    assert "32768" in str(ei.value)
    s.close()
