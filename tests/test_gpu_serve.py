"""Serving loop on the GPU: solves arriving over time are admitted, batched with the running
ones and returned; each result is bitwise the state the same solve reaches alone."""
import numpy as np
import pytest

from paper_2206_09733_amd import serve, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dg():
    from paper_2206_09733_amd import dgsem
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    dgsem.lib()
    return dgsem


def small_requests(n, seed, steps, mixed_precision=False):
    g = synth.rng(seed)
    arr = synth.poisson_arrivals(n, 400.0, seed)
    out = []
    for i in range(n):
        viscous = bool(g.integers(0, 2))
        out.append(serve.Request(id=i, E=int(g.integers(2, 6)), N=int(g.integers(3, 6)),
                                 Ma=float(g.uniform(0.1, 0.8)),
                                 Re=float(g.uniform(400.0, 3200.0)) if viscous else 0.0,
                                 steps=steps + int(g.integers(0, 9)), arrival=float(arr[i]),
                                 precision="fp32_bulk" if mixed_precision and i % 2 else "fp64"))
    return out


@pytest.mark.parametrize("mixed_precision", [False, True])
def test_served_results_equal_alone(dg, mixed_precision):
    """Each served result equals the same solve advanced alone, bitwise, also when FP64 and
    FP32-bulk requests share the loop (they are batched in groups of their own precision)."""
    reqs = small_requests(16, seed=5, steps=12, mixed_precision=mixed_precision)
    ex = serve.GpuExecutor()
    budget = 3 * max(ex.required_bytes(q) for q in reqs)   # memory, not arrivals, limits the mix
    sch = serve.Scheduler(ex, budget, max_active=8, chunk_steps=5)
    import time
    t0 = time.perf_counter()
    res = sch.run(reqs)
    wall = time.perf_counter() - t0
    ex.close()
    st = serve.summarize(reqs, res, wall)
    print(f"[serve 16] {st} chunks {sch.chunks} peak active {sch.peak_active} peak bytes {sch.peak_bytes}",
          flush=True)
    assert st["completed"] == 16
    assert sch.peak_bytes <= budget and sch.peak_active > 1
    for q, r in zip(reqs, res):
        s = dg.Solver(q.E, N=q.N, Ma=q.Ma, Re=q.Re, precision=q.precision)
        s.set_ic("tgv")
        dt = s.suggest_dt(q.cfl)
        s.rk_step(dt, q.steps)
        U = s.state()
        assert r.diagnostics["nonfinite"] == 0
        assert np.array_equal(U, r.state), (q, np.abs(U - r.state).max())
        s.close()
