"""Batches of independent solvers (one launch per order/precision group and RK stage): each
member's state after batched steps is bitwise the state it reaches when stepped alone."""
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


def members(dg):
    """Two uniform Euler N=3 solves of different sizes and Mach numbers (one group), two
    Navier-Stokes N=4 solves (one group), an FP32-bulk Navier-Stokes N=4 solve, N=5 Euler solves
    with LLF faces, with Ismail-Roe + entropy-stable fluxes and with Kennedy-Gruber + low-
    dissipation Roe fluxes, an N=3 Euler solve with the Pirozzoli volume flux, an N=4
    Navier-Stokes solve with the interior-penalty viscous flux, and a mixed-order solve."""
    specs = [dict(ex=4, N=3, Ma=0.1), dict(ex=3, ey=2, ez=5, N=3, Ma=0.4, deform=True),
             dict(ex=3, N=4, Ma=0.1, Re=1600.0, deform=True), dict(ex=2, N=4, Ma=0.3, Re=400.0),
             dict(ex=2, N=4, Ma=0.1, Re=800.0, precision="fp32_bulk"),
             dict(ex=2, N=5, Ma=0.2, surf="llf"), dict(ex=2, N=5, Ma=0.2, surf="es", vol="ir"),
             dict(ex=2, N=5, Ma=0.2, vol="kg", surf="ld_roe"), dict(ex=2, N=3, Ma=0.3, vol="pirozzoli"),
             dict(ex=2, N=4, Ma=0.2, Re=500.0, visc="ip"), dict(ex=3, N=5, Ma=0.3, surf="lf_global"),
             dict(ex=3, orders=synth.mixed_orders(27, seed=2), Ma=0.5, lo=(-10.0,) * 3, hi=(10.0,) * 3)]
    out = []
    for sp in specs:
        s = dg.Solver(**sp)
        if "orders" in sp:
            s.set_ic("vortex", [5.0, 0.0, 0.0, 0.4, 0.4])
        else:
            s.set_ic("tgv")
        out.append(s)
    return out


def test_batch_equals_alone(dg):
    import torch
    alone, batched = members(dg), members(dg)
    dts = [s.suggest_dt(0.4) for s in alone]
    for s, dt in zip(alone, dts):
        s.rk_step(dt, 4)
    for s in batched:
        s.synchronize()
    side = torch.cuda.Stream()  # a batch on a stream of its own
    b = dg.Batch(batched, stream=side)
    # groups: N=3 Euler, N=4 NS FP64, N=4 NS FP32, N=5 Euler, one group per extended flux
    # family (N=5 extended surface flux, N=5 both extensions, N=3 kinetic-energy-preserving
    # volume flux) and N=4 NS with the interior penalty -> 1+2+2+1+1+1+1+2 launches, mixed 1
    assert b.launches_per_stage() == 12
    b.rk_step(dts, 4)
    side.synchronize()
    for k, (a, c) in enumerate(zip(alone, batched)):
        Ua, Uc = a.state(), c.state()
        assert np.array_equal(Ua, Uc), (k, np.abs(Ua - Uc).max())
    b.close()


def test_batch_parities_graphs_and_many_members(dg):
    """40 members of one group (two launches of at most 32), a member that starts from its other
    state buffer, graph replay against eager batched steps, and single steps with recurring step
    sizes."""
    def make():
        out = []
        for i in range(40):
            s = dg.Solver(ex=2 + i % 3, N=3, Ma=0.1 + 0.01 * i)
            s.set_ic("density_wave", [0.1, 0.5, 0.2, 0.1, 1.0, 1.0, 1.0, 1.0, 0.1 * i])
            out.append(s)
        return out
    A, B, C = make(), make(), make()
    dts = [s.suggest_dt(0.3) for s in A]
    for grp in (A, B, C):
        grp[5].rk_step(dts[5], 1)  # member 5 now starts from its other buffer
    for s, dt in zip(A, dts):
        s.rk_step(dt, 7)
    bb = dg.Batch(B)
    assert bb.launches_per_stage() == 2
    bb.rk_step(dts, 5)  # replayed
    for _ in range(2):  # single steps, same dts: the first runs eagerly, the second replays
        bb.rk_step(dts, 1)
    bc = dg.Batch(C)
    bc.use_graphs(False)
    bc.rk_step(dts, 7)
    for k in range(40):
        Ua = A[k].state()
        assert np.array_equal(Ua, B[k].state()), k
        assert np.array_equal(Ua, C[k].state()), k
    bb.close()
    bc.close()


def test_batch_argument_errors(dg):
    s1 = dg.Solver(ex=2, N=3)
    with pytest.raises(dg.DgError) as ei:
        dg.Batch([s1, s1])
    assert ei.value.code == dg.DG_EINVAL
    s2 = dg.Solver(ex=2, N=3, bind=False)
    with pytest.raises(dg.DgError) as ei:  # not bound
        dg.Batch([s1, s2])
    assert ei.value.code == dg.DG_ESTATE
    s1.set_ic("tgv")
    b = dg.Batch([s1])
    with pytest.raises(dg.DgError):
        b.rk_step([-1.0])
    with pytest.raises(ValueError):
        b.rk_step([1e-3, 1e-3])
    b.close()


def test_batch_rk4_equals_alone(dg):
    """Members using the RK4 scheme advance in a batch exactly as alone; a batch refuses members
    with different schemes."""
    specs = [dict(ex=3, N=3, Ma=0.2), dict(ex=2, N=4, Ma=0.1, Re=800.0), dict(ex=2, N=5, Ma=0.3)]

    def make():
        out = []
        for sp in specs:
            s = dg.Solver(**sp)
            s.set_scheme("rk4")
            s.set_ic("tgv")
            out.append(s)
        return out
    alone, batched = make(), make()
    dts = [s.suggest_dt(0.6) for s in alone]
    for s, dt in zip(alone, dts):
        s.rk_step(dt, 3)
    b = dg.Batch(batched)
    b.rk_step(dts, 3)
    for a, c in zip(alone, batched):
        assert np.array_equal(a.state(), c.state())
    b.close()
    other = dg.Solver(ex=2, N=3)
    with pytest.raises(dg.DgError) as ei:
        dg.Batch([batched[0], other])
    assert ei.value.code == dg.DG_EINVAL


def test_batch_members_match_oracle(dg, orc):
    """One member of every launch group of a batch (uniform orders 3-5, Euler and Navier-Stokes,
    the extended flux families, the interior penalty, FP32-bulk, a mixed-order member) against
    the oracle run alone from the same state with the same step: FP64 members within the parity
    gate (GPU vs long-double oracle within max(1e-12 |U|, GATE e64) per variable), the FP32-bulk
    member's increment within the stated FP32-bulk tolerance of the FP64 oracle."""
    import torch
    from helpers import gate_ok
    from helpers import FP32_TOL
    fp32_tol = FP32_TOL["small"]
    specs = [dict(ex=3, ey=2, ez=5, N=3, Ma=0.4, deform=True),
             dict(ex=3, N=4, Ma=0.1, Re=1600.0, deform=True),
             dict(ex=2, N=4, Ma=0.1, Re=800.0, precision="fp32_bulk"),
             dict(ex=2, N=5, Ma=0.2, surf="llf"), dict(ex=2, N=5, Ma=0.2, surf="es", vol="ir"),
             dict(ex=2, N=3, Ma=0.3, vol="pirozzoli"),
             dict(ex=2, N=4, Ma=0.2, Re=500.0, visc="ip"),
             dict(ex=3, orders=synth.mixed_orders(27, seed=2), Ma=0.5, lo=(-10.0,) * 3, hi=(10.0,) * 3)]
    steps = 4
    gpu, ref = [], []
    for sp in specs:
        oc = {k: v for k, v in sp.items() if k != "precision"}
        o = orc.OracleSolver(**oc)
        if "orders" in sp:
            o.set_ic("vortex", [5.0, 0.0, 0.0, 0.4, 0.4])
        else:
            o.set_ic("tgv")
        U0 = o.state()
        dt = o.suggest_dt(0.4)
        s = dg.Solver(**sp)
        s.set_state(U0)
        gpu.append(s)
        ref.append((oc, U0, dt, o))
    b = dg.Batch(gpu, stream=torch.cuda.Stream())
    b.rk_step([r[2] for r in ref], steps)
    b.stream.synchronize()
    for sp, s, (oc, U0, dt, o64) in zip(specs, gpu, ref):
        o64.rk3(dt, steps)
        Ug, Uo = s.state(), o64.state()
        lay = [(o64.elem(e)[1], int(np.prod([n + 1 for n in o64.elem(e)[0]]))) for e in range(o64.E)]

        def pv(A):
            m = np.zeros(5)
            for off, nn in lay:
                m = np.maximum(m, np.abs(A[5 * off:5 * (off + nn)]).reshape(5, nn).max(axis=1))
            return m
        name = ",".join(f"{k}={v}" for k, v in sp.items() if k != "orders")
        if sp.get("precision") == "fp32_bulk":
            err = pv(Ug - Uo) / pv(Uo - U0)
            print(f"[batch member {name}] increment rel err vs fp64 oracle {err}", flush=True)
            assert np.all(err < fp32_tol), err
        else:
            o80 = orc.OracleSolver(**oc, precision="fp80")
            o80.set_state(U0)
            o80.rk3(dt, steps)
            U80 = o80.state()
            sc = pv(U80)
            print(f"[batch member {name}] gpu-vs-fp80 {pv(Ug - U80) / sc} fp64-vs-fp80 {pv(Uo - U80) / sc}",
                  flush=True)
            assert gate_ok(f"batch member {name}", pv(Ug - U80), pv(Uo - U80), sc, 1e-14), "parity gate"
    b.close()
