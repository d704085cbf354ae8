#!/usr/bin/env python3
"""Benchmark of the DGSEM residual + low-storage RK3 on one MI355X.

Workload: compressible Navier-Stokes Taylor-Green vortex, Re 1600, Ma 0.1, Pr 0.71, on a
periodic [0, 2pi]^3 box of 32^3 hexahedra deformed by x += 0.05 sin y sin z (and cyclic),
Gauss-Lobatto order N = 4 (4.096M nodes, 20.48M DOF), entropy-conserving split form, Roe
faces, BR1 viscous terms, FP64 state; time step from CFL 0.5, held fixed.

Metric: GDOF-updates/s per RK stage = 5 * nodes * 3 * steps / t / 1e9, with the state
resident in HBM when the timed region starts.  One JSON line on stdout.
"""
import argparse
import json
import math
import os
import sys
import time

WORKLOAD = dict(ex=32, N=4, deform=True, amp=0.05, Ma=0.1, Re=1600.0, Pr=0.71, gamma=1.4,
                vol="ec", surf="roe")
HBM_PEAK_GBS = 8000.0


def algorithmic_bytes_stage(nodes, N, viscous, fp32, frac_read_dU):
    """HBM bytes the stage kernel must move per launch: U in, U out, dU in (not in the first
    RK stage) and out, metric terms (9 Ja + 1/J) and, for Navier-Stokes, the element's share of
    the face viscous fluxes written by the gradient pass (4 values per face node, 6 faces)."""
    n = N + 1
    per_node = 8 * (5 + 5 + 5 + 10) + 8 * 5 * frac_read_dU
    if viscous:
        per_node += (4 if fp32 else 8) * 4 * 6 * n * n / n ** 3
    return per_node * nodes


def algorithmic_bytes_gradient(nodes, N, fp32):
    """Gradient pass: U in, metric terms in, face viscous fluxes out."""
    n = N + 1
    return nodes * (8 * 5 + 8 * 10 + (4 if fp32 else 8) * 4 * 6 * n * n / n ** 3)


def run_gpu(precision, steps, warmup):
    import torch
    from paper_2206_09733_amd import dgsem
    s = dgsem.Solver(**WORKLOAD, precision=precision)
    s.set_ic("tgv")
    dt = s.suggest_dt(0.5)
    s.rk_step(dt, warmup)
    s.synchronize()
    stream = torch.cuda.current_stream()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start.record(stream)
    s.rk_step(dt, steps)
    stop.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms = start.elapsed_time(stop)
    # the same steps again with per-kernel HIP events (recorded by the library on its stream)
    s.profile_begin()
    s.rk_step(dt, steps)
    prof = s.profile_end()
    d = s.diagnostics()
    out = dict(nodes=s.nodes, E=s.E, dt=dt, wall_s=wall, event_ms=ev_ms, prof=prof,
               finite=d["nonfinite"] == 0, ke=d["ke"])
    s.close()
    return out


def run_cpu_baseline(budget_s=12.0, max_steps=4):
    """The oracle (plain C, FP64, OpenMP over elements) on the host cores, on the same workload:
    whole RK3 steps of the full 32^3, N=4 mesh until about budget_s seconds have passed."""
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    oracle.set_threads(threads)
    o = oracle.OracleSolver(**{k: v for k, v in WORKLOAD.items()})
    o.set_ic("tgv")
    dt = o.suggest_dt(0.5)
    steps, t = 0, 0.0
    while steps < max_steps and t < budget_s:
        t0 = time.perf_counter()
        o.rk3(dt, 1)
        t += time.perf_counter() - t0
        steps += 1
    return dict(value=5 * o.nodes * 3 * steps / t / 1e9, unit="GDOF/s", cores=threads, kind="oracle",
                sample=f"{steps} RK3 step(s) of the full 32^3 N=4 Navier-Stokes TGV mesh "
                       f"({steps * 3} residual evaluations, {t:.1f} s)")


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--skip-fp32", action="store_true")
    ap.add_argument("--copy-reference-mib", type=int, default=0,
                    help="first run a plain device copy of this many MiB (a known-size reference "
                         "for hardware traffic counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the DGSEM path here is a single-GPU build "
              "(multi-GPU element sharding is a design note, not implemented)", file=sys.stderr)
        sys.exit(2)
    rank = int(os.environ.get("RANK", "0"))
    if args.copy_reference_mib:
        import torch
        src = torch.ones(args.copy_reference_mib << 17, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    r64 = run_gpu("fp64", args.steps, args.warmup)
    nodes, N = r64["nodes"], WORKLOAD["N"]
    t = r64["event_ms"] / 1e3
    value = 5 * nodes * 3 * args.steps / t / 1e9
    prof = r64["prof"]
    st = prof["stage"]
    gr = prof["gradient"]
    avg_stage_s = st["ms"] / st["launches"] / 1e3
    avg_grad_s = gr["ms"] / gr["launches"] / 1e3
    b_stage = algorithmic_bytes_stage(nodes, N, True, False, 2.0 / 3.0)
    b_grad = algorithmic_bytes_gradient(nodes, N, False)
    achieved = b_stage / avg_stage_s / 1e9
    result = {
        "metric": "GDOF-updates/s per RK stage",
        "value": round(value, 3),
        "unit": "GDOF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r64["event_ms"] / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "compressible NS Taylor-Green vortex Re1600 Ma0.1 Pr0.71, 32^3 hex "
                               "deformed (x+=0.05 sin y sin z, cyclic), Gauss-Lobatto N=4, EC split "
                               "form + Roe + BR1, low-storage RK3, CFL 0.5",
                   "elements": r64["E"], "nodes": nodes, "dof": 5 * nodes, "precision": "fp64"},
        "roofline": {"bound": "hbm", "kernel": "stage_kernel<4,double,NS>",
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "avg_launch_us": round(avg_stage_s * 1e6, 2),
                     "algorithmic_bytes_per_launch": int(b_stage)},
        "kernels": {"stage": {"avg_us": round(avg_stage_s * 1e6, 2), "launches": st["launches"],
                              "GB_s": round(achieved, 1)},
                    "gradient": {"avg_us": round(avg_grad_s * 1e6, 2), "launches": gr["launches"],
                                 "GB_s": round(b_grad / avg_grad_s / 1e9, 1)}},
        "state_finite": r64["finite"],
    }
    if not args.skip_fp32:
        r32 = run_gpu("fp32_bulk", args.steps, args.warmup)
        v32 = 5 * nodes * 3 * args.steps / (r32["event_ms"] / 1e3) / 1e9
        result["fp32_bulk"] = {"value": round(v32, 3), "unit": "GDOF/s",
                               "ms_per_step": round(r32["event_ms"] / args.steps, 4),
                               "speedup_vs_fp64": round(v32 / value, 3)}
    if rank == 0 and not args.no_cpu_baseline:
        result["cpu_baseline"] = run_cpu_baseline()
    if rank == 0:
        print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
