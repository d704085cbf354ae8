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


HERE = os.path.dirname(os.path.abspath(__file__))
TRAFFIC_PROFILE = os.path.join(HERE, "profiles", "stage_kernel_c2_ns_fp64.md")
KERNEL_SOURCES = ["paper_2206_09733_amd/csrc/kernels.hip", "paper_2206_09733_amd/csrc/stage_kernel.h",
                  "paper_2206_09733_amd/csrc/dg_device.h", "paper_2206_09733_amd/csrc/dg_internal.h",
                  "paper_2206_09733_amd/csrc/grad_body.h"]


def _profile_rows(kernel, shape):
    """Table rows of `kernel` (launch shape `shape`) in the committed rocprofv3 summary, or None when
    the kernel sources changed since the counters were taken."""
    import hashlib
    import re
    try:
        text = open(TRAFFIC_PROFILE).read()
        h = hashlib.sha256()
        for f in KERNEL_SOURCES:
            h.update(open(os.path.join(HERE, f), "rb").read())
    except OSError:
        return None
    m = re.search(r"Kernel sources \(sha256[^`]*`([0-9a-f]+)`", text)
    if not m or m.group(1) != h.hexdigest()[:len(m.group(1))]:
        return None
    rows = []
    for line in text.splitlines():
        cells = [c.strip() for c in line.strip().strip("|").split("|")]
        if len(cells) >= 2 and cells[0] == f"`{kernel}`" and cells[1] == shape:
            rows.append(cells)
    return rows


def profiled_traffic(kernel="dg::stage_kernel<4, double, true, 0, false>", shape="32768 x 128"):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE summary,
    or None when the kernel sources changed since the counters were taken."""
    for cells in _profile_rows(kernel, shape) or []:
        if len(cells) == 8:
            return float(cells[7])
    return None


def profiled_limiter(kernel="dg::stage_kernel<4, double, true, 0, false>", shape="32768 x 128"):
    """What binds `kernel`, from the committed rocprofv3 SQ counters (None when stale): VALU busy
    share, mean resident waves per SIMD and the share of wave time spent waiting."""
    for cells in _profile_rows(kernel, shape) or []:
        if len(cells) == 12:
            busy = float(cells[5].rstrip("%")) / 100
            return {"valu_busy": busy, "waves_per_simd": float(cells[10]),
                    "wait_share": float(cells[11].rstrip("%")) / 100, "vgprs": int(cells[2]),
                    "lds_bytes": int(cells[3]),
                    "reading": "issue/latency bound: neither the VALU nor HBM is saturated; residency "
                               "is capped by registers and LDS, and each element's loads are only "
                               "partly hidden behind other workgroups' compute"}
    return None


def timed_steps(s, dt, steps, profile=True):
    """Run `steps` RK3 steps between two events on the solver's stream.  With profile=True the
    library also brackets every kernel of the timed steps with HIP events on that stream."""
    import torch
    stream = s.stream
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    if profile:
        s.profile_begin()
    t0 = time.perf_counter()
    start.record(stream)
    s.rk_step(dt, steps)
    stop.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prof = s.profile_end() if profile else None
    return start.elapsed_time(stop), wall, prof


def run_gpu(precision, steps, warmup, scheme="rk3"):
    """The workload on the product path: `steps` steps of one dg_rk_step call (graph replay),
    timed with events on the solver's stream.  A second, profiled pass of steps/5 steps (at
    least 2), in which the library brackets every kernel with HIP events and launches eagerly,
    gives the per-kernel averages."""
    from paper_2206_09733_amd import dgsem
    s = dgsem.Solver(**WORKLOAD, precision=precision)
    s.set_scheme(scheme)
    s.set_ic("tgv")
    dt = s.suggest_dt(0.5)
    s.rk_step(dt, warmup)
    s.synchronize()
    ev_ms, wall, _ = timed_steps(s, dt, steps, profile=False)
    _, _, prof = timed_steps(s, dt, max(2, steps // 5), profile=True)
    d = s.diagnostics()
    out = dict(nodes=s.nodes, E=s.E, dt=dt, wall_s=wall, event_ms=ev_ms, prof=prof,
               finite=d["nonfinite"] == 0, ke=d["ke"])
    s.close()
    return out


def precision_error(steps=20):
    """FP32-bulk against the FP64 path (itself checked against the oracle by the GPU tests) on
    the benchmark workload: per conserved variable, the relative L-inf difference
    max|a - b| / max|b| of the residual of the Taylor-Green state and of the state after `steps`
    RK3 steps, and the change of the conserved totals (volume integrals) over those steps."""
    import numpy as np
    from paper_2206_09733_amd import dgsem
    keys = ["mass_rho", "mass_rhou", "mass_rhov", "mass_rhow", "mass_rhoE"]
    res, st, drift = {}, {}, {}
    for prec in ("fp64", "fp32_bulk"):
        s = dgsem.Solver(**WORKLOAD, precision=prec)
        s.set_ic("tgv")
        dt = s.suggest_dt(0.5)
        d0 = s.diagnostics()
        res[prec] = s.residual().reshape(s.E, 5, -1)
        s.rk_step(dt, steps)
        st[prec] = s.state().reshape(s.E, 5, -1)
        d1 = s.diagnostics()
        drift[prec] = [d1[k] - d0[k] for k in keys]
        s.close()

    def rel(a, b):
        return [float(np.abs(a[:, c] - b[:, c]).max() / np.abs(b[:, c]).max()) for c in range(5)]
    return {"variables": ["rho", "rho v1", "rho v2", "rho v3", "rho e"],
            "residual_rel_linf": rel(res["fp32_bulk"], res["fp64"]),
            "state_rel_linf_after_steps": rel(st["fp32_bulk"], st["fp64"]), "steps": steps,
            "conserved_total_change": drift}


def run_adaptive(steps, warmup, fixed_ms):
    """The same workload with the step size chosen on the device before every step (CFL 0.5):
    wall time of one dg_rk_step_adaptive call of `steps` steps (it synchronises once, at the end),
    against the fixed-step time per step."""
    from paper_2206_09733_amd import dgsem
    s = dgsem.Solver(**WORKLOAD)
    s.set_ic("tgv")
    s.rk_step_adaptive(0.5, warmup)
    s.synchronize()
    t0 = time.perf_counter()
    t_sim = s.rk_step_adaptive(0.5, steps)
    wall = time.perf_counter() - t0
    d = s.diagnostics()
    s.close()
    ms = wall * 1e3 / steps
    return {"ms_per_step": round(ms, 4), "steps": steps, "simulated_time": t_sim,
            "overhead_vs_fixed_pct": round(100.0 * (ms / fixed_ms - 1.0), 2),
            "state_finite": d["nonfinite"] == 0}


def run_small_latency(steps=24, warmup=24):
    """The tiny 4^3, N=3 Euler TGV case (64 elements): launch-latency bound, so reported as time
    per RK3 step, with the step graphs replayed and with eager launches (the warm-up runs as many
    steps as the timed run, so that every graph is captured before the timing)."""
    from paper_2206_09733_amd import dgsem
    out = {"workload": "Euler Taylor-Green vortex Ma 0.1, 4^3 hex, N=3, EC + Roe, RK3 CFL 0.5"}
    for graphs in (True, False):
        s = dgsem.Solver(ex=4, N=3, Ma=0.1, vol="ec", surf="roe")
        s.use_graphs(graphs)
        s.set_ic("tgv")
        dt = s.suggest_dt(0.5)
        s.rk_step(dt, warmup)
        ev_ms, wall, _ = timed_steps(s, dt, steps, profile=False)
        out["graph_replay" if graphs else "eager_launches"] = {
            "us_per_step_device": round(ev_ms / steps * 1e3, 2), "us_per_step_host": round(wall / steps * 1e6, 2)}
        s.close()
    return out


def run_gauss(steps, warmup):
    """Euler TGV on the undeformed 32^3 box at N=4 on Gauss-Legendre points (the plain weak form:
    a face-trace kernel and the stage kernel per RK stage), against the same mesh on Lobatto
    points with the central volume form; Navier-Stokes with BR1, BR2 and the interior penalty,
    and BR1 on the deformed box."""
    from paper_2206_09733_amd import dgsem
    out = {"workload": "Euler Taylor-Green vortex Ma 0.1, 32^3 hex undeformed, N=4, Roe faces, RK3 CFL 0.5, "
                       "plain (central) volume form"}
    for nodes, Re, visc, deform in (("gauss", 0.0, "br1", False), ("lobatto", 0.0, "br1", False),
                                    ("gauss", 1600.0, "br1", False), ("lobatto", 1600.0, "br1", False),
                                    ("gauss", 1600.0, "br2", False), ("gauss", 1600.0, "ip", False),
                                    ("gauss", 1600.0, "br1", True)):
        key = nodes if Re == 0.0 else f"{nodes}_navier_stokes_re1600"
        key += "" if visc == "br1" else f"_{visc}"
        key += "_deformed" if deform else ""
        s = dgsem.Solver(ex=32, N=4, Ma=0.1, Re=Re, vol="central", surf="roe", nodes=nodes, visc=visc,
                         deform=deform)
        s.set_ic("tgv")
        dt = s.suggest_dt(0.5)
        s.rk_step(dt, warmup)
        ev_ms, _, _ = timed_steps(s, dt, steps, profile=False)
        _, _, prof = timed_steps(s, dt, max(2, steps // 5))
        d = s.diagnostics()
        st = prof["stage"]
        out[key] = {"value": round(5 * s.nodes * 3 * steps / (ev_ms / 1e3) / 1e9, 3), "unit": "GDOF/s",
                    "ms_per_step": round(ev_ms / steps, 4),
                    "stage_launch_pair_avg_us": round(st["ms"] / st["launches"] * 1e3, 2),
                    "gradient_avg_us": round(prof["gradient"]["ms"] / max(1, prof["gradient"]["launches"]) * 1e3, 2),
                    "state_finite": d["nonfinite"] == 0}
        s.close()
    return out


def algorithmic_bytes_grad_svv(nodes):
    """Unique HBM bytes of the launch that forms the Navier-Stokes gradient pass and the SVV flux
    of one RK stage, FP64 (N = 4): it reads U (40 B per node), Ja, J, 1/J (88) and writes the
    face viscous fluxes (38.4) and the filtered contravariant flux (96).  The stage kernel then
    reads that flux (96) and its neighbours' values on the faces (38.4) and adds it to the
    viscous flux: no correction pass."""
    return nodes * (40 + 88 + 38.4 + 96)


def run_svv(steps, warmup, plain_ms):
    """The benchmark workload with spectral vanishing viscosity (Maday kernel, cutoff 2,
    artificial viscosity 1/1600): throughput, cost against the plain step, and the two SVV
    kernels' time per stage from the library's HIP events; the same in FP32-bulk, and the LES
    closures."""
    from paper_2206_09733_amd import dgsem
    s = dgsem.Solver(**WORKLOAD, svv_mu=1.0 / 1600.0, svv_kernel="maday", svv_cutoff=2)
    s.set_ic("tgv")
    dt = s.suggest_dt(0.5)
    s.rk_step(dt, warmup)
    ev_ms, _, _ = timed_steps(s, dt, steps, profile=False)
    _, _, prof = timed_steps(s, dt, max(2, steps // 5))
    d = s.diagnostics()
    gr, stg = prof["gradient"], prof["stage"]
    flux_s = gr["ms"] / gr["launches"] / 1e3
    out = {"workload": "the benchmark workload plus SVV (Maday kernel, cutoff 2, mu_a 1/1600, no sensor)",
           "value": round(5 * s.nodes * 3 * steps / (ev_ms / 1e3) / 1e9, 3), "unit": "GDOF/s",
           "ms_per_step": round(ev_ms / steps, 4),
           "overhead_vs_plain_pct": round(100.0 * (ev_ms / steps / plain_ms - 1.0), 2),
           "gradient_and_svv_flux_kernel_avg_us": round(flux_s * 1e6, 2),
           "gradient_and_svv_flux_kernel_GB_s": round(algorithmic_bytes_grad_svv(s.nodes) / flux_s / 1e9, 1),
           "stage_kernel_with_svv_avg_us": round(stg["ms"] / stg["launches"] * 1e3, 2),
           "state_finite": d["nonfinite"] == 0}
    s.close()
    # FP32-bulk with the same term: the FP32 gradient pass and the FP64 filtered flux in one
    # launch, then the FP32 stage kernel with that flux in its viscous flux
    s = dgsem.Solver(**WORKLOAD, svv_mu=1.0 / 1600.0, svv_kernel="maday", svv_cutoff=2, precision="fp32_bulk")
    s.set_ic("tgv")
    s.rk_step(dt, warmup)
    ev_ms, _, _ = timed_steps(s, dt, steps, profile=False)
    _, _, prof = timed_steps(s, dt, max(2, steps // 5))
    gr, stg = prof["gradient"], prof["stage"]
    out["fp32_bulk"] = {"value": round(5 * s.nodes * 3 * steps / (ev_ms / 1e3) / 1e9, 3), "unit": "GDOF/s",
                        "ms_per_step": round(ev_ms / steps, 4),
                        "gradient_and_svv_flux_kernel_avg_us": round(gr["ms"] / gr["launches"] * 1e3, 2),
                        "stage_kernel_with_svv_avg_us": round(stg["ms"] / stg["launches"] * 1e3, 2),
                        "state_finite": s.diagnostics()["nonfinite"] == 0}
    s.close()
    # the explicit LES closures on the same workload: the model's eddy viscosity in place of the
    # constant one, filtered (SVV-Smagorinsky) and unfiltered (the plain models), with the models'
    # usual constants (C_s 0.17, C_w 0.5, Vreman's c 0.07)
    for name, kernel, cut, model, cs in (("svv_smagorinsky", "maday", 2, "smagorinsky", 0.17),
                                         ("smagorinsky", "tadmor", -1, "smagorinsky", 0.17),
                                         ("wale", "tadmor", -1, "wale", 0.5), ("vreman", "tadmor", -1, "vreman", 0.07)):
        s = dgsem.Solver(**WORKLOAD, les_cs=cs, les_model=model, svv_kernel=kernel, svv_cutoff=cut)
        s.set_ic("tgv")
        s.rk_step(dt, warmup)
        ev_ms, _, _ = timed_steps(s, dt, steps, profile=False)
        _, _, prof = timed_steps(s, dt, max(2, steps // 5))
        gr = prof["gradient"]
        out[name] = {"value": round(5 * s.nodes * 3 * steps / (ev_ms / 1e3) / 1e9, 3), "unit": "GDOF/s",
                     "ms_per_step": round(ev_ms / steps, 4),
                     "gradient_and_svv_flux_kernel_avg_us": round(gr["ms"] / gr["launches"] * 1e3, 2),
                     "state_finite": s.diagnostics()["nonfinite"] == 0}
        s.close()
    return out


VARIANTS = [("ec", "roe", "br1"), ("ir", "ir", "br1"), ("kg", "es_matrix", "br1"), ("pirozzoli", "ld_roe", "br1"),
            ("ducros", "es", "br1"), ("ec", "lf_global", "br1"), ("ec", "roe", "br2"), ("ec", "roe", "ip")]


def run_variants(steps, warmup):
    """The benchmark workload with other volume / surface / viscous fluxes (FP64): throughput and
    the stage and gradient kernels' time per launch from the library's HIP events."""
    from paper_2206_09733_amd import dgsem
    out = {}
    for vol, surf, visc in VARIANTS:
        s = dgsem.Solver(**{**WORKLOAD, "vol": vol, "surf": surf}, visc=visc)
        s.set_ic("tgv")
        dt = s.suggest_dt(0.5)
        s.rk_step(dt, warmup)
        ev_ms, _, prof = timed_steps(s, dt, steps)
        d = s.diagnostics()
        st, gr = prof["stage"], prof["gradient"]
        out[f"{vol}+{surf}+{visc}"] = {
            "value": round(5 * s.nodes * 3 * steps / (ev_ms / 1e3) / 1e9, 3), "unit": "GDOF/s",
            "ms_per_step": round(ev_ms / steps, 4),
            "stage_avg_us": round(st["ms"] / st["launches"] * 1e3, 2),
            "gradient_avg_us": round(gr["ms"] / gr["launches"] * 1e3, 2),
            "state_finite": d["nonfinite"] == 0}
        s.close()
    return out


MIXED = dict(ex=24, lo=(-10.0,) * 3, hi=(10.0,) * 3, Ma=0.5, vol="ec", surf="roe")
# isentropic vortex of strength 5, free stream rho = p = 1 moving along (1, 1, 0)/sqrt 2 at Mach 0.5
VORTEX = [5.0, 0.0, 0.0, 0.5 * math.sqrt(1.4 / 2.0), 0.5 * math.sqrt(1.4 / 2.0)]


def run_mixed(steps, warmup):
    """24^3 elements with orders (Nx, Ny, Nz) uniform in {2..6} (seed 0), Euler, graph replay
    of the RK steps, launch shapes from the autotuner; FP64 and FP32-bulk.  For comparison the
    same mesh at the uniform order 6 that bounds the mixed orders (the plain form)."""
    from paper_2206_09733_amd import dgsem, synth
    orders = synth.mixed_orders(24 ** 3, seed=0)
    out = {"workload": "Euler isentropic vortex (strength 5, Mach 0.5, diagonal) on [-10,10]^3, "
                       "24^3 hex, per-element orders (Nx,Ny,Nz) uniform in {2..6} (seed 0), EC split "
                       "form + Roe, mortar faces, RK3 CFL 0.5, graph replay"}
    for prec in ("fp64", "fp32_bulk"):
        s = dgsem.Solver(**MIXED, orders=orders, precision=prec)
        s.set_ic("vortex", VORTEX)
        tiles, tune_us = s.autotune()
        dt = s.suggest_dt(0.5)
        s.rk_step(dt, warmup)
        ev_ms, _, _ = timed_steps(s, dt, steps, profile=False)
        _, _, prof = timed_steps(s, dt, max(2, steps // 5))
        st = prof["stage"]
        d = s.diagnostics()
        r = {"value": round(5 * s.nodes * 3 * steps / (ev_ms / 1e3) / 1e9, 3), "unit": "GDOF/s",
             "ms_per_step": round(ev_ms / steps, 4), "autotuned_tiles": f"{tiles:06b}",
             "stage_avg_us": round(st["ms"] / st["launches"] * 1e3, 2),
             "stage_us_replay": round(ev_ms / steps / 3 * 1e3, 2), "state_finite": d["nonfinite"] == 0}
        if prec == "fp64":
            out.update({"elements": s.E, "nodes": s.nodes, "dof": 5 * s.nodes, "dtype": "f64", "steps": steps})
            out.update(r)
            # the whole stage (face kernel and buckets) against its algorithmic bytes: those of the
            # Euler stage, U in/out, dU out and (two stages in three) in, metric terms
            b = algorithmic_bytes_stage(s.nodes, 0, False, False, 2.0 / 3.0)
            st_s = ev_ms / steps / 3 / 1e3
            out["roofline"] = {"bound": "hbm", "scope": "whole stage (face kernel + buckets), graph replay",
                               "achieved": round(b / st_s / 1e9, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                               "frac": round(b / st_s / 1e9 / HBM_PEAK_GBS, 4),
                               "algorithmic_bytes_per_stage": int(b)}
        else:
            r["speedup_vs_fp64"] = round(r["value"] / out["value"], 3)
            out["fp32_bulk"] = r
        s.close()
    u = dgsem.Solver(**MIXED, N=6)
    u.set_ic("vortex", VORTEX)
    dtu = u.suggest_dt(0.5)
    u.rk_step(dtu, warmup)
    ev_u, _, _ = timed_steps(u, dtu, steps, profile=False)
    out["uniform_order6_same_mesh"] = {
        "nodes": u.nodes, "ms_per_step": round(ev_u / steps, 4),
        "value": round(5 * u.nodes * 3 * steps / (ev_u / 1e3) / 1e9, 3), "unit": "GDOF/s",
        "mixed_step_speedup": round((ev_u / steps) / out["ms_per_step"], 3)}
    u.close()
    return out


def run_halo(steps, warmup):
    """One GPU's share of the 64^3 N=5 Navier-Stokes TGV split across eight GPUs: a 32^3 block run
    with its periodic neighbours reached through ghost elements and a halo exchange before every
    stage (state face values; after the gradient pass the face viscous fluxes), against the same
    block with direct neighbours.  The exchange moves its buffers with a device copy where a split
    run would send them between GPUs."""
    from paper_2206_09733_amd import dgsem
    out = {"workload": "compressible NS TGV Re1600 Ma0.1, 32^3 hex block of a deformed 64^3 N=5 mesh, "
                       "EC + Roe + BR1, RK3 CFL 0.5, FP64"}
    K, nf = 6 * 32 * 32, 36
    for halo in (False, True):
        s = dgsem.Solver(32, N=5, deform=True, Ma=0.1, Re=1600.0, halo=halo)
        s.set_ic("tgv")
        dt = s.suggest_dt(0.5)
        s.rk_step(dt, warmup)
        ev_ms, _, _ = timed_steps(s, dt, steps, profile=False)
        _, _, prof = timed_steps(s, dt, max(2, steps // 5))
        key = "halo" if halo else "direct"
        out[key] = {"value": round(5 * s.nodes * 3 * steps / (ev_ms / 1e3) / 1e9, 3), "unit": "GDOF/s",
                    "ms_per_step": round(ev_ms / steps, 4), "state_finite": s.diagnostics()["nonfinite"] == 0}
        if halo:
            ot = prof["other"]
            out[key]["exchange_us_per_stage"] = round(ot["ms"] / ot["launches"] * 2 * 1e3, 2)
            out[key]["exchanged_bytes_per_stage"] = K * nf * 8 * (5 + 4)
        s.close()
    out["halo"]["overhead_pct"] = round(100.0 * (out["halo"]["ms_per_step"] / out["direct"]["ms_per_step"] - 1), 2)
    return out


def run_large(steps, warmup):
    """The large comparison: 64^3 elements, N = 5 (56.6 M nodes), Navier-Stokes TGV Re 1600,
    Ma 0.1, deformed mesh; FP64 against FP32-bulk, time per RK3 step."""
    from paper_2206_09733_amd import dgsem
    out = {"workload": "compressible NS Taylor-Green vortex Re1600 Ma0.1 Pr0.71, 64^3 hex deformed, "
                       "Gauss-Lobatto N=5, EC split form + Roe + BR1, RK3 CFL 0.5"}
    for prec in ("fp64", "fp32_bulk"):
        s = dgsem.Solver(64, N=5, deform=True, Ma=0.1, Re=1600.0, precision=prec)
        s.set_ic("tgv")
        dt = s.suggest_dt(0.5)
        s.rk_step(dt, warmup)
        ev_ms, _, _ = timed_steps(s, dt, steps, profile=False)
        d = s.diagnostics()
        out[prec] = {"value": round(5 * s.nodes * 3 * steps / (ev_ms / 1e3) / 1e9, 3), "unit": "GDOF/s",
                     "ms_per_step": round(ev_ms / steps, 3), "steps": steps, "ke": d["ke"],
                     "enstrophy": d["enstrophy"], "state_finite": d["nonfinite"] == 0}
        series = []  # after the timed steps, outside the timed region: (step, KE, enstrophy)
        for k in range(5):
            s.rk_step(dt, 1)
            dk = s.diagnostics()
            series.append([warmup + steps + k + 1, dk["ke"], dk["enstrophy"]])
        out[prec]["ke_enstrophy_series"] = series
        out["nodes"], out["dof"] = s.nodes, 5 * s.nodes
        s.close()
    out["fp32_bulk"]["speedup_vs_fp64"] = round(out["fp32_bulk"]["value"] / out["fp64"]["value"], 3)
    return out


def small_ensemble(n=64, seed=1):
    """An ensemble of small solves (parameter sweep): E^3 boxes with E uniform in {4..8}, N in
    {3, 4, 5}, Mach in [0.1, 0.8], half Navier-Stokes (Re in [400, 3200])."""
    from paper_2206_09733_amd import synth
    g = synth.rng(seed)
    out = []
    for i in range(n):
        visc = bool(g.integers(0, 2))
        out.append(dict(id=i, E=int(g.integers(4, 9)), N=int(g.integers(3, 6)), Ma=float(g.uniform(0.1, 0.8)),
                        Re=float(g.uniform(400.0, 3200.0)) if visc else 0.0))
    return out


def run_batch_vs_solo(specs, steps=50):
    """The given solves run alone one after the other, and the same solves as one batch (all
    present at the start): aggregate throughput of both forms."""
    import torch
    from paper_2206_09733_amd import dgsem
    n = len(specs)
    work = sum(5 * q["E"] ** 3 * (q["N"] + 1) ** 3 * 3 * steps for q in specs)

    def make(precision="fp64"):
        out = []
        for q in specs:
            s = dgsem.Solver(q["E"], N=q["N"], Ma=q["Ma"], Re=q["Re"], precision=precision)
            s.set_ic("tgv")
            out.append((s, s.suggest_dt(0.5)))
        return out
    solo = make()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s, dt in solo:
        s.rk_step(dt, steps)
    torch.cuda.synchronize()
    t_solo = time.perf_counter() - t0
    ref = [s.state() for s, _ in solo]
    for s, _ in solo:
        s.close()
    members = make()
    b = dgsem.Batch([s for s, _ in members])
    dts = [dt for _, dt in members]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.rk_step(dts, steps)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    same = all((s.state() == r).all() for (s, _), r in zip(members, ref))
    launches = b.launches_per_stage()
    b.close()
    for s, _ in members:
        s.close()
    # the chosen form: the same solves batched in FP32-bulk, against the plain FP64 solo runs
    members = make("fp32_bulk")
    b = dgsem.Batch([s for s, _ in members])
    dts = [dt for _, dt in members]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.rk_step(dts, steps)
    torch.cuda.synchronize()
    t_b32 = time.perf_counter() - t0
    dev = 0.0
    for (s, _), r in zip(members, ref):
        U = s.state().reshape(-1, 5, (s.N + 1) ** 3)
        R = r.reshape(U.shape)
        dev = max(dev, float((abs(U - R).max(axis=(0, 2)) / abs(R).max(axis=(0, 2))).max()))
    b.close()
    for s, _ in members:
        s.close()
    return {"solves": n, "steps": steps, "solo_gdof_s": round(work / t_solo / 1e9, 3),
            "batch_gdof_s": round(work / t_batch / 1e9, 3), "speedup": round(t_solo / t_batch, 3),
            "launches_per_stage_batched": launches, "launches_per_stage_solo": n,
            "results_bitwise_equal": bool(same),
            "batch_fp32_bulk_gdof_s": round(work / t_b32 / 1e9, 3),
            "speedup_fp32_bulk_batch_vs_fp64_solo": round(t_solo / t_b32, 3),
            "fp32_bulk_state_rel_diff_vs_fp64": dev}


def run_serving(n, rate, steps, budget_gib, chunk, precision="fp64"):
    """The serving stream: n solves from synth.serving_requests (seed 0) arriving as a Poisson
    process of the given rate (seed 0), admitted under an HBM budget, continuously batched."""
    from paper_2206_09733_amd import serve, synth
    reqs = serve.requests_from_specs(synth.serving_requests(n, seed=0),
                                     synth.poisson_arrivals(n, rate, seed=0), steps=steps, precision=precision)
    ex = serve.GpuExecutor(keep_state=False)
    sch = serve.Scheduler(ex, budget_gib * 2 ** 30, max_active=64, chunk_steps=chunk)
    t0 = time.perf_counter()
    res = sch.run(reqs)
    wall = time.perf_counter() - t0
    ex.close()
    st = serve.summarize(reqs, res, wall)
    st.update({"precision": precision, "requests": n, "arrival_rate_per_s": rate, "steps_per_solve": steps,
               "hbm_budget_gib": budget_gib, "chunk_steps": chunk, "chunks": sch.chunks,
               "peak_active": sch.peak_active, "peak_gib": round(sch.peak_bytes / 2 ** 30, 2),
               "nonfinite_results": sum(1 for r in res if r.diagnostics and r.diagnostics["nonfinite"])})
    for k in ("p50_s", "p99_s", "mean_s", "wall_s", "gdof_stage_per_s"):
        st[k] = round(st[k], 4)
    return st


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
    # one residual evaluation of the same mesh on a single thread
    oracle.set_threads(1)
    t0 = time.perf_counter()
    o.residual()
    t1 = time.perf_counter() - t0
    oracle.set_threads(threads)
    return dict(value=5 * o.nodes * 3 * steps / t / 1e9, unit="GDOF/s", cores=threads, kind="oracle",
                sample=f"{steps} RK3 step(s) of the full 32^3 N=4 Navier-Stokes TGV mesh "
                       f"({steps * 3} residual evaluations, {t:.1f} s)",
                value_1_thread=5 * o.nodes / t1 / 1e9,
                sample_1_thread=f"one residual evaluation of the same mesh on 1 thread ({t1:.1f} s)")


LEGS = ["fp32", "rk4", "adaptive", "small", "gauss", "variants", "svv", "mixed", "large", "halo", "batch", "serve",
        "cpu"]


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--legs", default=",".join(LEGS),
                    help="comma-separated parts to run after the headline (default: all of "
                         + ",".join(LEGS) + "; 'none' for the headline alone)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--skip-fp32", action="store_true")
    ap.add_argument("--skip-mixed", action="store_true")
    ap.add_argument("--skip-serve", action="store_true")
    ap.add_argument("--skip-large", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=256)
    ap.add_argument("--serve-rate", type=float, default=12.0, help="Poisson arrivals per second")
    ap.add_argument("--serve-steps", type=int, default=200)
    ap.add_argument("--serve-budget-gib", type=float, default=32.0)
    ap.add_argument("--copy-reference-mib", type=int, default=0,
                    help="first run a plain device copy of this many MiB (a known-size reference "
                         "for hardware traffic counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library runs the DGSEM path on a single GPU. A split "
              "run's halo exchange is built and timed on one GPU (the 'halo' leg); the transfer "
              "between GPUs is not implemented", file=sys.stderr)
        sys.exit(2)
    legs = set() if args.legs == "none" else set(x for x in args.legs.split(",") if x)
    unknown = legs - set(LEGS)
    if unknown:
        ap.error(f"unknown legs {sorted(unknown)}")
    for flag, leg in ((args.no_cpu_baseline, "cpu"), (args.skip_fp32, "fp32"), (args.skip_mixed, "mixed"),
                      (args.skip_large, "large")):
        if flag:
            legs.discard(leg)
    if args.skip_serve:
        legs -= {"batch", "serve"}
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
    stage_s = t / (3 * args.steps)
    result = {
        "metric": "GDOF-updates/s per RK stage (plain FP64 vs batched FP32-bulk); p50/p99 solve latency",
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
                   "elements": r64["E"], "nodes": nodes, "dof": 5 * nodes, "precision": "fp64",
                   "timing": "one dg_rk_step call of all timed steps (graph replay), HIP events on the "
                             "solver's stream"},
        "roofline": {"bound": "hbm", "kernel": "stage_kernel<4,double,NS>",
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": profiled_traffic(),
                     "limiter": profiled_limiter(),
                     "avg_launch_us": round(avg_stage_s * 1e6, 2),
                     "avg_launch_from": f"library HIP events around each launch, a separate pass of "
                                        f"{st['launches'] // 3} steps",
                     "algorithmic_bytes_per_launch": int(b_stage)},
        "whole_stage": {"us_per_stage": round(stage_s * 1e6, 2),
                        "algorithmic_bytes": int(b_stage + b_grad),
                        "GB_s": round((b_stage + b_grad) / stage_s / 1e9, 1),
                        "frac_hbm_peak": round((b_stage + b_grad) / stage_s / 1e9 / HBM_PEAK_GBS, 4)},
        "kernels": {"stage": {"avg_us": round(avg_stage_s * 1e6, 2), "launches": st["launches"],
                              "GB_s": round(achieved, 1)},
                    "gradient": {"avg_us": round(avg_grad_s * 1e6, 2), "launches": gr["launches"],
                                 "GB_s": round(b_grad / avg_grad_s / 1e9, 1)}},
        "state_finite": r64["finite"],
    }
    if "fp32" in legs:
        r32 = run_gpu("fp32_bulk", args.steps, args.warmup)
        v32 = 5 * nodes * 3 * args.steps / (r32["event_ms"] / 1e3) / 1e9
        result["fp32_bulk"] = {"value": round(v32, 3), "unit": "GDOF/s",
                               "ms_per_step": round(r32["event_ms"] / args.steps, 4),
                               "speedup_vs_fp64": round(v32 / value, 3),
                               "error_vs_fp64": precision_error()}
    if "rk4" in legs:
        k4 = max(10, args.steps // 5)
        r4 = run_gpu("fp64", k4, args.warmup, scheme="rk4")
        st4 = r4["prof"]["stage"]
        result["rk4_carpenter_kennedy"] = {
            "ms_per_step": round(r4["event_ms"] / k4, 4),
            "stages_per_step": 5, "stage_avg_us": round(st4["ms"] / st4["launches"] * 1e3, 2),
            "value": round(5 * nodes * 5 * k4 / (r4["event_ms"] / 1e3) / 1e9, 3),
            "unit": "GDOF-updates/s per RK stage"}
    if "adaptive" in legs:
        result["adaptive_dt"] = run_adaptive(args.steps, args.warmup, r64["event_ms"] / args.steps)
    if "small" in legs:
        result["small_case_latency"] = run_small_latency()
    if "gauss" in legs:
        result["gauss_legendre_nodes"] = run_gauss(max(10, args.steps // 2), args.warmup)
    if "variants" in legs:
        result["flux_variants"] = run_variants(max(10, args.steps // 5), 2)
    if "svv" in legs:
        result["spectral_vanishing_viscosity"] = run_svv(max(10, args.steps // 2), args.warmup,
                                                         r64["event_ms"] / args.steps)
    if "mixed" in legs:
        result["mixed_order"] = run_mixed(max(10, args.steps // 2), args.warmup)
    if "large" in legs:
        result["large_64_n5"] = run_large(max(5, args.steps // 10), 2)
    if "halo" in legs:
        result["halo_block_32_n5"] = run_halo(max(10, args.steps // 2), 2)
    if "batch" in legs:
        from paper_2206_09733_amd import synth
        result["batch_vs_solo"] = {
            "serving_first_32": run_batch_vs_solo(synth.serving_requests(32, seed=0)),
            "small_ensemble_64": run_batch_vs_solo(small_ensemble(64), steps=100)}
    if "serve" in legs:
        # the served form computes in FP32-bulk; the same stream in FP64 for comparison
        result["serving"] = run_serving(args.serve_requests, args.serve_rate, args.serve_steps,
                                        args.serve_budget_gib, 20, precision="fp32_bulk")
        result["serving_fp64"] = run_serving(args.serve_requests, args.serve_rate, args.serve_steps,
                                             args.serve_budget_gib, 20, precision="fp64")
        # offered load at half and twice the default arrival rate (FP32-bulk, the first 64 requests)
        result["serving_load_sweep"] = {
            f"{f}x": run_serving(64, f * args.serve_rate, args.serve_steps, args.serve_budget_gib, 20,
                                 precision="fp32_bulk") for f in (0.5, 2.0)}
    if rank == 0 and "cpu" in legs:
        result["cpu_baseline"] = run_cpu_baseline()
    if rank == 0:
        print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
