"""Serving loop for independent DGSEM solves (ensembles, parameter sweeps): requests arrive over
time, are admitted first-come first-served while their device memory fits an HBM budget, and
every admitted solve is advanced in the same batched launches as the others (continuous
batching: the batch is re-formed at chunk boundaries as solves finish and new ones join).
New solves are set up (geometry, initial condition, step size) on a side stream while the
running batch computes, so their work overlaps on the device.

`Scheduler` holds the policy and needs no GPU; `GpuExecutor` drives libdgsem.so through its
Python binding.  Latency of a request = completion (state back on the host) - arrival.
"""
import collections
import dataclasses
import time

import numpy as np


@dataclasses.dataclass
class Request:
    """One solve: Taylor-Green vortex on the periodic box [0, 2 pi]^3 with E^3 elements of order
    N, Mach Ma, Reynolds number Re (0 = Euler), advanced `steps` RK3 steps in `precision`
    ("fp64" or "fp32_bulk"), with the fixed step `dt`, or (dt = 0) the step that CFL number
    `cfl` gives for the initial state."""
    id: int
    E: int
    N: int
    Ma: float
    Re: float
    steps: int = 200
    arrival: float = 0.0
    cfl: float = 0.5
    precision: str = "fp64"
    dt: float = 0.0

    @property
    def nodes(self):
        return self.E ** 3 * (self.N + 1) ** 3

    @property
    def dof_stage_updates(self):
        return 5 * self.nodes * 3 * self.steps


@dataclasses.dataclass
class Result:
    id: int
    arrival: float
    admitted: float = float("nan")
    finished: float = float("nan")
    error: str = ""
    state: object = None
    diagnostics: object = None

    @property
    def latency(self):
        return self.finished - self.arrival


class Job:
    """An admitted request: executor handle, bytes held and steps still to take."""

    def __init__(self, req, handle, nbytes, dt):
        self.req, self.handle, self.nbytes, self.dt = req, handle, nbytes, dt
        self.steps_left = req.steps


class Scheduler:
    """FCFS admission under a byte budget and a cap on concurrent solves; chunked batched steps.

    executor interface:
      required_bytes(req) -> int      device bytes the solve needs (host-only)
      admit(req) -> (handle, dt)      allocate, set up and size the step; may overlap a chunk
      launch(jobs, k) -> token        enqueue k steps of every job as one batch
      wait(token)                     block until those steps are done
      finish(job) -> (state, diag)    read the result back and release the job's memory
      release(job)                    release without reading (failed job)
    """

    def __init__(self, executor, budget_bytes, max_active=64, chunk_steps=20,
                 clock=time.perf_counter, sleep=time.sleep):
        self.ex = executor
        self.budget = int(budget_bytes)
        self.max_active = int(max_active)
        self.chunk = int(chunk_steps)
        self.clock, self.sleep = clock, sleep
        self.peak_bytes = 0
        self.peak_active = 0
        self.chunks = 0
        self.admission_order = []

    def run(self, requests):
        t0 = self.clock()
        now = lambda: self.clock() - t0
        pending = collections.deque(sorted(requests, key=lambda r: (r.arrival, r.id)))
        waiting = collections.deque()
        results = {r.id: Result(r.id, r.arrival) for r in requests}
        active, used = [], 0

        def arrivals():
            t = now()
            while pending and pending[0].arrival <= t:
                waiting.append(pending.popleft())

        def admit():
            nonlocal used
            while waiting and len(active) < self.max_active:
                r = waiting[0]
                need = self.ex.required_bytes(r)
                if need > self.budget:
                    waiting.popleft()
                    results[r.id].error = f"needs {need} bytes, more than the budget of {self.budget}"
                    results[r.id].finished = now()
                    continue
                if used + need > self.budget:
                    break  # head of line waits for memory
                waiting.popleft()
                try:
                    handle, dt = self.ex.admit(r)
                except Exception as exc:  # a failed setup is isolated from the other solves
                    results[r.id].error = f"setup failed: {exc}"
                    results[r.id].finished = now()
                    continue
                used += need
                self.peak_bytes = max(self.peak_bytes, used)
                active.append(Job(r, handle, need, dt))
                results[r.id].admitted = now()
                self.admission_order.append(r.id)
            self.peak_active = max(self.peak_active, len(active))

        while pending or waiting or active:
            arrivals()
            admit()
            if not active:
                if pending and not waiting:
                    self.sleep(max(0.0, pending[0].arrival - now()))
                continue
            k = min(self.chunk, min(j.steps_left for j in active))
            token = self.ex.launch(active, k)
            self.chunks += 1
            arrivals()
            admit_during = len(active)
            admit()  # set-up of new solves overlaps the chunk; they join the next one
            self.ex.wait(token)
            for j in active[:admit_during]:
                j.steps_left -= k
            done = [j for j in active if j.steps_left == 0]
            for j in done:
                try:
                    st, dg = self.ex.finish(j)
                    results[j.req.id].state, results[j.req.id].diagnostics = st, dg
                except Exception as exc:
                    results[j.req.id].error = f"result failed: {exc}"
                    self.ex.release(j)
                used -= j.nbytes
                results[j.req.id].finished = now()
            active = [j for j in active if j.steps_left > 0]
        return [results[r.id] for r in sorted(requests, key=lambda r: r.id)]


def summarize(requests, results, wall):
    """p50/p99 latency (s) and aggregate DOF-stage updates per second of the completed solves."""
    ok = [(q, r) for q, r in zip(sorted(requests, key=lambda q: q.id), results) if not r.error]
    lat = np.array([r.latency for _, r in ok]) if ok else np.array([np.nan])
    work = sum(q.dof_stage_updates for q, _ in ok)
    return {"completed": len(ok), "failed": len(results) - len(ok),
            "p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
            "mean_s": float(lat.mean()), "wall_s": wall,
            "gdof_stage_per_s": work / wall / 1e9 if wall > 0 else float("nan")}


class GpuExecutor:
    """Executor on libdgsem.so: solves are set up on a side stream and advanced as one batch
    (re-formed when membership changes) on a compute stream; both at default priority."""

    def __init__(self, device="cuda", keep_state=True, graphs=True):
        import torch
        from . import dgsem
        self.torch, self.dg = torch, dgsem
        self.device = torch.device(device)
        self.setup = torch.cuda.Stream(self.device)
        self.compute = torch.cuda.Stream(self.device)
        self.keep_state = keep_state
        self.graphs = graphs
        self.batch, self.batch_key = None, None
        self._probe = {}

    def required_bytes(self, req):
        key = (req.E, req.N, req.Re > 0, req.precision)
        if key not in self._probe:
            s = self.dg.Solver(req.E, N=req.N, Ma=req.Ma, Re=req.Re, precision=req.precision, bind=False)
            self._probe[key] = s.required_bytes
            s.close()
        return self._probe[key]

    def admit(self, req):
        s = self.dg.Solver(req.E, N=req.N, Ma=req.Ma, Re=req.Re, precision=req.precision, bind=False)
        with self.torch.cuda.stream(self.setup):
            s.bind(self.device, stream=self.setup)
        s.set_ic("tgv")
        dt = req.dt if req.dt > 0 else s.suggest_dt(req.cfl)  # synchronises the side stream only
        return s, dt

    def launch(self, jobs, k):
        key = tuple(id(j.handle) for j in jobs)
        if key != self.batch_key:
            if self.batch is not None:
                self.batch.close()
            self.batch = self.dg.Batch([j.handle for j in jobs], stream=self.compute)
            self.batch.use_graphs(self.graphs)
            self.batch_key = key
        self.batch.rk_step([j.dt for j in jobs], k)
        ev = self.torch.cuda.Event()
        ev.record(self.compute)
        return ev

    def wait(self, token):
        token.synchronize()

    def finish(self, job):
        s = job.handle
        st = s.state() if self.keep_state else None
        dg = s.diagnostics()
        self.release(job)
        return st, dg

    def release(self, job):
        if self.batch is not None and id(job.handle) in (self.batch_key or ()):
            self.batch.close()
            self.batch, self.batch_key = None, None
        job.handle.close()

    def close(self):
        if self.batch is not None:
            self.batch.close()
            self.batch, self.batch_key = None, None


def requests_from_specs(specs, arrivals, steps=200, precision="fp64"):
    """Requests from synth.serving_requests() specs and arrival times (seconds)."""
    return [Request(id=s["id"], E=s["E"], N=s["N"], Ma=s["Ma"], Re=s["Re"], steps=steps,
                    arrival=float(a), precision=precision) for s, a in zip(specs, arrivals)]
