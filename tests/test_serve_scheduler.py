"""Host logic of the serving loop on a virtual clock (no GPU): FCFS admission under the byte
budget, exact step counts per solve when solves join and leave the batch at chunk boundaries,
isolation of failed solves, and the latency statistics."""
import numpy as np
import pytest

from paper_2206_09733_amd import serve, synth


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 1e-9)


class FakeExecutor:
    """Charges k * (sum of member nodes) / rate virtual seconds per chunk."""

    def __init__(self, clock, rate=2e8, fail_ids=()):
        self.clock, self.rate = clock, rate
        self.steps = {}
        self.live = set()
        self.launches = []
        self.fail_ids = set(fail_ids)

    def required_bytes(self, req):
        return 300 * req.nodes

    def admit(self, req):
        if req.id in self.fail_ids:
            raise RuntimeError("bad request")
        self.live.add(req.id)
        self.steps[req.id] = 0
        return req.id, 1e-3

    def launch(self, jobs, k):
        ids = [j.handle for j in jobs]
        assert all(i in self.live for i in ids)
        self.launches.append((self.clock(), tuple(ids), k))
        for i in ids:
            self.steps[i] += k
        return k * sum(j.req.nodes for j in jobs) / self.rate

    def wait(self, cost):
        self.clock.t += cost

    def finish(self, job):
        self.release(job)
        return np.array([job.req.id]), {"id": job.req.id}

    def release(self, job):
        self.live.discard(job.handle)


def make_requests(n, seed, rate, steps=50):
    specs = synth.serving_requests(n, seed)
    arr = synth.poisson_arrivals(n, rate, seed)
    return serve.requests_from_specs(specs, arr, steps=steps)


def test_every_solve_takes_its_steps_within_budget():
    clock = Clock()
    ex = FakeExecutor(clock)
    reqs = make_requests(64, seed=1, rate=4.0)
    budget = 2_000_000_000
    sch = serve.Scheduler(ex, budget, max_active=16, chunk_steps=7, clock=clock, sleep=clock.sleep)
    res = sch.run(reqs)
    assert all(not r.error for r in res)
    assert all(ex.steps[q.id] == q.steps for q in reqs)
    assert not ex.live
    assert sch.peak_bytes <= budget and sch.peak_active <= 16
    # first come, first served
    order = [q.id for q in sorted(reqs, key=lambda q: (q.arrival, q.id))]
    assert sch.admission_order == order
    for q, r in zip(reqs, res):
        assert r.arrival <= r.admitted <= r.finished
        assert r.state[0] == q.id
    # batching: chunks carry several solves at once
    assert max(len(ids) for _, ids, _ in ex.launches) > 1
    st = serve.summarize(reqs, res, wall=clock.t)
    lat = np.array([r.latency for r in res])
    assert st["completed"] == 64 and st["failed"] == 0
    assert st["p50_s"] == pytest.approx(np.percentile(lat, 50))
    assert st["p99_s"] == pytest.approx(np.percentile(lat, 99))
    assert st["p50_s"] <= st["p99_s"]
    work = sum(q.dof_stage_updates for q in reqs)
    assert st["gdof_stage_per_s"] == pytest.approx(work / clock.t / 1e9)


def test_budget_limits_concurrency_and_oversize_is_rejected():
    clock = Clock()
    ex = FakeExecutor(clock)
    reqs = make_requests(24, seed=2, rate=100.0, steps=20)
    big = max(reqs, key=lambda q: q.nodes)
    budget = 300 * big.nodes + 1          # the largest fits alone
    reqs.append(serve.Request(id=999, E=40, N=7, Ma=0.2, Re=0.0, steps=5, arrival=0.01))
    sch = serve.Scheduler(ex, budget, max_active=64, chunk_steps=5, clock=clock, sleep=clock.sleep)
    res = {r.id: r for r in sch.run(reqs)}
    assert "budget" in res[999].error
    assert sch.peak_bytes <= budget
    assert all(not r.error for k, r in res.items() if k != 999)
    assert all(ex.steps[q.id] == q.steps for q in reqs if q.id != 999)


def test_failed_setup_is_isolated():
    clock = Clock()
    ex = FakeExecutor(clock, fail_ids={3, 7})
    reqs = make_requests(12, seed=3, rate=50.0, steps=10)
    sch = serve.Scheduler(ex, 10**12, max_active=8, chunk_steps=4, clock=clock, sleep=clock.sleep)
    res = {r.id: r for r in sch.run(reqs)}
    assert "setup failed" in res[3].error and "setup failed" in res[7].error
    assert all(not r.error for k, r in res.items() if k not in (3, 7))
    st = serve.summarize(reqs, [res[q.id] for q in sorted(reqs, key=lambda q: q.id)], clock.t)
    assert st["completed"] == 10 and st["failed"] == 2


def test_idle_gaps_wait_for_arrivals():
    clock = Clock()
    ex = FakeExecutor(clock, rate=1e12)
    reqs = [serve.Request(id=i, E=2, N=1, Ma=0.1, Re=0.0, steps=3, arrival=10.0 * i) for i in range(4)]
    sch = serve.Scheduler(ex, 10**9, clock=clock, sleep=clock.sleep)
    res = sch.run(reqs)
    for q, r in zip(reqs, res):
        assert r.admitted >= q.arrival
        assert r.latency < 1e-3   # served alone the moment it arrived
