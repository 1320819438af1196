"""Host-only tests of the continuous-batching loop with a fake executor:
admission by HBM footprint and slots, rejection, isolation of failures,
interleaving, and the FIFO baseline."""
import math

import pytest

from paper_2010_11847_amd import serve


class FakeJob:
    def __init__(self, req, slot_log):
        self.req = req
        self.remaining = req.n_steps
        self.ended = False
        self.event = True
        self.result = {"rid": req.rid}
        self.log = slot_log


class FakeExecutor:
    """Steps take no time; a request finishes one tick after its last step.
    Records the interleaving of steps across requests, the live plans and
    the HBM they and the running requests hold."""

    def __init__(self, ws=100, fail=(), plan=0):
        self.ws = ws
        self.plan = plan
        self.fail = set(fail)
        self.trace = []
        self.active_now = 0
        self.max_active = 0
        self.live_plans = set()
        self.dropped = []

    def request_bytes(self, req):
        return self.ws

    def plan_bytes(self, cls):
        return self.plan

    def drop_plan(self, cls):
        self.live_plans.discard(cls)
        self.dropped.append(cls)

    def start(self, req):
        if req.rid in self.fail:
            raise RuntimeError("forced failure")
        self.live_plans.add(req.shape_class)
        self.active_now += 1
        self.max_active = max(self.max_active, self.active_now)
        return FakeJob(req, self.trace)

    def step(self, job):
        self.trace.append(job.req.rid)
        job.remaining -= 1

    def finish(self, job):
        job.ended = True

    def tick(self, jobs):
        for job in jobs:
            if job.remaining > 0:
                self.step(job)
            elif not job.ended:
                self.finish(job)

    def done(self, job):
        return job.ended

    def release(self, job):
        self.active_now -= 1

    def abandon(self, job):
        self.active_now -= 1


def req(i, npart=8, steps=3, grad=False, arrival=0.0):
    return serve.SimRequest(i, npart, npart, 2.0 * npart, steps, 1000 + i, grad, arrival)


def test_footprint_counts_checkpoints():
    a = serve.footprint_bytes(req(0, 64, 5), 1000)
    b = serve.footprint_bytes(req(0, 64, 5, grad=True), 1000)
    assert b - a >= 6 * 2 * 12 * 64 ** 3
    assert serve.request_bytes(req(0, 64, 5)) == a - 1000


def test_admission_respects_budget_and_slots():
    fp = lambda r: 10  # noqa: E731
    s = serve.Scheduler(budget_bytes=25, slots_per_class=5, footprint=fp)
    for i in range(4):
        s.submit(req(i))
    adm, rej = s.admit()
    assert [r.rid for r in adm] == [0, 1] and not rej and s.used == 20
    s.release(adm[0])
    adm, _ = s.admit()
    assert [r.rid for r in adm] == [2]
    s2 = serve.Scheduler(budget_bytes=1000, slots_per_class=2, footprint=fp)
    for i in range(4):
        s2.submit(req(i))
    adm, _ = s2.admit()
    assert len(adm) == 2


def test_oversized_request_rejected_and_others_not_blocked():
    sizes = {0: 50, 1: 500, 2: 50}
    s = serve.Scheduler(budget_bytes=120, slots_per_class=8, footprint=lambda r: sizes[r.rid])
    for i in range(3):
        s.submit(req(i, npart=8 if i != 1 else 16))
    adm, rej = s.admit()
    assert [r.rid for r in adm] == [0, 2]
    assert [r.rid for r, _ in rej] == [1]


def test_no_head_of_line_blocking_across_classes():
    sizes = {0: 80, 1: 60, 2: 10}
    s = serve.Scheduler(budget_bytes=100, slots_per_class=8, footprint=lambda r: sizes[r.rid])
    s.submit(req(0, npart=16))
    s.submit(req(1, npart=32))
    s.submit(req(2, npart=8))
    adm, _ = s.admit()
    assert [r.rid for r in adm] == [0, 2]      # 1 waits, 2 is not blocked by it


def test_cancel_queued():
    s = serve.Scheduler(budget_bytes=10, slots_per_class=1, footprint=lambda r: 10)
    s.submit(req(0))
    s.submit(req(1))
    s.admit()
    assert s.cancel(1) and not s.cancel(1)


def test_serve_interleaves_and_isolates_failures():
    ex = FakeExecutor(ws=10, fail={3})
    trace = [req(i, steps=2 + i % 3) for i in range(6)]
    out = {}
    rep = serve.serve(trace, ex, budget_bytes=10 ** 9, slots_per_class=4, realtime=False, results=out)
    ok = {c.rid for c in rep.completions if c.ok}
    assert ok == {0, 1, 2, 4, 5}
    failed = [c for c in rep.completions if not c.ok]
    assert len(failed) == 1 and "forced failure" in failed[0].error
    assert set(out) == ok
    # steps of different requests are interleaved (continuous batching)
    first_two = ex.trace[:4]
    assert len(set(first_two)) > 1
    assert ex.max_active == 4        # slots per class bound concurrency
    assert rep.summary()["completed"] == 5


def test_tiny_budget_serialises_without_oom():
    ex = FakeExecutor(ws=1000, plan=500)
    trace = [req(i, steps=2) for i in range(5)]
    rep = serve.serve(trace, ex, budget_bytes=1500, slots_per_class=8, realtime=False)
    assert all(c.ok for c in rep.completions)
    assert ex.max_active == 1
    assert rep.max_used <= 1500


def test_plan_memory_is_charged_and_idle_plans_evicted():
    """Resident plans count against the budget from their first request until
    they are evicted; with several shape classes the HBM in use (plans plus
    running requests) never exceeds the budget, and an idle plan of another
    class is dropped when a request would not fit otherwise."""
    ex = FakeExecutor(ws=10, plan=100)
    trace = []
    for i in range(12):
        npart = (8, 16, 32)[i % 3]
        trace.append(req(i, npart=npart, steps=1 + i % 2, arrival=float(i // 3)))
    rep = serve.serve(trace, ex, budget_bytes=125, slots_per_class=2, realtime=False)
    assert all(c.ok for c in rep.completions)
    assert rep.max_used <= 125          # one plan + up to two requests
    assert len(ex.dropped) >= 2         # classes took turns
    sched = serve.Scheduler(budget_bytes=250, slots_per_class=2, footprint=lambda r: 10, plan_bytes=lambda c: 100)
    sched.submit(req(0, npart=8))
    sched.submit(req(1, npart=16))
    adm, _ = sched.admit()
    assert [r.rid for r in adm] == [0, 1] and sched.used == 220
    sched.submit(req(2, npart=32))      # a third plan does not fit while both classes run
    adm, _ = sched.admit()
    assert not adm and not sched.evicted
    sched.release(adm and adm[0] or req(0, npart=8))
    adm, _ = sched.admit()              # class 8 is idle now: evicted for class 32
    assert [r.rid for r in adm] == [2] and sched.evicted == [(8, 8, 16.0)]
    assert sched.used == 220
    # a request whose own bytes plus its plan exceed the budget is rejected
    sched2 = serve.Scheduler(budget_bytes=105, slots_per_class=2, footprint=lambda r: 10, plan_bytes=lambda c: 100)
    sched2.submit(req(0))
    adm, rej = sched2.admit()
    assert not adm and len(rej) == 1 and "exceeds the HBM budget" in rej[0][1]


def test_fifo_baseline_runs_in_order():
    ex = FakeExecutor()
    trace = [req(i, steps=2, arrival=0.0) for i in range(3)]
    rep = serve.serve_fifo(trace, ex, realtime=False)
    assert [c.rid for c in rep.completions] == [0, 1, 2]
    assert ex.trace == [0, 0, 1, 1, 2, 2]


def test_poisson_trace_mix():
    tr = serve.poisson_trace(1000, 20.0, seed=5)
    kinds = {}
    for r in tr:
        kinds[(r.n_part, r.n_mesh, r.with_grad)] = kinds.get((r.n_part, r.n_mesh, r.with_grad), 0) + 1
    assert abs(kinds[(64, 64, False)] / 1000 - 0.6) < 0.05
    assert abs(kinds[(128, 128, True)] / 1000 - 0.3) < 0.05
    assert abs(kinds[(256, 512, False)] / 1000 - 0.1) < 0.03
    gaps = [b.arrival - a.arrival for a, b in zip(tr[:-1], tr[1:])]
    assert all(g > 0 for g in gaps)
    assert math.isclose(sum(gaps) / len(gaps), 1 / 20.0, rel_tol=0.1)
    assert all(5 <= r.n_steps <= 10 for r in tr)
