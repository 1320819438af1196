"""Continuous-batching request loop for PM simulations on one GPU.

Requests (forward, or forward + gradient of a chi^2 loss on the final
density) of different shapes arrive over time.  The loop

* admits a queued request as soon as a slot of its shape class is free and
  the HBM it needs fits in the budget.  Each shape class runs on one batch
  plan of the library (``pm_batch_*``): its workspace, all slots of the
  class, is charged to the budget when the plan is created and returned
  when an idle plan is dropped to make room for another class; each
  request is charged its own arrays.  Requests of other classes are not
  blocked by one that does not fit yet; a request larger than the whole
  budget is rejected;
* keeps every admitted request's particle and mesh state on the device, in
  its slot of the class's plan;
* advances all running requests of a class with one batched step (every
  kernel of a KDK step launched once for the whole class, a captured graph),
  each class on its own HIP stream so that classes overlap on the GPU, and
  keeps at most ``depth`` batched steps of a class in flight so that a new
  request joins the next step instead of queueing behind a backlog;
* retires a request when its completion event has fired and records the
  latency from arrival to result ready.

The scheduling policy is host logic (``Scheduler``) and is unit-tested on
the CPU with a fake executor; ``BatchedExecutor`` drives the HIP library's
batch plans and ``GpuExecutor`` runs one context per request (the FIFO
baseline, one request at a time).
"""
from __future__ import annotations

import collections
import heapq
import math
import time
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Tuple

import numpy as np

from .inputs import Cosmology, Workload, a_linear


# ---------------------------------------------------------------------------
# requests and shape classes
# ---------------------------------------------------------------------------

@dataclass
class SimRequest:
    rid: int
    n_part: int
    n_mesh: int
    box_size: float
    n_steps: int
    seed: int
    with_grad: bool = False
    arrival: float = 0.0          # seconds from the start of the trace
    sigma: float = 0.1            # chi^2 noise level (with_grad)

    @property
    def shape_class(self) -> Tuple[int, int, float]:
        """Requests of one shape class share a batch plan (forward and
        forward + gradient alike: the adjoint runs on the request's slot)."""
        return (self.n_part, self.n_mesh, self.box_size)

    def workload(self, cosmo: Optional[Cosmology] = None) -> Workload:
        return Workload(f"req{self.rid}", self.box_size, self.n_mesh, self.n_part, self.seed,
                        a_linear(0.1, 1.0, self.n_steps), cosmo or Cosmology())


@dataclass
class Completion:
    rid: int
    ok: bool
    arrival: float
    admitted: float = math.nan
    done: float = math.nan
    error: str = ""

    @property
    def latency(self) -> float:
        return self.done - self.arrival


def poisson_trace(n: int, rate: float, seed: int, mix=None, max_steps: int = 10, min_steps: int = 5,
                  box_per_particle: float = 2.0) -> List[SimRequest]:
    """Seeded Poisson arrivals with the benchmark's serving mix:
    60% forward 64^3 on 64^3, 30% forward + gradient 128^3 on 128^3, 10%
    forward 256^3 on 512^3; steps uniform in [min_steps, max_steps]; box =
    box_per_particle Mpc/h per lattice spacing; request seed = 1000 + id."""
    mix = mix or [(0.6, 64, 64, False), (0.3, 128, 128, True), (0.1, 256, 512, False)]
    rng = np.random.default_rng(seed)
    t = 0.0
    probs = np.array([m[0] for m in mix], dtype=np.float64)
    probs /= probs.sum()
    out = []
    for i in range(n):
        t += rng.exponential(1.0 / rate)
        k = rng.choice(len(mix), p=probs)
        _, npart, nmesh, grad = mix[k]
        steps = int(rng.integers(min_steps, max_steps + 1))
        out.append(SimRequest(i, npart, nmesh, box_per_particle * npart, steps, 1000 + i, grad, t))
    return out


def request_bytes(req: SimRequest) -> int:
    """HBM of a request's own device arrays: noise, positions, momenta, final
    density; with the gradient also the checkpoints, the target, the density
    cotangent, the position/momentum cotangents and the noise gradient."""
    np3 = req.n_part ** 3
    ng3 = req.n_mesh ** 3
    b = 4 * np3 + 2 * 12 * np3 + 4 * ng3
    if req.with_grad:
        b += (req.n_steps + 1) * 2 * 12 * np3 + 4 * ng3 + 4 * ng3 + 2 * 12 * np3 + 4 * np3
    return b


def footprint_bytes(req: SimRequest, workspace_bytes: int) -> int:
    """HBM held by one request run on a context of its own: the library
    workspace plus the request's arrays."""
    return workspace_bytes + request_bytes(req)


# ---------------------------------------------------------------------------
# scheduling policy (host only)
# ---------------------------------------------------------------------------

class Scheduler:
    """Admission by HBM and per-class slot count.

    ``footprint(req)`` is the HBM a request holds while admitted;
    ``plan_bytes(cls)`` is the HBM of the resident state of a shape class
    (its batch plan), charged when the first request of the class is
    admitted and kept until the class is evicted.  ``used`` never exceeds
    the budget: when a request does not fit, plans of other classes with no
    admitted request are evicted (oldest first) and listed in ``evicted``
    for the executor to free."""

    def __init__(self, budget_bytes: int, slots_per_class: int, footprint, plan_bytes=None):
        self.budget = int(budget_bytes)
        self.slots_per_class = int(slots_per_class)
        self.footprint = footprint          # callable(req) -> bytes
        self.plan_bytes = plan_bytes or (lambda cls: 0)
        self.used = 0
        self.queue: List[SimRequest] = []
        self.active_per_class: Dict[tuple, int] = {}
        self.held: Dict[int, int] = {}
        self.plans: Dict[tuple, int] = {}   # resident classes (insertion order = age) -> bytes
        self.evicted: List[tuple] = []

    def submit(self, req: SimRequest):
        self.queue.append(req)

    def _evict_idle(self, need: int, keep_cls) -> bool:
        """Evict idle resident classes other than keep_cls until need more
        bytes fit; True if they do."""
        for cls in list(self.plans):
            if self.used + need <= self.budget:
                break
            if cls != keep_cls and self.active_per_class.get(cls, 0) == 0:
                self.used -= self.plans.pop(cls)
                self.evicted.append(cls)
        return self.used + need <= self.budget

    def admit(self) -> Tuple[List[SimRequest], List[Tuple[SimRequest, str]]]:
        """Requests to start now (arrival order), and requests rejected."""
        admitted, rejected, keep = [], [], []
        for req in self.queue:
            cls = req.shape_class
            own = self.footprint(req)
            plan = self.plan_bytes(cls)
            if own + plan > self.budget:
                rejected.append((req, f"footprint {own + plan} B exceeds the HBM budget {self.budget} B"))
                continue
            need = own + (0 if cls in self.plans else plan)
            fits = self.used + need <= self.budget or self._evict_idle(need, cls)
            if self.active_per_class.get(cls, 0) < self.slots_per_class and fits:
                if cls not in self.plans:
                    self.plans[cls] = plan
                self.used += need
                self.held[req.rid] = own
                self.active_per_class[cls] = self.active_per_class.get(cls, 0) + 1
                admitted.append(req)
            else:
                keep.append(req)
        self.queue = keep
        return admitted, rejected

    def release(self, req: SimRequest):
        self.used -= self.held.pop(req.rid, 0)
        cls = req.shape_class
        self.active_per_class[cls] = self.active_per_class.get(cls, 1) - 1

    def cancel(self, rid: int) -> bool:
        n = len(self.queue)
        self.queue = [r for r in self.queue if r.rid != rid]
        return len(self.queue) != n


# ---------------------------------------------------------------------------
# GPU executors
# ---------------------------------------------------------------------------

class _Job:
    def __init__(self, req: SimRequest, slot):
        self.req = req
        self.slot = slot
        self.remaining = req.n_steps
        self.ended = False
        self.event = None
        self.result = None
        self.tensors = {}


def _finish_outputs(torch, req, ctx, t, device, delta):
    """The gradient request's chi^2 against a seeded target and the adjoint
    of its run on the request's own context (slot)."""
    out = {"pos": t["pos"], "mom": t["mom"], "delta": delta}
    if req.with_grad:
        m = req.n_mesh
        gen = torch.Generator(device=device)
        gen.manual_seed(req.seed + 2000)
        target = torch.randn((m, m, m), generator=gen, device=device) * req.sigma
        loss, gdelta = ctx.pm_chi2(delta, target, req.sigma)
        _, _, gn = ctx.pm_run_adjoint(t["a"], t["ckpt"], noise=t["noise"], grad_delta=gdelta)
        out.update(loss=loss, grad_noise=gn)
    return out


class _Plan:
    def __init__(self, batch, stream, slots):
        self.batch = batch
        self.stream = stream
        self.free = list(range(slots))
        self.jobs: Dict[int, _Job] = {}          # slot -> running job
        self.inflight = collections.deque()      # events of enqueued batched steps
        self.grad_pool: List[list] = []          # [context, stream, busy] for adjoints


class BatchedExecutor:
    """Runs each shape class on one batch plan of the HIP library (one
    stream per class): a request takes a slot, its initial conditions are
    generated on the slot, and every tick enqueues one batched KDK step for
    all running requests of a class (at most ``depth`` in flight per class).
    A finished request leaves its slot at once; a gradient request's chi^2
    and adjoint (which need only its arrays: checkpoints, noise, final
    density) then run on a context of its own from a per-class pool, each on
    its own stream, so that adjoints overlap with each other and with the
    class's batched steps."""

    def __init__(self, device="cuda", cosmo: Optional[Cosmology] = None, slots_per_class: int = 4,
                 keep_results: bool = True, graphs: bool = True, depth: int = 2):
        import torch
        from .binding import PMBatch
        self.torch = torch
        self.PMBatch = PMBatch
        self.device = torch.device(device)
        self.cosmo = cosmo or Cosmology()
        self.slots = max(2, int(slots_per_class))
        self.keep_results = keep_results
        self.graphs = graphs
        self.depth = max(1, int(depth))
        self.plans: Dict[tuple, _Plan] = {}
        self._ws: Dict[tuple, int] = {}

    def plan_bytes(self, cls) -> int:
        """HBM of a class's resident state: the plan (every slot's workspace)
        and its pool of adjoint contexts (one workspace per slot, created on
        demand but charged up front)."""
        if cls not in self._ws:
            import ctypes as C
            from . import _lib
            from .binding import make_config
            npart, nmesh, box = cls
            w = Workload("plan", box, nmesh, npart, 0, (0.1, 1.0), self.cosmo)
            lib = _lib.load()
            self._ws[cls] = (int(lib.pm_workspace_bytes(C.byref(make_config(w, batch=self.slots))))
                             + self.slots * int(lib.pm_workspace_bytes(C.byref(make_config(w)))))
        return self._ws[cls]

    def request_bytes(self, req: SimRequest) -> int:
        return request_bytes(req)

    def _plan(self, req: SimRequest) -> _Plan:
        cls = req.shape_class
        p = self.plans.get(cls)
        if p is None:
            stream = self.torch.cuda.Stream(device=self.device)
            with self.torch.cuda.stream(stream):
                b = self.PMBatch(req.workload(self.cosmo), self.slots, device=self.device, stream=stream)
            if self.graphs:
                b.pm_use_graphs(True)
            p = self.plans[cls] = _Plan(b, stream, self.slots)
        return p

    def drop_plan(self, cls):
        p = self.plans.pop(cls, None)
        if p is not None:
            p.stream.synchronize()
            p.batch.close()
            for ctx, stream, _ in p.grad_pool:
                stream.synchronize()
                ctx.close()

    def _grad_ctx(self, p: _Plan, req: SimRequest):
        for e in p.grad_pool:
            if not e[2]:
                e[2] = True
                return e
        from .binding import PMContext
        stream = self.torch.cuda.Stream(device=self.device)
        with self.torch.cuda.stream(stream):
            ctx = PMContext(req.workload(self.cosmo), device=self.device, stream=stream)
        e = [ctx, stream, True]
        p.grad_pool.append(e)
        return e

    def start(self, req: SimRequest) -> _Job:
        torch = self.torch
        p = self._plan(req)
        if not p.free:
            raise RuntimeError("no free slot in the class's plan")
        slot = p.free.pop(0)
        job = _Job(req, (p, slot))
        w = req.workload(self.cosmo)
        mc = p.batch.member(slot)
        try:
            with torch.cuda.stream(p.stream):
                n = req.n_part
                noise = mc.pm_noise(req.seed)
                pos, mom = mc.pm_init_lpt(req.seed, w.a_list[0], noise=noise)
                ckpt = None
                if req.with_grad:
                    ckpt = torch.empty((req.n_steps + 1, 2, n ** 3, 3), dtype=torch.float32, device=self.device)
                p.batch.pm_batch_begin(slot, w.a_list, pos, mom, ckpt=ckpt)
        except Exception:
            p.free.append(slot)
            raise
        job.tensors = {"noise": noise, "pos": pos, "mom": mom, "ckpt": ckpt, "a": w.a_list}
        p.jobs[slot] = job
        return job

    def tick(self, jobs: List[_Job]):
        """One batched step per class with running requests (unless its
        in-flight limit of steps is reached), then finish the requests whose
        last step is enqueued.  The class with the most mesh cells among
        those running keeps 2 `depth` steps in flight (its queue then
        outlasts a longer pause of this loop), the lighter ones `depth`."""
        torch = self.torch
        active = [cls for cls, p in self.plans.items() if any(not j.ended for j in p.jobs.values())]
        heavy = max((cls[1] for cls in active), default=0)
        for cls, p in self.plans.items():
            while p.inflight and p.inflight[0].query():
                p.inflight.popleft()
            limit = 2 * self.depth if cls[1] >= heavy else self.depth
            if cls not in active or len(p.inflight) >= limit:
                continue
            with torch.cuda.stream(p.stream):
                if p.batch.pm_batch_advance() > 0:
                    ev = torch.cuda.Event()
                    ev.record(p.stream)
                    p.inflight.append(ev)
            for slot, job in list(p.jobs.items()):
                if not job.ended:
                    job.remaining = p.batch.pm_batch_remaining(slot)
                    if job.remaining == 0:
                        self._finish(p, slot, job)

    def _finish(self, p: _Plan, slot: int, job: _Job):
        torch = self.torch
        req, t = job.req, job.tensors
        with torch.cuda.stream(p.stream):
            m = req.n_mesh
            delta = torch.empty((m, m, m), dtype=torch.float32, device=self.device)
            p.batch.pm_batch_end(slot, delta_final=delta)
            ev = torch.cuda.Event()
            ev.record(p.stream)
        # the slot is free once its end is enqueued: a later begin on it runs
        # after the end on the plan's stream
        del p.jobs[slot]
        p.free.append(slot)
        job.slot = (p, None)
        if req.with_grad:
            g = self._grad_ctx(p, req)
            g[1].wait_event(ev)
            with torch.cuda.stream(g[1]):
                out = _finish_outputs(torch, req, g[0], t, self.device, delta)
                ev = torch.cuda.Event()
                ev.record(g[1])
            job.grad = g
        else:
            out = {"pos": t["pos"], "mom": t["mom"], "delta": delta}
        job.event = ev
        job.result = out if self.keep_results else None
        job.ended = True

    def done(self, job: _Job) -> bool:
        return job.ended and job.event.query()

    def release(self, job: _Job):
        p, slot = job.slot
        job.tensors = {}
        g = getattr(job, "grad", None)
        if g is not None:
            g[2] = False
            job.grad = None
        if slot is not None and p.jobs.get(slot) is job:
            del p.jobs[slot]
            p.free.append(slot)

    def abandon(self, job: _Job):
        """Drop a request that failed mid-run (its slot is not reused)."""
        p, slot = job.slot
        if slot is not None:
            p.jobs.pop(slot, None)


class _Slot:
    def __init__(self, ctx, stream):
        self.ctx = ctx
        self.stream = stream
        self.busy = False


class GpuExecutor:
    """Runs each request on a library context of its own (one stream per
    context).  Used for the one-at-a-time baseline (``serve_fifo``), and by
    ``serve`` as the unbatched comparison: every request then launches its
    own kernels.  Contexts are pooled per shape class; a class's pool (up to
    ``slots_per_class`` workspaces) is what ``plan_bytes`` charges."""

    def __init__(self, device="cuda", cosmo: Optional[Cosmology] = None, keep_results: bool = True,
                 graphs: bool = True, slots_per_class: int = 4):
        import torch
        from .binding import PMContext
        self.torch = torch
        self.PMContext = PMContext
        self.device = torch.device(device)
        self.cosmo = cosmo or Cosmology()
        self.slots: Dict[tuple, List[_Slot]] = {}
        self.keep_results = keep_results
        self.graphs = graphs   # each slot replays one captured graph per step
        self.slots_per_class = int(slots_per_class)
        self._ws_bytes: Dict[tuple, int] = {}

    def workspace_bytes(self, req: SimRequest) -> int:
        key = (req.n_part, req.n_mesh)
        if key not in self._ws_bytes:
            import ctypes as C
            from . import _lib
            from .binding import make_config
            lib = _lib.load()
            self._ws_bytes[key] = int(lib.pm_workspace_bytes(C.byref(make_config(req.workload(self.cosmo)))))
        return self._ws_bytes[key]

    def plan_bytes(self, cls) -> int:
        npart, nmesh, box = cls
        return self.slots_per_class * self.workspace_bytes(SimRequest(0, npart, nmesh, box, 1, 0))

    def request_bytes(self, req: SimRequest) -> int:
        return request_bytes(req)

    def drop_plan(self, cls):
        for s in self.slots.pop(cls, []):
            s.stream.synchronize()
            s.ctx.close()

    def _slot(self, req: SimRequest) -> _Slot:
        cls = req.shape_class
        pool = self.slots.setdefault(cls, [])
        for s in pool:
            if not s.busy:
                s.busy = True
                return s
        stream = self.torch.cuda.Stream(device=self.device)
        with self.torch.cuda.stream(stream):
            ctx = self.PMContext(req.workload(self.cosmo), device=self.device, stream=stream)
        if self.graphs:
            ctx.pm_use_graphs(True)
        s = _Slot(ctx, stream)
        s.busy = True
        pool.append(s)
        return s

    def start(self, req: SimRequest) -> _Job:
        torch = self.torch
        slot = self._slot(req)
        job = _Job(req, slot)
        w = req.workload(self.cosmo)
        ctx = slot.ctx
        with torch.cuda.stream(slot.stream):
            n = req.n_part
            noise = ctx.pm_noise(req.seed)
            pos, mom = ctx.pm_init_lpt(req.seed, w.a_list[0], noise=noise)
            ckpt = None
            if req.with_grad:
                ckpt = torch.empty((req.n_steps + 1, 2, n ** 3, 3), dtype=torch.float32, device=self.device)
            ctx.pm_run_begin(w.a_list, pos, mom, ckpt=ckpt)
            job.tensors = {"noise": noise, "pos": pos, "mom": mom, "ckpt": ckpt, "a": w.a_list}
        return job

    def step(self, job: _Job):
        with self.torch.cuda.stream(job.slot.stream):
            job.remaining = job.slot.ctx.pm_run_advance(1)

    def finish(self, job: _Job):
        torch = self.torch
        req, ctx, t = job.req, job.slot.ctx, job.tensors
        with torch.cuda.stream(job.slot.stream):
            m = req.n_mesh
            delta = torch.empty((m, m, m), dtype=torch.float32, device=self.device)
            ctx.pm_run_end(delta_final=delta)
            out = _finish_outputs(torch, req, ctx, t, self.device, delta)
            ev = torch.cuda.Event()
            ev.record(job.slot.stream)
        job.event = ev
        job.result = out if self.keep_results else None
        job.ended = True

    def tick(self, jobs: List[_Job]):
        """One step of every running request (each on its own stream)."""
        for job in jobs:
            if job.remaining > 0:
                self.step(job)
            elif not job.ended:
                self.finish(job)

    def done(self, job: _Job) -> bool:
        return job.ended and job.event.query()

    def release(self, job: _Job):
        job.tensors = {}
        job.slot.busy = False

    def abandon(self, job: _Job):
        job.tensors = {}


# ---------------------------------------------------------------------------
# the loop
# ---------------------------------------------------------------------------

@dataclass
class ServeReport:
    completions: List[Completion] = field(default_factory=list)
    wall: float = 0.0
    max_active: int = 0
    max_queue: int = 0
    max_used: int = 0

    def summary(self) -> dict:
        ok = [c for c in self.completions if c.ok]
        lat = np.array([c.latency for c in ok]) if ok else np.array([math.nan])
        span = (max(c.done for c in ok) - min(c.arrival for c in ok)) if ok else math.nan
        return {"completed": len(ok), "failed": len(self.completions) - len(ok),
                "sims_per_s": len(ok) / span if ok and span > 0 else math.nan,
                "p50_latency_s": float(np.percentile(lat, 50)), "p99_latency_s": float(np.percentile(lat, 99)),
                "mean_latency_s": float(lat.mean()), "wall_s": self.wall, "max_active": self.max_active,
                "max_queue": self.max_queue}


def serve(trace: List[SimRequest], executor, budget_bytes: int, slots_per_class: int = 4,
          realtime: bool = True, results: Optional[dict] = None, clock=time.perf_counter,
          sleep=time.sleep) -> ServeReport:
    """Continuous batching over a trace of requests (sorted by arrival)."""
    sched = Scheduler(budget_bytes, slots_per_class, executor.request_bytes, executor.plan_bytes)
    pending = list(sorted(trace, key=lambda r: r.arrival))
    rep = ServeReport()
    comp: Dict[int, Completion] = {}
    active: List[_Job] = []
    t0 = clock()
    i = 0
    while i < len(pending) or sched.queue or active:
        now = clock() - t0 if realtime else math.inf
        while i < len(pending) and pending[i].arrival <= now:
            sched.submit(pending[i])
            comp[pending[i].rid] = Completion(pending[i].rid, False, pending[i].arrival)
            i += 1
        rep.max_queue = max(rep.max_queue, len(sched.queue))
        admitted, rejected = sched.admit()
        for cls in sched.evicted:
            executor.drop_plan(cls)
        sched.evicted.clear()
        rep.max_used = max(rep.max_used, sched.used)
        for req, why in rejected:
            c = comp[req.rid]
            c.done, c.error = clock() - t0, why
        for req in admitted:
            comp[req.rid].admitted = clock() - t0
            try:
                active.append(executor.start(req))
            except Exception as e:   # isolate a failing request
                c = comp[req.rid]
                c.done, c.error = clock() - t0, f"start failed: {e}"
                sched.release(req)
        rep.max_active = max(rep.max_active, len(active))
        try:
            executor.tick(active)
        except Exception as e:       # a failing step fails the requests it carried
            for job in active:
                if not job.ended:
                    job.ended, job.event = True, None
                    comp[job.req.rid].error = f"run failed: {e}"
                    executor.abandon(job)
        still = []
        for job in active:
            failed = job.ended and job.event is None
            if failed or executor.done(job):
                c = comp[job.req.rid]
                c.done = clock() - t0
                c.ok = not failed
                if results is not None and job.result is not None:
                    results[job.req.rid] = job.result
                if not failed:
                    executor.release(job)
                sched.release(job.req)
            else:
                still.append(job)
        active = still
        if not active and not sched.queue and i < len(pending) and realtime:
            sleep(max(0.0, min(0.01, pending[i].arrival - (clock() - t0))))
    rep.wall = clock() - t0
    rep.completions = [comp[r.rid] for r in trace]
    return rep


def serve_fifo(trace: List[SimRequest], executor, realtime: bool = True, results: Optional[dict] = None,
               clock=time.perf_counter, sleep=time.sleep) -> ServeReport:
    """Baseline: the same trace served one request at a time, in arrival
    order, each run whole on a context of its own."""
    rep = ServeReport()
    t0 = clock()
    for req in sorted(trace, key=lambda r: r.arrival):
        if realtime:
            wait = req.arrival - (clock() - t0)
            if wait > 0:
                sleep(wait)
        c = Completion(req.rid, False, req.arrival, admitted=clock() - t0)
        try:
            job = executor.start(req)
            while job.remaining > 0:
                executor.step(job)
            executor.finish(job)
            while not executor.done(job):
                sleep(0)
            c.ok = True
            if results is not None and job.result is not None:
                results[req.rid] = job.result
            executor.release(job)
        except Exception as e:
            c.error = str(e)
        c.done = clock() - t0
        rep.completions.append(c)
    rep.wall = clock() - t0
    rep.max_active = 1
    return rep
