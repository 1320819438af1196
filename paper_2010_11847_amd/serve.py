"""Continuous-batching request loop for PM simulations on one GPU.

Requests (forward, or forward + gradient of a chi^2 loss on the final
density) of different shapes arrive over time.  The loop

* admits a queued request as soon as a slot of its shape class is free and
  its HBM footprint fits in the budget (requests of other classes are not
  blocked by one that does not fit yet; a request larger than the whole
  budget is rejected);
* keeps every admitted request's particle and mesh state on the device (one
  library context, i.e. one workspace, per slot, reused across requests);
* advances every active request by one KDK step per tick, each slot on its
  own HIP stream, so the kernels of different requests overlap on the GPU
  and new requests join while others are mid-run;
* retires a request when its completion event has fired and records the
  latency from arrival to result ready.

The scheduling policy is host logic (``Scheduler``) and is unit-tested on
the CPU with a fake executor; ``GpuExecutor`` drives the HIP library.
"""
from __future__ import annotations

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
    def shape_class(self) -> Tuple[int, int, float, bool]:
        return (self.n_part, self.n_mesh, self.box_size, self.with_grad)

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


def footprint_bytes(req: SimRequest, workspace_bytes: int) -> int:
    """HBM held by one admitted request: the library workspace plus its own
    device arrays (noise, positions, momenta, final density; with the
    gradient also the checkpoints, target, cotangents and noise gradient)."""
    np3 = req.n_part ** 3
    ng3 = req.n_mesh ** 3
    b = workspace_bytes + 4 * np3 + 2 * 12 * np3 + 4 * ng3
    if req.with_grad:
        b += (req.n_steps + 1) * 2 * 12 * np3 + 4 * ng3 + 2 * 12 * np3 + 4 * np3 + 4 * ng3
    return b


# ---------------------------------------------------------------------------
# scheduling policy (host only)
# ---------------------------------------------------------------------------

class Scheduler:
    """Admission by HBM footprint and per-class slot count."""

    def __init__(self, budget_bytes: int, slots_per_class: int, footprint):
        self.budget = int(budget_bytes)
        self.slots_per_class = int(slots_per_class)
        self.footprint = footprint          # callable(req) -> bytes
        self.used = 0
        self.queue: List[SimRequest] = []
        self.active_per_class: Dict[tuple, int] = {}
        self.held: Dict[int, int] = {}

    def submit(self, req: SimRequest):
        self.queue.append(req)

    def admit(self) -> Tuple[List[SimRequest], List[Tuple[SimRequest, str]]]:
        """Requests to start now (arrival order), and requests rejected."""
        admitted, rejected, keep = [], [], []
        for req in self.queue:
            need = self.footprint(req)
            if need > self.budget:
                rejected.append((req, f"footprint {need} B exceeds the HBM budget {self.budget} B"))
                continue
            cls = req.shape_class
            if self.active_per_class.get(cls, 0) < self.slots_per_class and self.used + need <= self.budget:
                self.used += need
                self.held[req.rid] = need
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
# GPU executor
# ---------------------------------------------------------------------------

class _Slot:
    def __init__(self, ctx, stream):
        self.ctx = ctx
        self.stream = stream
        self.busy = False


class _Job:
    def __init__(self, req: SimRequest, slot: _Slot):
        self.req = req
        self.slot = slot
        self.remaining = req.n_steps
        self.ended = False
        self.event = None
        self.result = None
        self.tensors = {}


class GpuExecutor:
    """Runs requests with the HIP library, one context and stream per slot."""

    def __init__(self, device="cuda", cosmo: Optional[Cosmology] = None, keep_results: bool = True,
                 graphs: bool = True):
        import torch
        from .binding import PMContext
        self.torch = torch
        self.PMContext = PMContext
        self.device = torch.device(device)
        self.cosmo = cosmo or Cosmology()
        self.slots: Dict[tuple, List[_Slot]] = {}
        self.keep_results = keep_results
        self.graphs = graphs   # each slot replays one captured graph per step
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

    def _slot(self, req: SimRequest) -> _Slot:
        cls = (req.n_part, req.n_mesh, req.box_size)
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
            out = {"pos": t["pos"], "mom": t["mom"], "delta": delta}
            if req.with_grad:
                gen = torch.Generator(device=self.device)
                gen.manual_seed(req.seed + 2000)
                target = torch.randn((m, m, m), generator=gen, device=self.device) * req.sigma
                loss, gdelta = ctx.pm_chi2(delta, target, req.sigma)
                _, _, gn = ctx.pm_run_adjoint(t["a"], t["ckpt"], noise=t["noise"], grad_delta=gdelta)
                out.update(loss=loss, grad_noise=gn)
            ev = torch.cuda.Event()
            ev.record(job.slot.stream)
        job.event = ev
        job.result = out if self.keep_results else None
        job.ended = True

    def done(self, job: _Job) -> bool:
        return job.ended and job.event.query()

    def release(self, job: _Job):
        job.tensors = {}
        job.slot.busy = False


# ---------------------------------------------------------------------------
# the loop
# ---------------------------------------------------------------------------

@dataclass
class ServeReport:
    completions: List[Completion] = field(default_factory=list)
    wall: float = 0.0
    max_active: int = 0
    max_queue: int = 0

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
    sched = Scheduler(budget_bytes, slots_per_class,
                      lambda r: footprint_bytes(r, executor.workspace_bytes(r)))
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
        # one KDK step of every running request, then close finished ones
        for job in active:
            try:
                if job.remaining > 0:
                    executor.step(job)
                elif not job.ended:
                    executor.finish(job)
            except Exception as e:
                job.ended, job.event = True, None
                comp[job.req.rid].error = f"run failed: {e}"
        still = []
        for job in active:
            failed = job.ended and job.event is None
            if failed or executor.done(job):
                c = comp[job.req.rid]
                c.done = clock() - t0
                c.ok = not failed
                if results is not None and job.result is not None:
                    results[job.req.rid] = job.result
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
    """Baseline: the same trace served one request at a time, in arrival order."""
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
