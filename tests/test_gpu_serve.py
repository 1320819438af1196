"""Continuous batching on the GPU: requests of a shape class share a batch
plan and advance together in batched steps; every request's result in the
mix equals its result when run alone on a context of its own, bit for bit
(same kernels, integer paint sums), for forward and forward + gradient
requests of different shapes, and one request of each serving class
matches the FP64 oracle."""
import json
import os

import numpy as np
import pytest
import torch

from oracle import pm as opm
from paper_2010_11847_amd import serve
from tests.golden import make_golden as G
from tests.gpu_helpers import banner, record, rel, to_np

pytestmark = pytest.mark.gpu


def small_trace():
    mix = []
    for i in range(10):
        if i % 3 == 0:
            mix.append(serve.SimRequest(i, 16, 64, 32.0, 3 + i % 3, 1000 + i, True, 0.0))
        elif i % 3 == 1:
            mix.append(serve.SimRequest(i, 32, 64, 64.0, 4 + i % 4, 1000 + i, False, 0.0))
        else:
            mix.append(serve.SimRequest(i, 32, 128, 64.0, 5, 1000 + i, False, 0.0))
    return mix


def test_results_same_alone_and_in_mix(gpu):
    banner("served in batch plans vs alone")
    trace = small_trace()
    ex = serve.BatchedExecutor(slots_per_class=3)
    mixed = {}
    rep = serve.serve(trace, ex, budget_bytes=8 << 30, slots_per_class=3, realtime=False, results=mixed)
    s = rep.summary()
    banner(f"  {s}")
    assert s["completed"] == len(trace) and rep.max_active > 1
    alone_ex = serve.GpuExecutor(graphs=False)
    for req in trace:
        alone = {}
        serve.serve_fifo([req], alone_ex, realtime=False, results=alone)
        a, m = alone[req.rid], mixed[req.rid]
        for k in ("pos", "mom", "delta") + (("grad_noise",) if req.with_grad else ()):
            assert torch.equal(m[k], a[k]), (req.rid, k, float((m[k] - a[k]).abs().max()))
        if req.with_grad:
            assert float(m["loss"]) == float(a["loss"])


def test_served_requests_match_the_oracle(gpu):
    """One request of each serving class (64^3 forward, 128^3 forward +
    gradient, 256^3 particles on a 512^3 mesh), served together with small
    requests, against the FP64 oracle's run from the same seed (stored by
    tests/golden/make_golden.py serve): final positions rms < 1e-3 cell and
    momenta within 1e-2 at 1024 sampled particles (independent trajectories
    from the seed on both sides)."""
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "serve_classes.json")
    if not os.path.exists(path):
        pytest.skip("golden file serve_classes.json not generated")
    with open(path) as fh:
        g = json.load(fh)
    banner("served requests vs the oracle")
    trace = [serve.SimRequest(rid, npart, nmesh, box, steps, seed, grad, 0.0)
             for rid, npart, nmesh, box, steps, seed, grad in G.SERVE_REQS]
    trace += small_trace()[:4]
    for i, r in enumerate(trace[3:]):
        r.rid = 100 + i
    results = {}
    rep = serve.serve(trace, serve.BatchedExecutor(slots_per_class=4), budget_bytes=64 << 30, slots_per_class=4,
                      realtime=False, results=results)
    assert rep.summary()["completed"] == len(trace)
    for r in g["requests"]:
        m = results[r["rid"]]
        idx = torch.tensor(r["particles"], device="cuda", dtype=torch.long)
        x = to_np(m["pos"][idx]).astype(np.float64)
        p = to_np(m["mom"][idx]).astype(np.float64)
        d = opm.min_image(x - np.array(r["x"]), r["n_mesh"])
        rms = float(np.sqrt((d ** 2).sum(1).mean()))
        rp = rel(p, np.array(r["p"]))
        banner(f"  request {r['rid']} ({r['n_part']}^3 / {r['n_mesh']}^3): positions rms {rms:.2e} cells, "
               f"momenta rel {rp:.2e}")
        record(f"serve_class_{r['n_part']}_{r['n_mesh']}_pos_rms_cells", rms, 1e-3)
        record(f"serve_class_{r['n_part']}_{r['n_mesh']}_mom_rel", rp, 1e-2)
        assert rms < 1e-3
        assert rp < 1e-2


def test_tiny_budget_and_oversize_rejection(gpu):
    banner("serve tiny budget")
    ex = serve.BatchedExecutor(slots_per_class=2, keep_results=False)
    trace = [serve.SimRequest(i, 16, 64, 32.0, 3, 1000 + i, False, 0.0) for i in range(4)]
    big = serve.SimRequest(99, 64, 128, 128.0, 3, 7, False, 0.0)
    budget = ex.plan_bytes(trace[0].shape_class) + ex.request_bytes(trace[0])
    rep = serve.serve(trace + [big], ex, budget_bytes=budget, slots_per_class=2, realtime=False)
    ok = [c for c in rep.completions if c.ok]
    assert len(ok) == 4 and rep.max_active == 1 and rep.max_used <= budget
    bad = [c for c in rep.completions if c.rid == 99][0]
    assert not bad.ok and "exceeds the HBM budget" in bad.error


@pytest.mark.gpu
def test_graph_step_loop_equals_eager(gpu):
    """One captured graph per step, replayed over the run, with eager work on
    the same stream between replays: every replay's result equals the eager
    loop's bit for bit, with and without checkpoints, run after run."""
    import torch
    from dataclasses import replace
    from paper_2010_11847_amd import inputs
    from paper_2010_11847_amd.binding import PMContext
    w = inputs.scaled(inputs.MEDIUM, 64, 32, n_steps=6)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        eager = PMContext(w, stream=s)
        graph = PMContext(w, stream=s)
        graph.pm_use_graphs(True)
        n = w.n_part ** 3
        for rep, with_ckpt in enumerate((False, True, True)):
            pos0, mom0 = eager.pm_init_lpt(w.seed + rep, w.a_list[0])
            outs = []
            for c in (eager, graph):
                pos, mom = pos0.clone(), mom0.clone()
                ck = torch.empty((len(w.a_list), 2, n, 3), device="cuda") if with_ckpt else None
                d = torch.empty((64, 64, 64), device="cuda")
                c.pm_run_begin(w.a_list, pos, mom, ckpt=ck)
                while c.pm_run_advance(1) > 0:
                    torch.zeros(1000, device="cuda").add_(1.0)   # eager work between replays
                c.pm_run_end(delta_final=d)
                outs.append((pos, mom, ck, d))
            torch.cuda.synchronize()
            for a, b in zip(outs[0], outs[1]):
                if a is not None:
                    assert torch.equal(a, b)
