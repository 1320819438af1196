"""Batched steps of same-shape simulations (continuous batching) against
runs on contexts of their own and against the oracle.

Members join a plan while others are mid-run and leave when done; each
member's final positions, momenta and overdensity must equal, bit for bit,
the same run on a context of its own (the same kernels, and the paint sums
integers, so the result does not depend on the order of the sort), and the
oracle's run from the same float32 start within the run bar (rms < 1e-3
cell).  Covered: eager and graph-captured batched steps, the raw
descriptor-table entry point, checkpoints and the adjoint of a member.
"""
import ctypes as C

import numpy as np
import pytest
import torch

from oracle import lpt, pm
from paper_2010_11847_amd import inputs
from paper_2010_11847_amd.inputs import Workload, a_linear
from tests.gpu_helpers import banner, record, to_dev, to_np

pytestmark = pytest.mark.gpu


def shape(n_steps=5, seed=0):
    # 32^3 particles on a 64^3 mesh, 128 Mpc/h, no-wiggle P(k)
    return Workload(f"b{seed}", 128.0, 64, 32, seed, a_linear(0.1, 1.0, n_steps))


# (member slot, seed, steps, tick at which it joins)
SCHEDULE = [(0, 1000, 5, 0), (2, 1001, 7, 2), (1, 1002, 6, 3), (0, 1003, 4, 6)]


def standalone(w, ckpt=False):
    from paper_2010_11847_amd.binding import PMContext
    c = PMContext(w)
    pos, mom = c.pm_init_lpt(w.seed, w.a_list[0])
    ck = torch.zeros((len(w.a_list), 2, w.n_particles, 3), device="cuda") if ckpt else None
    delta = torch.empty((w.n_mesh,) * 3, device="cuda")
    c.pm_run(w.a_list, pos, mom, ckpt=ck, delta_final=delta)
    out = (to_np(pos), to_np(mom), to_np(delta), None if ck is None else to_np(ck))
    c.close()
    return out


def run_schedule(graphs, stream):
    """Drive a 3-slot plan through SCHEDULE; returns {seed: (pos, mom, delta)}."""
    from paper_2010_11847_amd.binding import PMBatch
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        plan = PMBatch(shape(), 3, stream=stream)
        if graphs:
            plan.pm_use_graphs(True)
        pending = list(SCHEDULE)
        live = {}
        done = {}
        tick = 0
        while pending or live:
            for item in [p for p in pending if p[3] <= tick and p[0] not in live]:
                m, seed, steps, _ = item
                pending.remove(item)
                w = shape(steps, seed)
                mc = plan.member(m)
                pos, mom = mc.pm_init_lpt(seed, w.a_list[0])
                plan.pm_batch_begin(m, w.a_list, pos, mom)
                live[m] = (seed, w, pos, mom)
            plan.pm_batch_advance()
            for m in list(live):
                if plan.pm_batch_remaining(m) == 0:
                    seed, w, pos, mom = live.pop(m)
                    delta = torch.empty((w.n_mesh,) * 3, device="cuda")
                    plan.pm_batch_end(m, delta_final=delta)
                    done[seed] = (pos, mom, delta)
            tick += 1
        stream.synchronize()
        out = {k: tuple(to_np(t) for t in v) for k, v in done.items()}
        plan.close()
    return out


@pytest.mark.parametrize("graphs", [False, True])
def test_batched_members_equal_their_own_runs(gpu, graphs):
    banner(f"batch plan, 3 slots, 4 requests joining mid-run, graphs={graphs}")
    stream = torch.cuda.Stream()
    got = run_schedule(graphs, stream)
    assert sorted(got) == sorted(s for _, s, _, _ in SCHEDULE)
    for _, seed, steps, _ in SCHEDULE:
        ref = standalone(shape(steps, seed))
        for name, a, b in zip(("pos", "mom", "delta"), got[seed], ref[:3]):
            assert np.array_equal(a, b), (seed, name, float(np.abs(a - b).max()))


def test_batched_member_matches_the_oracle(gpu):
    """One member, started from the oracle's 2LPT state rounded to float32,
    stepped in a plan beside a second member, against the oracle's run."""
    from paper_2010_11847_amd.binding import PMBatch
    w = shape(6, 7)
    x0, p0 = (np.asarray(v, dtype=np.float32) for v in lpt.generate(w))
    plan = PMBatch(w, 2)
    pos, mom = to_dev(x0), to_dev(p0)
    other = shape(8, 8)
    opos, omom = plan.member(1).pm_init_lpt(other.seed, other.a_list[0])
    plan.pm_batch_begin(1, other.a_list, opos, omom)
    plan.pm_batch_advance()
    plan.pm_batch_begin(0, w.a_list, pos, mom)
    while plan.pm_batch_remaining(0) > 0:
        plan.pm_batch_advance()
    plan.pm_batch_end(0)
    gx = to_np(pos).astype(np.float64)
    ox, op_, _ = pm.kdk_run(x0.astype(np.float64), p0.astype(np.float64), w.a_list, w.n_mesh, w.n_particles,
                            w.cosmo.omega_m)
    d = pm.min_image(gx - ox, w.n_mesh)
    rms = float(np.sqrt((d ** 2).sum(1).mean()))
    rp = float(np.linalg.norm(to_np(mom) - op_) / np.linalg.norm(op_))
    banner(f"  batched member vs oracle: position rms {rms:.2e} cells, momentum rel {rp:.2e}")
    record("batch_member_vs_oracle_pos_rms", rms, 1e-3)
    record("batch_member_vs_oracle_mom_rel", rp, 1e-4)
    plan.close()
    assert rms < 1e-3
    assert rp < 1e-4


def test_raw_descriptor_steps_and_member_adjoint(gpu):
    """pm_kdk_step_batched over a caller's descriptor table (with
    checkpoints) equals pm_run on a context of its own, checkpoints
    included, and the member's adjoint equals the standalone adjoint."""
    from paper_2010_11847_amd import _lib
    from paper_2010_11847_amd.binding import PMBatch, PMContext, req_descs
    w = shape(5, 21)
    plan = PMBatch(w, 2)
    mc = plan.member(1)
    noise = mc.pm_noise(w.seed)
    pos, mom = mc.pm_init_lpt(w.seed, w.a_list[0], noise=noise)
    ck = torch.zeros((len(w.a_list), 2, w.n_particles, 3), device="cuda")
    plan.pm_batch_begin(1, w.a_list, pos, mom, ckpt=ck)
    k1, dr, k2 = plan.pm_kdk_factors(w.a_list)
    n3 = w.n_particles
    descs = torch.empty(2 * C.sizeof(_lib.pm_req_desc), dtype=torch.uint8, device="cuda")
    for i in range(w.n_steps):
        cx = ck[i, 0].data_ptr()
        cp = ck[i, 1].data_ptr()
        host = req_descs([(-1, 0, 0.0, 0.0, 0.0, None, None),
                          (1, _lib.PM_REQ_CKPT, k2[i - 1] if i else 0.0, k1[i], dr[i], cx, cp)])
        descs.copy_(torch.frombuffer(bytearray(host), dtype=torch.uint8))
        plan.pm_kdk_step_batched(descs, 2)
    delta = torch.empty((w.n_mesh,) * 3, device="cuda")
    plan.pm_batch_end(1, delta_final=delta, check_steps=False)
    ref_pos, ref_mom, ref_delta, ref_ck = standalone(w, ckpt=True)
    assert np.array_equal(to_np(pos), ref_pos)
    assert np.array_equal(to_np(mom), ref_mom)
    assert np.array_equal(to_np(delta), ref_delta)
    assert np.array_equal(to_np(ck), ref_ck)
    # adjoint on the member's slot against a context of its own
    g = torch.from_numpy(inputs.normal_array((w.n_mesh,) * 3, seed=5)).cuda()
    _, _, gn = mc.pm_run_adjoint(w.a_list, ck, noise=noise, grad_delta=g)
    c = PMContext(w)
    _, _, gn_ref = c.pm_run_adjoint(w.a_list, ck, noise=noise, grad_delta=g)
    assert np.array_equal(to_np(gn), to_np(gn_ref))
    c.close()
    plan.close()


def test_batch_plan_errors(gpu):
    from paper_2010_11847_amd import _lib
    from paper_2010_11847_amd.binding import PMBatch, PMContext, PMError
    w = shape(3, 1)
    plan = PMBatch(w, 2)
    lib = plan.lib
    h = C.c_void_p()
    assert lib.pm_batch_member(plan.ctx, 2, C.byref(h)) == _lib.PM_EINVAL
    assert lib.pm_batch_remaining(plan.ctx, 0) == _lib.PM_ESTATE      # not running
    assert lib.pm_batch_end(plan.ctx, 0, None) == _lib.PM_ESTATE
    assert lib.pm_destroy(plan.member(1).ctx) == _lib.PM_EINVAL      # owned by the plan
    k = C.c_int(-1)
    assert lib.pm_batch_advance(plan.ctx, C.byref(k)) == _lib.PM_OK and k.value == 0
    single = PMContext(w)
    assert lib.pm_kdk_step_batched(single.ctx, C.c_void_p(plan.ws.data_ptr()), 1) == _lib.PM_EINVAL
    pos, mom = plan.member(0).pm_init_lpt(1, w.a_list[0])
    plan.pm_batch_begin(0, w.a_list, pos, mom)
    with pytest.raises(PMError):
        plan.pm_batch_begin(0, w.a_list, pos, mom)   # already running
    with pytest.raises(PMError):
        plan.pm_batch_end(0)                         # steps left
    single.close()
    plan.close()
