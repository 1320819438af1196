"""Element-wise parity at the full sizes, against stored FP64 oracle values.

The oracle cannot run these sizes inside a test, so tests/golden/make_golden.py
(oracle only) stored its outputs at sampled cells and particles; the inputs
are drawn here again from the same seeded generators.  Bars are norm-wise
over the sample: 1e-5 for the painted overdensity and the force (the
per-step bar), 1e-4 for adjoint cotangents and noise gradients.

* 512^3 particles on the 1024^3 mesh: overdensity at 4096 cells and the PM
  force at 1024 particles, for a perturbed lattice (the 2LPT start's
  displacement scale) and a clustered set (heavy tiles).  This covers the
  1024^3 instantiations of every force kernel.
* One reverse KDK step on a 512^3 mesh: the transposed force at that size.
* The 5-step reverse sweep at 128^3 particles / 256^3 mesh (the larger
  differentiable configuration), down to the white-noise gradient.
* The gradient of the 64^3 / 128^3 chi^2 run at 32 seeded cells: along the
  oracle's trajectory against the oracle, and end to end against central
  finite differences of the FP64 oracle.
"""
import json
import os

import numpy as np
import pytest
import torch

from tests.golden import make_golden as G
from oracle.rng import white_noise
from paper_2010_11847_amd import inputs
from tests.gpu_helpers import banner, record, rel, to_dev, to_np

pytestmark = pytest.mark.gpu
HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load(name):
    path = os.path.join(HERE, name + ".json")
    if not os.path.exists(path):
        pytest.skip(f"golden file {name}.json not generated")
    with open(path) as fh:
        return json.load(fh)


@pytest.fixture(scope="module")
def large_ctx(gpu):
    from paper_2010_11847_amd.binding import PMContext
    c = PMContext(inputs.LARGE)
    yield c
    c.close()
    torch.cuda.empty_cache()


@pytest.mark.parametrize("name", list(G.FORCE_SETS))
def test_force_and_paint_at_1024_match_golden(large_ctx, name):
    g = load("force_pm512_mesh1024")["sets"][name]
    banner(f"paint + force 512^3 / 1024^3, {name} positions")
    x = to_dev(G.force_positions(name))
    delta = large_ctx.pm_paint(x)
    cells = torch.tensor(g["cells"], device="cuda", dtype=torch.long)
    d_s = to_np(delta.reshape(-1)[cells]).astype(np.float64)
    del delta
    r_d = rel(d_s, np.array(g["delta"]))
    f = large_ctx.pm_force(x)
    parts = torch.tensor(g["particles"], device="cuda", dtype=torch.long)
    f_s = to_np(f[parts]).astype(np.float64)
    ref = np.array(g["force"])
    r_f = rel(f_s, ref)
    r_max = float(np.abs(f_s - ref).max() / np.sqrt(np.mean(ref ** 2)))
    banner(f"  delta rel {r_d:.2e}, force rel {r_f:.2e} (max element / rms {r_max:.2e})")
    record(f"fullsize_{name}_delta_rel", r_d, 1e-5)
    record(f"fullsize_{name}_force_rel", r_f, 1e-5)
    record(f"fullsize_{name}_force_max_over_rms", r_max)
    assert r_d < 1e-5
    assert r_f < 1e-5


def test_adjoint_step_on_512_mesh_matches_golden(gpu):
    from paper_2010_11847_amd.binding import PMContext
    g = load("adjoint_step_mesh512")
    c = G.ADJ512
    banner("reverse KDK step, 256^3 particles on a 512^3 mesh")
    w = inputs.scaled(inputs.ADJ_SMALL, c["n_mesh"], c["n_part"], n_steps=1)
    ctx = PMContext(w)
    x0, x1, pbar = G.adj512_inputs()
    n = c["n_part"] ** 3
    ck = torch.zeros((2, 2, n, 3), device="cuda")
    ck[0, 0] = to_dev(x0)
    ck[1, 0] = to_dev(x1)
    gx, gp, _ = ctx.pm_run_adjoint(list(c["a"]), ck, grad_mom=to_dev(pbar), want_noise_grad=False)
    parts = torch.tensor(g["particles"], device="cuda", dtype=torch.long)
    rx = rel(to_np(gx[parts]), np.array(g["x0_bar"]))
    rp = rel(to_np(gp[parts]), np.array(g["p0_bar"]))
    banner(f"  x0_bar rel {rx:.2e}, p0_bar rel {rp:.2e}")
    record("adjoint_step_mesh512_x0bar_rel", rx, 1e-4)
    record("adjoint_step_mesh512_p0bar_rel", rp, 1e-4)
    ctx.close()
    assert rx < 1e-4 and rp < 1e-4


def test_adjoint_sweep_128_on_256_matches_golden(gpu):
    from paper_2010_11847_amd.binding import PMContext
    g = load("adjoint_adj128_mesh256")
    w = G.c4b_workload()
    banner(f"reverse sweep {w.name} ({w.n_steps} steps) along a seeded trajectory")
    xs, noise, dbar = G.c4b_inputs(w)
    ctx = PMContext(w)
    ck = torch.zeros((len(w.a_list), 2, w.n_particles, 3), device="cuda")
    for i, x in enumerate(xs):
        ck[i, 0] = to_dev(x)
    gx, gp, gn = ctx.pm_run_adjoint(w.a_list, ck, noise=to_dev(noise), grad_delta=to_dev(dbar))
    parts = torch.tensor(g["particles"], device="cuda", dtype=torch.long)
    cells = torch.tensor(g["cells"], device="cuda", dtype=torch.long)
    rx = rel(to_np(gx[parts]), np.array(g["x0_bar"]))
    rp = rel(to_np(gp[parts]), np.array(g["p0_bar"]))
    rn = rel(to_np(gn.reshape(-1)[cells]), np.array(g["grad_noise"]))
    banner(f"  x0_bar rel {rx:.2e}, p0_bar rel {rp:.2e}, noise gradient rel {rn:.2e}")
    record("adjoint_c4b_x0bar_rel", rx, 1e-4)
    record("adjoint_c4b_p0bar_rel", rp, 1e-4)
    record("adjoint_c4b_grad_noise_rel", rn, 1e-4)
    ctx.close()
    assert rx < 1e-4 and rp < 1e-4 and rn < 1e-4


def test_adjoint_of_64_on_128_run_vs_fd_golden(gpu):
    """The GPU adjoint of the chi^2 loss of the 64^3 / 128^3 5-step run at 32
    seeded white-noise cells, scaled by the rms over all cells of the
    oracle's gradient.

    (1) Along the oracle's trajectory rounded to float32 (only the adjoint
    runs on the GPU): equal to the oracle's gradient along that same rounded
    trajectory (stored), max |g - g_o| / rms <= 1e-5.
    (2) End to end (the GPU's float32 forward run and its adjoint) against
    Richardson-extrapolated central differences of the FP64 oracle: within
    2e-3.  The oracle's own adjoint along its FP64 trajectory meets those
    differences to 3.1e-5 (pinned on the CPU), but a float32 state moves
    positions by up to 8e-6 cells, enough to put a few particles on the
    other side of a CIC kink, and the oracle's own gradient along its
    float32-rounded trajectory is already 4.9e-4 from the differences at
    one of the cells; the GPU's float32 trajectory carries the same
    sensitivity."""
    from oracle import adjoint as A
    from oracle import lpt as olpt
    from paper_2010_11847_amd.binding import PMContext
    g = load("fd_adj64_mesh128_box200")
    gt = load("grad_f32traj_adj64_mesh128_box200")
    w = inputs.ADJ_SMALL
    banner(f"adjoint vs FD golden, {w.name}")
    sigma = g["sigma"]
    noise = white_noise(w.seed, w.n_part)
    target = G.chi2_target(w, sigma)
    cells = np.array(g["cells"])
    assert cells.tolist() == gt["cells"]
    fd = np.array(g["fd"])
    c = PMContext(w)
    z = to_dev(noise.astype(np.float32))
    # (1) the oracle's trajectory rounded to float32, the GPU's adjoint
    x0, p0 = olpt.generate(w, noise=noise)
    xs, _, _ = A.run_forward_trajectory(x0, p0, w.a_list, w.n_mesh, w.n_particles, w.cosmo.omega_m)
    ck = torch.zeros((len(w.a_list), 2, w.n_particles, 3), device="cuda")
    for i, x in enumerate(xs):
        ck[i, 0] = to_dev(x)
    delta = c.pm_paint(ck[-1, 0])
    _, gdelta = c.pm_chi2(delta, to_dev(target.astype(np.float32)), sigma)
    _, _, gn = c.pm_run_adjoint(w.a_list, ck, noise=z, grad_delta=gdelta)
    got = to_np(gn).reshape(-1)[cells].astype(np.float64)
    err1 = float(np.abs(got - np.array(gt["grad"])).max() / gt["grad_rms"])
    # (2) end to end on the GPU
    pos, mom = c.pm_init_lpt(0, w.a_list[0], noise=z)
    ckpt = torch.empty((len(w.a_list), 2, w.n_particles, 3), device="cuda")
    d_gpu = torch.empty((w.n_mesh,) * 3, device="cuda")
    c.pm_run(w.a_list, pos, mom, ckpt=ckpt, delta_final=d_gpu)
    _, gd_gpu = c.pm_chi2(d_gpu, to_dev(target.astype(np.float32)), sigma)
    _, _, gn2 = c.pm_run_adjoint(w.a_list, ckpt, noise=z, grad_delta=gd_gpu)
    got2 = to_np(gn2).reshape(-1)[cells].astype(np.float64)
    err2 = float(np.abs(got2 - fd).max() / g["grad_rms"])
    err_traj_fd = float(np.abs(got - fd).max() / g["grad_rms"])
    banner(f"  along the float32-rounded oracle trajectory vs the oracle there: max / rms {err1:.2e}; "
           f"that gradient vs fd {err_traj_fd:.2e}; end to end vs fd {err2:.2e} (rel norm {rel(got2, fd):.2e}); "
           f"oracle (FP64 trajectory) vs fd {g['oracle_adjoint_vs_fd_max_rel_to_rms']:.2e}")
    record("fd_c4a_gpu_vs_oracle_f32_trajectory_max_over_rms", err1, 1e-5)
    record("fd_c4a_f32_trajectory_vs_fd_max_over_rms", err_traj_fd)
    record("fd_c4a_end_to_end_max_over_rms", err2, 2e-3)
    record("fd_c4a_end_to_end_rel_norm", rel(got2, fd))
    c.close()
    assert err1 < 1e-5
    assert err2 < 2e-3
