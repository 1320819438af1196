"""Hand-written GPU adjoint against the FP64 oracle.

* Implementation parity: the oracle differentiates along the GPU's own
  checkpointed (float32) trajectory, so both sides evaluate every operator
  at the same points; bound 1e-4 (norm-wise).
* Independent trajectories and finite differences: the CIC weights have
  kinks at cell faces, so a float32 and a float64 trajectory can put a few
  particles on different sides of a face and their derivatives legitimately
  differ there; these comparisons carry that sensitivity.
"""
import json
import os

import numpy as np
import pytest
import torch

from oracle import adjoint as A
from oracle import lpt, pm
from oracle.rng import white_noise
from paper_2010_11847_amd import inputs
from tests.gpu_helpers import banner, rel, to_dev, to_np

pytestmark = pytest.mark.gpu
SIGMA = 0.1
METRICS = {}


def setup(w):
    noise = white_noise(w.seed, w.n_part)
    xt, _, _ = pm.kdk_run(*lpt.generate(w, noise=white_noise(w.seed + 1000, w.n_part)), w.a_list, w.n_mesh,
                          w.n_particles, w.cosmo.omega_m)
    target = pm.density_contrast(xt, w.n_mesh, w.n_particles)
    target = target + np.random.default_rng(w.seed + 2000).normal(0.0, SIGMA, target.shape)
    return noise, target


def gpu_run_and_grad(w, noise, target):
    from paper_2010_11847_amd.binding import PMContext
    c = PMContext(w)
    z = to_dev(noise.astype(np.float32))
    pos, mom = c.pm_init_lpt(0, w.a_list[0], noise=z)
    ckpt = torch.empty((len(w.a_list), 2, w.n_particles, 3), device="cuda")
    delta = torch.empty((w.n_mesh,) * 3, device="cuda")
    c.pm_run(w.a_list, pos, mom, ckpt=ckpt, delta_final=delta)
    t = to_dev(target.astype(np.float32))
    gdelta = (2.0 / SIGMA ** 2) * (delta - t)
    _, _, gn = c.pm_run_adjoint(w.a_list, ckpt, noise=z, grad_delta=gdelta)
    return to_np(ckpt).astype(np.float64), to_np(gn)


def record(name, value):
    """Keep a measured error; written to $PM_METRICS_DIR/adjoint_metrics.json when set."""
    METRICS[name] = value
    out = os.environ.get("PM_METRICS_DIR")
    if out:
        os.makedirs(out, exist_ok=True)
        with open(os.path.join(out, "adjoint_metrics.json"), "w") as fh:
            json.dump(METRICS, fh, indent=1)


@pytest.mark.parametrize("n_mesh,n_part,steps", [(32, 16, 3), (64, 32, 5), (128, 64, 5)])
def test_adjoint_matches_oracle_on_same_trajectory(gpu, n_mesh, n_part, steps):
    banner(f"adjoint same-trajectory n={n_mesh} np={n_part} steps={steps}")
    w = inputs.scaled(inputs.ADJ_SMALL, n_mesh, n_part, n_steps=steps)
    noise, target = setup(w)
    ck, g_g = gpu_run_and_grad(w, noise, target)
    xs = [ck[i, 0] for i in range(len(w.a_list))]
    g_o = A.grad_along_trajectory(xs, noise, w, target, SIGMA)
    r = rel(g_g, g_o)
    record(f"same_traj_{n_mesh}_{n_part}_{steps}", r)
    assert r < 1e-4


@pytest.mark.parametrize("opts", [{"deconv_order": 2}, {"split_mode": 1, "split_rs": 2.0},
                                  {"split_mode": 2, "split_rs": 2.0}])
def test_adjoint_with_force_filters_on_same_trajectory(gpu, opts):
    # the deconvolution and split filters are real and even in k, so the
    # transposed force applies them unchanged
    banner(f"adjoint same-trajectory with {opts}")
    w = inputs.scaled(inputs.ADJ_SMALL, 64, 32, n_steps=3, **opts)
    noise, target = setup(w)
    ck, g_g = gpu_run_and_grad(w, noise, target)
    xs = [ck[i, 0] for i in range(len(w.a_list))]
    g_o = A.grad_along_trajectory(xs, noise, w, target, SIGMA, **opts)
    r = rel(g_g, g_o)
    record("same_traj_filters_" + "_".join(f"{k}{v}" for k, v in opts.items()), r)
    assert r < 1e-4


def test_autograd_function_matches_direct_call(gpu):
    banner("autograd")
    from paper_2010_11847_amd.autograd import simulate
    from paper_2010_11847_amd.binding import PMContext
    w = inputs.scaled(inputs.ADJ_SMALL, 32, 16, n_steps=3)
    noise, target = setup(w)
    c = PMContext(w)
    z = to_dev(noise.astype(np.float32)).requires_grad_(True)
    delta = simulate(z, c, w.a_list)
    loss = (((delta - to_dev(target.astype(np.float32))) / SIGMA) ** 2).sum()
    loss.backward()
    _, g_direct = gpu_run_and_grad(w, noise, target)
    assert rel(to_np(z.grad), g_direct) < 1e-5


@pytest.mark.parametrize("n_mesh,n_part,steps", [(32, 16, 3), (128, 64, 5)])
def test_adjoint_vs_independent_fp64_run(gpu, n_mesh, n_part, steps):
    banner(f"adjoint independent n={n_mesh}")
    w = inputs.scaled(inputs.ADJ_SMALL, n_mesh, n_part, n_steps=steps)
    noise, target = setup(w)
    _, g_o = A.loss_and_grad(noise, w, target, SIGMA)
    _, g_g = gpu_run_and_grad(w, noise, target)
    r = rel(g_g, g_o)
    record(f"independent_{n_mesh}_{n_part}_{steps}", r)
    assert r < 1e-2


def test_adjoint_vs_central_fd(gpu):
    banner("adjoint vs FD")
    w = inputs.scaled(inputs.ADJ_SMALL, 32, 16, n_steps=5)
    noise, target = setup(w)
    _, g_g = gpu_run_and_grad(w, noise, target)
    cells = inputs.sample_indices(noise.size, 32, seed=3)
    flat = noise.reshape(-1)
    refs = []
    for c in cells:
        def f(e):
            z = flat.copy()
            z[c] += e
            return A.forward_loss(z.reshape(noise.shape), w, target, SIGMA)[0]
        h = 1e-4
        d1 = (f(h) - f(-h)) / (2 * h)
        d2 = (f(h / 2) - f(-h / 2)) / h
        refs.append((4 * d2 - d1) / 3)
    refs = np.array(refs)
    got = g_g.reshape(-1)[cells]
    scale = np.sqrt(np.mean(g_g ** 2))
    err = float(np.abs(got - refs).max() / scale)
    record("fd_max_rel_to_rms", err)
    record("fd_rel_norm", rel(got, refs))
    assert rel(got, refs) < 1e-3


def test_adjoint_with_force_checkpoints_is_identical(gpu):
    """Reading the forward's force meshes instead of recomputing them changes
    nothing: paint and FFTs are deterministic, so the gradients are equal bit
    for bit."""
    from paper_2010_11847_amd.binding import PMContext
    banner("adjoint with force checkpoints 64/32 5 steps")
    w = inputs.scaled(inputs.ADJ_SMALL, 64, 32, n_steps=5)
    c = PMContext(w)
    noise = to_dev(white_noise(w.seed, 32))
    gd = to_dev(np.random.default_rng(3).normal(size=(64, 64, 64)))
    outs = []
    for fck in (False, True):
        c.pm_set_force_ckpt(len(w.a_list) if fck else 0)
        pos, mom = c.pm_init_lpt(0, w.a_list[0], noise=noise)
        ck = torch.empty((len(w.a_list), 2, 32 ** 3, 3), device="cuda")
        c.pm_run(w.a_list, pos, mom, ckpt=ck)
        gx, gp, gn = c.pm_run_adjoint(w.a_list, ck, noise=noise, grad_delta=gd)
        outs.append((pos, mom, gx, gp, gn))
    c.pm_set_force_ckpt(0)
    for a, b in zip(*outs):
        assert torch.equal(a, b)
