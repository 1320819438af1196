"""Hand-written GPU adjoint against the FP64 oracle.

* Implementation parity: both adjoints sweep back over the same trajectory,
  the oracle's own FP64 run rounded to float32 (the GPU reads it as its
  checkpoints), so both evaluate every operator at the same points; bound
  1e-4 (norm-wise).  The larger sizes (128^3 particles on 256^3, a 512^3
  mesh) are compared against stored oracle values in test_gpu_fullsize.py.
* Independent trajectories and finite differences: the CIC weights have
  kinks at cell faces, so a float32 and a float64 trajectory can put a few
  particles on different sides of a face and their derivatives legitimately
  differ there; these comparisons carry that sensitivity.
"""
import numpy as np
import pytest
import torch

from oracle import adjoint as A
from oracle import lpt, pm
from oracle.rng import white_noise
from paper_2010_11847_amd import inputs
from tests.gpu_helpers import banner, f32, record, rel, to_dev, to_np

pytestmark = pytest.mark.gpu
SIGMA = 0.1


def setup(w):
    noise = white_noise(w.seed, w.n_part)
    xt, _, _ = pm.kdk_run(*lpt.generate(w, noise=white_noise(w.seed + 1000, w.n_part)), w.a_list, w.n_mesh,
                          w.n_particles, w.cosmo.omega_m)
    target = pm.density_contrast(xt, w.n_mesh, w.n_particles)
    target = target + np.random.default_rng(w.seed + 2000).normal(0.0, SIGMA, target.shape)
    return noise, target


def gpu_run_and_grad(w, noise, target):
    """The GPU's own forward run (with checkpoints) and adjoint."""
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
    return to_np(gn)


def oracle_trajectory(w, noise, **kw):
    """Positions at every scale factor of the oracle's FP64 run from the
    noise, rounded to float32."""
    x0, p0 = lpt.generate(w, noise=noise)
    xs, _, _ = A.run_forward_trajectory(x0, p0, w.a_list, w.n_mesh, w.n_particles, w.cosmo.omega_m, **kw)
    return [f32(x) for x in xs]


def gpu_grad_along(w, xs, noise, target):
    """The GPU adjoint swept back over the given trajectory (its checkpoints;
    the adjoint reads only their positions), for the chi^2 loss of the
    density painted from the last positions."""
    from paper_2010_11847_amd.binding import PMContext
    c = PMContext(w)
    z = to_dev(noise.astype(np.float32))
    ck = torch.zeros((len(xs), 2, w.n_particles, 3), device="cuda")
    for i, x in enumerate(xs):
        ck[i, 0] = to_dev(x)
    delta = c.pm_paint(ck[-1, 0])
    _, gdelta = c.pm_chi2(delta, to_dev(target.astype(np.float32)), SIGMA)
    _, _, gn = c.pm_run_adjoint(w.a_list, ck, noise=z, grad_delta=gdelta)
    return to_np(gn)


@pytest.mark.parametrize("n_mesh,n_part,steps", [(32, 16, 3), (64, 32, 5), (128, 64, 5)])
def test_adjoint_matches_oracle_on_same_trajectory(gpu, n_mesh, n_part, steps):
    # 128 / 64 / 5 steps is the 64^3-on-128^3 differentiable configuration
    banner(f"adjoint same-trajectory n={n_mesh} np={n_part} steps={steps}")
    w = inputs.scaled(inputs.ADJ_SMALL, n_mesh, n_part, n_steps=steps)
    noise, target = setup(w)
    xs = oracle_trajectory(w, noise)
    g_g = gpu_grad_along(w, xs, noise, target)
    g_o = A.grad_along_trajectory(xs, noise, w, target, SIGMA)
    r = rel(g_g, g_o)
    banner(f"  rel {r:.2e}")
    record(f"adjoint_same_traj_{n_mesh}_{n_part}_{steps}", r, 1e-4)
    assert r < 1e-4


@pytest.mark.parametrize("opts", [{"deconv_order": 2}, {"split_mode": 1, "split_rs": 2.0},
                                  {"split_mode": 2, "split_rs": 2.0}])
def test_adjoint_with_force_filters_on_same_trajectory(gpu, opts):
    # the deconvolution and split filters are real and even in k, so the
    # transposed force applies them unchanged
    banner(f"adjoint same-trajectory with {opts}")
    w = inputs.scaled(inputs.ADJ_SMALL, 64, 32, n_steps=3, **opts)
    noise, target = setup(w)
    xs = oracle_trajectory(w, noise, **opts)
    g_g = gpu_grad_along(w, xs, noise, target)
    g_o = A.grad_along_trajectory(xs, noise, w, target, SIGMA, **opts)
    r = rel(g_g, g_o)
    record("adjoint_same_traj_filters_" + "_".join(f"{k}{v}" for k, v in opts.items()), r, 1e-4)
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
    g_direct = gpu_run_and_grad(w, noise, target)
    assert rel(to_np(z.grad), g_direct) < 1e-5


@pytest.mark.parametrize("n_mesh,n_part,steps", [(32, 16, 3), (128, 64, 5)])
def test_adjoint_vs_independent_fp64_run(gpu, n_mesh, n_part, steps):
    banner(f"adjoint independent n={n_mesh}")
    w = inputs.scaled(inputs.ADJ_SMALL, n_mesh, n_part, n_steps=steps)
    noise, target = setup(w)
    _, g_o = A.loss_and_grad(noise, w, target, SIGMA)
    g_g = gpu_run_and_grad(w, noise, target)
    r = rel(g_g, g_o)
    record(f"independent_{n_mesh}_{n_part}_{steps}", r, 1e-2)
    assert r < 1e-2


def test_adjoint_vs_central_fd(gpu):
    """GPU gradient (its own float32 run) against Richardson-extrapolated
    central differences of the FP64 oracle's forward run at 32 cells."""
    banner("adjoint vs FD")
    w = inputs.scaled(inputs.ADJ_SMALL, 32, 16, n_steps=5)
    noise, target = setup(w)
    g_g = gpu_run_and_grad(w, noise, target)
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
    record("fd_16_32_max_over_rms", err, 1e-4)
    record("fd_16_32_rel_norm", rel(got, refs), 1e-4)
    assert err < 1e-4
    assert rel(got, refs) < 1e-4


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
