"""Pins for oracle.adjoint: every transpose against finite differences of the
forward oracle (directional derivatives in float64) and dot-product identities."""
from dataclasses import replace

import numpy as np
import pytest

from oracle import adjoint as A
from oracle import lpt, pm
from oracle.rng import white_noise
from paper_2010_11847_amd import inputs

OM = 0.3


def fd(f, x, v, eps):
    return (f(x + eps * v) - f(x - eps * v)) / (2 * eps)


def test_readout_position_grad_matches_fd():
    rng = np.random.default_rng(1)
    g = rng.normal(size=(8, 8, 8))
    x = inputs.uniform_positions(50, 8, seed=1).astype(np.float64)
    v = rng.normal(size=x.shape)
    lhs = np.sum(A.readout_position_grad(g, x) * v)
    rhs = np.sum(fd(lambda y: pm.readout(g, y), x, v, 1e-7))
    assert lhs == pytest.approx(rhs, rel=1e-6)


def test_multiplier_transpose_dot_product():
    n = 12
    rng = np.random.default_rng(2)
    u, w = rng.normal(size=(n, n, n)), rng.normal(size=(n, n, n))
    for m in pm.force_multipliers(n, OM, deconv_order=1):
        lhs = np.vdot(A.apply_multiplier(u, m), w)
        rhs = np.vdot(u, A.apply_multiplier(w, np.conj(m)))
        assert lhs == pytest.approx(rhs, rel=1e-12)
        # the FD force kernel is antisymmetric
        np.testing.assert_allclose(A.apply_multiplier(w, np.conj(m)), -A.apply_multiplier(w, m), atol=1e-12)


@pytest.mark.parametrize("opts", [{}, {"deconv_order": 2}, {"split_mode": 1, "split_rs": 1.5},
                                  {"split_mode": 2, "split_rs": 1.5}])
def test_force_vjp_matches_fd(opts):
    n = 16
    x = inputs.clustered_positions(300, n, seed=3).astype(np.float64)
    rng = np.random.default_rng(3)
    fb = rng.normal(size=x.shape)
    v = rng.normal(size=x.shape)
    lhs = np.sum(A.force_vjp(x, n, 300, OM, fb, **opts) * v)
    rhs = np.sum(fb * fd(lambda y: pm.force(y, n, 300, OM, **opts), x, v, 1e-7))
    assert lhs == pytest.approx(rhs, rel=1e-5)


def test_lpt_vjp_matches_fd():
    w = replace(inputs.scaled(inputs.MEDIUM, 16, 8), lpt_order=2)
    noise = white_noise(4, 8)
    rng = np.random.default_rng(4)
    xb, pb = rng.normal(size=(512, 3)), rng.normal(size=(512, 3))
    v = rng.normal(size=noise.shape)
    lhs = np.sum(A.lpt_vjp(noise, w, xb, pb) * v)

    def f(z):
        x, p = lpt.generate(w, noise=z)
        q = lpt.lattice(8, 2)
        return np.sum(pm.min_image(x - q, 16) * xb) + np.sum(p * pb)
    rhs = fd(f, noise, v, 1e-6)
    assert lhs == pytest.approx(rhs, rel=1e-7)


def test_run_vjp_matches_fd():
    w = inputs.scaled(inputs.MEDIUM, 16, 8, n_steps=3)
    x0, p0 = lpt.generate(w)
    rng = np.random.default_rng(5)
    xb, pb = rng.normal(size=x0.shape), rng.normal(size=x0.shape)
    vx, vp = rng.normal(size=x0.shape), rng.normal(size=x0.shape)
    xs, xn, pn = A.run_forward_trajectory(x0, p0, w.a_list, 16, 512, OM)
    gx, gp = A.run_vjp(xs, w.a_list, 16, 512, OM, xb, pb)
    lhs = np.sum(gx * vx) + np.sum(gp * vp)

    def f(e):
        x, p, _ = pm.kdk_run(x0 + e * vx, p0 + e * vp, w.a_list, 16, 512, OM)
        return np.sum(pm.min_image(x - xn, 16) * xb) + np.sum(p * pb)
    rhs = (f(1e-7) - f(-1e-7)) / 2e-7
    assert lhs == pytest.approx(rhs, rel=1e-5)


def test_chi2_gradient_matches_central_fd_on_random_cells():
    # the full chain noise -> LPT -> KDK -> paint -> chi^2, 32 random cells,
    # Richardson-extrapolated central differences in float64
    w = inputs.scaled(inputs.ADJ_SMALL, 16, 8, n_steps=3)
    noise = white_noise(w.seed, 8)
    target = pm.density_contrast(lpt.generate(w, noise=white_noise(w.seed + 1000, 8))[0], 16, 512)
    target = target + np.random.default_rng(w.seed + 2000).normal(0, 0.1, target.shape)
    loss, g = A.loss_and_grad(noise, w, target, 0.1)
    cells = inputs.sample_indices(noise.size, 32, seed=3)
    flat = noise.reshape(-1)
    errs = []
    for c in cells:
        def f(e):
            z = flat.copy()
            z[c] += e
            return A.forward_loss(z.reshape(noise.shape), w, target, 0.1)[0]
        h = 1e-4
        d1 = (f(h) - f(-h)) / (2 * h)
        d2 = (f(h / 2) - f(-h / 2)) / h
        ref = (4 * d2 - d1) / 3
        errs.append(abs(g.reshape(-1)[c] - ref))
    scale = np.sqrt(np.mean(g ** 2))
    assert max(errs) / scale < 1e-6


def test_stored_c4a_gradient_meets_finite_differences():
    """At the 64^3 / 128^3 differentiable configuration (5 steps) the oracle's
    adjoint (along its FP64 trajectory) meets Richardson-extrapolated central
    differences of its forward run to 1e-4 of the gradient's rms at 32
    seeded cells (written by tests/golden/make_golden.py fd_c4a), while the
    same adjoint along the trajectory rounded to float32 (fd_c4a_f32traj)
    moves by CIC-kink crossings at some cell: the float32 state, not the
    adjoint, sets the end-to-end agreement of a float32 run."""
    import json
    import os
    here = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
    g = json.load(open(os.path.join(here, "fd_adj64_mesh128_box200.json")))
    gt = json.load(open(os.path.join(here, "grad_f32traj_adj64_mesh128_box200.json")))
    fd, ga = np.array(g["fd"]), np.array(g["oracle_adjoint"])
    assert np.abs(ga - fd).max() / g["grad_rms"] < 1e-4
    assert g["oracle_adjoint_vs_fd_max_rel_to_rms"] < 1e-4
    assert g["cells"] == gt["cells"]
    d32 = np.abs(np.array(gt["grad"]) - fd).max() / g["grad_rms"]
    assert 1e-4 < d32 < 2e-3
