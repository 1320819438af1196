"""Pins for oracle.recon: the Adam rule against its closed forms and
invariances, the posterior gradient against finite differences of the
forward oracle, and descent of the posterior on a small problem."""
import numpy as np
import pytest

from oracle import lpt, pm, recon
from oracle.rng import white_noise
from paper_2010_11847_amd import inputs


def test_adam_first_step_is_a_sign_step():
    # at t = 1 the bias-corrected moments are g and g^2: the step is lr g / (|g| + eps)
    rng = np.random.default_rng(0)
    g = rng.normal(size=1000) * 10.0 ** rng.uniform(-3, 3, size=1000)
    w = rng.normal(size=1000)
    w1, m1, v1 = recon.adam_update(w, g, np.zeros(1000), np.zeros(1000), 1, lr=0.01, eps=1e-8)
    np.testing.assert_allclose(w - w1, 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)
    np.testing.assert_allclose(m1, 0.1 * g, rtol=1e-12)
    np.testing.assert_allclose(v1, 0.001 * g * g, rtol=1e-12)


def test_adam_is_invariant_to_gradient_scale():
    # with eps = 0 the update depends only on the direction of the gradient history
    rng = np.random.default_rng(1)
    gs = [rng.normal(size=50) for _ in range(4)]
    def run(c):
        w, m, v = np.zeros(50), np.zeros(50), np.zeros(50)
        for t, g in enumerate(gs, 1):
            w, m, v = recon.adam_update(w, c * g, m, v, t, lr=0.1, eps=0.0)
        return w
    np.testing.assert_allclose(run(1.0), run(1e4), rtol=1e-12)


def test_adam_zero_gradient_does_not_move():
    w = np.arange(5.0)
    w1, m1, v1 = recon.adam_update(w, np.zeros(5), np.zeros(5), np.zeros(5), 1, lr=0.1)
    np.testing.assert_array_equal(w1, w)


def test_adam_minimises_a_quadratic():
    # f(w) = 1/2 sum a_i (w_i - c_i)^2 with condition number 100
    rng = np.random.default_rng(2)
    a = 10.0 ** rng.uniform(0, 2, size=20)
    c = rng.normal(size=20)
    w, m, v = np.zeros(20), np.zeros(20), np.zeros(20)
    for t in range(1, 3001):
        w, m, v = recon.adam_update(w, a * (w - c), m, v, t, lr=0.01)
    assert np.max(np.abs(w - c)) < 1e-3


def _problem():
    w = inputs.scaled(inputs.ADJ_SMALL, 16, 8, n_steps=3)
    noise = white_noise(w.seed, 8)
    target = pm.density_contrast(lpt.generate(w, noise=white_noise(w.seed + 1000, 8))[0], 16, 512)
    target = target + np.random.default_rng(w.seed + 2000).normal(0, 0.1, target.shape)
    return w, noise, target


def test_posterior_gradient_matches_central_fd():
    w, noise, target = _problem()
    chi2, pr, g = recon.posterior_loss_and_grad(noise, w, target, 0.1)
    assert pr == pytest.approx(float(np.sum(noise.astype(np.float64) ** 2)), rel=1e-14)
    flat = noise.reshape(-1).astype(np.float64)
    errs = []
    for c in inputs.sample_indices(noise.size, 12, seed=5):
        def f(e):
            z = flat.copy()
            z[c] += e
            zz = z.reshape(noise.shape)
            return recon.posterior_loss_and_grad(zz, w, target, 0.1)[0] + float(np.sum(zz ** 2))
        h = 1e-4
        d1 = (f(h) - f(-h)) / (2 * h)
        d2 = (f(h / 2) - f(-h / 2)) / h
        errs.append(abs(g.reshape(-1)[c] - (4 * d2 - d1) / 3))
    assert max(errs) / np.sqrt(np.mean(g ** 2)) < 1e-6


def test_reconstruction_lowers_the_posterior():
    w, noise, target = _problem()
    # Adam is not monotone; over ten iterations the posterior falls by > 3x
    _, hist = recon.reconstruct(np.zeros_like(noise, dtype=np.float64), w, target, 0.1, n_iter=10, lr=0.03)
    tot = [a + b for a, b in hist]
    assert tot[-1] < tot[0] / 3
