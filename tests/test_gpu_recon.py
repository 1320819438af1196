"""Reconstruction (section 7, dark-matter observable) on the GPU against the
oracle: the posterior terms and the gradient handed to Adam at one
iteration, the Adam update itself, and descent over ten iterations."""
import numpy as np
import pytest
import torch

from oracle import lpt, pm, recon as orecon
from oracle.rng import white_noise
from paper_2010_11847_amd import inputs
from paper_2010_11847_amd.binding import PMContext, PMError
from paper_2010_11847_amd.recon import Reconstruction
from tests.gpu_helpers import banner, to_dev, to_np

SIGMA = 0.1


def problem(n_mesh=32, n_part=16, n_steps=3):
    w = inputs.scaled(inputs.ADJ_SMALL, n_mesh, n_part, n_steps=n_steps)
    noise = white_noise(w.seed, n_part)
    xt = lpt.generate(w, noise=white_noise(w.seed + 1000, n_part))[0]
    target = pm.density_contrast(xt, n_mesh, n_part ** 3)
    target = target + np.random.default_rng(w.seed + 2000).normal(0, SIGMA, target.shape)
    return w, noise, target


@pytest.mark.gpu
def test_recon_step_matches_oracle(gpu):
    banner("recon step 32/16 3 steps")
    w, noise, target = problem()
    # both sides start from the same float32 noise
    noise = noise.astype(np.float32).astype(np.float64)
    c = PMContext(w)
    r = Reconstruction(c, w.a_list, to_dev(target.astype(np.float32)), SIGMA,
                       noise0=to_dev(noise.astype(np.float32)), lr=0.01)
    chi2, prior = r.step()
    chi2_o, prior_o, g_o = orecon.posterior_loss_and_grad(noise, w, target, SIGMA)
    assert chi2 == pytest.approx(chi2_o, rel=1e-4)
    assert prior == pytest.approx(prior_o, rel=1e-10)
    # the gradient Adam received: m = (1 - beta1) g, v = (1 - beta2) g^2 at t = 1
    g = to_np(r.m).astype(np.float64) / 0.1
    assert np.linalg.norm(g - g_o) / np.linalg.norm(g_o) < 1e-4
    v = to_np(r.v).astype(np.float64) / 0.001
    assert np.linalg.norm(v - g_o ** 2) / np.linalg.norm(g_o ** 2) < 2e-4
    # the update is the Adam step of that gradient
    w1 = to_np(r.noise).astype(np.float64)
    w1_self, _, _ = orecon.adam_update(noise, g, 0.0, 0.0, 1, 0.01)
    assert np.max(np.abs(w1 - w1_self)) < 1e-6
    # and the oracle's own step, up to sign flips where the gradient is ~0
    w1_o, _, _ = orecon.adam_update(noise, g_o, 0.0, 0.0, 1, 0.01)
    bad = np.abs(w1 - w1_o) > 1e-5
    assert np.all(np.abs(g_o[bad]) < 1e-3 * np.sqrt(np.mean(g_o ** 2)))


@pytest.mark.gpu
def test_recon_descends_like_the_oracle(gpu):
    banner("recon 10 iterations 16/8")
    w, noise, target = problem(16, 8, 3)
    c = PMContext(w)
    r = Reconstruction(c, w.a_list, to_dev(target.astype(np.float32)), SIGMA, lr=0.03)
    hist = r.run(10)
    tot = [a + b for a, b in hist]
    _, ho = orecon.reconstruct(np.zeros_like(noise, dtype=np.float64), w, target, SIGMA, n_iter=10, lr=0.03)
    to = [a + b for a, b in ho]
    assert tot[0] == pytest.approx(to[0], rel=1e-4)
    assert tot[-1] < tot[0] / 3


@pytest.mark.gpu
def test_recon_rejects_bad_arguments(gpu):
    w, noise, target = problem(16, 8, 2)
    c = PMContext(w)
    d = to_dev(target.astype(np.float32))
    z = torch.zeros((8, 8, 8), device="cuda")
    small = torch.empty(1024, dtype=torch.uint8, device="cuda")
    with pytest.raises(PMError):
        c.pm_recon_step(w.a_list, d, SIGMA, z.clone(), z.clone(), z.clone(), 1, 0.01, work=small)
    with pytest.raises(PMError):
        c.pm_recon_step(w.a_list, d, SIGMA, z.clone(), z.clone(), z.clone(), 0, 0.01)
    with pytest.raises(PMError):
        c.pm_recon_step(w.a_list, d, -1.0, z.clone(), z.clone(), z.clone(), 1, 0.01)


@pytest.mark.gpu
def test_chi2_matches_oracle(gpu):
    from oracle import adjoint as A
    w, _, _ = problem(32, 16, 2)
    c = PMContext(w)
    rng = np.random.default_rng(9)
    d = rng.normal(size=(32, 32, 32)).astype(np.float32)
    t = rng.normal(size=(32, 32, 32)).astype(np.float32)
    chi2, g = c.pm_chi2(to_dev(d), to_dev(t), SIGMA)
    d64, t64 = d.astype(np.float64), t.astype(np.float64)
    assert float(chi2.item()) == pytest.approx(A.chi2(d64, t64, SIGMA), rel=1e-6)
    np.testing.assert_allclose(to_np(g), 2.0 * (d64 - t64) / SIGMA ** 2, rtol=1e-5, atol=1e-4)
    with pytest.raises(PMError):
        c.pm_chi2(to_dev(d), to_dev(t), 0.0)
