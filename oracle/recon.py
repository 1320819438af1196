"""MAP reconstruction of the initial conditions from the final dark-matter
overdensity (float64).

Test infrastructure: see the package docstring.

Section 7 ("Reconstruction from Dark Matter") minimises the negative log
posterior of the initial field given the evolved overdensity: a Gaussian
likelihood with constant variance sigma^2 in configuration space plus the
Gaussian prior of the initial field, and updates the field with Adam.  The
listing of that section writes both terms without the factor 1/2 (the
chi^2 of the model against the data, and the squared Fourier modes of the
field over the fiducial power).

Readings (the paper leaves the normalisations implicit):
  * The variable is the white noise w that sets the initial field (the
    Gen-IC input), so the prior term over the field's modes is the squared
    norm of w: with s^(k) = DFT(w) T(k) and T^2 = P / V_cell, the listing's
    sum of |s^|^2 / P is the sum of |DFT(w)|^2 up to the DFT normalisation,
    and the weight that makes chi^2 + prior equal -2 log posterior for unit
    white noise is sum_x w(x)^2.
  * loss(w) = sum_cells ((delta_m(w) - delta_e) / sigma)^2 + sum_lattice w^2.
  * The adiabatic (smoothing) schedule is left out, as in the listing.

Adam is the update rule of Kingma & Ba (2015, Algorithm 1): biased first and
second moment estimates, bias correction by 1 - beta^t, step
lr * m_hat / (sqrt(v_hat) + eps).  The paper uses it with learning rate 0.01
in the text (0.1 in the listing).
"""
from __future__ import annotations

import numpy as np

from . import adjoint


def prior(noise):
    """Negative double log-density of unit white noise: sum_x w(x)^2."""
    w = np.asarray(noise, dtype=np.float64)
    return float(np.sum(w * w))


def posterior_loss_and_grad(noise, workload, target, sigma):
    """(chi^2, prior, d(chi^2 + prior)/dw) at the white noise w."""
    w = np.asarray(noise, dtype=np.float64)
    chi2, g = adjoint.loss_and_grad(w, workload, target, sigma)
    return chi2, prior(w), g + 2.0 * w


def adam_update(w, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step at step count t >= 1; returns the new (w, m, v)."""
    w = np.asarray(w, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    m = beta1 * np.asarray(m, dtype=np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, dtype=np.float64) + (1.0 - beta2) * g * g
    m_hat = m / (1.0 - beta1 ** t)
    v_hat = v / (1.0 - beta2 ** t)
    return w - lr * m_hat / (np.sqrt(v_hat) + eps), m, v


def reconstruct(noise0, workload, target, sigma, n_iter, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """n_iter Adam iterations from noise0; returns (w, [(chi2, prior) per iteration])."""
    w = np.array(noise0, dtype=np.float64)
    m = np.zeros_like(w)
    v = np.zeros_like(w)
    hist = []
    for t in range(1, n_iter + 1):
        chi2, pr, g = posterior_loss_and_grad(w, workload, target, sigma)
        hist.append((chi2, pr))
        w, m, v = adam_update(w, g, m, v, t, lr, beta1, beta2, eps)
    return w, hist
