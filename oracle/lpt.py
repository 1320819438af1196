"""Gaussian linear field and Lagrangian perturbation theory initial conditions.

Test infrastructure: see the package docstring.

Follows the Gen-IC algorithm of section 6 (sample a normal field, scale it by
the power spectrum, estimate the "force" of the linear field on the grid,
scale it to a displacement, displace the particles and scale to a velocity).
The paper uses first order (Zel'dovich) in its text and second order in one
figure caption; both are implemented (``order``).  The derivative kernels are
the same FD kernels as the force (section 2), applied on the particle lattice.

Lattice: particle (i, j, l) sits at q = B (i, j, l) + shift (shift = 0: mesh
nodes; the paper is silent), with B = Ng / Np; particle index = (i Np + j) Np + l.
With shift = 0 the CIC deposit of a particle that sits on a node is not
differentiable in its displacement at zero (the deposit moves to the left or
right neighbour by the sign of the displacement); shift = 0.5 avoids that.
"""
from __future__ import annotations

import numpy as np

from . import cosmology as cosmo_mod
from .pm import omega_axes, laplace_symbol, gradient_symbol, wrap, rfftn, irfftn


def linear_field_k(noise, box_size, cosmo, fixed_amplitude=False):
    """delta_L^(n) = DFT(w)(n) sqrt(P(k)/V_cell), delta_L^(0) = 0.

    With unit white noise <|w^|^2> = N^3, so <|delta_L^|^2> = N^6 P / L^3.
    ``fixed_amplitude`` replaces |w^| by sqrt(N^3) (test mode).
    """
    n = noise.shape[0]
    wk = rfftn(np.asarray(noise, dtype=np.float64))
    if fixed_amplitude:
        mag = np.abs(wk)
        wk = np.where(mag > 0, wk / np.where(mag > 0, mag, 1.0), 0.0) * np.sqrt(float(n) ** 3)
    nx = np.fft.fftfreq(n, 1.0 / n)
    nz = np.fft.rfftfreq(n, 1.0 / n)
    n2 = nx[:, None, None] ** 2 + nx[None, :, None] ** 2 + nz[None, None, :] ** 2
    k = 2 * np.pi * np.sqrt(n2) / box_size
    v_cell = (box_size / n) ** 3
    dk = wk * np.sqrt(cosmo_mod.linear_power(k, cosmo) / v_cell)
    dk[0, 0, 0] = 0.0
    return dk


def lpt_displacements(dk, order=2):
    """Lattice-unit displacement fields s1 (and s2) from delta_L^.

    s1^_d = i D(w_d)/K^2 delta_L^                 (s1 = -grad lap^-1 delta_L)
    phi,ij^ = D(w_i) D(w_j)/K^2 delta_L^           (phi = lap^-1 delta_L... up to sign)
    delta2 = sum_{i<j} phi,ii phi,jj - phi,ij^2    (real space)
    s2^_d = -i D(w_d)/K^2 delta2^                 (s2 = grad lap^-1 delta2)
    """
    n = dk.shape[0]
    shape = (n, n, n)
    ws = omega_axes(n)
    k2 = laplace_symbol(*ws)
    inv = np.where(k2 > 0, 1.0 / np.where(k2 > 0, k2, 1.0), 0.0)
    dsym = [gradient_symbol(w) for w in ws]
    s1 = np.stack([irfftn(1j * d * inv * dk, shape) for d in dsym], -1)
    if order < 2:
        return s1, np.zeros_like(s1)
    phi = {}
    for i in range(3):
        for j in range(i, 3):
            phi[i, j] = irfftn(dsym[i] * dsym[j] * inv * dk, shape)
    delta2 = (phi[0, 0] * phi[1, 1] + phi[0, 0] * phi[2, 2] + phi[1, 1] * phi[2, 2]
              - phi[0, 1] ** 2 - phi[0, 2] ** 2 - phi[1, 2] ** 2)
    d2k = rfftn(delta2)
    s2 = np.stack([irfftn(-1j * d * inv * d2k, shape) for d in dsym], -1)
    return s1, s2


def lattice(n_part, ratio, shift=0.0):
    i = np.arange(n_part, dtype=np.float64)
    q = np.stack(np.meshgrid(i, i, i, indexing="ij"), -1).reshape(-1, 3)
    return q * ratio + shift


def initial_state(s1, s2, a0, n_mesh, omega_m, order=2, shift=0.0):
    """x = B (q + D1 s1 + D2 s2) (wrapped), p = B a0^2 E(a0) (f1 D1 s1 + f2 D2 s2).

    p = a^3 E dx/da is the momentum conjugate to x in the drift equation.
    """
    n_part = s1.shape[0]
    b = n_mesh // n_part
    d1, f1, d2, f2 = (float(v[0]) for v in cosmo_mod.growth(a0, omega_m))
    if order < 2:
        d2 = 0.0
    s1 = s1.reshape(-1, 3)
    s2 = s2.reshape(-1, 3)
    x = wrap(lattice(n_part, b, shift) + b * (d1 * s1 + d2 * s2), n_mesh)
    e0 = float(cosmo_mod.hubble(a0, omega_m))
    p = b * a0 ** 2 * e0 * (f1 * d1 * s1 + f2 * d2 * s2)
    return x, p


def generate(workload, noise=None, fixed_amplitude=False):
    """Gen-IC: white noise -> delta_L -> LPT -> (x, p) at a_list[0]."""
    from .rng import white_noise
    if noise is None:
        noise = white_noise(workload.seed, workload.n_part)
    dk = linear_field_k(noise, workload.box_size, workload.cosmo, fixed_amplitude)
    s1, s2 = lpt_displacements(dk, workload.lpt_order)
    return initial_state(s1, s2, workload.a_list[0], workload.n_mesh,
                         workload.cosmo.omega_m, workload.lpt_order, workload.lattice_shift)
