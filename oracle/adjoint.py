"""Reverse-mode derivative (vector-Jacobian products) of the PM run (float64).

Test infrastructure: see the package docstring.

The paper obtains gradients of a loss on the final density with respect to
the initial Gaussian field by automatic differentiation (section 7, the
reconstruction posterior and its chi^2 term).  Here the same derivative is
written out by hand, operator by operator, in the order the forward pass
applies them:

  noise w --Gen-IC (LPT)--> (x0, p0) --KDK steps--> x_n --paint--> delta
  loss = sum_cells ((delta - d) / sigma)^2           (section 7 listing form)

Transposes used (each pinned by a dot-product test):
  * paint^T on masses = readout; the position derivative of the CIC weight
    of corner o along d is (+1 if o_d else -1) times the other two factors;
  * a real Fourier multiplier IDFT(m DFT(.)) with Hermitian m has transpose
    IDFT(conj(m) DFT(.)); the FD force kernel i D / K^2 is odd, so the force
    operator is antisymmetric;
  * delta2 = sum_{i<j} phi_ii phi_jj - phi_ij^2 gives
    phi_bar_ii += delta2_bar (phi_jj + phi_kk), phi_bar_ij += -2 delta2_bar phi_ij.
"""
from __future__ import annotations

import numpy as np

from . import cosmology as cosmo_mod
from . import lpt as lpt_mod
from . import pm
from . import pyramid as pyramid_mod
from .pm import omega_axes, laplace_symbol, gradient_symbol


# ---------------------------------------------------------------------------
# building blocks
# ---------------------------------------------------------------------------

def _corner_terms(x, n):
    x = np.asarray(x, dtype=np.float64)
    i = np.floor(x)
    t = x - i
    i = i.astype(np.int64) % n
    for ox in (0, 1):
        for oy in (0, 1):
            for oz in (0, 1):
                o = (ox, oy, oz)
                f = [t[:, d] if o[d] else 1 - t[:, d] for d in range(3)]
                s = [1.0 if o[d] else -1.0 for d in range(3)]
                w = f[0] * f[1] * f[2]
                dw = np.stack([s[0] * f[1] * f[2], f[0] * s[1] * f[2], f[0] * f[1] * s[2]], 1)
                idx = (((i[:, 0] + ox) % n) * n + (i[:, 1] + oy) % n) * n + (i[:, 2] + oz) % n
                yield idx, w, dw


def readout_position_grad(mesh, x):
    """d/dx_p of readout(mesh, x_p): per particle, per axis."""
    n = mesh.shape[0]
    flat = np.asarray(mesh, dtype=np.float64).reshape(-1)
    g = np.zeros((len(x), 3))
    for idx, _, dw in _corner_terms(x, n):
        g += dw * flat[idx][:, None]
    return g


def paint_vjp(x, n, rho_bar, mass=None):
    """Cotangent of positions (and masses) for rho = paint(x, n, mass)."""
    xb = readout_position_grad(rho_bar, x)
    if mass is not None:
        xb = xb * np.asarray(mass, dtype=np.float64)[:, None]
    return xb


def apply_multiplier(field, mult):
    """IDFT(mult * DFT(field)) for a real field and a Hermitian multiplier."""
    return np.fft.irfftn(mult * np.fft.rfftn(field), s=field.shape, axes=(0, 1, 2))


def force_vjp(x, n_mesh, n_particles, omega_m, f_bar, **kw):
    """x_bar of F = readout(G delta(x), x) for a cotangent f_bar [np, 3]
    (G: the single-grid force, or with pyramid_levels = f the pyramid force).

    delta = paint(x) Ng^3/Np - 1, M_d = G_d delta, F_pd = readout(M_d, x_p).
    Two terms: the positions at which M is read out, and the positions that
    paint delta (through M_bar_d = paint(x, f_bar_d), delta_bar = sum G_d^T M_bar_d).
    """
    levels = kw.pop("pyramid_levels", 0)
    delta = pm.density_contrast(x, n_mesh, n_particles)
    if levels:
        meshes = pyramid_mod.force_meshes(delta, omega_m, levels)
    else:
        mult = pm.force_multipliers(n_mesh, omega_m, **kw)
        meshes = [apply_multiplier(delta, m) for m in mult]
    xb = np.zeros((len(x), 3))
    for d in range(3):
        xb += readout_position_grad(meshes[d], x) * f_bar[:, d:d + 1]
    mbar = [pm.paint(x, n_mesh, mass=f_bar[:, d]) for d in range(3)]
    if levels:
        delta_bar = pyramid_mod.force_meshes_T(mbar, omega_m, levels)
    else:
        delta_bar = np.zeros((n_mesh,) * 3)
        for d in range(3):
            delta_bar += apply_multiplier(mbar[d], np.conj(mult[d]))
    xb += paint_vjp(x, n_mesh, delta_bar * (n_mesh ** 3 / n_particles))
    return xb


# ---------------------------------------------------------------------------
# KDK run
# ---------------------------------------------------------------------------

def run_forward_trajectory(x0, p0, a_list, n_mesh, n_particles, omega_m, **kw):
    """Forward run that records the positions at every force evaluation."""
    xs = [np.array(x0, dtype=np.float64)]

    def cb(step, x, p, f):
        xs.append(np.array(x))
    xn, pn, _ = pm.kdk_run(x0, p0, a_list, n_mesh, n_particles, omega_m, callback=cb, **kw)
    return xs, xn, pn


def run_vjp(xs, a_list, n_mesh, n_particles, omega_m, x_bar, p_bar, **kw):
    """Cotangents (x0_bar, p0_bar) of a KDK run given (x_n_bar, p_n_bar).

    Reverse of, for each step ai -> aj (half step ac):
      q = p + F(x_i) K1;  x_j = x_i + q D;  p_j = q + F(x_j) K2.
    """
    xb = np.array(x_bar, dtype=np.float64)
    pb = np.array(p_bar, dtype=np.float64)
    n = len(a_list) - 1
    for s in range(n - 1, -1, -1):
        ai, aj = a_list[s], a_list[s + 1]
        ac = cosmo_mod.half_step(ai, aj)
        k1 = cosmo_mod.kick_factor(ai, ac, ai, omega_m)
        dr = cosmo_mod.drift_factor(ai, aj, ac, omega_m)
        k2 = cosmo_mod.kick_factor(ac, aj, aj, omega_m)
        # p_j = q + F(x_j) K2
        qb = pb.copy()
        xb = xb + force_vjp(xs[s + 1], n_mesh, n_particles, omega_m, pb * k2, **kw)
        # x_j = x_i + q D
        qb = qb + xb * dr
        # q = p_i + F(x_i) K1
        pb = qb
        xb = xb + force_vjp(xs[s], n_mesh, n_particles, omega_m, qb * k1, **kw)
    return xb, pb


# ---------------------------------------------------------------------------
# Gen-IC (LPT)
# ---------------------------------------------------------------------------

def _lpt_symbols(n):
    ws = omega_axes(n)
    k2 = laplace_symbol(*ws)
    inv = np.where(k2 > 0, 1.0 / np.where(k2 > 0, k2, 1.0), 0.0)
    dsym = [gradient_symbol(w) for w in ws]
    return inv, dsym


def _linear_scale(n, box_size, cosmo):
    nx = np.fft.fftfreq(n, 1.0 / n)
    nz = np.fft.rfftfreq(n, 1.0 / n)
    n2 = nx[:, None, None] ** 2 + nx[None, :, None] ** 2 + nz[None, None, :] ** 2
    k = 2 * np.pi * np.sqrt(n2) / box_size
    t = np.sqrt(cosmo_mod.linear_power(k, cosmo) / (box_size / n) ** 3)
    t[0, 0, 0] = 0.0
    return t


def lpt_vjp(noise, workload, x0_bar, p0_bar):
    """Cotangent of the white noise for (x0, p0) = generate(workload, noise)."""
    n = noise.shape[0]
    shape = (n, n, n)
    a0 = workload.a_list[0]
    om = workload.cosmo.omega_m
    b = workload.n_mesh // n
    order = workload.lpt_order
    d1, f1, d2, f2 = (float(v[0]) for v in cosmo_mod.growth(a0, om))
    if order < 2:
        d2 = 0.0
    e0 = float(cosmo_mod.hubble(a0, om))
    xb = np.asarray(x0_bar, dtype=np.float64).reshape(n, n, n, 3)
    pb = np.asarray(p0_bar, dtype=np.float64).reshape(n, n, n, 3)
    s1b = b * d1 * xb + b * a0 ** 2 * e0 * f1 * d1 * pb
    s2b = b * d2 * xb + b * a0 ** 2 * e0 * f2 * d2 * pb
    inv, dsym = _lpt_symbols(n)
    tk = _linear_scale(n, workload.box_size, workload.cosmo)
    dk = np.fft.rfftn(np.asarray(noise, dtype=np.float64)) * tk
    # adjoint of s1_d = IDFT(i D_d / K^2 delta_L^): conj multiplier
    acc = np.zeros_like(dk)
    for d in range(3):
        acc += np.conj(1j * dsym[d] * inv) * np.fft.rfftn(s1b[..., d])
    if order >= 2:
        phi = {}
        for i in range(3):
            for j in range(i, 3):
                phi[i, j] = np.fft.irfftn(dsym[i] * dsym[j] * inv * dk, s=shape, axes=(0, 1, 2))
        # s2_d = IDFT(-i D_d / K^2 DFT(delta2))
        d2b = np.zeros(shape)
        for d in range(3):
            d2b += apply_multiplier(s2b[..., d], np.conj(-1j * dsym[d] * inv))
        phib = {
            (0, 0): d2b * (phi[1, 1] + phi[2, 2]),
            (1, 1): d2b * (phi[0, 0] + phi[2, 2]),
            (2, 2): d2b * (phi[0, 0] + phi[1, 1]),
            (0, 1): -2 * d2b * phi[0, 1],
            (0, 2): -2 * d2b * phi[0, 2],
            (1, 2): -2 * d2b * phi[1, 2],
        }
        for (i, j), v in phib.items():
            acc += dsym[i] * dsym[j] * inv * np.fft.rfftn(v)
    # delta_L^ = DFT(w) T with T real: the transpose of w -> irfftn(m T rfftn(w))
    # is irfftn(conj(m) T rfftn(.)) with the same normalisation
    return np.fft.irfftn(acc * tk, s=shape, axes=(0, 1, 2))


# ---------------------------------------------------------------------------
# chi^2 loss of the final density and its full gradient
# ---------------------------------------------------------------------------

def chi2(delta, target, sigma):
    return float(np.sum(((delta - target) / sigma) ** 2))


def forward_loss(noise, workload, target, sigma):
    x0, p0 = lpt_mod.generate(workload, noise=noise)
    xn, _, _ = pm.kdk_run(x0, p0, workload.a_list, workload.n_mesh, workload.n_particles,
                          workload.cosmo.omega_m)
    delta = pm.density_contrast(xn, workload.n_mesh, workload.n_particles)
    return chi2(delta, target, sigma), delta


def loss_and_grad(noise, workload, target, sigma):
    """chi^2 and its gradient with respect to the white noise."""
    x0, p0 = lpt_mod.generate(workload, noise=noise)
    n, npart, om = workload.n_mesh, workload.n_particles, workload.cosmo.omega_m
    xs, xn, pn = run_forward_trajectory(x0, p0, workload.a_list, n, npart, om)
    delta = pm.density_contrast(xn, n, npart)
    loss = chi2(delta, target, sigma)
    delta_bar = 2.0 * (delta - target) / sigma ** 2
    xb = paint_vjp(xn, n, delta_bar * (n ** 3 / npart))
    pb = np.zeros_like(xb)
    x0b, p0b = run_vjp(xs, workload.a_list, n, npart, om, xb, pb)
    return loss, lpt_vjp(noise, workload, x0b, p0b)


def grad_along_trajectory(xs, noise, workload, target, sigma, **kw):
    """chi^2 gradient with respect to the noise, differentiating along a given
    trajectory xs (positions at every scale factor) instead of re-running the
    forward pass: the same reverse sweep, at externally supplied points
    (kw: force options, e.g. pyramid_levels)."""
    n, npart, om = workload.n_mesh, workload.n_particles, workload.cosmo.omega_m
    xs = [np.asarray(x, dtype=np.float64) for x in xs]
    delta = pm.density_contrast(xs[-1], n, npart)
    delta_bar = 2.0 * (delta - target) / sigma ** 2
    xb = paint_vjp(xs[-1], n, delta_bar * (n ** 3 / npart))
    x0b, p0b = run_vjp(xs, workload.a_list, n, npart, om, xb, np.zeros_like(xb), **kw)
    return lpt_vjp(noise, workload, x0b, p0b)
