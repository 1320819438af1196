"""Particle-mesh force and kick-drift-kick integration (float64).

Test infrastructure: see the package docstring.

Conventions (a reading; the paper fixes none of them): positions and momenta
in mesh-cell units, periodic box [0, Ng)^3, meshes C-ordered [x][y][z],
integer frequencies n in {0..N/2, -N/2+1..-1}, circular frequency
omega = 2 pi n / N in (-pi, pi], particle mass 1, delta = rho Ng^3/Np - 1.
"""
from __future__ import annotations

import math
import os

import numpy as np
import scipy.fft as sfft

from . import cosmology as cosmo_mod

# threads of the library DFT: the CPUs this process may run on, or
# ORACLE_FFT_WORKERS; painting and readout are single-threaded NumPy
_WORKERS = int(os.environ.get("ORACLE_FFT_WORKERS", "0")) or len(os.sched_getaffinity(0)) or 1


def rfftn(a):
    """3D real DFT (unnormalised), library routine (pocketfft)."""
    return sfft.rfftn(a, axes=(0, 1, 2), workers=_WORKERS)


def irfftn(a, shape, overwrite=False):
    """Inverse of rfftn, normalised by 1/N^3, library routine (pocketfft)."""
    return sfft.irfftn(a, s=shape, axes=(0, 1, 2), workers=_WORKERS, overwrite_x=overwrite)

SPLIT_NONE, SPLIT_LONG, SPLIT_SHORT = 0, 1, 2


# ---------------------------------------------------------------------------
# Fourier-space kernels (section 2, the FD transfer function)
# ---------------------------------------------------------------------------

def omega_axes(n, rfft_last=True):
    """Circular frequencies along the three axes, broadcastable to the half spectrum."""
    w = 2.0 * np.pi * np.fft.fftfreq(n) 
    wz = 2.0 * np.pi * np.fft.rfftfreq(n) if rfft_last else w
    return w[:, None, None], w[None, :, None], wz[None, None, :]


def laplace_symbol(wx, wy, wz):
    """K^2 = sum_d (2 sin(w_d/2))^2: the FD Laplacian is -K^2.

    This is the inverse of the paper's FD inverse-Laplacian kernel
    (k_d sinc(w_d/2))^2 summed over d, with k_d = w_d / x0 and x0 = 1.
    """
    return (2 * np.sin(wx / 2)) ** 2 + (2 * np.sin(wy / 2)) ** 2 + (2 * np.sin(wz / 2)) ** 2


def gradient_symbol(w):
    """Fourth-order FD gradient: grad <-> i (8 sin w - sin 2w) / 6 (section 2)."""
    return (8.0 * np.sin(w) - np.sin(2.0 * w)) / 6.0


def cic_window(wx, wy, wz):
    """Fourier transform of the CIC assignment: prod_d sinc^2(w_d/2)."""
    def s(w):
        return np.sinc(w / (2 * np.pi))   # numpy sinc(x) = sin(pi x)/(pi x)
    return (s(wx) * s(wy) * s(wz)) ** 2


def green_function(n, omega_m, deconv_order=0, split_rs=0.0, split_mode=SPLIT_NONE):
    """Real part common to the three force multipliers: 1.5 Om / K^2 W^-n S."""
    wx, wy, wz = omega_axes(n)
    k2 = laplace_symbol(wx, wy, wz)
    with np.errstate(divide="ignore", invalid="ignore"):
        green = np.where(k2 > 0, 1.5 * omega_m / np.where(k2 > 0, k2, 1.0), 0.0)
    del k2
    if deconv_order:
        green /= cic_window(wx, wy, wz) ** deconv_order
    if split_mode != SPLIT_NONE:
        kk = wx ** 2 + wy ** 2 + wz ** 2
        s = np.exp(-kk * split_rs ** 2)
        green *= (s if split_mode == SPLIT_LONG else 1.0 - s)
    return green


def force_multipliers(n, omega_m, deconv_order=0, split_rs=0.0, split_mode=SPLIT_NONE):
    """Complex multipliers G_d such that F_d^ = G_d delta^ (d = x, y, z).

    G_d = 1.5 Omega_m i D(w_d) / K^2 * W^-deconv * S(k), G_d(0) = 0.
    The factor 1.5 Omega_m and the sign (attractive force F = -grad phi with
    lap phi = 1.5 Omega_m delta) are omitted by the paper's force equation;
    they are the reading taken here.
    """
    wx, wy, wz = omega_axes(n)
    k2 = laplace_symbol(wx, wy, wz)
    with np.errstate(divide="ignore", invalid="ignore"):
        green = np.where(k2 > 0, 1.5 * omega_m / np.where(k2 > 0, k2, 1.0), 0.0)
    if deconv_order:
        green = green / cic_window(wx, wy, wz) ** deconv_order
    if split_mode != SPLIT_NONE:
        kk = wx ** 2 + wy ** 2 + wz ** 2
        s = np.exp(-kk * split_rs ** 2)
        green = green * (s if split_mode == SPLIT_LONG else 1.0 - s)
    return [1j * gradient_symbol(w) * green for w in (wx, wy, wz)]


# ---------------------------------------------------------------------------
# CIC paint / readout (section 2: linear window of unit size)
# ---------------------------------------------------------------------------

def _cic_corners(x, n):
    x = np.asarray(x, dtype=np.float64)
    i = np.floor(x)
    t = x - i
    i = i.astype(np.int64) % n
    for ox in (0, 1):
        for oy in (0, 1):
            for oz in (0, 1):
                w = ((t[:, 0] if ox else 1 - t[:, 0]) *
                     (t[:, 1] if oy else 1 - t[:, 1]) *
                     (t[:, 2] if oz else 1 - t[:, 2]))
                idx = (((i[:, 0] + ox) % n) * n + (i[:, 1] + oy) % n) * n + (i[:, 2] + oz) % n
                yield idx, w, (ox, oy, oz), t


def paint(x, n, mass=None):
    """Mass assignment rho(c) = sum_p m_p prod_d w(x_pd - c_d), w(t) = 1 - |t|."""
    rho = np.zeros(n ** 3, dtype=np.float64)
    m = None if mass is None else np.asarray(mass, dtype=np.float64)
    for idx, w, _, _ in _cic_corners(x, n):
        rho += np.bincount(idx, weights=w if m is None else w * m, minlength=n ** 3)
        del idx, w
    return rho.reshape(n, n, n)


def readout(mesh, x):
    """CIC interpolation of mesh values at positions, the transpose of paint."""
    n = mesh.shape[0]
    flat = np.asarray(mesh, dtype=np.float64).reshape(-1)
    out = np.zeros(len(x), dtype=np.float64)
    for idx, w, _, _ in _cic_corners(x, n):
        out += w * flat[idx]
    return out


def density_contrast(x, n_mesh, n_particles):
    delta = paint(x, n_mesh)
    delta *= n_mesh ** 3 / n_particles
    delta -= 1.0
    return delta


# ---------------------------------------------------------------------------
# Force (section 2: paint -> FFT -> grad lap^-1 -> inverse FFTs -> readout)
# ---------------------------------------------------------------------------

def force_mesh(dk, green, d, n):
    """Force component d on the mesh: IDFT(i D(w_d) green DFT(delta))."""
    w = omega_axes(n)[d]
    spec = green * (1j * gradient_symbol(w))
    spec *= dk
    return irfftn(spec, (n, n, n), overwrite=True)


def force_meshes(delta, omega_m, **kw):
    """Three real force meshes F_d = IDFT(G_d DFT(delta))."""
    n = delta.shape[0]
    dk = rfftn(delta)
    green = green_function(n, omega_m, **kw)
    return [force_mesh(dk, green, d, n) for d in range(3)]


def force(x, n_mesh, n_particles, omega_m, **kw):
    """Per-particle PM force at positions x (mesh units); one component at a time."""
    delta = density_contrast(x, n_mesh, n_particles)
    dk = rfftn(delta)
    del delta
    green = green_function(n_mesh, omega_m, **kw)
    out = np.empty((len(x), 3))
    for d in range(3):
        mesh = force_mesh(dk, green, d, n_mesh)
        out[:, d] = readout(mesh, x)
        del mesh
    return out


# ---------------------------------------------------------------------------
# Kick-drift-kick leapfrog (section 2, the drift and kick update equations)
# ---------------------------------------------------------------------------

def wrap(x, n):
    x = np.mod(x, n)
    x[x >= n] = 0.0
    return x


def kdk_run(x, p, a_list, n_mesh, n_particles, omega_m, force_fn=None, callback=None, **kw):
    """Integrate from a_list[0] to a_list[-1].

    For each step ai -> aj with half-step ac (geometric mean):
      kick  p += F(x_i) K(ai -> ac; ai)
      drift x += p D(ai -> aj; ac), wrapped into the box
      force F(x_j)
      kick  p += F(x_j) K(ac -> aj; aj)
    Returns (x, p, F) at the final time.
    """
    fn = force_fn or (lambda xx: force(xx, n_mesh, n_particles, omega_m, **kw))
    x = np.array(x, dtype=np.float64)
    p = np.array(p, dtype=np.float64)
    f = fn(x)
    for s, (ai, aj) in enumerate(zip(a_list[:-1], a_list[1:])):
        ac = cosmo_mod.half_step(ai, aj)
        p = p + f * cosmo_mod.kick_factor(ai, ac, ai, omega_m)
        x = wrap(x + p * cosmo_mod.drift_factor(ai, aj, ac, omega_m), n_mesh)
        f = fn(x)
        p = p + f * cosmo_mod.kick_factor(ac, aj, aj, omega_m)
        if callback is not None:
            callback(s, x, p, f)
    return x, p, f


def min_image(d, n):
    """Minimum-image separation in a periodic box."""
    return d - n * np.round(d / n)
