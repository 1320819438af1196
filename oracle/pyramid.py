"""Multi-grid (pyramid) force of section 5.2 (float64).

Test infrastructure: see the package docstring.

The paper builds a two-level force from a multiresolution pyramid
(section 3.1 and Algorithms 2 and 3):
  * REDUCE: f times, convolve with a 3-D B-spline kernel and subsample by a
    stride of 2 (a strided convolution);
  * EXPAND: f times, a transposed strided convolution with the same kernel
    times 8, the inverse of the subsampling's loss of 2^3 samples per cell;
  * force: the long-range force on the reduced (coarse) grid, expanded back,
    plus the short-range force on the fine grid minus the part of it that
    the coarse grid represents (its reduce-then-expand), per component.

Readings (the paper's algorithms leave these open; each is listed with the
design notes):
  * "B-spline kernel of order n": the discrete B-spline of order n, the n-fold
    convolution of the two-tap box [1, 1]/2, i.e. n + 1 binomial weights
    C(n, k) / 2^n (n = 6: 7 taps, sum 1); the 3-D kernel is the tensor product
    of three such 1-D kernels.
  * The loop "for i in 0..f" runs f times: the text repeats the operation
    twice for a grid four times coarser (f = 2).
  * One device holds the whole periodic mesh, so the "local" fine-grid FFT of
    the distributed scheme is the global one, and every convolution wraps
    periodically; coarse cell i is centred on fine cell 2 i.
  * Forces are in cells of the grid they are computed on; a coarse-grid force
    is converted to fine cells by the factor 2^f (the Green's function scales
    as the inverse square and the gradient as the first power of the cell).
"""
from __future__ import annotations

import numpy as np

from . import pm


def bspline_kernel(order: int = 6) -> np.ndarray:
    """1-D discrete B-spline of the given order: order + 1 binomial weights / 2^order."""
    k = np.array([1.0])
    for _ in range(order):
        k = np.convolve(k, [0.5, 0.5])
    return k


def _conv_axis(a, k, axis):
    """Centred periodic convolution along one axis: out[i] = sum_t k[t] a[i + t - r]."""
    r = len(k) // 2
    out = np.zeros_like(a, dtype=np.float64)
    for t, kt in enumerate(k):
        out += kt * np.roll(a, -(t - r), axis=axis)
    return out


def reduce_field(field, levels: int = 2, order: int = 6):
    """REDUCE (Algorithm 2): levels times a B-spline convolution with stride 2."""
    k = bspline_kernel(order)
    d = np.asarray(field, dtype=np.float64)
    for _ in range(levels):
        for ax in range(3):
            d = _conv_axis(d, k, ax)
        d = d[::2, ::2, ::2]
    return d


def expand_field(field, levels: int = 2, order: int = 6):
    """EXPAND (Algorithm 2): levels times a transposed stride-2 convolution
    with the kernel times 8 (zeros inserted, then the kernel times 2 per axis)."""
    k = 2.0 * bspline_kernel(order)
    h = np.asarray(field, dtype=np.float64)
    for _ in range(levels):
        n = h.shape[0]
        up = np.zeros((2 * n, 2 * n, 2 * n))
        up[::2, ::2, ::2] = h
        for ax in range(3):
            up = _conv_axis(up, k, ax)
        h = up
    return h


def force_meshes(delta, omega_m, levels: int = 2, order: int = 6):
    """Force meshes of Algorithm 3: F = EXPAND(F_L) + F_S - EXPAND(REDUCE(F_S))."""
    delta = np.asarray(delta, dtype=np.float64)
    coarse = reduce_field(delta, levels, order)
    f_long = [f * 2.0 ** levels for f in pm.force_meshes(coarse, omega_m)]
    f_short = pm.force_meshes(delta, omega_m)
    out = []
    for d in range(3):
        f_l = expand_field(f_long[d], levels, order)
        f_ll = expand_field(reduce_field(f_short[d], levels, order), levels, order)
        out.append(f_l + f_short[d] - f_ll)
    return out


def force(x, n_mesh, n_particles, omega_m, levels: int = 2, order: int = 6):
    """Per-particle pyramid force at positions x (mesh units)."""
    delta = pm.density_contrast(x, n_mesh, n_particles)
    meshes = force_meshes(delta, omega_m, levels, order)
    return np.stack([pm.readout(m, x) for m in meshes], axis=1)


def force_meshes_T(mbar, omega_m, levels: int = 2, order: int = 6):
    """Transpose of force_meshes in the real-space inner product:
    delta_bar = sum_d F_d^T mbar_d.  With R = REDUCE, E = EXPAND = 8^f R^T and
    F_d = G_d delta - E R G_d delta + 2^f E G_c,d R delta, each term's
    transpose gives
        F_d^T m = G_d^T (m - E R m) + 2^f E G_c,d^T R m,
    with G^T the conjugate multiplier (the FD force kernel is odd)."""
    mbar = [np.asarray(m, dtype=np.float64) for m in mbar]
    n = mbar[0].shape[0]
    mult = pm.force_multipliers(n, omega_m)
    mult_c = pm.force_multipliers(n >> levels, omega_m)
    fine = np.zeros((n, n, n))
    coarse = np.zeros((n >> levels,) * 3)
    for d in range(3):
        r = reduce_field(mbar[d], levels, order)
        fine += np.fft.irfftn(np.conj(mult[d]) * np.fft.rfftn(mbar[d] - expand_field(r, levels, order)),
                              s=(n, n, n), axes=(0, 1, 2))
        coarse += np.fft.irfftn(np.conj(mult_c[d]) * np.fft.rfftn(r), s=r.shape, axes=(0, 1, 2))
    return fine + 2.0 ** levels * expand_field(coarse, levels, order)
