"""Binned power spectrum and two-point comparison statistics (float64).

Test infrastructure: see the package docstring.

Section 6.1 compares fields with the transfer function T_f = sqrt(P_a/P_b)
and the cross-correlation r_c = P_ab / sqrt(P_a P_b).  Estimator (a reading):
P(k_j) = (L^3/N^6) sum_w |delta^|^2 / sum_w over the half spectrum with mode
weight 2 on interior planes (0 < n_z < N/2) and 1 on the n_z = 0 and N/2
planes; bin j (j = 1..N/2) holds |n| in [j - 1/2, j + 1/2).
"""
from __future__ import annotations

import numpy as np

from .pm import omega_axes, cic_window


def _modes(n, n_max=0):
    nx = np.fft.fftfreq(n, 1.0 / n)
    nz = np.fft.rfftfreq(n, 1.0 / n)
    n2 = nx[:, None, None] ** 2 + nx[None, :, None] ** 2 + nz[None, None, :] ** 2
    w = np.full(n2.shape, 2.0)
    w[:, :, 0] = 1.0
    if n % 2 == 0:
        w[:, :, -1] = 1.0
    if n_max > 0:
        keep = ((np.abs(nx)[:, None, None] < n_max) & (np.abs(nx)[None, :, None] < n_max)
                & (np.abs(nz)[None, None, :] < n_max))
        w = np.where(keep, w, 0.0)
    return np.sqrt(n2), w


def cross_power(ak, bk, box_size, n, n_bins=None, n_max=0):
    """Binned Re(a^ b^*) -> (k_mean [h/Mpc], P [(Mpc/h)^3], N_modes)."""
    nb = n // 2 if n_bins is None else n_bins
    mag, w = _modes(n, n_max)
    j = np.floor(mag + 0.5).astype(np.int64)
    sel = (j >= 1) & (j <= nb) & (w > 0)
    j, ww, mm = j[sel], w[sel], mag[sel]
    p = np.real(ak[sel] * np.conj(bk[sel]))
    sw = np.bincount(j, ww, nb + 1)[1:]
    sp = np.bincount(j, ww * p, nb + 1)[1:]
    sk = np.bincount(j, ww * mm, nb + 1)[1:]
    with np.errstate(invalid="ignore", divide="ignore"):
        pk = sp / sw * box_size ** 3 / float(n) ** 6
        kk = sk / sw * 2 * np.pi / box_size
    return kk, pk, sw


def power(delta, box_size, n_bins=None, deconvolve_cic=False, n_max=0):
    """Auto power spectrum of a real mesh."""
    n = delta.shape[0]
    dk = np.fft.rfftn(np.asarray(delta, dtype=np.float64))
    if deconvolve_cic:
        dk = dk / cic_window(*omega_axes(n))
    return cross_power(dk, dk, box_size, n, n_bins, n_max)


def power_k(dk, box_size, n, n_bins=None, n_max=0):
    return cross_power(dk, dk, box_size, n, n_bins, n_max)


def transfer_and_correlation(a, b, box_size):
    """T_f = sqrt(P_a/P_b), r_c = P_ab / sqrt(P_a P_b) (section 6.1)."""
    n = a.shape[0]
    ak = np.fft.rfftn(np.asarray(a, dtype=np.float64))
    bk = np.fft.rfftn(np.asarray(b, dtype=np.float64))
    k, paa, _ = cross_power(ak, ak, box_size, n)
    _, pbb, _ = cross_power(bk, bk, box_size, n)
    _, pab, _ = cross_power(ak, bk, box_size, n)
    return k, np.sqrt(paa / pbb), pab / np.sqrt(paa * pbb)
