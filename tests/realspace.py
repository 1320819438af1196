"""Independent real-space operators used to pin the oracle's Fourier kernels.

The FD kernels of the paper's section 2 are the Fourier symbols of two
periodic stencils: the 7-point Laplacian (symbol -K^2) and the fourth-order
central difference [f(x-2) - 8 f(x-1) + 8 f(x+1) - f(x+2)] / 12 (symbol
i (8 sin w - sin 2w) / 6).  These helpers apply the stencils with np.roll and
solve the Poisson equation with conjugate gradients, never touching an FFT,
so they pin sign, factors, symbols and FFT layout of the oracle at once.
"""
import numpy as np


def lap7(f):
    out = -6.0 * f
    for ax in range(3):
        out += np.roll(f, 1, ax) + np.roll(f, -1, ax)
    return out


def grad4(f, ax):
    return (8.0 * (np.roll(f, -1, ax) - np.roll(f, 1, ax))
            - (np.roll(f, -2, ax) - np.roll(f, 2, ax))) / 12.0


def solve_poisson_cg(rhs, tol=1e-13, maxiter=5000):
    """Zero-mean solution of lap7(phi) = rhs - mean(rhs) by conjugate gradients."""
    b = -(rhs - rhs.mean())          # -lap7 is positive semi-definite
    x = np.zeros_like(b)
    r = b.copy()
    p = r.copy()
    rs = np.vdot(r, r)
    bn = np.sqrt(np.vdot(b, b)) + 1e-300
    for _ in range(maxiter):
        ap = -lap7(p)
        alpha = rs / np.vdot(p, ap)
        x += alpha * p
        r -= alpha * ap
        rs_new = np.vdot(r, r)
        if np.sqrt(rs_new) < tol * bn:
            break
        p = r + (rs_new / rs) * p
        rs = rs_new
    return x - x.mean()


def direct_paint(x, n):
    """Per-particle, per-corner loop (tiny inputs only)."""
    rho = np.zeros((n, n, n))
    for xp in np.asarray(x, dtype=np.float64):
        base = [int(np.floor(v)) for v in xp]
        for ox in (0, 1):
            for oy in (0, 1):
                for oz in (0, 1):
                    c = (base[0] + ox, base[1] + oy, base[2] + oz)
                    w = 1.0
                    for d in range(3):
                        w *= max(0.0, 1.0 - abs(xp[d] - c[d]))
                    rho[c[0] % n, c[1] % n, c[2] % n] += w
    return rho
