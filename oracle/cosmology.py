"""Background cosmology, growth and FastPM time-step factors (float64).

Test infrastructure: see the package docstring.

Units: H0 = 1, the scale factor a is the time variable, lengths in mesh cells
for the dynamics (the box size only enters the power spectrum).

The paper's kick/drift operators (section 2, the pair of update equations)
are the FastPM ones, which the paper only cites.  They are *derived* here from
the equations of motion

    dx/da = p / (a^3 E(a)),     dp/da = F / (a^2 E(a)),

with F = -1.5 Omega_m grad(lap^-1 delta) (the transfer function of the force
equation in section 2), by requiring the Zel'dovich (linear) solution to be
reproduced exactly:

    drift(ai -> aj; ac) = [D1(aj) - D1(ai)] / G_f(ac),   G_f = a^3 E dD1/da
    kick (ai -> aj; ar) = [G_f(aj) - G_f(ai)] / g_f(ar), g_f = a^2 E dG_f/da
                                                        = 1.5 Omega_m D1.
"""
from __future__ import annotations

import math
from functools import lru_cache

import numpy as np
from scipy.integrate import quad, solve_ivp

A_INIT = 1e-5


def hubble(a, omega_m):
    """E(a) = H(a)/H0 for flat LCDM without radiation."""
    a = np.asarray(a, dtype=np.float64)
    return np.sqrt(omega_m / a ** 3 + (1.0 - omega_m))


def dlnE_dlna(a, omega_m):
    a = np.asarray(a, dtype=np.float64)
    return -1.5 * omega_m / a ** 3 / hubble(a, omega_m) ** 2


def omega_m_a(a, omega_m):
    a = np.asarray(a, dtype=np.float64)
    return omega_m / a ** 3 / hubble(a, omega_m) ** 2


@lru_cache(maxsize=64)
def _growth_solution(omega_m: float):
    """Integrate the first- and second-order growth ODEs in ln a.

    With ' = d/dln a:
      D1'' + (2 + dlnE/dlna) D1' - 1.5 Om(a) D1 = 0
      D2'' + (2 + dlnE/dlna) D2' - 1.5 Om(a) D2 = -1.5 Om(a) D1^2
    started in the matter era where D1 = a and D2 = -3/7 a^2.
    """
    def rhs(lna, y):
        a = math.exp(lna)
        c = 2.0 + float(dlnE_dlna(a, omega_m))
        om = float(omega_m_a(a, omega_m))
        d1, d1p, d2, d2p = y
        return [d1p, -c * d1p + 1.5 * om * d1,
                d2p, -c * d2p + 1.5 * om * d2 - 1.5 * om * d1 * d1]

    a0 = A_INIT
    y0 = [a0, a0, -3.0 / 7.0 * a0 ** 2, -6.0 / 7.0 * a0 ** 2]
    sol = solve_ivp(rhs, (math.log(a0), math.log(4.0)), y0, method="DOP853",
                    rtol=1e-13, atol=1e-30, dense_output=True)
    y1 = sol.sol(0.0)
    return sol.sol, float(y1[0])


def growth(a, omega_m):
    """Return (D1, f1, D2, f2) at a, with D1(1) = 1 and D2 scaled by D1(1)^2.

    f_i = dln D_i / dln a.
    """
    sol, d1_today = _growth_solution(float(omega_m))
    a = np.atleast_1d(np.asarray(a, dtype=np.float64))
    y = sol(np.log(a))
    d1 = y[0] / d1_today
    f1 = y[1] / y[0]
    d2 = y[2] / d1_today ** 2
    f2 = y[3] / y[2]
    return d1, f1, d2, f2


def D1(a, omega_m):
    return growth(a, omega_m)[0]


def G_f(a, omega_m):
    """a^3 E dD1/da = a^2 E f1 D1."""
    d1, f1, _, _ = growth(a, omega_m)
    a = np.atleast_1d(np.asarray(a, dtype=np.float64))
    return a ** 2 * hubble(a, omega_m) * f1 * d1


def g_f(a, omega_m):
    """a^2 E dG_f/da, equal to 1.5 Omega_m D1 by the growth equation."""
    return 1.5 * omega_m * D1(a, omega_m)


def drift_factor(ai, aj, ac, omega_m):
    """Position update per unit momentum, drift from ai to aj with p known at ac."""
    return float((D1(aj, omega_m) - D1(ai, omega_m))[0] / G_f(ac, omega_m)[0])


def kick_factor(ai, aj, ar, omega_m):
    """Momentum update per unit force, kick from ai to aj with F evaluated at ar."""
    return float((G_f(aj, omega_m) - G_f(ai, omega_m))[0] / g_f(ar, omega_m)[0])


def half_step(ai, aj):
    """Staggered half-step time of the leapfrog (geometric mean; a reading)."""
    return math.sqrt(ai * aj)


# ---- independent closed forms (used only as pins) -------------------------

def D1_hypergeometric(a, omega_m):
    """Flat LCDM linear growth a 2F1(1/3, 1; 11/6; -a^3 (1-Om)/Om), normalised."""
    from scipy.special import hyp2f1
    a = np.atleast_1d(np.asarray(a, dtype=np.float64))
    r = (1.0 - omega_m) / omega_m
    g = a * hyp2f1(1.0 / 3.0, 1.0, 11.0 / 6.0, -a ** 3 * r)
    return g / (1.0 * hyp2f1(1.0 / 3.0, 1.0, 11.0 / 6.0, -r))


def D1_heath(a, omega_m):
    """Heath (1977) integral D1 propto E(a) int_0^a da'/(a' E(a'))^3, normalised."""
    def raw(x):
        val = quad(lambda t: 1.0 / (t * hubble(t, omega_m)) ** 3, 0.0, x,
                   epsabs=0, epsrel=1e-13, limit=200)[0]
        return float(hubble(x, omega_m)) * val
    a = np.atleast_1d(np.asarray(a, dtype=np.float64))
    return np.array([raw(x) for x in a]) / raw(1.0)


# ---- linear power spectrum -------------------------------------------------

def tophat_window(x):
    x = np.asarray(x, dtype=np.float64)
    out = np.empty_like(x)
    small = np.abs(x) < 1e-3
    xs = x[small]
    out[small] = 1.0 - xs ** 2 / 10.0 + xs ** 4 / 280.0
    xl = x[~small]
    out[~small] = 3.0 * (np.sin(xl) - xl * np.cos(xl)) / xl ** 3
    return out


def eh_nowiggle_transfer(k, cosmo):
    """Eisenstein & Hu (1998) zero-baryon-wiggle transfer function T0(k).

    k in h/Mpc.  Sound horizon fit s, shape suppression alpha_Gamma, effective
    shape Gamma_eff(k), and T0(q) = L0 / (L0 + C0 q^2).

    Parity unpinned beyond its limits: the tests pin T0 -> 1 as k -> 0, the
    monotone fall-off and the sigma8 normalisation of the resulting P(k); the
    fitting formula's intermediate values have no independent source here
    (the paper names no linear P(k); this spectrum stands in for it).
    """
    k = np.asarray(k, dtype=np.float64)
    om, ob, h = cosmo.omega_m, cosmo.omega_b, cosmo.h
    omh2, obh2 = om * h * h, ob * h * h
    fb = ob / om
    theta = cosmo.t_cmb / 2.7
    s = 44.5 * np.log(9.83 / omh2) / np.sqrt(1.0 + 10.0 * obh2 ** 0.75)   # Mpc
    alpha = 1.0 - 0.328 * np.log(431.0 * omh2) * fb + 0.38 * np.log(22.3 * omh2) * fb * fb
    gamma_eff = om * h * (alpha + (1.0 - alpha) / (1.0 + (0.43 * k * h * s) ** 4))
    q = k * theta * theta / gamma_eff
    L0 = np.log(2.0 * math.e + 1.8 * q)
    C0 = 14.2 + 731.0 / (1.0 + 62.5 * q)
    return L0 / (L0 + C0 * q * q)


def table_power(k, table):
    """A caller's tabulated P(k), interpolated linearly in (ln k, ln P); beyond
    the first or last point the end segment's line continues."""
    lk = np.log(np.asarray(table[0], dtype=np.float64))
    lp = np.log(np.maximum(np.asarray(table[1], dtype=np.float64), 1e-300))
    x = np.log(np.asarray(k, dtype=np.float64))
    i = np.clip(np.searchsorted(lk, x, side="right"), 1, len(lk) - 1)
    t = (x - lk[i - 1]) / (lk[i] - lk[i - 1])
    return np.exp(lp[i - 1] + t * (lp[i] - lp[i - 1]))


def _pk_shape(k, cosmo):
    k = np.asarray(k, dtype=np.float64)
    if cosmo.pk_kind == 0:
        return k ** cosmo.pk_index
    if cosmo.pk_kind == 1:
        return k ** cosmo.n_s * eh_nowiggle_transfer(k, cosmo) ** 2
    if cosmo.pk_kind == 2:
        return table_power(k, cosmo.pk_table)
    raise ValueError("unsupported pk_kind for the oracle")


def sigma_r(shape, r):
    """sigma(R)^2 = 1/(2 pi^2) int k^2 P(k) W(kR)^2 dk, integrated in ln k."""
    def integrand(lnk):
        k = math.exp(lnk)
        return k ** 3 * float(shape(k)) * float(tophat_window(np.array([k * r]))[0]) ** 2
    lo, hi = math.log(1e-5), math.log(1e2)
    edges = np.linspace(lo, hi, 57)
    tot = 0.0
    for a0, a1 in zip(edges[:-1], edges[1:]):
        tot += quad(integrand, a0, a1, epsabs=0, epsrel=1e-10, limit=400)[0]
    return math.sqrt(tot / (2.0 * math.pi ** 2))


def powerlaw_amplitude_sigma8(cosmo, r=8.0):
    """Closed form for P = A k^n with n = -2: A = sigma8^2 2 pi^2 R / (3 pi / 5)."""
    if cosmo.pk_index != -2.0:
        raise ValueError("closed form only for n = -2")
    return cosmo.sigma8 ** 2 * 2.0 * math.pi ** 2 * r / (3.0 * math.pi / 5.0)


@lru_cache(maxsize=64)
def pk_amplitude(cosmo):
    """Amplitude A so that sigma8 of the linear P(k) at a = 1 matches cosmo.sigma8."""
    if cosmo.pk_amp > 0:
        return float(cosmo.pk_amp)
    if cosmo.pk_kind == 2:   # a table is taken as given
        return 1.0
    if cosmo.pk_kind == 0 and cosmo.pk_index == -2.0:
        return powerlaw_amplitude_sigma8(cosmo)
    s = sigma_r(lambda k: _pk_shape(k, cosmo), 8.0)
    return (cosmo.sigma8 / s) ** 2


def linear_power(k, cosmo):
    """Linear P(k) at a = 1 in (Mpc/h)^3, k in h/Mpc; P(0) = 0."""
    k = np.asarray(k, dtype=np.float64)
    out = np.zeros_like(k)
    nz = k > 0
    out[nz] = pk_amplitude(cosmo) * _pk_shape(k[nz], cosmo)
    return out
