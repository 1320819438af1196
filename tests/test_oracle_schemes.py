"""Pins of the oracle's other time-stepping schemes (oracle/schemes.py):
closed forms of the leapfrog factors in Einstein-de Sitter, the LPT force as
the time derivative of the LPT momentum, exactness of the LPT-frame scheme
on a Zel'dovich trajectory, second-order convergence of the leapfrog, and
agreement of every scheme with FastPM's at many steps."""
import math

import numpy as np
import pytest

from oracle import cosmology as cm
from oracle import lpt, pm
from oracle import schemes as S
from paper_2010_11847_amd import inputs


def test_leapfrog_factors_closed_form_eds():
    # Omega_m = 1: E = a^-3/2, int da a^-1/2 and int da a^-3/2
    for ai, aj in [(0.1, 0.2), (0.3, 1.0), (0.05, 0.051)]:
        assert S.std_kick(ai, aj, 1.0) == pytest.approx(2 * (math.sqrt(aj) - math.sqrt(ai)), rel=1e-12)
        assert S.std_drift(ai, aj, 1.0) == pytest.approx(2 * (1 / math.sqrt(ai) - 1 / math.sqrt(aj)), rel=1e-12)


def test_leapfrog_factors_lcdm_by_simpson():
    a = np.linspace(0.2, 0.7, 20001)
    e = cm.hubble(a, 0.3)
    h = a[1] - a[0]

    def simpson(y):
        return h / 3 * (y[0] + y[-1] + 4 * y[1:-1:2].sum() + 2 * y[2:-1:2].sum())
    assert S.std_kick(0.2, 0.7, 0.3) == pytest.approx(simpson(1 / (a * a * e)), rel=1e-10)
    assert S.std_drift(0.2, 0.7, 0.3) == pytest.approx(simpson(1 / (a ** 3 * e)), rel=1e-10)


@pytest.mark.parametrize("a", [0.1, 0.37, 1.0])
def test_lpt_force_is_the_derivative_of_the_lpt_momentum(a):
    """F_LPT = a^2 E dp_LPT/da, coefficient by coefficient (central
    differences of the momentum coefficients)."""
    om, h = 0.3, 1e-5 * a
    dq = [(u - v) / (2 * h) for u, v in zip(S.lpt_momentum_coeffs(a + h, om), S.lpt_momentum_coeffs(a - h, om))]
    e = float(cm.hubble(a, om))
    c1, c2 = S.lpt_force_coeffs(a, om)
    assert a * a * e * dq[0] == pytest.approx(c1, rel=1e-7)
    assert a * a * e * dq[1] == pytest.approx(c2, rel=1e-7)
    # and the momentum coefficients are a^3 E times the growth rates dD/da
    d1 = lambda b: float(cm.growth(b, om)[0][0])  # noqa: E731
    d2 = lambda b: float(cm.growth(b, om)[2][0])  # noqa: E731
    q1, q2 = S.lpt_momentum_coeffs(a, om)
    assert q1 == pytest.approx(a ** 3 * e * (d1(a + h) - d1(a - h)) / (2 * h), rel=1e-7)
    assert q2 == pytest.approx(a ** 3 * e * (d2(a + h) - d2(a - h)) / (2 * h), rel=1e-7)


def _zeldovich_setup(n=64, amp=0.3, seed=3):
    """1D-like Zel'dovich flow: particles at q with displacements D1 Psi1,
    Psi1 along x only, and the exact force of a one-dimensional flow before
    shell crossing, F = 1.5 Omega_m (x - q) (Gauss's law in 1D)."""
    rng = np.random.default_rng(seed)
    q = rng.random((n, 3)) * 32.0
    psi1 = np.zeros((n, 3))
    psi1[:, 0] = amp * np.sin(2 * np.pi * q[:, 0] / 32.0) * 10
    return q, psi1


@pytest.mark.parametrize("steps", [1, 3])
def test_lpt_frame_scheme_exact_on_zeldovich(steps):
    om = 0.3
    q, psi1 = _zeldovich_setup()
    psi2 = np.zeros_like(psi1)
    force = lambda x: 1.5 * om * (x - q)  # noqa: E731  (no wrap: displacements stay inside)
    a_list = inputs.a_linear(0.1, 1.0, steps)
    d0 = float(cm.D1(a_list[0], om)[0])
    q1, _ = S.lpt_momentum_coeffs(a_list[0], om)
    x0, p0 = q + d0 * psi1, q1 * psi1
    x, p, f = S.cola_run(x0, p0, psi1, psi2, a_list, 10 ** 6, 1, om, force_fn=force)
    d1 = float(cm.D1(1.0, om)[0])
    q1e, _ = S.lpt_momentum_coeffs(1.0, om)
    np.testing.assert_allclose(x, q + d1 * psi1, rtol=0, atol=1e-10)
    np.testing.assert_allclose(p, q1e * psi1, rtol=0, atol=1e-10)
    # the plain leapfrog is not exact on it at a few steps, FastPM's scheme is
    xl, _, _ = S.leapfrog_run(x0, p0, a_list, 10 ** 6, 1, om, force_fn=force)
    xf, _, _ = pm.kdk_run(x0, p0, a_list, 10 ** 6, 1, om, force_fn=force)
    assert np.abs(xl - (q + d1 * psi1)).max() > 1e-3
    np.testing.assert_allclose(xf, q + d1 * psi1, rtol=0, atol=1e-9)


def test_leapfrog_converges_at_second_order():
    om = 0.3
    q, psi1 = _zeldovich_setup()
    force = lambda x: 1.5 * om * (x - q)  # noqa: E731
    d0 = float(cm.D1(0.1, om)[0])
    q1, _ = S.lpt_momentum_coeffs(0.1, om)
    x0, p0 = q + d0 * psi1, q1 * psi1
    exact = q + float(cm.D1(1.0, om)[0]) * psi1
    errs = []
    for steps in (8, 16, 32):
        x, _, _ = S.leapfrog_run(x0, p0, inputs.a_linear(0.1, 1.0, steps), 10 ** 6, 1, om, force_fn=force)
        errs.append(np.abs(x - exact).max())
    assert 3.3 < errs[0] / errs[1] < 4.7 and 3.3 < errs[1] / errs[2] < 4.7, errs


def test_schemes_agree_with_fastpm_at_many_steps():
    """On a 16^3 PM run from 2LPT initial conditions (strong second-order
    fields), the LPT-frame scheme and the leapfrog reach FastPM's trajectory
    as the steps grow; at 3 steps the LPT-frame scheme is the closer one."""
    w = inputs.scaled(inputs.SMALL, 16, 16, box_size=40.0)
    x0, p0 = lpt.generate(w)
    psi1, psi2 = S.displacement_fields(w)
    assert np.abs(psi2).max() > 1e-3 * np.abs(psi1).max()
    om = w.cosmo.omega_m

    def runs(steps):
        a = inputs.a_linear(0.1, 1.0, steps)
        xf, _, _ = pm.kdk_run(x0, p0, a, 16, w.n_particles, om)
        xc, pc, _ = S.cola_run(x0, p0, psi1, psi2, a, 16, w.n_particles, om)
        xl, _, _ = S.leapfrog_run(x0, p0, a, 16, w.n_particles, om)
        return xf, xc, xl, pc
    ref, _, _, _ = runs(160)

    def dist(x):
        d = pm.min_image(x - ref, 16)
        return float(np.sqrt((d ** 2).sum(1).mean()))
    xf, xc, xl, _ = runs(80)
    assert dist(xf) < 2e-3 and dist(xc) < 2e-3 and dist(xl) < 2e-3
    xf3, xc3, xl3, _ = runs(3)
    assert dist(xc3) < dist(xl3)


def test_lpt_frame_initial_state_round_trip():
    """With zero steps of residual motion the scheme returns the LPT state:
    p_LPT from the displacement fields equals Gen-IC's momenta."""
    w = inputs.scaled(inputs.SMALL, 16, 8, box_size=50.0)
    x0, p0 = lpt.generate(w)
    psi1, psi2 = S.displacement_fields(w)
    q1, q2 = S.lpt_momentum_coeffs(w.a_list[0], w.cosmo.omega_m)
    np.testing.assert_allclose(p0, q1 * psi1 + q2 * psi2, rtol=1e-12, atol=1e-14)
    d1, _, d2, _ = (float(v[0]) for v in cm.growth(w.a_list[0], w.cosmo.omega_m))
    qlat = lpt.lattice(w.n_part, w.n_mesh // w.n_part)
    d = pm.min_image(x0 - (qlat + d1 * psi1 + d2 * psi2), w.n_mesh)
    assert np.abs(d).max() < 1e-12
