"""Pins for oracle.cosmology: closed forms, limits and exactness identities."""
import math

import numpy as np
import pytest

from oracle import cosmology as C
from paper_2010_11847_amd.inputs import Cosmology, POWERLAW

A = np.array([0.05, 0.1, 0.19, 0.37, 0.5, 0.82, 1.0])


@pytest.mark.parametrize("om", [0.3, 0.25, 0.8])
def test_growth_ode_matches_hypergeometric_and_heath(om):
    d_ode = C.D1(A, om)
    d_hyp = C.D1_hypergeometric(A, om)
    d_heath = C.D1_heath(A, om)
    np.testing.assert_allclose(d_ode, d_hyp, rtol=1e-10)
    np.testing.assert_allclose(d_ode, d_heath, rtol=1e-9)


def test_growth_rate_matches_closed_form_derivative():
    om = 0.3
    h = 1e-5
    for a in (0.1, 0.5, 1.0):
        lo, hi = C.D1_hypergeometric(a * math.exp(-h), om), C.D1_hypergeometric(a * math.exp(h), om)
        f_fd = float((math.log(hi[0]) - math.log(lo[0])) / (2 * h))
        assert abs(C.growth(a, om)[1][0] - f_fd) < 1e-8


def test_einstein_de_sitter_limits():
    om = 1.0
    d1, f1, d2, f2 = C.growth(A, om)
    np.testing.assert_allclose(d1, A, rtol=1e-10)
    np.testing.assert_allclose(f1, 1.0, rtol=1e-9)
    np.testing.assert_allclose(d2, -3.0 / 7.0 * A ** 2, rtol=1e-9)
    np.testing.assert_allclose(f2, 2.0, rtol=1e-9)
    np.testing.assert_allclose(C.G_f(A, om), A ** 1.5, rtol=1e-9)
    ai, aj = 0.3, 0.45
    ac = math.sqrt(ai * aj)
    assert C.drift_factor(ai, aj, ac, om) == pytest.approx((aj - ai) / ac ** 1.5, rel=1e-9)
    assert C.kick_factor(ai, aj, ai, om) == pytest.approx((aj ** 1.5 - ai ** 1.5) / (1.5 * ai), rel=1e-9)


def test_second_order_growth_matches_bouchet_fit():
    # Bouchet et al. (1995): D2 ~ -3/7 D1^2 Om(a)^(-1/143), accurate to ~0.1%.
    om = 0.3
    d1, _, d2, _ = C.growth(A, om)
    fit = -3.0 / 7.0 * d1 ** 2 * C.omega_m_a(A, om) ** (-1.0 / 143.0)
    np.testing.assert_allclose(d2, fit, rtol=2e-3)


def test_gf_identity():
    # a^2 E dG_f/da = 1.5 Om D1 (the growth ODE multiplied by a^3 E).
    om = 0.3
    for a in (0.1, 0.4, 1.0):
        h = 1e-6 * a
        dg = (C.G_f(a + h, om)[0] - C.G_f(a - h, om)[0]) / (2 * h)
        lhs = a ** 2 * float(C.hubble(a, om)) * dg
        assert lhs == pytest.approx(float(C.g_f(a, om)[0]), rel=1e-7)


def test_kdk_factors_reproduce_zeldovich_exactly():
    # Linear theory: x = q + D1 s, p = G_f s, F = g_f s = 1.5 Om (x - q).
    from oracle.pm import kdk_run
    om = 0.3
    rng = np.random.default_rng(0)
    q = 10 + rng.random((50, 3)) * 80
    s = rng.normal(0, 0.3, (50, 3))
    a_list = [0.1 + 0.09 * i for i in range(11)]
    x0 = q + C.D1(a_list[0], om)[0] * s
    p0 = C.G_f(a_list[0], om)[0] * s
    seen = []

    def cb(step, x, p, f):
        a = a_list[step + 1]
        np.testing.assert_allclose(x, q + C.D1(a, om)[0] * s, rtol=0, atol=1e-10)
        np.testing.assert_allclose(p, C.G_f(a, om)[0] * s, rtol=0, atol=1e-10)
        seen.append(step)

    kdk_run(x0, p0, a_list, 1000, 50, om, force_fn=lambda x: 1.5 * om * (x - q), callback=cb)
    assert seen == list(range(10))


def test_powerlaw_sigma8_closed_form():
    a_closed = C.powerlaw_amplitude_sigma8(POWERLAW)
    assert a_closed == pytest.approx(53.6165, rel=1e-5)
    s8 = C.sigma_r(lambda k: a_closed * k ** -2.0, 8.0)
    assert s8 == pytest.approx(0.8, rel=5e-5)   # quadrature truncated at k = 100 h/Mpc


def test_eh_nowiggle_limits_and_normalisation():
    cos = Cosmology()
    assert C.eh_nowiggle_transfer(np.array([1e-6]), cos)[0] == pytest.approx(1.0, abs=1e-4)
    t = C.eh_nowiggle_transfer(np.logspace(-4, 1, 200), cos)
    assert np.all(np.diff(t) < 0)
    s8 = C.sigma_r(lambda k: float(C.linear_power(np.array([k]), cos)[0]), 8.0)
    assert s8 == pytest.approx(0.8, rel=1e-8)
    # large-k slope of T0 approaches ln(q)/q^2
    k = np.array([50.0, 100.0])
    tk = C.eh_nowiggle_transfer(k, cos)
    assert -2.3 < np.log(tk[1] / tk[0]) / np.log(2.0) < -1.6


def test_table_power_is_exact_on_a_sampled_power_law():
    # log-log interpolation reproduces a power law at any k, extrapolation
    # beyond both ends included, so a sampled A k^-2 is the power law itself
    ks = np.logspace(-3, 0, 20)
    table = (tuple(ks), tuple(53.6 * ks ** -2.0))
    k = np.array([2e-4, 1e-3, 3.3e-3, 0.047, 0.5, 1.0, 7.5])
    np.testing.assert_allclose(C.table_power(k, table), 53.6 * k ** -2.0, rtol=1e-12)
    cos = Cosmology(pk_kind=2, pk_table=table)
    np.testing.assert_allclose(C.linear_power(k, cos), 53.6 * k ** -2.0, rtol=1e-12)   # amplitude 1
    assert C.linear_power(np.array([0.0]), cos)[0] == 0.0


def test_table_power_interpolates_between_points():
    # a kink between two points: the midpoint in ln k gets the geometric mean
    table = ((0.1, 1.0), (2.0, 8.0))
    np.testing.assert_allclose(C.table_power(np.array([math.sqrt(0.1)]), table), [4.0], rtol=1e-12)
