"""Pins for oracle.lpt and oracle.power."""
import math

import numpy as np
import pytest

from oracle import cosmology as C
from oracle import lpt, pm, power
from oracle.rng import white_noise
from paper_2010_11847_amd import inputs
from tests.realspace import grad4, solve_poisson_cg


def _wave_k(field):
    return np.fft.rfftn(field)


def test_lpt_matches_realspace_stencils():
    n = 12
    rng = np.random.default_rng(1)
    d = rng.normal(size=(n, n, n))
    d -= d.mean()
    s1, s2 = lpt.lpt_displacements(np.fft.rfftn(d), order=2)
    psi = solve_poisson_cg(d)
    for ax in range(3):
        np.testing.assert_allclose(s1[..., ax], -grad4(psi, ax), atol=1e-10)
    phi = {(i, j): grad4(grad4(psi, i), j) for i in range(3) for j in range(3)}
    d2 = (phi[0, 0] * phi[1, 1] + phi[0, 0] * phi[2, 2] + phi[1, 1] * phi[2, 2]
          - phi[0, 1] ** 2 - phi[0, 2] ** 2 - phi[1, 2] ** 2)
    psi2 = solve_poisson_cg(d2)
    for ax in range(3):
        np.testing.assert_allclose(s2[..., ax], grad4(psi2, ax), atol=1e-10 * np.abs(s2).max())


def test_single_plane_wave_has_no_second_order():
    n = 16
    x = np.arange(n)
    d = 0.3 * np.cos(2 * np.pi * 2 * x / n)[None, :, None] * np.ones((n, n, n))
    s1, s2 = lpt.lpt_displacements(_wave_k(d), order=2)
    assert np.abs(s2).max() < 1e-14
    w = 2 * np.pi * 2 / n
    ref = -0.3 * ((8 * math.sin(w) - math.sin(2 * w)) / 6) / (2 * math.sin(w / 2)) ** 2 * np.sin(w * x)
    np.testing.assert_allclose(s1[0, :, 0, 1], ref, atol=1e-13)


def test_two_orthogonal_waves_closed_form():
    n = 16
    x = np.arange(n)
    a, b, m = 0.2, 0.1, 1
    w = 2 * np.pi * m / n
    c = ((8 * math.sin(w) - math.sin(2 * w)) / 6) ** 2 / (2 * math.sin(w / 2)) ** 2
    cx = np.cos(w * x)[:, None, None]
    cy = np.cos(w * x)[None, :, None]
    d = (a * cx + b * cy) * np.ones((n, n, n))
    # phi_xx = -c a cos(wx), phi_yy = -c b cos(wy), mixed terms vanish
    d2 = (c * a * cx) * (c * b * cy) * np.ones((n, n, n))
    s1, s2 = lpt.lpt_displacements(_wave_k(d), order=2)
    _, s2_ref = None, None
    psi2 = solve_poisson_cg(d2)
    np.testing.assert_allclose(s2[..., 0], grad4(psi2, 0), atol=1e-12)
    np.testing.assert_allclose(s2[..., 1], grad4(psi2, 1), atol=1e-12)


def test_lpt_scaling_and_zero_mean():
    n = 16
    d = np.random.default_rng(2).normal(size=(n, n, n))
    dk = np.fft.rfftn(d)
    dk[0, 0, 0] = 0
    s1a, s2a = lpt.lpt_displacements(dk)
    s1b, s2b = lpt.lpt_displacements(3.0 * dk)
    np.testing.assert_allclose(s1b, 3 * s1a, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(s2b, 9 * s2a, rtol=1e-10, atol=1e-12)
    assert np.abs(s1a.sum((0, 1, 2))).max() < 1e-10
    assert np.abs(s2a.sum((0, 1, 2))).max() < 1e-10


def test_linear_field_fixed_amplitude_recovers_input_power_exactly():
    w = inputs.scaled(inputs.MEDIUM, 32, 32)
    noise = white_noise(w.seed, 32)
    dk = lpt.linear_field_k(noise, w.box_size, w.cosmo, fixed_amplitude=True)
    k, pk, nm = power.power_k(dk, w.box_size, 32)
    # expected: mode-weighted bin average of P(k_n), by an explicit mode loop
    n = 32
    acc = np.zeros(n // 2 + 1)
    wsum = np.zeros(n // 2 + 1)
    f = np.fft.fftfreq(n, 1 / n)
    for ix in f:
        for iy in f:
            for iz in range(n // 2 + 1):
                mag = math.sqrt(ix * ix + iy * iy + iz * iz)
                j = int(math.floor(mag + 0.5))
                if j < 1 or j > n // 2:
                    continue
                wt = 1.0 if iz in (0, n // 2) else 2.0
                acc[j] += wt * C.linear_power(np.array([2 * math.pi * mag / w.box_size]), w.cosmo)[0]
                wsum[j] += wt
    np.testing.assert_allclose(pk, acc[1:] / wsum[1:], rtol=1e-10)
    np.testing.assert_allclose(nm, wsum[1:])


def test_linear_field_random_power_within_cosmic_variance():
    w = inputs.scaled(inputs.MEDIUM, 64, 64)
    dk = lpt.linear_field_k(white_noise(5, 64), w.box_size, w.cosmo)
    k, pk, nm = power.power_k(dk, w.box_size, 64)
    ref = C.linear_power(k, w.cosmo)
    sel = nm > 200
    dev = (pk[sel] / ref[sel] - 1) / np.sqrt(2.0 / nm[sel])
    assert np.abs(dev).max() < 5.0
    assert abs(dev.mean()) < 1.5
    real = np.fft.irfftn(dk, s=(64, 64, 64), axes=(0, 1, 2))
    assert np.isrealobj(real)


def test_power_plane_wave_amplitude():
    n, m, amp, box = 32, 3, 0.7, 50.0
    x = np.arange(n)
    d = amp * np.cos(2 * np.pi * m * x / n)[:, None, None] * np.ones((n, n, n))
    k, pk, nm = power.power(d, box)
    expect = box ** 3 * amp ** 2 / (2 * nm[m - 1])
    assert pk[m - 1] == pytest.approx(expect, rel=1e-12)
    assert k[m - 1] == pytest.approx(2 * math.pi * m / box, rel=0.05)
    others = np.delete(pk, m - 1)
    assert np.abs(others).max() < 1e-20


def test_transfer_and_correlation_identities():
    d = np.random.default_rng(3).normal(size=(16, 16, 16))
    _, tf, rc = power.transfer_and_correlation(d, d, 100.0)
    np.testing.assert_allclose(tf, 1, rtol=1e-12)
    np.testing.assert_allclose(rc, 1, rtol=1e-12)
    _, tf, rc = power.transfer_and_correlation(2 * d, -d, 100.0)
    np.testing.assert_allclose(tf, 2, rtol=1e-12)
    np.testing.assert_allclose(rc, -1, rtol=1e-12)


def test_power_subcube_and_weights_by_explicit_full_spectrum_loop():
    """Brute force: every mode of the full complex spectrum (numpy's fftn, no
    half-spectrum weights) counted once, selected by |n_d| < n_max and binned
    by round(|n|), reproduces power()'s mode counts and band powers."""
    n, box = 12, 30.0
    d = np.random.default_rng(8).normal(size=(n, n, n))
    full = np.fft.fftn(d)
    freqs = [int(v) for v in np.fft.fftfreq(n, 1.0 / n)]
    for n_max in (0, 3, 4, 6):
        cnt = np.zeros(n // 2)
        acc = np.zeros(n // 2)
        for ix, fx in enumerate(freqs):
            for iy, fy in enumerate(freqs):
                for iz, fz in enumerate(freqs):
                    if n_max and not (abs(fx) < n_max and abs(fy) < n_max and abs(fz) < n_max):
                        continue
                    j = int(math.floor(math.sqrt(fx * fx + fy * fy + fz * fz) + 0.5))
                    if 1 <= j <= n // 2:
                        cnt[j - 1] += 1
                        acc[j - 1] += abs(full[ix, iy, iz]) ** 2
        k, pk, nm = power.power(d, box, n_max=n_max)
        np.testing.assert_array_equal(nm, cnt)
        sel = cnt > 0
        np.testing.assert_allclose(pk[sel], acc[sel] / cnt[sel] * box ** 3 / n ** 6, rtol=1e-12)
        assert np.all(np.isnan(pk[~sel]))


@pytest.mark.parametrize("m", [(3, 0, 0), (1, 2, 3), (5, 0, 6)])
def test_power_deconvolution_divides_a_plane_wave_by_the_window_squared(m):
    """A single plane wave: the CIC-deconvolved band power is the plain one
    divided by W^2, W = prod_d (sin(w_d/2)/(w_d/2))^2 at the wave's mode."""
    n, box = 16, 40.0
    g = np.arange(n)
    ph = 2 * np.pi * (m[0] * g[:, None, None] + m[1] * g[None, :, None] + m[2] * g[None, None, :]) / n
    d = 0.3 * np.cos(ph)
    _, p0, nm0 = power.power(d, box)
    _, p1, nm1 = power.power(d, box, deconvolve_cic=True)
    np.testing.assert_array_equal(nm0, nm1)
    j = int(math.floor(math.sqrt(sum(v * v for v in m)) + 0.5))
    win = 1.0
    for v in m:
        h = math.pi * v / n
        win *= (math.sin(h) / h) ** 2 if v else 1.0
    assert p1[j - 1] == pytest.approx(p0[j - 1] / win ** 2, rel=1e-12)
    assert p0[j - 1] > 0
