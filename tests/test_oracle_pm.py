"""Pins for oracle.pm: paint, readout, force kernels and invariants."""
import math

import numpy as np
import pytest

from oracle import pm
from paper_2010_11847_amd import inputs
from tests.realspace import direct_paint, grad4, lap7, solve_poisson_cg

OM = 0.3


def test_paint_matches_direct_loop():
    x = inputs.uniform_positions(40, 6, seed=1).astype(np.float64)
    x[0] = [5.999, 0.0, 3.5]          # wraps in x
    np.testing.assert_allclose(pm.paint(x, 6), direct_paint(x, 6), atol=1e-13)


def test_paint_conserves_mass_and_deposits_nodes():
    x = inputs.clustered_positions(5000, 16, seed=2)
    rho = pm.paint(x, 16)
    assert rho.sum() == pytest.approx(5000.0, rel=1e-12)
    assert rho.min() >= 0
    nodes = np.array([[0, 0, 0], [3, 15, 7], [3, 15, 7]], dtype=np.float64)
    r = pm.paint(nodes, 16)
    assert r[0, 0, 0] == 1.0 and r[3, 15, 7] == 2.0 and r.sum() == 3.0


def test_paint_integer_shift_rolls_mesh():
    x = inputs.uniform_positions(300, 8, seed=3).astype(np.float64)
    shift = np.array([3, 5, 7])
    a = pm.paint(x, 8)
    b = pm.paint((x + shift) % 8, 8)
    np.testing.assert_allclose(np.roll(a, tuple(shift), (0, 1, 2)), b, atol=1e-12)


def test_readout_is_transpose_of_paint():
    rng = np.random.default_rng(4)
    x = inputs.clustered_positions(700, 12, seed=4).astype(np.float64)
    m = rng.normal(size=700)
    g = rng.normal(size=(12, 12, 12))
    lhs = np.vdot(pm.paint(x, 12, mass=m), g)
    rhs = np.vdot(m, pm.readout(g, x))
    assert lhs == pytest.approx(rhs, rel=1e-12)


def test_readout_reproduces_trilinear_function():
    n = 16
    c = np.arange(n, dtype=np.float64)
    X, Y, Z = np.meshgrid(c, c, c, indexing="ij")
    f = 1.0 + 0.5 * X - 0.25 * Y + 0.125 * Z + 0.01 * X * Y * Z
    x = 1 + np.random.default_rng(5).random((100, 3)) * 13   # away from the periodic seam
    exact = 1.0 + 0.5 * x[:, 0] - 0.25 * x[:, 1] + 0.125 * x[:, 2] + 0.01 * x.prod(1)
    np.testing.assert_allclose(pm.readout(f, x), exact, rtol=1e-12)


@pytest.mark.parametrize("n", [8, 16])
def test_force_mesh_matches_realspace_poisson_and_stencil(n):
    # F = -grad4(phi) with lap7(phi) = 1.5 Om delta, solved with CG in real space.
    delta = np.random.default_rng(6 + n).normal(size=(n, n, n))
    delta -= delta.mean()
    phi = solve_poisson_cg(1.5 * OM * delta)
    ref = [-grad4(phi, ax) for ax in range(3)]
    got = pm.force_meshes(delta, OM)
    for g, r in zip(got, ref):
        np.testing.assert_allclose(g, r, atol=1e-10 * np.abs(r).max())


def test_force_mesh_matches_brute_force_dft_8():
    n = 8
    rng = np.random.default_rng(8)
    delta = rng.normal(size=(n, n, n))
    idx = np.arange(n)
    e = np.exp(-2j * np.pi * np.outer(idx, idx) / n)
    # full-spectrum DFT by explicit summation over each axis
    dk = np.einsum("ax,by,cz,xyz->abc", e, e, e, delta)
    w = 2 * np.pi * np.fft.fftfreq(n)
    wx, wy, wz = w[:, None, None], w[None, :, None], w[None, None, :]
    k2 = (2 * np.sin(wx / 2)) ** 2 + (2 * np.sin(wy / 2)) ** 2 + (2 * np.sin(wz / 2)) ** 2
    inv = np.where(k2 > 0, 1 / np.where(k2 > 0, k2, 1), 0)
    einv = np.conj(e) / n
    got = pm.force_meshes(delta, OM)
    for g, wd in zip(got, (wx, wy, wz)):
        fk = 1.5 * OM * 1j * (8 * np.sin(wd) - np.sin(2 * wd)) / 6 * inv * dk
        ref = np.einsum("xa,yb,zc,abc->xyz", einv, einv, einv, fk)
        np.testing.assert_allclose(g, ref.real, atol=1e-12)
        assert np.abs(ref.imag).max() < 1e-12


def test_plane_wave_force_continuum_limit():
    n, m, amp = 64, 1, 0.01
    x = np.arange(n)
    delta = amp * np.cos(2 * np.pi * m * x / n)[:, None, None] * np.ones((n, n, n))
    fx, fy, fz = pm.force_meshes(delta, OM)
    k = 2 * np.pi * m / n
    cont = -1.5 * OM * amp / k * np.sin(k * x)   # attractive: F = -grad phi, lap phi = 1.5 Om delta
    np.testing.assert_allclose(fx[:, 3, 5], cont, atol=2e-3 * np.abs(cont).max())
    assert np.abs(fy).max() < 1e-14 and np.abs(fz).max() < 1e-14


def test_self_force_zero_and_momentum_conservation():
    for x in (np.array([[3.3, 7.71, 1.05]]), inputs.clustered_positions(2000, 16, seed=9)):
        f = pm.force(x, 16, len(x), OM)
        scale = 1.5 * OM * 16 ** 3 / len(x)
        assert np.abs(f.sum(0)).max() < 1e-12 * scale * len(x)
        if len(x) == 1:
            assert np.abs(f).max() < 1e-13 * scale


@pytest.mark.parametrize("r", [6.0, 8.0])
def test_two_particle_inverse_square_law(r):
    n = 128
    x = np.array([[40.3, 50.2, 60.1], [40.3 + r, 50.2, 60.1]])
    f = pm.force(x, n, 2, OM)
    nbar = 2.0 / n ** 3
    expect = 1.5 * OM / (4 * np.pi * nbar * r ** 2)
    assert f[0, 0] > 0 and f[1, 0] < 0                 # attraction
    assert f[0, 0] == pytest.approx(expect, rel=0.05)
    assert abs(f[0, 1]) < 0.02 * expect


def test_cic_window_is_triangle_transform():
    from scipy.integrate import quad
    for w in (0.3, 1.1, 2.7):
        ref = quad(lambda t: (1 - abs(t)) * math.cos(w * t), -1, 1)[0]
        assert float(pm.cic_window(np.array(w), np.array(0.0), np.array(0.0))) == pytest.approx(ref, rel=1e-10)


def test_split_parts_sum_to_full_force():
    n = 16
    delta = np.random.default_rng(10).normal(size=(n, n, n))
    full = pm.force_meshes(delta, OM)
    lo = pm.force_meshes(delta, OM, split_rs=1.5, split_mode=pm.SPLIT_LONG)
    hi = pm.force_meshes(delta, OM, split_rs=1.5, split_mode=pm.SPLIT_SHORT)
    for a, b, c in zip(full, lo, hi):
        np.testing.assert_allclose(b + c, a, atol=1e-12)
    # long part equals the full force on a long-wavelength field
    x = np.arange(n)
    wave = np.cos(2 * np.pi * x / n)[:, None, None] * np.ones((n, n, n))
    f = pm.force_meshes(wave, OM)[0]
    fl = pm.force_meshes(wave, OM, split_rs=0.2, split_mode=pm.SPLIT_LONG)[0]
    np.testing.assert_allclose(fl, f * math.exp(-(2 * np.pi / n) ** 2 * 0.04), atol=1e-12)


def test_deconvolution_divides_by_window():
    n = 16
    x = np.arange(n)
    m = 3
    wave = np.cos(2 * np.pi * m * x / n)[:, None, None] * np.ones((n, n, n))
    f0 = pm.force_meshes(wave, OM)[0]
    f2 = pm.force_meshes(wave, OM, deconv_order=2)[0]
    w = 2 * np.pi * m / n
    win = (math.sin(w / 2) / (w / 2)) ** 2
    np.testing.assert_allclose(f2, f0 / win ** 2, atol=1e-12)
