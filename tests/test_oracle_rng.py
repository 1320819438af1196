"""Pins for oracle.rng: published SplitMix64 outputs and Gaussian statistics."""
import numpy as np

from oracle import rng


def test_splitmix64_published_vectors():
    # Reference outputs of the SplitMix64 generator (Steele, Lea & Flood 2014):
    # state 0 -> first output; state 1234567 -> first five outputs.
    assert int(rng.splitmix64(np.uint64(0))) == 0xE220A8397B1DCDAF
    g = np.uint64(0x9E3779B97F4A7C15)
    with np.errstate(over="ignore"):
        out = [int(rng.splitmix64(np.uint64(1234567) + np.uint64(i) * g)) for i in range(5)]
    assert out == [6457827717110365317, 3203168211198807973, 9817491932198370423,
                   4593380528125082431, 16408922859458223821]


def test_counter_layout():
    b = rng.counter_bits(3, 10, 4)
    with np.errstate(over="ignore"):
        ref = rng.splitmix64(np.uint64(3) * np.uint64(1 << 40) + np.arange(10, 14, dtype=np.uint64))
    assert np.array_equal(b, ref)


def test_gaussian_moments():
    w = rng.white_noise(7, 64).ravel()
    n = w.size
    assert abs(w.mean()) < 5 / np.sqrt(n)
    assert abs(w.var() - 1) < 5 * np.sqrt(2 / n)
    assert abs((w ** 4).mean() - 3) < 5 * np.sqrt(96 / n)
    assert abs((w ** 3).mean()) < 5 * np.sqrt(15 / n)


def test_box_muller_extremes():
    bits = np.array([0, 0xFFFFFFFF00000000, 0x00000000FFFFFFFF], dtype=np.uint64)
    v = rng.box_muller(bits)
    assert np.all(np.isfinite(v))
    assert v[1] == 0.0                              # u1 = 1 -> radius 0
    assert abs(v[0] - np.sqrt(2 * 32 * np.log(2))) < 1e-12   # u1 = 2^-32, u2 = 0
