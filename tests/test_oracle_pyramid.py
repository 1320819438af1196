"""Pins for oracle.pyramid: the B-spline kernel against its binomial closed
form, the separable strided convolution against a brute-force 3-D one,
constants, the transpose relation of EXPAND and REDUCE, the filter's
transfer function on plane waves, and the paper's claim that the pyramid
force stays within a percent of the single-grid force."""
import itertools
from math import comb

import numpy as np
import pytest

from oracle import pm, pyramid as P
from paper_2010_11847_amd import inputs

OM = 0.3


def test_bspline_kernel_is_binomial():
    k = P.bspline_kernel(6)
    np.testing.assert_allclose(k, [comb(6, i) / 64.0 for i in range(7)], rtol=0, atol=1e-16)
    assert k.sum() == pytest.approx(1.0, abs=1e-15)
    np.testing.assert_array_equal(k, k[::-1])


def test_reduce_matches_brute_force_3d_strided_convolution():
    rng = np.random.default_rng(0)
    a = rng.normal(size=(8, 8, 8))
    k1 = P.bspline_kernel(6)
    k3 = np.einsum("i,j,k->ijk", k1, k1, k1)
    ref = np.zeros((4, 4, 4))
    for i, j, l in itertools.product(range(4), repeat=3):
        for t, u, v in itertools.product(range(7), repeat=3):
            ref[i, j, l] += k3[t, u, v] * a[(2 * i + t - 3) % 8, (2 * j + u - 3) % 8, (2 * l + v - 3) % 8]
    np.testing.assert_allclose(P.reduce_field(a, levels=1), ref, rtol=1e-13, atol=1e-14)


def test_reduce_and_expand_keep_constants():
    c = np.full((16, 16, 16), 2.5)
    np.testing.assert_allclose(P.reduce_field(c, 2), np.full((4, 4, 4), 2.5), rtol=1e-14)
    np.testing.assert_allclose(P.expand_field(np.full((4, 4, 4), 2.5), 2), c, rtol=1e-14)


@pytest.mark.parametrize("levels", [1, 2])
def test_expand_is_8_to_the_levels_times_reduce_transpose(levels):
    rng = np.random.default_rng(levels)
    x = rng.normal(size=(16 >> levels,) * 3)
    y = rng.normal(size=(16, 16, 16))
    lhs = np.sum(P.expand_field(x, levels) * y)
    rhs = 8.0 ** levels * np.sum(x * P.reduce_field(y, levels))
    assert lhs == pytest.approx(rhs, rel=1e-12)


@pytest.mark.parametrize("axis,m", [(0, 1), (1, 2), (2, 3)])
def test_reduce_transfer_function_on_plane_waves(axis, m):
    # one level on cos(w x): the symmetric binomial kernel of order 6 has
    # response cos(w/2)^6, so the coarse samples are cos(w 2i) cos(w/2)^6
    n = 32
    w = 2 * np.pi * m / n
    idx = np.arange(n)
    shape = [1, 1, 1]
    shape[axis] = n
    f = np.broadcast_to(np.cos(w * idx).reshape(shape), (n, n, n))
    r = P.reduce_field(f, levels=1)
    shape[axis] = n // 2
    expect = np.broadcast_to((np.cos(w * 2 * np.arange(n // 2)) * np.cos(w / 2) ** 6).reshape(shape), r.shape)
    np.testing.assert_allclose(r, expect, atol=1e-13)


def test_pyramid_force_is_within_a_percent_of_single_grid():
    # clustered particles on a 64^3 mesh
    x = inputs.clustered_positions(20000, 64, seed=4).astype(np.float64)
    single = pm.force(x, 64, len(x), OM)
    pyr = P.force(x, 64, len(x), OM, levels=2)
    err = np.linalg.norm(pyr - single) / np.linalg.norm(single)
    assert err < 1e-2
    # and it is not the single-grid force itself: the long-range part differs
    assert err > 1e-6


@pytest.mark.parametrize("levels", [1, 2])
def test_pyramid_force_transpose_dot_product(levels):
    # sum_d <F_d(delta), m_d> = <delta, F^T(m)> for the pyramid force meshes
    rng = np.random.default_rng(10 + levels)
    n = 32
    delta = rng.normal(size=(n, n, n))
    m = [rng.normal(size=(n, n, n)) for _ in range(3)]
    lhs = sum(np.sum(f * mm) for f, mm in zip(P.force_meshes(delta, OM, levels), m))
    rhs = np.sum(delta * P.force_meshes_T(m, OM, levels))
    assert lhs == pytest.approx(rhs, rel=1e-11)


def test_pyramid_force_vjp_matches_fd():
    from oracle import adjoint as A
    n = 32
    x = inputs.clustered_positions(300, n, seed=5).astype(np.float64)
    rng = np.random.default_rng(5)
    fb = rng.normal(size=x.shape)
    v = rng.normal(size=x.shape)
    lhs = np.sum(A.force_vjp(x, n, 300, OM, fb, pyramid_levels=2) * v)
    f = lambda y: P.force(y, n, 300, OM, levels=2)
    rhs = np.sum(fb * (f(x + 1e-7 * v) - f(x - 1e-7 * v)) / 2e-7)
    assert lhs == pytest.approx(rhs, rel=1e-5)
