"""Run-level pins for the oracle: conservation laws and linear-theory growth."""
import math
from dataclasses import replace

import numpy as np
import pytest

from oracle import cosmology as C
from oracle import lpt, pm, power
from paper_2010_11847_amd import inputs


def test_momentum_conserved_through_run():
    w = inputs.scaled(inputs.SMALL, 16, 16, n_steps=4)
    x, p = lpt.generate(w)
    scale = np.abs(p).mean() * len(p)
    assert np.abs(p.sum(0)).max() < 1e-11 * scale

    def cb(step, x, p, f):
        assert np.abs(p.sum(0)).max() < 1e-11 * scale
        assert np.abs(f.sum(0)).max() < 1e-11 * np.abs(f).mean() * len(f)

    pm.kdk_run(x, p, w.a_list, w.n_mesh, w.n_particles, w.cosmo.omega_m, callback=cb)


def _fundamental_growth(n_part, n_mesh):
    base = inputs.scaled(inputs.SMALL, n_mesh, n_part, box_size=100.0)
    cos = replace(base.cosmo, pk_amp=C.powerlaw_amplitude_sigma8(base.cosmo) * 1e-4)
    w = replace(base, cosmo=cos)
    x0, p0 = lpt.generate(w)
    q = lpt.lattice(n_part, n_mesh // n_part)
    x1, _, _ = pm.kdk_run(x0, p0, w.a_list, n_mesh, w.n_particles, cos.omega_m)
    shape = (n_part,) * 3 + (3,)
    f0 = np.fft.rfftn(pm.min_image(x0 - q, n_mesh).reshape(shape), axes=(0, 1, 2))
    f1 = np.fft.rfftn(pm.min_image(x1 - q, n_mesh).reshape(shape), axes=(0, 1, 2))
    nx = np.fft.fftfreq(n_part, 1.0 / n_part)
    nz = np.fft.rfftfreq(n_part, 1.0 / n_part)
    sel = (nx[:, None, None] ** 2 + nx[None, :, None] ** 2 + nz[None, None, :] ** 2) == 1
    r = np.real((f1[sel] * np.conj(f0[sel])).sum()) / (np.abs(f0[sel]) ** 2).sum()
    return r / float((C.D1(1.0, cos.omega_m) / C.D1(0.1, cos.omega_m))[0]) - 1.0


def test_linear_growth_recovered_at_large_scales():
    # Displacements of the fundamental modes grow as D1(a) (linear theory) up
    # to the O(w^2) error of the FD kernels and CIC, which must shrink ~4x per
    # doubling of resolution at fixed box.
    assert float((C.D1(1.0, 0.3) / C.D1(0.1, 0.3))[0]) ** 2 == pytest.approx(60.73, rel=1e-3)
    e32 = _fundamental_growth(32, 32)
    e64 = _fundamental_growth(64, 64)
    assert abs(e32) < 0.015
    assert abs(e64) < 0.004
    assert abs(e64) < abs(e32) / 3


def test_zeldovich_pancake_before_shell_crossing():
    n, amp, om = 32, 0.02, 0.3
    q1 = np.arange(n)
    d = amp * np.cos(2 * np.pi * q1 / n)[:, None, None] * np.ones((n, n, n))
    s1, s2 = lpt.lpt_displacements(np.fft.rfftn(d), order=2)
    a_list = inputs.a_linear(0.1, 1.0, 10)
    # lattice at cell centres: the CIC deposit is then linear in the displacement
    x0, p0 = lpt.initial_state(s1, s2, a_list[0], n, om, shift=0.5)
    q = lpt.lattice(n, 1, 0.5)
    x1, _, _ = pm.kdk_run(x0, p0, a_list, n, n ** 3, om)
    disp0 = pm.min_image(x0 - q, n)[:, 0]
    disp1 = pm.min_image(x1 - q, n)[:, 0]
    growth = float((C.D1(1.0, om) / C.D1(0.1, om))[0])
    assert np.abs(disp1).max() < 0.5 * n / (2 * np.pi)         # still before shell crossing
    np.testing.assert_allclose(disp1, growth * disp0, atol=0.01 * np.abs(growth * disp0).max())
    assert np.abs(pm.min_image(x1 - q, n)[:, 1:]).max() < 1e-12
