"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Tolerances: relative 1e-5 (norm-wise) on painted density
and forces per step, positions rms < 1e-3 cell after a full run.  FFTs and
spectra are compared at the float32 rounding level of the transform.
"""
from dataclasses import replace

import numpy as np
import pytest
import torch

from oracle import cosmology, lpt, pm, power
from oracle.rng import white_noise
from paper_2010_11847_amd import inputs
from paper_2010_11847_amd.binding import PMError
from tests.gpu_helpers import banner, f32, record, rel, to_dev, to_np

pytestmark = pytest.mark.gpu

OM = 0.3


def ctx_for(w, max_particles=0):
    from paper_2010_11847_amd.binding import PMContext
    return PMContext(w, max_particles=max_particles)


def wl(n_mesh, n_part, **kw):
    return inputs.scaled(inputs.MEDIUM, n_mesh, n_part, **kw)


@pytest.mark.parametrize("n", [8, 16, 32, 64, 128, 256])
def test_rfft_irfft_match_numpy(gpu, n):
    banner(f"rfft n={n}")
    c = ctx_for(wl(n, 8))
    x = inputs.normal_array((n, n, n), seed=n)
    spec = to_np(c.pm_rfft(to_dev(x)))
    ref = np.fft.rfftn(x.astype(np.float64))
    record(f"rfft_{n}_rel", rel(spec, ref), 2e-6)
    assert rel(spec, ref) < 2e-6
    back = to_np(c.pm_irfft(to_dev(ref.astype(np.complex64), torch.complex64)))
    assert rel(back, x) < 2e-6


def test_noise_matches_counter_generator(gpu):
    banner("noise")
    w = wl(64, 64)
    c = ctx_for(w)
    for seed in (0, 7, 123456):
        g = to_np(c.pm_noise(seed))
        o = white_noise(seed, 64).astype(np.float32)
        assert np.max(np.abs(g - o)) <= 2e-6 * max(1.0, np.abs(o).max())
        assert np.mean(g == o) > 0.999


@pytest.mark.parametrize("n_mesh,n_p,kind", [(32, 5001, "uniform"), (64, 70001, "clustered"),
                                             (128, 100003, "clustered"), (16, 999, "uniform")])
def test_paint_matches_oracle(gpu, n_mesh, n_p, kind):
    banner(f"paint n={n_mesh} np={n_p} {kind}")
    w = wl(n_mesh, 8)
    c = ctx_for(w, max_particles=n_p)
    x = (inputs.uniform_positions if kind == "uniform" else inputs.clustered_positions)(n_p, n_mesh, seed=n_mesh)
    g = to_np(c.pm_paint(to_dev(x)))
    o = pm.density_contrast(x.astype(np.float64), n_mesh, n_p)
    record(f"paint_{n_mesh}_{n_p}_{kind}_rel", rel(g, o), 1e-5)
    assert rel(g, o) < 1e-5
    # mass conservation: sum(delta) = 0 <=> sum(rho) = np
    assert abs(g.astype(np.float64).sum()) < 1e-5 * n_mesh ** 3


def test_paint_lattice_and_edges(gpu):
    banner("paint lattice/edges")
    n = 32
    w = wl(n, 16)
    c = ctx_for(w, max_particles=16 ** 3 + 4)
    x = inputs.perturbed_lattice(16, n, seed=3, amp=0.3)
    extra = np.array([[0, 0, 0], [n - 1e-4, n - 1e-4, n - 1e-4], [15.999, 16.0, 0.5], [31.0, 0.0, 31.0]],
                     dtype=np.float32)
    x = np.concatenate([x, extra])
    g = to_np(c.pm_paint(to_dev(x)))
    o = pm.density_contrast(x.astype(np.float64), n, len(x))
    assert rel(g, o) < 1e-5


@pytest.mark.parametrize("n_mesh,n_p,opts", [(32, 4000, {}), (64, 30011, {}), (128, 60000, {}),
                                             (256, 50000, {}), (512, 50000, {}),
                                             (64, 20000, {"deconv_order": 2}),
                                             (64, 20000, {"split_mode": 1, "split_rs": 2.0}),
                                             (64, 20000, {"split_mode": 2, "split_rs": 2.0})])
def test_force_matches_oracle(gpu, n_mesh, n_p, opts):
    banner(f"force n={n_mesh} np={n_p} {opts}")
    w = replace(wl(n_mesh, 8), **opts)
    c = ctx_for(w, max_particles=n_p)
    x = inputs.clustered_positions(n_p, n_mesh, seed=11 + n_mesh)
    g = to_np(c.pm_force(to_dev(x)))
    o = pm.force(x.astype(np.float64), n_mesh, n_p, OM, deconv_order=w.deconv_order,
                 split_rs=w.split_rs, split_mode=w.split_mode)
    record(f"force_{n_mesh}_{n_p}_" + "_".join(f"{k}{v}" for k, v in opts.items()) + "_rel", rel(g, o), 1e-5)
    assert rel(g, o) < 1e-5
    # momentum conservation of the force
    assert np.abs(g.astype(np.float64).sum(0)).max() < 1e-5 * np.abs(o).sum(0).max()


@pytest.mark.parametrize("n_mesh,n_part,order", [(32, 32, 2), (64, 32, 2), (64, 64, 1)])
def test_init_lpt_matches_oracle(gpu, n_mesh, n_part, order):
    banner(f"lpt n={n_mesh} np={n_part} order={order}")
    w = replace(wl(n_mesh, n_part), lpt_order=order)
    c = ctx_for(w)
    pos, mom = c.pm_init_lpt(w.seed, w.a_list[0])
    gx, gp = to_np(pos), to_np(mom)
    ox, op = lpt.generate(w)
    dx = pm.min_image(gx - ox, n_mesh)
    record(f"lpt_{n_part}_{n_mesh}_order{order}_mom_rel", rel(gp, op), 1e-5)
    assert np.abs(dx).max() < 1e-4 * max(1.0, n_mesh / 64)
    assert rel(gp, op) < 1e-5


def test_init_lpt_with_tabulated_pk_matches_oracle(gpu):
    # a caller's table (here the no-wiggle spectrum at 96 log-spaced k),
    # interpolated in (ln k, ln P) on both sides and taken as given
    banner("lpt with a tabulated P(k)")
    base = wl(64, 32)
    ks = np.logspace(-4, 2, 96)
    pk = cosmology.linear_power(ks, base.cosmo)
    cos = replace(base.cosmo, pk_kind=inputs.PK_TABLE, pk_table=(tuple(ks), tuple(pk)))
    w = replace(base, cosmo=cos)
    c = ctx_for(w)
    pos, mom = c.pm_init_lpt(w.seed, w.a_list[0])
    gx, gp = to_np(pos), to_np(mom)
    ox, op = lpt.generate(w)
    assert np.abs(pm.min_image(gx - ox, 64)).max() < 1e-4
    assert rel(gp, op) < 1e-5
    # and it is the analytic spectrum's field to the table's interpolation
    # error (measured 6e-4 on the momenta)
    _, ap = lpt.generate(base)
    assert rel(gp, ap) < 5e-3


def test_init_lpt_with_short_table_extrapolates_like_the_oracle(gpu):
    # a table that ends at k = 0.4 h/Mpc, below the largest lattice mode of
    # 32^3 particles in 200 Mpc/h (0.87 h/Mpc): the modes above it take the
    # end segment's power law on both sides (and a table starting above the
    # smallest nonzero mode, 0.031 h/Mpc, the first segment's)
    banner("lpt with a tabulated P(k) extrapolated at both ends")
    base = wl(64, 32)
    ks = np.logspace(np.log10(0.05), np.log10(0.4), 24)
    pk = cosmology.linear_power(ks, base.cosmo)
    cos = replace(base.cosmo, pk_kind=inputs.PK_TABLE, pk_table=(tuple(ks), tuple(pk)))
    w = replace(base, cosmo=cos)
    c = ctx_for(w)
    pos, mom = c.pm_init_lpt(w.seed, w.a_list[0])
    gx, gp = to_np(pos), to_np(mom)
    ox, op = lpt.generate(w)
    d = float(np.abs(pm.min_image(gx - ox, 64)).max())
    record("lpt_short_table_pos_max", d, 1e-4)
    record("lpt_short_table_mom_rel", rel(gp, op), 1e-5)
    assert d < 1e-4
    assert rel(gp, op) < 1e-5


def oracle_start(w):
    """The 2LPT start of the oracle, rounded to float32: the state both sides
    are fed (so that no oracle input comes from the GPU)."""
    x0, p0 = lpt.generate(w)
    return f32(x0), f32(p0)


def test_kdk_step_matches_oracle(gpu):
    banner("kdk step")
    w = wl(64, 32)
    c = ctx_for(w)
    x0, p0 = oracle_start(w)
    pos, mom = to_dev(x0), to_dev(p0)
    force = c.pm_force(pos)
    f0 = pm.force(x0, 64, 32 ** 3, OM)
    assert rel(to_np(force), f0) < 1e-5
    c.pm_kdk_step(pos, mom, force, 0.1, 0.3)
    from oracle import cosmology as Cm
    ac = np.sqrt(0.1 * 0.3)
    p = p0 + f0 * Cm.kick_factor(0.1, ac, 0.1, OM)
    x = pm.wrap(x0 + p * Cm.drift_factor(0.1, 0.3, ac, OM), 64)
    f = pm.force(x, 64, 32 ** 3, OM)
    p = p + f * Cm.kick_factor(ac, 0.3, 0.3, OM)
    dx = np.abs(pm.min_image(to_np(pos) - x, 64)).max()
    r_f, r_p = rel(to_np(force), f), rel(to_np(mom), p)
    record("kdk_step_pos_max_abs_cells", dx, 1e-4)
    record("kdk_step_force_rel", r_f, 1e-5)
    record("kdk_step_mom_rel", r_p, 1e-5)
    assert dx < 1e-4
    assert r_f < 1e-5
    assert r_p < 1e-5


@pytest.mark.parametrize("n_mesh,n_part", [(32, 32), (64, 32)])
def test_run_matches_oracle(gpu, n_mesh, n_part):
    banner(f"run n={n_mesh} np={n_part}")
    base = inputs.SMALL if n_mesh == n_part else wl(n_mesh, n_part)
    w = replace(base, n_mesh=n_mesh, n_part=n_part)
    c = ctx_for(w)
    x0, p0 = oracle_start(w)
    pos, mom = to_dev(x0), to_dev(p0)
    delta = torch.empty((n_mesh,) * 3, device="cuda")
    c.pm_run(w.a_list, pos, mom, delta_final=delta)
    ox, op, _ = pm.kdk_run(x0, p0, w.a_list, n_mesh, w.n_particles, OM)
    d = pm.min_image(to_np(pos) - ox, n_mesh)
    rms = float(np.sqrt((d ** 2).sum(1).mean()))
    banner(f"  rms position error {rms:.3e} cells")
    record(f"run_{n_part}_{n_mesh}_pos_rms_cells", rms, 1e-3)
    assert rms < 1e-3
    assert rel(to_np(mom), op) < 1e-3
    od = pm.density_contrast(ox, n_mesh, w.n_particles)
    assert rel(to_np(delta), od) < 1e-3


@pytest.mark.parametrize("n,deconv,n_max", [(32, False, 0), (64, True, 0), (64, False, 12)])
def test_power_matches_oracle(gpu, n, deconv, n_max):
    banner(f"power n={n} deconv={deconv} nmax={n_max}")
    w = wl(n, 8)
    c = ctx_for(w)
    x = inputs.clustered_positions(20000, n, seed=5)
    d = pm.density_contrast(x.astype(np.float64), n, 20000).astype(np.float32)
    k, p, m = c.pm_power(to_dev(d), n_max=n_max, deconv=deconv)
    ok, op, om = power.power(d.astype(np.float64), w.box_size, deconvolve_cic=deconv, n_max=n_max)
    sel = om > 0
    np.testing.assert_array_equal(m, om)
    np.testing.assert_allclose(k[sel], ok[sel], rtol=1e-12)
    np.testing.assert_allclose(p[sel], op[sel], rtol=1e-5)


def test_growth_factors_match_oracle(gpu):
    from oracle import cosmology as Cm
    c = ctx_for(wl(32, 32))
    for a in (0.1, 0.55, 1.0):
        g = c.pm_growth(a)
        d1, f1, d2, f2 = (float(v[0]) for v in Cm.growth(a, OM))
        assert g["D1"] == pytest.approx(d1, rel=1e-9)
        assert g["f1"] == pytest.approx(f1, rel=1e-9)
        assert g["D2"] == pytest.approx(d2, rel=1e-9)
        assert g["f2"] == pytest.approx(f2, rel=1e-9)


def test_kdk_factors_match_oracle(gpu):
    from oracle import cosmology as Cm
    c = ctx_for(wl(32, 32))
    a = np.array([0.02, 0.1, 0.13, 0.4, 0.41, 1.0])
    k1, dr, k2 = c.pm_kdk_factors(a)
    for i in range(len(a) - 1):
        ai, aj = a[i], a[i + 1]
        ac = np.sqrt(ai * aj)
        assert k1[i] == pytest.approx(float(Cm.kick_factor(ai, ac, ai, OM)), rel=1e-9)
        assert dr[i] == pytest.approx(float(Cm.drift_factor(ai, aj, ac, OM)), rel=1e-9)
        assert k2[i] == pytest.approx(float(Cm.kick_factor(ac, aj, aj, OM)), rel=1e-9)
    with pytest.raises(PMError):
        c.pm_kdk_factors([0.5, 0.4])
