"""Edge and degenerate cases of the HIP path through the C ABI: a single
particle, an unperturbed lattice, positions outside the box, the smallest
mesh, and the errors the entry points return for invalid arguments and
call orders."""
import numpy as np
import pytest
import torch

from oracle import lpt, pm
from paper_2010_11847_amd import inputs
from paper_2010_11847_amd.binding import PMContext, PMError
from tests.gpu_helpers import banner, f32, rel, to_dev, to_np

pytestmark = pytest.mark.gpu
OM = 0.3


def wl(n_mesh, n_part, **kw):
    return inputs.scaled(inputs.MEDIUM, n_mesh, n_part, **kw)


def test_single_particle_paint_and_zero_self_force(gpu):
    banner("one particle")
    c = PMContext(wl(32, 8), max_particles=512)
    x = np.array([[7.3, 20.9, 0.4]], dtype=np.float32)
    d = to_np(c.pm_paint(to_dev(x)))
    o = pm.density_contrast(x.astype(np.float64), 32, 1)
    assert rel(d, o) < 1e-6
    f = to_np(c.pm_force(to_dev(x)))
    # one particle in a periodic box feels no force from itself (paint and
    # readout share the CIC weights and the FD kernel is odd): zero up to
    # float32 rounding, against the force of a partner two cells away
    pair = np.array([[7.3, 20.9, 0.4], [9.3, 20.9, 0.4]], dtype=np.float32)
    fp = to_np(c.pm_force(to_dev(pair)))
    assert np.abs(fp[0, 0]) == pytest.approx(abs(pm.force(pair.astype(np.float64), 32, 2, OM)[0, 0]), rel=1e-5)
    assert np.abs(f).max() < 1e-5 * np.abs(fp[0, 0])


def test_lattice_has_no_force(gpu):
    # particles on every node of a B = 2 lattice: each sits at a centre of
    # symmetry of the painted density, so the force read out there vanishes
    banner("unperturbed lattice")
    c = PMContext(wl(32, 16))
    q = np.stack(np.meshgrid(*(np.arange(16) * 2.0,) * 3, indexing="ij"), -1).reshape(-1, 3).astype(np.float32)
    f = to_np(c.pm_force(to_dev(q)))
    assert np.abs(f).max() < 1e-6


def test_positions_outside_the_box_wrap(gpu):
    banner("positions outside the box")
    n = 32
    c = PMContext(wl(n, 8), max_particles=4096)
    x = inputs.clustered_positions(4096, n, seed=17)
    shift = np.random.default_rng(1).integers(-2, 3, size=x.shape).astype(np.float32) * n
    f_in = to_np(c.pm_force(to_dev(x)))
    f_out = to_np(c.pm_force(to_dev(x + shift)))
    # the same cells and weights up to the float32 rounding of the shift
    assert rel(f_out, f_in) < 1e-4


def test_smallest_mesh_run(gpu):
    banner("8^3 mesh run")
    w = inputs.scaled(inputs.SMALL, 8, 8, n_steps=3)
    c = PMContext(w)
    x0, p0 = (f32(v) for v in lpt.generate(w))   # the oracle's start, fed to both sides
    pos, mom = to_dev(x0), to_dev(p0)
    c.pm_run(w.a_list, pos, mom)
    xo, _, _ = pm.kdk_run(x0, p0, w.a_list, 8, 512, w.cosmo.omega_m)
    d = pm.min_image(to_np(pos).astype(np.float64) - xo, 8)
    assert np.sqrt(np.mean(d ** 2)) < 1e-3


def test_argument_and_order_errors(gpu):
    w = wl(32, 16)
    c = PMContext(w, max_particles=16 ** 3)
    ok = torch.zeros((16 ** 3, 3), device="cuda")
    with pytest.raises(PMError):
        c.pm_paint(torch.zeros((16 ** 3 + 1, 3), device="cuda"))     # beyond the capacity
    with pytest.raises(PMError):
        c.pm_force(torch.zeros((0, 3), device="cuda"))               # no particles
    with pytest.raises(PMError):
        c.pm_kdk_step(ok.clone(), ok.clone(), ok.clone(), 0.5, 0.5)   # a1 must exceed a0
    with pytest.raises(PMError):
        c.pm_run([0.1, 0.3, 0.2], ok.clone(), ok.clone())           # a not increasing
    with pytest.raises(PMError):
        c.pm_run_advance(1)                                           # no run in progress
    pos, mom = c.pm_init_lpt(w.seed, w.a_list[0])
    c.pm_run_begin(w.a_list, pos, mom)
    with pytest.raises(PMError):
        c.pm_run_end()                                                # steps still to go
    while c.pm_run_advance(4) > 0:
        pass
    c.pm_run_end()
    with pytest.raises(PMError):
        c.pm_power(to_dev(np.zeros((32, 32, 32), np.float32)), n_bins=17)   # more bins than n/2
