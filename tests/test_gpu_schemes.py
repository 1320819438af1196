"""The plain leapfrog and the LPT-frame (COLA-like) integrators on the GPU
against the oracle's schemes (oracle/schemes.py), from the same float32
start: positions rms < 1e-3 cell and momenta within 1e-4 (norm-wise) after
the run, as for the FastPM runs.  The LPT fields the library writes in
pm_init_lpt match the oracle's."""
import numpy as np
import pytest
import torch
from dataclasses import replace

from oracle import lpt, pm
from oracle import schemes as S
from paper_2010_11847_amd import inputs
from tests.gpu_helpers import banner, f32, record, rel, to_dev, to_np

pytestmark = pytest.mark.gpu


def compare(name, gx, gp, ox, op_, n_mesh):
    d = pm.min_image(gx.astype(np.float64) - ox, n_mesh)
    rms = float(np.sqrt((d ** 2).sum(1).mean()))
    rp = rel(gp, op_)
    banner(f"  {name}: position rms {rms:.2e} cells, momentum rel {rp:.2e}")
    record(f"{name}_pos_rms", rms, 1e-3)
    record(f"{name}_mom_rel", rp, 1e-4)
    assert rms < 1e-3
    assert rp < 1e-4


@pytest.mark.parametrize("n_mesh,n_part,steps", [(32, 32, 10), (64, 32, 6)])
def test_leapfrog_run_matches_oracle(gpu, n_mesh, n_part, steps):
    from paper_2010_11847_amd.binding import PMContext
    w = replace(inputs.scaled(inputs.SMALL, n_mesh, n_part, n_steps=steps), integrator=inputs.INT_LEAPFROG)
    banner(f"leapfrog {n_part}^3 / {n_mesh}^3, {steps} steps")
    x0, p0 = (f32(v) for v in lpt.generate(w))
    c = PMContext(w)
    k1, dr, k2 = c.pm_kdk_factors(w.a_list)
    om = w.cosmo.omega_m
    for i, (ai, aj) in enumerate(zip(w.a_list[:-1], w.a_list[1:])):
        ac = np.sqrt(ai * aj)
        assert k1[i] == pytest.approx(S.std_kick(ai, ac, om), rel=1e-9)
        assert dr[i] == pytest.approx(S.std_drift(ai, aj, om), rel=1e-9)
        assert k2[i] == pytest.approx(S.std_kick(ac, aj, om), rel=1e-9)
    pos, mom = to_dev(x0), to_dev(p0)
    c.pm_run(w.a_list, pos, mom)
    ox, op_, _ = S.leapfrog_run(x0, p0, w.a_list, n_mesh, w.n_particles, om)
    compare(f"leapfrog_{n_part}_{n_mesh}", to_np(pos), to_np(mom), ox, op_, n_mesh)
    c.close()


@pytest.mark.parametrize("n_mesh,n_part,steps,order", [(32, 32, 10, 2), (64, 32, 5, 2), (64, 32, 3, 1)])
def test_cola_run_matches_oracle(gpu, n_mesh, n_part, steps, order):
    from paper_2010_11847_amd.binding import PMContext
    w = replace(inputs.scaled(inputs.SMALL, n_mesh, n_part, n_steps=steps), integrator=inputs.INT_COLA,
                lpt_order=order)
    banner(f"COLA {n_part}^3 / {n_mesh}^3, {steps} steps, {order}LPT")
    c = PMContext(w)
    psi1_d, psi2_d = c.pm_set_lpt_frame()
    c.pm_init_lpt(w.seed, w.a_list[0])          # fills the frame
    o1, o2 = S.displacement_fields(w)
    r1, r2 = rel(to_np(psi1_d), o1), (rel(to_np(psi2_d), o2) if order >= 2 else float(np.abs(to_np(psi2_d)).max()))
    banner(f"  LPT fields vs oracle: Psi1 rel {r1:.2e}, Psi2 {r2:.2e}")
    assert r1 < 1e-5 and r2 < 1e-5
    # both sides from the oracle's start and fields rounded to float32
    x0, p0 = (f32(v) for v in lpt.generate(w))
    psi1, psi2 = f32(o1), f32(o2)
    psi1_d.copy_(to_dev(psi1))
    psi2_d.copy_(to_dev(psi2))
    pos, mom = to_dev(x0), to_dev(p0)
    c.pm_run(w.a_list, pos, mom)
    ox, op_, _ = S.cola_run(x0, p0, psi1, psi2, w.a_list, n_mesh, w.n_particles, w.cosmo.omega_m)
    compare(f"cola_{n_part}_{n_mesh}_{order}lpt", to_np(pos), to_np(mom), ox, op_, n_mesh)
    c.close()


def test_cola_graphs_and_errors(gpu):
    """The COLA step loop as captured graphs equals the eager loop bit for
    bit; COLA refuses checkpoints, the adjoint, pm_kdk_step and a run with
    no frame."""
    from paper_2010_11847_amd.binding import PMContext, PMError
    w = replace(inputs.scaled(inputs.SMALL, 64, 32, n_steps=4), integrator=inputs.INT_COLA)
    s = torch.cuda.Stream()
    outs = []
    with torch.cuda.stream(s):
        for graphs in (False, True):
            c = PMContext(w, stream=s)
            c.pm_use_graphs(graphs)
            c.pm_set_lpt_frame()
            pos, mom = c.pm_init_lpt(w.seed, w.a_list[0])
            c.pm_run(w.a_list, pos, mom)
            outs.append((pos, mom))
            if graphs:
                ck = torch.empty((len(w.a_list), 2, w.n_particles, 3), device="cuda")
                with pytest.raises(PMError):
                    c.pm_run(w.a_list, pos, mom, ckpt=ck)
                with pytest.raises(PMError):
                    c.pm_run_adjoint(w.a_list, ck, want_noise_grad=False)
                f = torch.zeros_like(pos)
                with pytest.raises(PMError):
                    c.pm_kdk_step(pos, mom, f, 0.1, 0.2)
                c.pm_clear_lpt_frame()
                with pytest.raises(PMError):
                    c.pm_run(w.a_list, pos, mom)
            c.close()
        s.synchronize()
    for a, b in zip(*outs):
        assert torch.equal(a, b)
