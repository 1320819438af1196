"""The allocation-free force entry point against pm_force on a context with
its own workspace: two calls in a row (the second with a smaller mesh and
fewer particles, so stale contents of the shared static array would show),
bitwise equal, since both run the same deterministic kernels."""
import ctypes as C

import numpy as np
import pytest
import torch

from paper_2010_11847_amd import inputs

pytestmark = pytest.mark.gpu


def _force_both(w, x):
    from paper_2010_11847_amd.binding import PMContext, pm_force_static
    pos = torch.from_numpy(x).cuda()
    ctx = PMContext(w, max_particles=len(x))
    ref = ctx.pm_force(pos)
    torch.cuda.synchronize()
    ctx.close()
    out = torch.full_like(pos, float("nan"))
    pm_force_static(w, pos, out=out, max_particles=len(x))
    torch.cuda.synchronize()
    return ref.cpu().numpy(), out.cpu().numpy()


def test_static_force_matches_workspace_force_twice(gpu):
    cases = [
        (inputs.scaled(inputs.SMALL, 64, 64, n_steps=1), inputs.clustered_positions(64 ** 3, 64, seed=91)),
        (inputs.scaled(inputs.SMALL, 32, 8, n_steps=1), inputs.uniform_positions(3001, 32, seed=92)),
    ]
    for w, x in cases:
        print(f"[gpu] pm_force_static vs pm_force: mesh {w.n_mesh}^3, {len(x)} particles", flush=True)
        ref, got = _force_both(w, x)
        assert np.isfinite(got).all()
        assert np.array_equal(ref, got), float(np.abs(ref - got).max())
        assert np.abs(ref).max() > 0


def test_static_force_rejects_what_does_not_fit(gpu):
    from paper_2010_11847_amd import _lib
    from paper_2010_11847_amd.binding import make_config
    lib = _lib.load()
    w = inputs.scaled(inputs.SMALL, 128, 128, n_steps=1)   # 179 MiB of workspace
    cfg = make_config(w)
    pos = torch.zeros((8, 3), device="cuda")
    out = torch.zeros((8, 3), device="cuda")
    rc = lib.pm_force_static(C.byref(cfg), C.c_void_p(pos.data_ptr()), 8, C.c_void_p(out.data_ptr()), None)
    assert rc == _lib.PM_ENOMEM
    rc = lib.pm_force_static(None, C.c_void_p(pos.data_ptr()), 8, C.c_void_p(out.data_ptr()), None)
    assert rc == _lib.PM_EINVAL
