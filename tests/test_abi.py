"""Host-only checks of the C ABI: the library loads, exports every symbol the
header declares, and sizes workspaces / rejects bad configurations without
touching a GPU."""
import ctypes as C
import os
import re
from dataclasses import replace

import pytest

from paper_2010_11847_amd import inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(pm_[a-z0-9_]+)\s*\(", txt))
    return names


@pytest.fixture(scope="module")
def lib():
    from paper_2010_11847_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libpm.so is not built; run __graft_entry__.build()")
    return _lib.load()


def test_every_declared_symbol_is_exported(lib):
    from paper_2010_11847_amd import _lib
    declared = header_symbols()
    assert {"pm_init_lpt", "pm_paint", "pm_force", "pm_kdk_step", "pm_run"} <= declared
    for name in sorted(declared):
        assert hasattr(lib, name), f"{name} declared in include/ but not exported"
        assert name in _lib._SIGS, f"{name} has no ctypes signature"


def test_workspace_sizes_and_validation(lib):
    from paper_2010_11847_amd.binding import make_config
    sizes = {}
    for w in (inputs.SMALL, inputs.MEDIUM, inputs.LARGE, inputs.ADJ_SMALL):
        cfg = make_config(w)
        sizes[w.name] = lib.pm_workspace_bytes(C.byref(cfg))
        assert sizes[w.name] > 0
    # the 1024^3 mesh needs three float32 meshes plus particle scratch
    assert 3 * 1024 ** 3 * 4 < sizes[inputs.LARGE.name] < 40e9
    bad = [replace(inputs.SMALL, n_mesh=48), replace(inputs.SMALL, n_part=64),
           replace(inputs.SMALL, box_size=-1.0), replace(inputs.SMALL, lpt_order=3),
           replace(inputs.SMALL, n_mesh=2048), replace(inputs.SMALL, deconv_order=5),
           replace(inputs.SMALL, lattice_shift=1.5),
           replace(inputs.SMALL, split_mode=1, split_rs=0.0)]
    for w in bad:
        assert lib.pm_workspace_bytes(C.byref(make_config(w))) == 0, w
    assert lib.pm_workspace_bytes(None) == 0
    cfg = make_config(inputs.SMALL, max_particles=10)   # below n_part^3
    assert lib.pm_workspace_bytes(C.byref(cfg)) == 0


def test_tabulated_power_spectrum_validation(lib):
    """A caller's P(k) table must hold finite k > 0 (increasing) and finite
    P >= 0; anything else is an invalid configuration (workspace size 0)."""
    from paper_2010_11847_amd.binding import make_config
    import numpy as np
    ks = tuple(np.logspace(-3, 1, 8))
    ps = tuple(np.linspace(1.0, 8.0, 8))

    def cfg(k, p):
        cos = replace(inputs.SMALL.cosmo, pk_kind=inputs.PK_TABLE, pk_table=(k, p))
        return make_config(replace(inputs.SMALL, cosmo=cos))
    assert lib.pm_workspace_bytes(C.byref(cfg(ks, ps))) > 0
    # a numpy table is accepted too
    assert lib.pm_workspace_bytes(C.byref(cfg(np.array(ks), np.array(ps)))) > 0
    inf, nan = float("inf"), float("nan")
    for k, p in [(ks[:-1] + (inf,), ps), (ks, ps[:-1] + (inf,)), (ks, (nan,) + ps[1:]),
                 ((nan,) + ks[1:], ps), (ks, (-1.0,) + ps[1:]), (ks[::-1], ps), (ks[:1], ps[:1])]:
        assert lib.pm_workspace_bytes(C.byref(cfg(k, p))) == 0, (k, p)


def test_strerror(lib):
    assert lib.pm_strerror(0) == b"ok"
    assert lib.pm_strerror(-2) == b"workspace too small"


def test_no_kernel_uses_scratch():
    """Every HIP kernel keeps its state in registers and LDS: a kernel that
    spills to (or builds arrays in) private scratch memory pays HBM traffic
    per lane.  Reads the compiler's resource report written by the build."""
    import glob
    import re
    build = os.path.join(ROOT, "paper_2010_11847_amd", "_build")
    reports = glob.glob(os.path.join(build, "*.usage.txt"))
    if not reports:
        pytest.skip("library not built")
    bad = []
    for path in reports:
        name = None
        for line in open(path):
            m = re.search(r"Function Name: (\S+)", line)
            if m:
                name = m.group(1)
            m = re.search(r"ScratchSize \[bytes/lane\]: (\d+)", line)
            if m and int(m.group(1)) > 0:
                bad.append((os.path.basename(path), name, int(m.group(1))))
    assert not bad, bad


def test_batch_plan_sizes_and_validation(lib):
    """A batch plan of B members takes B single-simulation workspaces; it
    needs n_mesh >= 64, no pyramid and B <= PM_MAX_BATCH."""
    from paper_2010_11847_amd import _lib
    from paper_2010_11847_amd.binding import make_config
    w = inputs.scaled(inputs.MEDIUM, 64, 32)
    one = lib.pm_workspace_bytes(C.byref(make_config(w)))
    assert one > 0
    assert lib.pm_workspace_bytes(C.byref(make_config(w, batch=1))) == one
    for b in (2, 5, _lib.PM_MAX_BATCH):
        assert lib.pm_workspace_bytes(C.byref(make_config(w, batch=b))) == b * one
    assert lib.pm_workspace_bytes(C.byref(make_config(w, batch=_lib.PM_MAX_BATCH + 1))) == 0
    assert lib.pm_workspace_bytes(C.byref(make_config(w, batch=-1))) == 0
    assert lib.pm_workspace_bytes(C.byref(make_config(inputs.scaled(inputs.SMALL, 32, 32), batch=2))) == 0
    assert lib.pm_workspace_bytes(C.byref(make_config(replace(w, pyramid_levels=1), batch=2))) == 0
    assert C.sizeof(_lib.pm_req_desc) == 48
    # the batch entry points reject a missing plan without touching a GPU
    assert lib.pm_kdk_step_batched(None, None, 1) == _lib.PM_EINVAL
    assert lib.pm_batch_advance(None, None) == _lib.PM_EINVAL
    assert lib.pm_batch_remaining(None, 0) == _lib.PM_EINVAL
    assert lib.pm_batch_end(None, 0, None) == _lib.PM_EINVAL
    assert lib.pm_batch_begin(None, 0, None, 0, None, None, None) == _lib.PM_EINVAL
    h = C.c_void_p()
    assert lib.pm_batch_member(None, 0, C.byref(h)) == _lib.PM_EINVAL


def test_integrator_validation(lib):
    """PM_INT_FASTPM / LEAPFROG / COLA are valid; other values and a COLA
    batch plan are not; the LPT-frame call rejects a half-given frame."""
    from paper_2010_11847_amd import _lib
    from paper_2010_11847_amd.binding import make_config
    w = inputs.scaled(inputs.MEDIUM, 64, 32)
    for k in (inputs.INT_FASTPM, inputs.INT_LEAPFROG, inputs.INT_COLA):
        assert lib.pm_workspace_bytes(C.byref(make_config(replace(w, integrator=k)))) > 0
    for k in (-1, 3):
        assert lib.pm_workspace_bytes(C.byref(make_config(replace(w, integrator=k)))) == 0
    assert lib.pm_workspace_bytes(C.byref(make_config(replace(w, integrator=inputs.INT_COLA), batch=2))) == 0
    assert lib.pm_workspace_bytes(C.byref(make_config(replace(w, integrator=inputs.INT_LEAPFROG), batch=2))) > 0
    assert lib.pm_set_lpt_frame(None, None, None) == _lib.PM_EINVAL
