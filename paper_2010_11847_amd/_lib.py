"""ctypes declarations of the C ABI in include/pm.h (argument marshalling only).

The shared library must be built beforehand (``__graft_entry__.build()`` or
``python -m paper_2010_11847_amd.build``).  There is no fallback: if the
library is missing or fails to load, importing the binding raises.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# PM_LIBRARY may name another build of the same library (same ABI), e.g.
# one compiled with different kernel options, to compare builds
LIB_PATH = os.environ.get("PM_LIBRARY") or os.path.join(HERE, "libpm.so")

PM_OK, PM_EINVAL, PM_ENOMEM, PM_EHIP, PM_ESTATE = 0, -1, -2, -3, -4


class pm_cosmo(C.Structure):
    _fields_ = [("omega_m", C.c_double), ("omega_b", C.c_double), ("h", C.c_double),
                ("n_s", C.c_double), ("sigma8", C.c_double), ("t_cmb", C.c_double),
                ("pk_kind", C.c_int), ("pk_amp", C.c_double), ("pk_index", C.c_double),
                ("pk_k", C.POINTER(C.c_double)), ("pk_p", C.POINTER(C.c_double)),
                ("pk_n", C.c_int)]


class pm_config(C.Structure):
    _fields_ = [("box_size", C.c_double), ("n_mesh", C.c_int), ("n_part", C.c_int),
                ("cosmo", pm_cosmo), ("lpt_order", C.c_int), ("deconv_order", C.c_int),
                ("split_rs", C.c_double), ("split_mode", C.c_int),
                ("lattice_shift", C.c_double), ("max_particles", C.c_int64), ("pyramid_levels", C.c_int),
                ("batch", C.c_int), ("integrator", C.c_int)]


class pm_req_desc(C.Structure):
    _fields_ = [("member", C.c_int32), ("flags", C.c_int32), ("kick_close", C.c_float), ("kick_open", C.c_float),
                ("drift", C.c_float), ("reserved", C.c_float), ("ckpt_x", C.c_void_p), ("ckpt_p", C.c_void_p),
                ("reserved2", C.c_int64)]


PM_MAX_BATCH = 256
PM_REQ_CKPT = 1


# name -> (restype, argtypes)
_SIGS = {
    "pm_workspace_bytes": (C.c_size_t, [C.POINTER(pm_config)]),
    "pm_create": (C.c_int, [C.POINTER(pm_config), C.c_void_p, C.c_size_t, C.c_void_p, C.POINTER(C.c_void_p)]),
    "pm_destroy": (C.c_int, [C.c_void_p]),
    "pm_set_stream": (C.c_int, [C.c_void_p, C.c_void_p]),
    "pm_sync": (C.c_int, [C.c_void_p]),
    "pm_strerror": (C.c_char_p, [C.c_int]),
    "pm_last_error": (C.c_char_p, [C.c_void_p]),
    "pm_growth": (C.c_int, [C.c_void_p, C.c_double, C.POINTER(C.c_double)]),
    "pm_kdk_factors": (C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.c_int, C.POINTER(C.c_double),
                                 C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "pm_noise": (C.c_int, [C.c_void_p, C.c_uint64, C.c_void_p]),
    "pm_init_lpt": (C.c_int, [C.c_void_p, C.c_uint64, C.c_double, C.c_void_p, C.c_void_p, C.c_void_p,
                              C.c_void_p]),
    "pm_paint": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p]),
    "pm_force": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p]),
    "pm_kdk_step": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_double, C.c_double]),
    "pm_run": (C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.c_int, C.c_void_p, C.c_void_p, C.c_void_p,
                         C.c_void_p]),
    "pm_run_begin": (C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.c_int, C.c_void_p, C.c_void_p,
                               C.c_void_p]),
    "pm_run_advance": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_int)]),
    "pm_run_end": (C.c_int, [C.c_void_p, C.c_void_p]),
    "pm_run_adjoint": (C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.c_int, C.c_void_p, C.c_void_p,
                                 C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "pm_chi2": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_double, C.c_void_p, C.c_void_p]),
    "pm_recon_work_bytes": (C.c_size_t, [C.c_void_p, C.c_int]),
    "pm_recon_step": (C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.c_int, C.c_void_p, C.c_double, C.c_void_p,
                                C.c_void_p, C.c_void_p, C.c_int, C.c_double, C.c_double, C.c_double, C.c_double,
                                C.c_void_p, C.c_size_t, C.POINTER(C.c_double)]),
    "pm_use_graphs": (C.c_int, [C.c_void_p, C.c_int]),
    "pm_set_force_ckpt": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64]),
    "pm_rfft": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "pm_irfft": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "pm_profile": (C.c_int, [C.c_void_p, C.c_int]),
    "pm_profile_read": (C.c_int, [C.c_void_p, C.c_int, C.c_char_p, C.POINTER(C.c_double), C.POINTER(C.c_int)]),
    "pm_power": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.c_int, C.POINTER(C.c_double),
                           C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "pm_force_static": (C.c_int, [C.POINTER(pm_config), C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p]),
    "pm_kdk_step_batched": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int]),
    "pm_set_lpt_frame": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "pm_batch_member": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_void_p)]),
    "pm_batch_begin": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_double), C.c_int, C.c_void_p, C.c_void_p,
                                 C.c_void_p]),
    "pm_batch_advance": (C.c_int, [C.c_void_p, C.POINTER(C.c_int)]),
    "pm_batch_remaining": (C.c_int, [C.c_void_p, C.c_int]),
    "pm_batch_end": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p]),
}

_lib = None


def exported_symbols():
    return sorted(_SIGS)


def load():
    """Load libpm.so (once).  The HIP runtime must be the one torch uses, so
    torch is imported first; libpm.so then binds to the already-loaded
    libamdhip64 by soname."""
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401  (loads torch's HIP runtime first)
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name, None)
        if fn is None:
            continue
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib
