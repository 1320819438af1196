"""Thin Python binding of the C ABI (include/pm.h) on torch device memory.

Only argument marshalling lives here: tensors are checked for device, dtype,
shape and contiguity and their pointers passed to libpm.so together with the
current HIP stream.  Every step of the computation runs in the library's
kernels.
"""
from __future__ import annotations

import ctypes as C
from typing import Optional, Sequence

import numpy as np
import torch

from . import _lib
from .inputs import Workload


class PMError(RuntimeError):
    pass


def make_config(w: Workload, max_particles: int = 0, batch: int = 0) -> _lib.pm_config:
    c = w.cosmo
    tk = tp = None
    n_tab = 0
    if len(c.pk_table):
        n_tab = len(c.pk_table[0])
        tk = (C.c_double * n_tab)(*c.pk_table[0])
        tp = (C.c_double * n_tab)(*c.pk_table[1])
    cos = _lib.pm_cosmo(c.omega_m, c.omega_b, c.h, c.n_s, c.sigma8, c.t_cmb, c.pk_kind,
                        c.pk_amp, c.pk_index, tk, tp, n_tab)
    cfg = _lib.pm_config(w.box_size, w.n_mesh, w.n_part, cos, w.lpt_order, w.deconv_order,
                         w.split_rs, w.split_mode, w.lattice_shift, max_particles, w.pyramid_levels, batch,
                         w.integrator)
    cfg.keep_alive = (tk, tp)   # the library copies the table in pm_create
    return cfg


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


class PMContext:
    """A library context with its device workspace, bound to one GPU stream."""

    def __init__(self, workload: Workload, device="cuda", max_particles: int = 0, stream=None, batch: int = 0):
        self.lib = _lib.load()
        self.workload = workload
        dev = torch.device(device)
        if dev.type == "cuda" and dev.index is None:
            dev = torch.device("cuda", torch.cuda.current_device())
        self.device = dev
        self.cfg = make_config(workload, max_particles, batch)
        nbytes = self.lib.pm_workspace_bytes(C.byref(self.cfg))
        if nbytes == 0:
            raise PMError(f"invalid configuration for {workload.name}")
        self.workspace_bytes = int(nbytes)
        self.ws = torch.empty(self.workspace_bytes + 256, dtype=torch.uint8, device=self.device)
        base = self.ws.data_ptr()
        self._ws_ptr = (base + 255) // 256 * 256
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        ctx = C.c_void_p()
        rc = self.lib.pm_create(C.byref(self.cfg), C.c_void_p(self._ws_ptr), self.workspace_bytes,
                                C.c_void_p(self.stream.cuda_stream), C.byref(ctx))
        self._check(rc, "pm_create", ctx=None)
        self.ctx = ctx
        self.np3 = workload.n_part ** 3
        self._owner = True

    @classmethod
    def _view(cls, parent: "PMContext", handle: C.c_void_p) -> "PMContext":
        """A context handle owned by the library (a batch plan's member)."""
        v = cls.__new__(cls)
        v.lib, v.workload, v.device, v.cfg = parent.lib, parent.workload, parent.device, parent.cfg
        v.workspace_bytes, v.ws, v._ws_ptr = 0, parent.ws, 0
        v.stream, v.ctx, v.np3, v._owner = parent.stream, handle, parent.np3, False
        return v

    # ---- helpers -------------------------------------------------------------
    def _check(self, rc, what, ctx="self"):
        if rc != _lib.PM_OK:
            msg = self.lib.pm_strerror(rc).decode()
            if ctx == "self" and getattr(self, "ctx", None):
                msg += ": " + self.lib.pm_last_error(self.ctx).decode()
            raise PMError(f"{what} failed ({rc}): {msg}")

    def _dev(self, t: torch.Tensor, shape=None, dtype=torch.float32, name="array"):
        if not isinstance(t, torch.Tensor) or t.device != self.device or t.dtype != dtype:
            raise PMError(f"{name} must be a {dtype} tensor on {self.device}")
        if not t.is_contiguous():
            raise PMError(f"{name} must be contiguous")
        if shape is not None and tuple(t.shape) != tuple(shape):
            raise PMError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
        return t

    def close(self):
        if getattr(self, "ctx", None) and getattr(self, "_owner", True):
            self.lib.pm_destroy(self.ctx)
        self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_stream(self, stream):
        self.stream = stream
        self._check(self.lib.pm_set_stream(self.ctx, C.c_void_p(stream.cuda_stream)), "pm_set_stream")

    # ---- entry points (same names as the C ABI) --------------------------------
    def pm_sync(self):
        self._check(self.lib.pm_sync(self.ctx), "pm_sync")

    def pm_growth(self, a: float):
        out = (C.c_double * 6)()
        self._check(self.lib.pm_growth(self.ctx, a, out), "pm_growth")
        return dict(zip(("D1", "f1", "D2", "f2", "E", "Gf"), list(out)))

    def pm_kdk_factors(self, a_list: Sequence[float]):
        """(k1, dr, k2) arrays of the KDK steps over a_list."""
        a = np.ascontiguousarray(a_list, dtype=np.float64)
        ns = max(len(a) - 1, 0)
        k1, dr, k2 = (C.c_double * max(ns, 1))(), (C.c_double * max(ns, 1))(), (C.c_double * max(ns, 1))()
        self._check(self.lib.pm_kdk_factors(self.ctx, a.ctypes.data_as(C.POINTER(C.c_double)), len(a), k1, dr, k2),
                    "pm_kdk_factors")
        return np.array(k1[:ns]), np.array(dr[:ns]), np.array(k2[:ns])

    def pm_noise(self, seed: int, out: Optional[torch.Tensor] = None):
        n = self.workload.n_part
        out = torch.empty((n, n, n), dtype=torch.float32, device=self.device) if out is None else out
        self._dev(out, (n, n, n), name="noise")
        self._check(self.lib.pm_noise(self.ctx, seed, _ptr(out)), "pm_noise")
        return out

    def pm_init_lpt(self, seed: int, a0: float, noise: Optional[torch.Tensor] = None,
                    noise_out: Optional[torch.Tensor] = None, pos=None, mom=None):
        n = self.workload.n_part
        pos = torch.empty((self.np3, 3), dtype=torch.float32, device=self.device) if pos is None else pos
        mom = torch.empty((self.np3, 3), dtype=torch.float32, device=self.device) if mom is None else mom
        self._dev(pos, (self.np3, 3), name="pos")
        self._dev(mom, (self.np3, 3), name="mom")
        if noise is not None:
            self._dev(noise, (n, n, n), name="noise")
        if noise_out is not None:
            self._dev(noise_out, (n, n, n), name="noise_out")
        self._check(self.lib.pm_init_lpt(self.ctx, seed, a0, _ptr(noise), _ptr(noise_out), _ptr(pos), _ptr(mom)),
                    "pm_init_lpt")
        return pos, mom

    def pm_paint(self, pos: torch.Tensor, out: Optional[torch.Tensor] = None):
        n = self.workload.n_mesh
        self._dev(pos, name="pos")
        if pos.ndim != 2 or pos.shape[1] != 3:
            raise PMError("pos must have shape (np, 3)")
        out = torch.empty((n, n, n), dtype=torch.float32, device=self.device) if out is None else out
        self._dev(out, (n, n, n), name="delta")
        self._check(self.lib.pm_paint(self.ctx, _ptr(pos), pos.shape[0], _ptr(out)), "pm_paint")
        return out

    def pm_force(self, pos: torch.Tensor, out: Optional[torch.Tensor] = None):
        self._dev(pos, name="pos")
        if pos.ndim != 2 or pos.shape[1] != 3:
            raise PMError("pos must have shape (np, 3)")
        out = torch.empty_like(pos) if out is None else out
        self._dev(out, tuple(pos.shape), name="force")
        self._check(self.lib.pm_force(self.ctx, _ptr(pos), pos.shape[0], _ptr(out)), "pm_force")
        return out

    def pm_kdk_step(self, pos, mom, force, a0: float, a1: float):
        for t, nm in ((pos, "pos"), (mom, "mom"), (force, "force")):
            self._dev(t, (self.np3, 3), name=nm)
        self._check(self.lib.pm_kdk_step(self.ctx, _ptr(pos), _ptr(mom), _ptr(force), a0, a1), "pm_kdk_step")
        return pos, mom, force

    def pm_run(self, a_list: Sequence[float], pos, mom, ckpt: Optional[torch.Tensor] = None,
               delta_final: Optional[torch.Tensor] = None):
        self._dev(pos, (self.np3, 3), name="pos")
        self._dev(mom, (self.np3, 3), name="mom")
        a = np.ascontiguousarray(a_list, dtype=np.float64)
        if ckpt is not None:
            self._dev(ckpt, (len(a), 2, self.np3, 3), name="ckpt")
        if delta_final is not None:
            n = self.workload.n_mesh
            self._dev(delta_final, (n, n, n), name="delta_final")
        ap = a.ctypes.data_as(C.POINTER(C.c_double))
        self._check(self.lib.pm_run(self.ctx, ap, len(a), _ptr(pos), _ptr(mom), _ptr(ckpt), _ptr(delta_final)),
                    "pm_run")
        return pos, mom

    def pm_power(self, delta: torch.Tensor, n_bins: Optional[int] = None, n_max: int = 0, deconv: bool = False):
        n = self.workload.n_mesh
        self._dev(delta, (n, n, n), name="delta")
        nb = n // 2 if n_bins is None else n_bins
        k = (C.c_double * nb)()
        p = (C.c_double * nb)()
        m = (C.c_double * nb)()
        self._check(self.lib.pm_power(self.ctx, _ptr(delta), nb, n_max, int(deconv), k, p, m), "pm_power")
        return np.array(k), np.array(p), np.array(m)

    def pm_rfft(self, real: torch.Tensor):
        n = self.workload.n_mesh
        self._dev(real, (n, n, n), name="real")
        spec = torch.empty((n, n, n // 2 + 1), dtype=torch.complex64, device=self.device)
        self._check(self.lib.pm_rfft(self.ctx, _ptr(real), _ptr(spec)), "pm_rfft")
        return spec

    def pm_irfft(self, spec: torch.Tensor):
        n = self.workload.n_mesh
        self._dev(spec, (n, n, n // 2 + 1), dtype=torch.complex64, name="spec")
        real = torch.empty((n, n, n), dtype=torch.float32, device=self.device)
        self._check(self.lib.pm_irfft(self.ctx, _ptr(spec), _ptr(real)), "pm_irfft")
        return real

    def pm_set_force_ckpt(self, n_slots: int, fckpt: Optional[torch.Tensor] = None):
        """Keep the force meshes of runs of up to n_slots scale factors for the
        adjoint (0 switches it off).  Returns the buffer (allocated here when
        not given); it must stay alive while in use."""
        if n_slots <= 0:
            self._check(self.lib.pm_set_force_ckpt(self.ctx, None, 0), "pm_set_force_ckpt")
            self._fck = None
            return None
        m = self.workload.n_mesh
        if fckpt is None:
            fckpt = torch.empty(n_slots * m ** 3 * 3, dtype=torch.float32, device=self.device)
        self._dev(fckpt, (n_slots * m ** 3 * 3,), name="fckpt")
        self._check(self.lib.pm_set_force_ckpt(self.ctx, _ptr(fckpt), n_slots), "pm_set_force_ckpt")
        self._fck = fckpt
        return fckpt

    def pm_set_lpt_frame(self, psi1: Optional[torch.Tensor] = None, psi2: Optional[torch.Tensor] = None):
        """Register the LPT displacement fields of the COLA integrator, [np][3]
        each (created here, zeroed, when not given: pm_init_lpt then fills
        them).  pm_clear_lpt_frame unsets them."""
        if psi1 is None and psi2 is None:
            psi1 = torch.zeros((self.np3, 3), dtype=torch.float32, device=self.device)
            psi2 = torch.zeros((self.np3, 3), dtype=torch.float32, device=self.device)
        self._dev(psi1, (self.np3, 3), name="psi1")
        self._dev(psi2, (self.np3, 3), name="psi2")
        self._check(self.lib.pm_set_lpt_frame(self.ctx, _ptr(psi1), _ptr(psi2)), "pm_set_lpt_frame")
        self._frame = (psi1, psi2)
        return psi1, psi2

    def pm_clear_lpt_frame(self):
        self._check(self.lib.pm_set_lpt_frame(self.ctx, None, None), "pm_set_lpt_frame")
        self._frame = None

    def pm_use_graphs(self, enable: bool):
        self._check(self.lib.pm_use_graphs(self.ctx, int(enable)), "pm_use_graphs")

    def pm_profile(self, enable: bool):
        self._check(self.lib.pm_profile(self.ctx, int(enable)), "pm_profile")

    def pm_profile_read(self):
        """{class name: (total ms, launches)} of the kernels timed since pm_profile(True)."""
        mx = 64
        names = C.create_string_buffer(32 * mx)
        ms = (C.c_double * mx)()
        cnt = (C.c_int * mx)()
        k = self.lib.pm_profile_read(self.ctx, mx, names, ms, cnt)
        if k < 0:
            self._check(k, "pm_profile_read")
        out = {}
        for i in range(min(k, mx)):
            nm = names.raw[32 * i:32 * (i + 1)].split(b"\0", 1)[0].decode()
            out[nm] = (ms[i], cnt[i])
        return out

    def pm_run_adjoint(self, a_list, ckpt, noise=None, grad_delta=None, grad_pos=None, grad_mom=None,
                       want_noise_grad=True):
        """Cotangents of (x0, p0) and of the white noise for a loss on the final
        overdensity (grad_delta) and/or final state (grad_pos/grad_mom)."""
        a = np.ascontiguousarray(a_list, dtype=np.float64)
        n = self.workload.n_part
        self._dev(ckpt, (len(a), 2, self.np3, 3), name="ckpt")
        gx = torch.zeros((self.np3, 3), dtype=torch.float32, device=self.device) if grad_pos is None else grad_pos
        gp = torch.zeros((self.np3, 3), dtype=torch.float32, device=self.device) if grad_mom is None else grad_mom
        self._dev(gx, (self.np3, 3), name="grad_pos")
        self._dev(gp, (self.np3, 3), name="grad_mom")
        if grad_delta is not None:
            m = self.workload.n_mesh
            self._dev(grad_delta, (m, m, m), name="grad_delta")
        gn = None
        if want_noise_grad:
            if noise is None:
                raise PMError("the noise gradient needs the forward noise")
            self._dev(noise, (n, n, n), name="noise")
            gn = torch.empty((n, n, n), dtype=torch.float32, device=self.device)
        ap = a.ctypes.data_as(C.POINTER(C.c_double))
        self._check(self.lib.pm_run_adjoint(self.ctx, ap, len(a), _ptr(ckpt), _ptr(noise), _ptr(grad_delta),
                                            _ptr(gx), _ptr(gp), _ptr(gn)), "pm_run_adjoint")
        return gx, gp, gn

    # ---- MAP reconstruction ----------------------------------------------------
    def pm_chi2(self, delta, data, sigma: float, grad=None):
        """(chi^2 as a device float64 scalar, d chi^2 / d delta) of a model
        overdensity against data; asynchronous on the context's stream."""
        m = self.workload.n_mesh
        self._dev(delta, (m, m, m), name="delta")
        self._dev(data, (m, m, m), name="data")
        grad = torch.empty_like(delta) if grad is None else grad
        self._dev(grad, (m, m, m), name="grad")
        chi2 = torch.empty((), dtype=torch.float64, device=self.device)
        self._check(self.lib.pm_chi2(self.ctx, _ptr(delta), _ptr(data), sigma, _ptr(grad), _ptr(chi2)), "pm_chi2")
        return chi2, grad

    def pm_recon_work_bytes(self, n_a: int) -> int:
        return int(self.lib.pm_recon_work_bytes(self.ctx, n_a))

    def pm_recon_step(self, a_list, data, sigma: float, noise, adam_m, adam_v, t: int, lr: float,
                      beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8, work=None):
        """One Adam iteration of the reconstruction; updates noise, adam_m,
        adam_v in place and returns (chi^2, prior) before the update."""
        a = np.ascontiguousarray(a_list, dtype=np.float64)
        n, m = self.workload.n_part, self.workload.n_mesh
        self._dev(data, (m, m, m), name="data")
        for arr, nm in ((noise, "noise"), (adam_m, "adam_m"), (adam_v, "adam_v")):
            self._dev(arr, (n, n, n), name=nm)
        need = self.pm_recon_work_bytes(len(a))
        if work is None:
            work = torch.empty(need, dtype=torch.uint8, device=self.device)
        self._dev(work, dtype=torch.uint8, name="work")
        out = (C.c_double * 2)()
        self._check(self.lib.pm_recon_step(self.ctx, a.ctypes.data_as(C.POINTER(C.c_double)), len(a), _ptr(data),
                                           sigma, _ptr(noise), _ptr(adam_m), _ptr(adam_v), t, lr, beta1, beta2, eps,
                                           _ptr(work), work.numel(), out), "pm_recon_step")
        return float(out[0]), float(out[1])

    # ---- resumable run (continuous batching) ---------------------------------
    def pm_run_begin(self, a_list, pos, mom, ckpt: Optional[torch.Tensor] = None):
        self._dev(pos, (self.np3, 3), name="pos")
        self._dev(mom, (self.np3, 3), name="mom")
        a = np.ascontiguousarray(a_list, dtype=np.float64)
        if ckpt is not None:
            self._dev(ckpt, (len(a), 2, self.np3, 3), name="ckpt")
        self._run_refs = (pos, mom, ckpt)   # keep the arrays alive until pm_run_end
        ap = a.ctypes.data_as(C.POINTER(C.c_double))
        self._check(self.lib.pm_run_begin(self.ctx, ap, len(a), _ptr(pos), _ptr(mom), _ptr(ckpt)), "pm_run_begin")

    def pm_run_advance(self, max_steps: int = 1) -> int:
        rem = C.c_int(0)
        self._check(self.lib.pm_run_advance(self.ctx, max_steps, C.byref(rem)), "pm_run_advance")
        return rem.value

    def pm_run_end(self, delta_final: Optional[torch.Tensor] = None):
        if delta_final is not None:
            n = self.workload.n_mesh
            self._dev(delta_final, (n, n, n), name="delta_final")
        self._check(self.lib.pm_run_end(self.ctx, _ptr(delta_final)), "pm_run_end")
        refs = getattr(self, "_run_refs", None)
        self._run_refs = None
        return refs


def pm_force_static(workload: Workload, pos: torch.Tensor, out: Optional[torch.Tensor] = None,
                    max_particles: int = 0, stream=None) -> torch.Tensor:
    """PM force through the library's allocation-free entry point (its
    scratch is a fixed device array inside the library, so no workspace is
    created).  pos: (np, 3) float32 on the current GPU; out: the same shape,
    allocated here when not given (pass it to keep the call allocation-free)."""
    lib = _lib.load()
    if not isinstance(pos, torch.Tensor) or pos.device.type != "cuda" or pos.dtype != torch.float32:
        raise PMError("pos must be a float32 tensor on a GPU")
    if pos.ndim != 2 or pos.shape[1] != 3 or not pos.is_contiguous():
        raise PMError("pos must be a contiguous (np, 3) tensor")
    out = torch.empty_like(pos) if out is None else out
    if out.shape != pos.shape or out.dtype != torch.float32 or out.device != pos.device or not out.is_contiguous():
        raise PMError("out must be a contiguous float32 tensor shaped like pos on its device")
    cfg = make_config(workload, max_particles)
    s = stream if stream is not None else torch.cuda.current_stream(pos.device)
    with torch.cuda.device(pos.device):
        rc = lib.pm_force_static(C.byref(cfg), _ptr(pos), pos.shape[0], _ptr(out), C.c_void_p(s.cuda_stream))
    if rc != _lib.PM_OK:
        raise PMError(f"pm_force_static failed ({rc}): {lib.pm_strerror(rc).decode()}")
    return out


class PMBatch(PMContext):
    """A batch plan of `batch` member slots of one workload's shape
    (continuous batching): members join and leave while others run, and one
    batched step launches every kernel of a KDK step once for all running
    members.  Member m's context (``member(m)``) takes every single-simulation
    call (initial conditions, adjoint, chi^2, power spectrum) on its slot."""

    def __init__(self, workload: Workload, batch: int, device="cuda", stream=None):
        if batch < 2:
            raise PMError("a batch plan has at least 2 members")
        super().__init__(workload, device=device, stream=stream, batch=batch)
        self.batch = batch
        self._members = []
        for m in range(batch):
            h = C.c_void_p()
            self._check(self.lib.pm_batch_member(self.ctx, m, C.byref(h)), "pm_batch_member")
            self._members.append(PMContext._view(self, h))
        self._refs = {}

    def member(self, m: int) -> PMContext:
        return self._members[m]

    def set_stream(self, stream):
        super().set_stream(stream)
        for v in self._members:
            v.stream = stream

    def pm_batch_begin(self, m: int, a_list, pos, mom, ckpt: Optional[torch.Tensor] = None):
        self._dev(pos, (self.np3, 3), name="pos")
        self._dev(mom, (self.np3, 3), name="mom")
        a = np.ascontiguousarray(a_list, dtype=np.float64)
        if ckpt is not None:
            self._dev(ckpt, (len(a), 2, self.np3, 3), name="ckpt")
        ap = a.ctypes.data_as(C.POINTER(C.c_double))
        self._check(self.lib.pm_batch_begin(self.ctx, m, ap, len(a), _ptr(pos), _ptr(mom), _ptr(ckpt)),
                    "pm_batch_begin")
        self._refs[m] = (pos, mom, ckpt)   # the library writes them at pm_batch_end

    def pm_batch_advance(self) -> int:
        k = C.c_int(0)
        self._check(self.lib.pm_batch_advance(self.ctx, C.byref(k)), "pm_batch_advance")
        return k.value

    def pm_batch_remaining(self, m: int) -> int:
        r = self.lib.pm_batch_remaining(self.ctx, m)
        if r < 0:
            self._check(r, "pm_batch_remaining")
        return r

    def pm_batch_end(self, m: int, delta_final: Optional[torch.Tensor] = None, check_steps: bool = True):
        """check_steps: require every step counted by pm_batch_advance (pass
        False for a member stepped through pm_kdk_step_batched)."""
        if delta_final is not None:
            n = self.workload.n_mesh
            self._dev(delta_final, (n, n, n), name="delta_final")
        if check_steps and self.pm_batch_remaining(m) != 0:
            raise PMError(f"member {m} still has steps to take")
        self._check(self.lib.pm_batch_end(self.ctx, m, _ptr(delta_final)), "pm_batch_end")
        return self._refs.pop(m, None)

    def pm_kdk_step_batched(self, descs: torch.Tensor, n: int):
        """descs: a uint8 device tensor holding n pm_req_desc entries."""
        if descs.device != self.device or descs.dtype != torch.uint8 or not descs.is_contiguous():
            raise PMError("descs must be a contiguous uint8 tensor on the plan's device")
        if descs.numel() < n * C.sizeof(_lib.pm_req_desc):
            raise PMError("descs holds fewer than n descriptors")
        self._check(self.lib.pm_kdk_step_batched(self.ctx, _ptr(descs), n), "pm_kdk_step_batched")

    def close(self):
        for v in getattr(self, "_members", []):
            v.ctx = None
        super().close()


def req_descs(entries) -> bytes:
    """Pack (member, flags, kick_close, kick_open, drift, ckpt_x_ptr, ckpt_p_ptr)
    tuples as pm_req_desc structures (host bytes, to be copied to the device)."""
    arr = (_lib.pm_req_desc * len(entries))()
    for i, (m, fl, kc, ko, dr, cx, cp) in enumerate(entries):
        arr[i] = _lib.pm_req_desc(m, fl, kc, ko, dr, 0.0, cx, cp, 0)
    return bytes(arr)
