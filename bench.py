"""Benchmark of the PM kick-drift-kick hot path on one MI355X.

A "step" is one KDK step of the whole path: CIC readout + kick + drift,
counting sort by tile, LDS-tiled CIC paint, r2c FFT, fused Green/gradient
x pass, inverse FFTs to three force meshes.  Each timed region is one
``pm_run`` over K steps (it includes the force at the first scale factor and
the closing half kick) on 512^3 particles / 1024^3 mesh / 1024 Mpc/h, with
the initial conditions already resident in HBM; after the warm-up, R such
runs (default 5) are timed and the median one is reported.

Prints one JSON line.  Extra objects: ``roofline`` (dominant kernel class,
algorithmic bytes / average event-timed duration vs 8 TB/s) and
``cpu_baseline`` (the FP64 oracle timed on a bounded sample on this host).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def kernel_bytes(w, np3):
    """Algorithmic HBM bytes per launch of each timed kernel class (float32).

    Mesh field F = N^3 reals = N^2 (N/2) complex, plus the Nyquist plane of
    N^2 complex values.  Particle state 24 B (x, p), id 4 B, sort key 4 B.
    The x_force and y_inv figures are those of meshes from 64^3 up, where F_y
    and F_z share one inverse x transform.
    """
    n = w.n_mesh
    real = 4.0 * n ** 3
    spec = 4.0 * n ** 3 + 8.0 * n * n
    return {
        "fft_z_r2c": real + spec,                       # 1 field
        "fft_y_fwd": 2 * spec,                          # 1 field, in place
        "fft_x_force": 3 * spec,                        # spectrum in; F_x and i g X (shared by F_y, F_z) out
        "fft_y_inv": 2 * spec + 3 * spec,               # F_x and the shared factor in; F_x, F_y, F_z out
        "fft_z_c2r": 3 * (spec + real),                 # 3 fields
        "paint": 12.0 * np3 + real,                     # positions in, mesh out
        "readout_kdk": 3 * real + np3 * (24 + 24 + 4),  # 3 meshes + x,p in; x,p,key out
        "scatter": np3 * (4 + 28 + 28),                 # key, state in, state out
    }


def end_to_end(w, np3, sec_per_step):
    """Bytes the method itself must move per step (paint: positions in, mesh
    out; r2c; Green + 3 inverse transforms: spectrum in once, 3 meshes out;
    readout: 3 meshes and 48 B of particle state) against the step time."""
    n = w.n_mesh
    real = 4.0 * n ** 3
    spec = 4.0 * n ** 3 + 8.0 * n * n
    b = (12.0 * np3 + real) + (real + spec) + (spec + 3 * real) + (3 * real + 48.0 * np3)
    gbs = b / sec_per_step / 1e9
    return {"method_bytes_per_step": b, "achieved_GBps": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4)}


def kernel_source_hash():
    """sha256 over the kernel sources (csrc/*.hip, *.h, *.cpp and include/pm.h),
    the key that ties a committed counter summary to the code it measured."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_2010_11847_amd", "csrc")
    files = sorted(f for f in os.listdir(csrc) if f.endswith((".hip", ".h", ".cpp")))
    h = hashlib.sha256()
    paths = [os.path.join(csrc, f) for f in files] + [os.path.join(ROOT, "include", "pm.h")]
    for f, path in zip(files + ["pm.h"], paths):
        with open(path, "rb") as fh:
            h.update(f.encode())
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload, kernel_class):
    """HBM bytes per launch of one kernel class from the committed rocprofv3
    counter summary profiles/hbm_traffic_<workload>.txt, or None when the
    summary is missing or was taken on other kernel sources."""
    path = os.path.join(ROOT, "profiles", f"hbm_traffic_{workload}.txt")
    if not os.path.exists(path):
        return None
    sha, rows = None, {}
    with open(path) as fh:
        for line in fh:
            parts = line.split()
            if len(parts) >= 2 and parts[0] == "sources_sha256:":
                sha = parts[1]
            elif len(parts) >= 4 and parts[0] == "class":
                rows[parts[1]] = float(parts[2]) + float(parts[3])
    if sha != kernel_source_hash() or kernel_class not in rows:
        return None
    return rows[kernel_class]


def cpu_baseline():
    """The oracle (FP64 NumPy/SciPy, unmodified) timed on this host at the
    small configurations, about 30 s of CPU work in all:
      - 32^3 particles on 32^3 (100 Mpc/h, power law), 10 KDK steps;
      - 128^3 particles on 256^3 (256 Mpc/h, no-wiggle), 10 KDK steps: the
        headline figure, in particle-steps/s (same B = 2 and 1 Mpc/h cells as
        the 512^3 / 1024^3 workload);
      - 64^3 particles on 128^3 (200 Mpc/h), 5 steps: forward run plus the
        adjoint (gradient of the chi^2 loss w.r.t. the white noise).
    Each run starts from the oracle's own 2LPT initial conditions (not
    timed)."""
    import numpy as np
    from oracle import adjoint as A
    from oracle import lpt, pm
    from oracle.rng import white_noise
    from paper_2010_11847_amd import inputs
    out = {}

    def run(w):
        x, p = lpt.generate(w)
        t0 = time.perf_counter()
        pm.kdk_run(x, p, w.a_list, w.n_mesh, w.n_particles, w.cosmo.omega_m)
        dt = time.perf_counter() - t0
        return {"particle_steps_per_s": w.n_particles * w.n_steps / dt, "s": round(dt, 2)}
    out["pm32_box100_powerlaw"] = run(inputs.SMALL)
    out["pm128_mesh256_box256"] = run(inputs.MEDIUM)
    w = inputs.ADJ_SMALL
    noise = white_noise(w.seed, w.n_part)
    target = np.zeros((w.n_mesh,) * 3)
    t0 = time.perf_counter()
    A.loss_and_grad(noise, w, target, 0.1)
    dt = time.perf_counter() - t0
    out["adj64_mesh128_box200"] = {"gradients_per_s": 1.0 / dt, "s": round(dt, 2),
                                   "what": "2LPT + 5-step forward run + adjoint to the white noise"}
    med = out["pm128_mesh256_box256"]
    cores = len(os.sched_getaffinity(0))
    return {"value": med["particle_steps_per_s"], "unit": "particle-steps/s", "cores": pm._WORKERS,
            "kind": "oracle",
            "sample": f"128^3 particles on 256^3 mesh, 256 Mpc/h, 10 KDK steps incl. first force, {med['s']} s wall "
                      f"(same B=2, 1 Mpc/h cell, no-wiggle P(k) as the headline workload); DFTs on {pm._WORKERS} "
                      f"threads (scipy.fft), paint/readout 1 thread; host cpu_count {os.cpu_count()}, "
                      f"affinity {cores}",
            "configs": out}


def adjoint_section(names=("adj128_mesh256_box400", "pm512_mesh1024_box1024"), reps=2):
    """Forward run with per-step checkpoints plus the reverse sweep (gradient
    of a loss on the final overdensity with respect to the white noise),
    timed with HIP events; one untimed warm-up each."""
    import torch
    from paper_2010_11847_amd import inputs
    from paper_2010_11847_amd.binding import PMContext
    out = {}
    for name in names:
        w = inputs.PRESETS[name]
        c = PMContext(w)
        n, m = w.n_part, w.n_mesh
        g = torch.Generator(device="cuda").manual_seed(w.seed + 2000)
        noise = torch.randn((n, n, n), device="cuda", generator=g)
        gd = torch.randn((m, m, m), device="cuda", generator=g)
        ckpt = torch.empty((len(w.a_list), 2, c.np3, 3), device="cuda")
        delta = torch.empty((m, m, m), device="cuda")

        def once():
            pos, mom = c.pm_init_lpt(0, w.a_list[0], noise=noise)
            e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
            e0.record()
            c.pm_run(w.a_list, pos, mom, ckpt=ckpt, delta_final=delta)
            e1.record()
            c.pm_run_adjoint(w.a_list, ckpt, noise=noise, grad_delta=gd)
            e2.record()
            torch.cuda.synchronize()
            return e0.elapsed_time(e1), e1.elapsed_time(e2)

        once()
        fw, bw = zip(*[once() for _ in range(reps)])
        f, b = min(fw), min(bw)
        # the same with the forward's force meshes kept for the reverse sweep
        c.pm_set_force_ckpt(len(w.a_list))
        once()
        fw2, bw2 = zip(*[once() for _ in range(reps)])
        c.pm_set_force_ckpt(0)
        f2, b2 = min(fw2), min(bw2)
        out[name] = {"n_part": n, "n_mesh": m, "steps": w.n_steps, "forward_ckpt_ms": round(f, 2),
                     "adjoint_ms": round(b, 2), "gradients_per_s": round(1e3 / (f + b), 3),
                     "adjoint_over_forward": round(b / f, 2),
                     "with_force_ckpt": {"forward_ms": round(f2, 2), "adjoint_ms": round(b2, 2),
                                         "gradients_per_s": round(1e3 / (f2 + b2), 3),
                                         "extra_hbm_gb": round(len(w.a_list) * m ** 3 * 12 / 1e9, 1)}}
        print(f"[bench] adjoint {name} {out[name]}", file=sys.stderr, flush=True)
        del c, noise, gd, ckpt, delta
        torch.cuda.empty_cache()
    return out


def pyramid_section(w, steps):
    """The same run with the two-level pyramid force (section 5.2, f = 2):
    step time and the extra kernel classes (the paper's scheme targets
    distributed meshes; on one device it adds its passes to the full force)."""
    import torch
    from dataclasses import replace
    from paper_2010_11847_amd.binding import PMContext
    wp = replace(w, pyramid_levels=2)
    c = PMContext(wp)
    pos, mom = c.pm_init_lpt(wp.seed, wp.a_list[0])
    a = inputs_a(wp, steps)
    c.pm_run(a, pos.clone(), mom.clone())
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    c.pm_run(a, pos, mom)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    c.pm_profile(True)
    c.pm_run(a, pos, mom)
    prof = c.pm_profile_read()
    c.pm_profile(False)
    out = {"levels": 2, "coarse_mesh": wp.n_mesh >> 2, "ms_per_step": round(ms, 2),
           "kernels_ms_per_step": {k: round(v[0] / (steps + 1), 3) for k, v in prof.items() if k.startswith("pyr")}}
    print(f"[bench] pyramid {out}", file=sys.stderr, flush=True)
    del c, pos, mom
    torch.cuda.empty_cache()
    return out


def inputs_a(w, steps):
    from paper_2010_11847_amd import inputs
    return inputs.a_linear(w.a_list[0], w.a_list[-1], steps)


def recon_section(n_iter=10):
    """Iterations of the section 7 reconstruction (dark-matter observable):
    the paper's own problem (5 KDK steps, 128^3 grid, 400 Mpc/h, force
    resolution 1) and the 128^3/256^3 adjoint workload.  Data: the final
    overdensity of another noise realisation plus Gaussian noise (sigma 0.1)."""
    import torch
    from paper_2010_11847_amd import inputs
    from paper_2010_11847_amd.binding import PMContext
    from paper_2010_11847_amd.recon import Reconstruction
    out = {}
    from dataclasses import replace
    paper = replace(inputs.ADJ_MEDIUM, name="recon128_mesh128_box400", n_mesh=128)
    for w in (paper, inputs.ADJ_MEDIUM):
        c = PMContext(w)
        m = w.n_mesh
        pos, mom = c.pm_init_lpt(w.seed + 1000, w.a_list[0])
        data = torch.empty((m, m, m), device="cuda")
        c.pm_run(w.a_list, pos, mom, delta_final=data)
        g = torch.Generator(device="cuda").manual_seed(w.seed + 2000)
        data += 0.1 * torch.randn((m, m, m), device="cuda", generator=g)
        r = Reconstruction(c, w.a_list, data, 0.1, lr=0.01)
        r.run(2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        hist = r.run(n_iter)
        dt = (time.perf_counter() - t0) / n_iter
        out[w.name] = {"n_part": w.n_part, "n_mesh": w.n_mesh, "box_mpc_h": w.box_size, "steps": w.n_steps,
                       "ms_per_iteration": round(dt * 1e3, 2), "iterations": n_iter,
                       "loss_first": round(sum(hist[0]), 1), "loss_last": round(sum(hist[-1]), 1)}
        print(f"[bench] recon {w.name} {out[w.name]}", file=sys.stderr, flush=True)
        del r, c, data, pos, mom
        torch.cuda.empty_cache()
    out["paper_s_per_iteration_v100"] = 1.1
    return out


def serving_section(n_requests, rate=20.0, seed=5, budget_gb=64.0, slots=4):
    """Continuous batching (batch plans, batched steps) vs one request at a
    time on the same Poisson trace, then the same requests arriving at once
    (throughput), and the forward+gradient requests alone."""
    from paper_2010_11847_amd import serve
    trace = serve.poisson_trace(n_requests, rate, seed)
    warm = serve.poisson_trace(24, 1000.0, seed + 1)
    budget = int(budget_gb * (1 << 30))
    ex = serve.BatchedExecutor(slots_per_class=slots, keep_results=False)
    fifo_ex = serve.GpuExecutor(keep_results=False)
    serve.serve(warm, ex, budget, slots, realtime=False)          # builds the plans and their graphs
    serve.serve_fifo(warm, fifo_ex, realtime=False)               # builds the per-class contexts
    print(f"[bench] serving: Poisson trace of {n_requests} requests at {rate}/s, continuous batching",
          file=sys.stderr, flush=True)
    cb = serve.serve(trace, ex, budget, slots, realtime=True).summary()
    print(f"[bench] serving continuous {cb}", file=sys.stderr, flush=True)
    fifo = serve.serve_fifo(trace, fifo_ex, realtime=True).summary()
    print(f"[bench] serving fifo {fifo}", file=sys.stderr, flush=True)
    # saturated: the same requests all arriving at once (maximum throughput)
    burst = [serve.SimRequest(r.rid, r.n_part, r.n_mesh, r.box_size, r.n_steps, r.seed, r.with_grad, 0.0)
             for r in trace]
    cb_sat = serve.serve(burst, ex, budget, slots, realtime=True).summary()
    print(f"[bench] serving burst continuous {cb_sat}", file=sys.stderr, flush=True)
    fifo_sat = serve.serve_fifo(burst, fifo_ex, realtime=True).summary()
    print(f"[bench] serving burst fifo {fifo_sat}", file=sys.stderr, flush=True)
    # forward + gradient requests alone (128^3 particles on 128^3, chi^2 adjoint)
    grad = [r for r in burst if r.with_grad]
    cb_grad = serve.serve(grad, ex, budget, slots, realtime=True).summary()
    print(f"[bench] serving fwd+grad burst continuous {cb_grad}", file=sys.stderr, flush=True)
    fifo_grad = serve.serve_fifo(grad, fifo_ex, realtime=True).summary()
    print(f"[bench] serving fwd+grad burst fifo {fifo_grad}", file=sys.stderr, flush=True)
    del ex, fifo_ex
    return {"requests": n_requests, "rate_per_s": rate, "arrival_seed": seed, "hbm_budget_gb": budget_gb,
            "slots_per_class": slots, "grad_requests": len(grad),
            "mix": "60% fwd 64^3/64^3, 30% fwd+grad 128^3/128^3, 10% fwd 256^3/512^3, 5-10 steps",
            "continuous": "one batch plan per shape class (all slots' workspaces), one batched step per class "
                          "per tick (captured graph), classes on separate streams, <= 2 steps in flight per class",
            "fifo": "one request at a time, each on a context of its own (captured step graphs)",
            "poisson": {"continuous": cb, "fifo": fifo},
            "burst": {"continuous": cb_sat, "fifo": fifo_sat},
            "fwd_grad_burst": {"continuous": cb_grad, "fifo": fifo_grad}}


def optional(name, fn, *args):
    """Run a secondary section; its failure (e.g. device memory) is reported
    in the JSON line instead of losing the headline measurement."""
    import torch
    try:
        return fn(*args)
    except Exception as e:   # noqa: BLE001 - any failure of a side section
        print(f"[bench] {name} section failed: {e!r}", file=sys.stderr, flush=True)
        torch.cuda.empty_cache()
        return {"error": repr(e)[:300]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--repeats", type=int, default=5,
                    help="timed runs of --steps steps each; the median is reported")
    ap.add_argument("--workload", default="pm512_mesh1024_box1024")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-profile", action="store_true", help="skip the event-timed profile pass")
    ap.add_argument("--calibrate-copy", type=float, default=0.0, metavar="GIB",
                    help="only run a plain device-to-device copy of GIB GiB (counter calibration) and exit")
    ap.add_argument("--no-adjoint", action="store_true",
                    help="skip the pyramid, gradient (adjoint) and reconstruction timing sections")
    ap.add_argument("--serve", type=int, default=1000,
                    help="requests of the serving trace (Poisson 20/s); 0 skips the serving section")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs one GPU only: the PM hot path here is the single-GPU share; "
              "multi-GPU sharding is not built (use --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2010_11847_amd import inputs
    from paper_2010_11847_amd.binding import PMContext

    if args.calibrate_copy > 0:
        n = int(args.calibrate_copy * (1 << 30)) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes_read": 4 * n, "calibrate_copy_bytes_written": 4 * n,
                          "launches": 3}))
        return

    w = inputs.PRESETS[args.workload]
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    ctx = PMContext(w, device=dev)
    np3 = w.n_particles

    t0 = time.perf_counter()
    pos0, mom0 = ctx.pm_init_lpt(w.seed, w.a_list[0])
    torch.cuda.synchronize()
    init_s = time.perf_counter() - t0
    print(f"[bench] init_lpt {init_s * 1e3:.1f} ms", file=sys.stderr, flush=True)
    pos = torch.empty_like(pos0)
    mom = torch.empty_like(mom0)

    def run(nsteps):
        a = inputs.a_linear(w.a_list[0], w.a_list[-1], nsteps)
        pos.copy_(pos0)
        mom.copy_(mom0)
        torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record()
        ctx.pm_run(a, pos, mom)
        ev1.record()
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1) / 1e3

    for _ in range(max(0, args.warmup)):
        run(max(1, args.steps))
        print("[bench] warmup done", file=sys.stderr, flush=True)
    # R timed runs of exactly K steps each (each bracketed by device
    # synchronisation); the median run is reported
    runs = []
    for _ in range(max(1, args.repeats)):
        runs.append(run(args.steps))
        print(f"[bench] timed {args.steps} steps: {runs[-1] * 1e3:.1f} ms", file=sys.stderr, flush=True)
    t = sorted(runs)[len(runs) // 2]
    value = np3 * args.steps / t

    roofline = None
    kernels = {}
    if not args.no_profile:
        ctx.pm_profile(True)
        run(args.steps)
        prof = ctx.pm_profile_read()
        ctx.pm_profile(False)
        nbytes = kernel_bytes(w, np3)
        for name, (ms, cnt) in prof.items():
            avg = ms / cnt
            ent = {"total_ms": round(ms, 3), "launches": cnt, "avg_ms": round(avg, 4)}
            if name in nbytes:
                ent["GBps"] = round(nbytes[name] / (avg / 1e3) / 1e9, 1)
                ent["frac"] = round(ent["GBps"] / HBM_PEAK_GBS, 4)
            kernels[name] = ent
        dom = max((k for k in kernels if k in nbytes), key=lambda k: kernels[k]["total_ms"])
        ach = kernels[dom]["GBps"]
        traffic = measured_traffic(w.name, dom)
        roofline = {"bound": "hbm", "kernel": dom, "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": traffic,
                    "bytes_per_launch": nbytes[dom], "avg_launch_ms": kernels[dom]["avg_ms"]}
        print(f"[bench] kernels {json.dumps(kernels)}", file=sys.stderr, flush=True)

    # the particle kernels at the start and at the end of the run: one force
    # evaluation on the 2LPT positions (a = 0.1, nearly uniform) and on the
    # final ones (a = 1, clustered: heavy tiles)
    by_epoch = None
    if not args.no_profile:
        by_epoch = {}
        for label, p in (("a0.1", pos0), ("a1.0", pos)):
            f = ctx.pm_force(p)
            ctx.pm_profile(True)
            ctx.pm_force(p, out=f)
            pr = ctx.pm_profile_read()
            ctx.pm_profile(False)
            for k in ("scatter", "paint", "readout_kdk"):
                if k in pr:
                    by_epoch[f"{label}_{k}_ms"] = round(pr[k][0] / pr[k][1], 4)
            del f
        print(f"[bench] particle kernels by epoch {by_epoch}", file=sys.stderr, flush=True)

    del ctx, pos, mom, pos0, mom0
    torch.cuda.empty_cache()
    pyramid = None if args.no_adjoint else optional("pyramid", pyramid_section, w, args.steps)
    adjoint = None if args.no_adjoint else optional("adjoint", adjoint_section)
    reconstruction = None if args.no_adjoint else optional("reconstruction", recon_section)
    serving = None
    if args.serve > 0:
        serving = optional("serving", serving_section, args.serve)

    base = None
    if not args.no_cpu:
        base = optional("cpu_baseline", cpu_baseline)

    out = {
        "metric": "particle-steps/s (PM KDK) at 512^3/1024^3",
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t * 1e3 / args.steps,
        "runs_ms_per_step": [round(r * 1e3 / args.steps, 3) for r in runs],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "n_part": w.n_part, "n_mesh": w.n_mesh, "box_mpc_h": w.box_size,
                   "seed": w.seed, "a0": w.a_list[0], "a1": w.a_list[-1], "lpt_order": w.lpt_order,
                   "pk": "eisenstein_hu_nowiggle", "init_lpt_ms": round(init_s * 1e3, 1)},
        "roofline": roofline,
        "end_to_end": end_to_end(w, np3, t / args.steps),
        "cpu_baseline": base,
        "pyramid": pyramid,
        "adjoint": adjoint,
        "reconstruction": reconstruction,
        "serving": serving,
        "kernels": kernels,
        "particle_kernels_by_epoch": by_epoch,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
