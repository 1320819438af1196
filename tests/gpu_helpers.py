"""Shared helpers of the GPU parity tests."""
import json
import os

import numpy as np
import torch

_METRICS = {}


def rel(a, b):
    """Norm-wise relative error ||a - b|| / ||b||; complex arrays keep their
    imaginary parts."""
    a = np.asarray(a)
    b = np.asarray(b)
    dt = np.complex128 if (np.iscomplexobj(a) or np.iscomplexobj(b)) else np.float64
    a = a.astype(dt)
    b = b.astype(dt)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def to_dev(x, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(x)).to(device="cuda", dtype=dtype)


def to_np(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def f32(x):
    """Round to float32 and back: the state both sides are fed."""
    return np.asarray(x, dtype=np.float32).astype(np.float64)


def banner(msg):
    print(f"[gpu] {msg}", flush=True)


def record(name, value, bar=None):
    """Keep a measured error and the bar its test asserts (None: reported,
    not asserted); written to $PM_METRICS_DIR/parity_margins.json when that
    variable is set."""
    _METRICS[name] = {"value": float(value), "bar": None if bar is None else float(bar)}
    out = os.environ.get("PM_METRICS_DIR")
    if out:
        os.makedirs(out, exist_ok=True)
        path = os.path.join(out, "parity_margins.json")
        old = {}
        if os.path.exists(path):
            with open(path) as fh:
                old = json.load(fh)
        old.update(_METRICS)
        with open(path, "w") as fh:
            json.dump(old, fh, indent=1, sort_keys=True)
