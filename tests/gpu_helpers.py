"""Shared helpers of the GPU parity tests."""
import numpy as np
import torch


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def to_dev(x, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(x)).to(device="cuda", dtype=dtype)


def to_np(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def banner(msg):
    print(f"[gpu] {msg}", flush=True)
