"""Counter-based Gaussian white noise (float64).

Test infrastructure: see the package docstring.

The paper only says that the initial condition generator samples a 3D normal
random field (Gen-IC algorithm, section 6).  Reading: a counter-based stream
that any implementation can reproduce bit for bit:

* integer stream: the SplitMix64 output function of Steele, Lea & Flood,
  "Fast splittable pseudorandom number generators" (OOPSLA 2014), applied to
  the counter  c = seed * 2^40 + i  (lattice site i in C order), i.e. the
  first output of a SplitMix64 generator whose state is c;
* normal deviate: the Box-Muller transform (cosine branch only) with
  u1 = (hi32 + 1) 2^-32 in (0, 1] and u2 = lo32 2^-32 in [0, 1).
"""
from __future__ import annotations

import numpy as np

GOLDEN = np.uint64(0x9E3779B97F4A7C15)
M1 = np.uint64(0xBF58476D1CE4E5B9)
M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(state):
    """First SplitMix64 output for each 64-bit state (vectorised, wrapping)."""
    with np.errstate(over="ignore"):
        z = np.asarray(state, dtype=np.uint64) + GOLDEN
        z = (z ^ (z >> np.uint64(30))) * M1
        z = (z ^ (z >> np.uint64(27))) * M2
        return z ^ (z >> np.uint64(31))


def counter_bits(seed: int, start: int, count: int):
    with np.errstate(over="ignore"):
        base = np.uint64(seed) * np.uint64(1 << 40)
        idx = np.arange(start, start + count, dtype=np.uint64)
        return splitmix64(base + idx)


def box_muller(bits):
    hi = (bits >> np.uint64(32)).astype(np.float64)
    lo = (bits & np.uint64(0xFFFFFFFF)).astype(np.float64)
    u1 = (hi + 1.0) * 2.0 ** -32
    u2 = lo * 2.0 ** -32
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)


def white_noise(seed: int, n: int):
    """Unit-variance Gaussian field on an n^3 lattice, C order [x][y][z]."""
    out = np.empty(n ** 3, dtype=np.float64)
    chunk = 1 << 22
    for s in range(0, n ** 3, chunk):
        c = min(chunk, n ** 3 - s)
        out[s:s + c] = box_muller(counter_bits(seed, s, c))
    return out.reshape(n, n, n)
