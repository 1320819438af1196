"""Seeded synthetic inputs and workload presets.

This module is shared by the oracle-based tests and the GPU path.  It holds
no arithmetic of the particle-mesh method: only workload descriptions (sizes,
seeds, scale-factor lists, cosmological parameters) and seeded random arrays
(particle positions, cotangents) drawn with NumPy's PCG64 generator.

The white noise that seeds the initial conditions is *not* drawn here: both
the oracle and the HIP library implement the same counter-based generator
(SplitMix64 finaliser + Box-Muller) from its published definition and draw it
from the seed themselves.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import Optional, Tuple

import numpy as np

PK_POWERLAW = 0
PK_EH_NOWIGGLE = 1
PK_TABLE = 2

SPLIT_NONE = 0
SPLIT_LONG = 1
SPLIT_SHORT = 2

INT_FASTPM = 0      # FastPM kick/drift factors
INT_LEAPFROG = 1    # plain leapfrog factors
INT_COLA = 2        # plain leapfrog in the LPT frame


@dataclass(frozen=True)
class Cosmology:
    """Flat LCDM background and linear power spectrum parameters.

    The method needs Omega_m for the Poisson equation and growth factors
    (the paper's FastPM scheme, section 2) and a linear P(k) to scale the
    Gaussian field (Gen-IC algorithm, section 6).  Omega_b, h, n_s and
    T_cmb only enter the no-wiggle transfer function.
    """
    omega_m: float = 0.3
    omega_b: float = 0.05
    h: float = 0.7
    n_s: float = 0.96
    sigma8: float = 0.8
    t_cmb: float = 2.7255
    pk_kind: int = PK_EH_NOWIGGLE
    pk_amp: float = 0.0      # 0: normalise to sigma8 (PK_TABLE: 0 means 1, the table as given)
    pk_index: float = -2.0   # power-law index (PK_POWERLAW)
    pk_table: Tuple[Tuple[float, ...], Tuple[float, ...]] = ()   # PK_TABLE: (k in h/Mpc increasing, P)


@dataclass(frozen=True)
class Workload:
    name: str
    box_size: float          # Mpc/h
    n_mesh: int              # mesh cells per side
    n_part: int              # particles per side
    seed: int
    a_list: Tuple[float, ...]
    cosmo: Cosmology = field(default_factory=Cosmology)
    lpt_order: int = 2
    deconv_order: int = 0
    split_rs: float = 0.0
    split_mode: int = SPLIT_NONE
    lattice_shift: float = 0.0   # particle lattice offset from mesh nodes, in cells
    pyramid_levels: int = 0      # 0: single-grid force; f: two-level pyramid force, grid n_mesh / 2^f
    integrator: int = INT_FASTPM

    @property
    def n_particles(self) -> int:
        return self.n_part ** 3

    @property
    def n_steps(self) -> int:
        return len(self.a_list) - 1

    @property
    def ratio(self) -> int:
        return self.n_mesh // self.n_part


def a_linear(a0: float, a1: float, n_steps: int) -> Tuple[float, ...]:
    """Scale factors linearly spaced in a (the paper's steps are linear in a)."""
    return tuple(float(v) for v in np.linspace(a0, a1, n_steps + 1))


POWERLAW = Cosmology(pk_kind=PK_POWERLAW, pk_index=-2.0)

# 32^3 particles on a 32^3 mesh, 100 Mpc/h, P = A k^-2 with A fixed by sigma8.
SMALL = Workload("pm32_box100_powerlaw", 100.0, 32, 32, 0, a_linear(0.1, 1.0, 10), POWERLAW)
# 128^3 particles on a 256^3 mesh, 256 Mpc/h, no-wiggle P(k).
MEDIUM = Workload("pm128_mesh256_box256", 256.0, 256, 128, 1, a_linear(0.1, 1.0, 10))
# 512^3 particles on a 1024^3 mesh, 1024 Mpc/h (the single-GPU headline size).
LARGE = Workload("pm512_mesh1024_box1024", 1024.0, 1024, 512, 2, a_linear(0.1, 1.0, 10))
# Differentiable runs: 5 KDK steps.
ADJ_SMALL = Workload("adj64_mesh128_box200", 200.0, 128, 64, 3, a_linear(0.1, 1.0, 5))
ADJ_MEDIUM = Workload("adj128_mesh256_box400", 400.0, 256, 128, 4, a_linear(0.1, 1.0, 5))

PRESETS = {w.name: w for w in (SMALL, MEDIUM, LARGE, ADJ_SMALL, ADJ_MEDIUM)}


def scaled(w: Workload, n_mesh: int, n_part: int, box_size: Optional[float] = None,
           n_steps: Optional[int] = None, **kw) -> Workload:
    """Same physics recipe at another size (for tests that must finish fast)."""
    box = box_size if box_size is not None else w.box_size * n_mesh / w.n_mesh
    a = w.a_list if n_steps is None else a_linear(w.a_list[0], w.a_list[-1], n_steps)
    return replace(w, name=f"{w.name}@{n_part}/{n_mesh}", n_mesh=n_mesh, n_part=n_part,
                   box_size=box, a_list=a, **kw)


# ---------------------------------------------------------------------------
# Seeded random arrays (PCG64).  Used for operator-level tests: paint, force,
# readout and adjoint dot-product tests need particle sets and cotangents.
# ---------------------------------------------------------------------------

def uniform_positions(n: int, n_mesh: int, seed: int) -> np.ndarray:
    """n particles uniformly in the periodic box [0, n_mesh)^3, float32."""
    rng = np.random.default_rng(seed)
    x = rng.random((n, 3), dtype=np.float64) * n_mesh
    x = x.astype(np.float32)
    x[x >= n_mesh] = 0.0
    return x


def clustered_positions(n: int, n_mesh: int, seed: int, n_clumps: int = 8,
                        width: float = 1.5, frac: float = 0.6) -> np.ndarray:
    """A mix of uniform particles and tight Gaussian clumps (late-time halos)."""
    rng = np.random.default_rng(seed)
    n_c = int(n * frac)
    centres = rng.random((n_clumps, 3)) * n_mesh
    which = rng.integers(0, n_clumps, n_c)
    xc = centres[which] + rng.normal(0.0, width, (n_c, 3))
    xu = rng.random((n - n_c, 3)) * n_mesh
    x = np.concatenate([xc, xu], 0) % n_mesh
    x = x[rng.permutation(n)].astype(np.float32)
    x[x >= n_mesh] = 0.0
    return x


def perturbed_lattice(n_part: int, n_mesh: int, seed: int, amp: float = 0.5) -> np.ndarray:
    """Particles on the n_part^3 lattice (spacing n_mesh/n_part) with random offsets."""
    rng = np.random.default_rng(seed)
    b = n_mesh // n_part
    i = np.arange(n_part)
    q = np.stack(np.meshgrid(i, i, i, indexing="ij"), -1).reshape(-1, 3).astype(np.float64) * b
    x = (q + rng.normal(0.0, amp, q.shape)) % n_mesh
    x = x.astype(np.float32)
    x[x >= n_mesh] = 0.0
    return x


def normal_array(shape, seed: int, scale: float = 1.0) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return (rng.standard_normal(shape) * scale).astype(np.float32)


def sample_indices(n_total: int, n: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(n_total, size=min(n, n_total), replace=False))
