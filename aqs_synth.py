"""Seeded synthetic inputs shared by the GPU path's tests/benchmark and the
CPU oracle.

This module draws random numbers and lays out boxes; it holds none of the
method's arithmetic (no potential, no minimiser, no deformation step).

The paper's 1000 melt-quenched 2D samples (Sec. 2.2, "The benchmark
problem") are not available, so binary Lennard-Jones glasses of the
Kob-Andersen type stand in for them: uniform random positions in a square or
cubic periodic box at number density 1.2, an exact A:B count drawn by a
seeded permutation, then an energy minimisation (done by the caller) to an
inherent structure.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

DENSITY = 1.2
X_A = {2: 0.65, 3: 0.80}
SEED_BASE = (2507, 20802)


def rng_for(*words: int) -> np.random.Generator:
    """PCG64 generator seeded from SeedSequence([2507, 20802, *words])."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(list(SEED_BASE) + [int(w) for w in words])))


def box_length(n: int, dim: int, density: float = DENSITY) -> float:
    """Edge of the square/cubic box holding n atoms at the given density."""
    return float((n / density) ** (1.0 / dim))


@dataclass
class Sample:
    pos: np.ndarray      # (n, dim) float64, atom-major
    types: np.ndarray    # (n,) uint8, 0 = A, 1 = B
    L: float             # unstrained box edge (square / cube)
    dim: int

    @property
    def n(self) -> int:
        return int(self.types.shape[0])


def uniform_glass_start(dim: int, n: int, *seed: int, density: float = DENSITY,
                        x_a: float | None = None) -> Sample:
    """Uniform random positions in [0, L)^dim and exactly floor(x_A n + 1/2)
    A atoms, the rest B, assigned by a random permutation."""
    if x_a is None:
        x_a = X_A[dim]
    rng = rng_for(*seed)
    L = box_length(n, dim, density)
    pos = rng.uniform(0.0, L, size=(n, dim))
    n_a = int(math.floor(x_a * n + 0.5))
    perm = rng.permutation(n)
    types = np.zeros(n, dtype=np.uint8)
    types[perm[n_a:]] = 1
    return Sample(np.ascontiguousarray(pos, dtype=np.float64), types, L, dim)


def jittered_lattice_start(dim: int, m: int, *seed: int, jitter: float = 0.05,
                           density: float = DENSITY, x_a: float | None = None) -> Sample:
    """m^dim atoms on a simple square/cubic lattice at the given density, each
    displaced by a uniform random vector in [-jitter, jitter]^dim (in units of
    the lattice spacing), with randomly assigned types.  A start with no
    overlapping atoms, for short fixed-iteration comparisons at large n."""
    if x_a is None:
        x_a = X_A[dim]
    rng = rng_for(*seed)
    n = m ** dim
    L = box_length(n, dim, density)
    a = L / m
    grid = np.stack(np.meshgrid(*[np.arange(m)] * dim, indexing="ij"), axis=-1).reshape(n, dim)
    pos = (grid + 0.5 + rng.uniform(-jitter, jitter, size=(n, dim))) * a
    n_a = int(math.floor(x_a * n + 0.5))
    perm = rng.permutation(n)
    types = np.zeros(n, dtype=np.uint8)
    types[perm[n_a:]] = 1
    return Sample(np.ascontiguousarray(pos, dtype=np.float64), types, L, dim)


def log_uniform_sizes(count: int, lo: int, hi: int, *seed: int) -> np.ndarray:
    """count atom numbers round(exp(U[ln lo, ln hi])) (uneven batches)."""
    rng = rng_for(*seed)
    return np.rint(np.exp(rng.uniform(math.log(lo), math.log(hi), size=count))).astype(np.int64)


def choice_of(values, count: int, *seed: int) -> np.ndarray:
    """count draws, equally likely, from a short list of values."""
    rng = rng_for(*seed)
    return np.asarray(values)[rng.integers(0, len(values), size=count)]


def mlp_init(dim: int, *seed: int, n_in: int = 64, hidden: int = 128) -> dict:
    """Initial parameters of the per-atom network n_in -> hidden -> hidden ->
    dim: every weight and bias drawn uniform in (-1/sqrt(fan_in),
    1/sqrt(fan_in)) (FP32), weights in the [in, out] layout."""
    rng = rng_for(*seed)
    out = {}
    for name, fi, fo in (("1", n_in, hidden), ("2", hidden, hidden), ("3", hidden, dim)):
        k = 1.0 / math.sqrt(fi)
        out["w" + name] = rng.uniform(-k, k, size=(fi, fo)).astype(np.float32)
        out["b" + name] = rng.uniform(-k, k, size=fo).astype(np.float32)
    return out


def epoch_orders(n: int, epochs: int, *seed: int) -> np.ndarray:
    """One random order of the n training samples per epoch, int32 [epochs, n]."""
    rng = rng_for(*seed)
    return np.stack([rng.permutation(n) for _ in range(epochs)]).astype(np.int32)


# The paper's benchmark problem (Sec. 2.2): 400 atoms of two types at one
# atom per unit area (square cell of side 20), large to small in the golden
# mean ratio N_L / N_S = (1 + sqrt 5) / 4.  Type 0 = small (S), 1 = large (L).
PAPER_N = 400
PAPER_DENSITY = 1.0
PAPER_RATIO_LS = (1.0 + math.sqrt(5.0)) / 4.0


def paper_sample_start(*seed: int) -> Sample:
    """Uniform random positions in the paper's 20 x 20 cell with round(400 x_S)
    small atoms, x_S = 1 / (1 + r), r = N_L / N_S; the melt-quenched samples
    of the paper are not available, the caller minimises this start."""
    x_s = 1.0 / (1.0 + PAPER_RATIO_LS)
    return uniform_glass_start(2, PAPER_N, *seed, density=PAPER_DENSITY, x_a=x_s)
