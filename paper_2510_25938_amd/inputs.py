"""Seeded synthetic workloads (random Lennard-Jones cluster starts).

This module only draws numbers and lays them out: it holds none of the
method's arithmetic.  Both the HIP path and the CPU oracle consume exactly the
arrays it returns, so every comparison starts from identical bytes.

A start of N atoms is uniform in a cube of side L = 1.2 * N^(1/3) centred at
the origin (the paper reads its start from a file; the benchmark workloads use
random cubes of this side instead).  Coordinates are returned as three planes
[3][total_atoms] with an int32 prefix-sum offset[B+1] per cluster.
"""
from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 25102593800


def cube_side(n: int) -> float:
    return 1.2 * float(np.cbrt(float(n)))


def offsets_from_sizes(sizes) -> np.ndarray:
    sizes = np.asarray(sizes, dtype=np.int64)
    off = np.zeros(sizes.size + 1, dtype=np.int64)
    np.cumsum(sizes, out=off[1:])
    if off[-1] >= 2 ** 31:
        raise ValueError("total atom count exceeds int32 offsets")
    return off.astype(np.int32)


def random_starts(sizes, seed: int, side=None):
    """Random cube starts for clusters of the given sizes.

    Returns (offset int32[B+1], xyz float64[3][T]).  `side` overrides the cube
    side (a scalar or one value per cluster).
    """
    sizes = np.asarray(sizes, dtype=np.int64)
    off = offsets_from_sizes(sizes)
    T = int(off[-1])
    rng = np.random.Generator(np.random.Philox(key=np.uint64(seed)))
    u = rng.random((T, 3))  # atom-major, as the paper's flattened [x0, y0, z0, x1, ...]
    if side is None:
        L = np.array([cube_side(int(n)) for n in sizes])
    else:
        L = np.broadcast_to(np.asarray(side, dtype=np.float64), sizes.shape)
    Lat = np.repeat(L, sizes)
    xyz = np.ascontiguousarray(((u - 0.5) * Lat[:, None]).T)
    return off, xyz


def uniform_sizes(count: int, lo: int, hi: int, seed: int) -> np.ndarray:
    rng = np.random.Generator(np.random.Philox(key=np.uint64(seed ^ 0x5A5A5A5A)))
    return rng.integers(lo, hi + 1, size=count)


def aos_to_planes(flat: np.ndarray) -> np.ndarray:
    """[x0, y0, z0, x1, ...] -> planes [3][n]."""
    return np.ascontiguousarray(np.asarray(flat, dtype=np.float64).reshape(-1, 3).T)


def planes_to_aos(xyz: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(xyz).T).reshape(-1)


@dataclass
class Workload:
    name: str
    sizes: np.ndarray
    seed: int
    precision: str = "fp64"
    max_iter: int = 10000
    polish: bool = True
    chains: int = 0
    cands: int = 0
    steps: int = 0
    kT: float = 0.8
    step0: float = 0.4
    extra: dict = field(default_factory=dict)

    def starts(self):
        return random_starts(self.sizes, self.seed)


def lj13_bh(steps: int = 200) -> Workload:
    """LJ13 plain basin hopping in FP64: 1 chain, 8 candidates, 200 steps."""
    return Workload("lj13-bh-1x8x200-fp64", np.array([13]), SEED_BASE + 1, "fp64",
                    chains=1, cands=8, steps=steps)


def lj38_batch(count: int = 1024) -> Workload:
    """1024 independent LJ38 candidates from random cube starts, one launch."""
    return Workload(f"lj38-batch-{count}", np.full(count, 38), SEED_BASE + 2, "mixed")


def uneven_batch(count: int = 4096, lo: int = 13, hi: int = 150) -> Workload:
    """4096 candidates with N uniform on the integers 13..150."""
    seed = SEED_BASE + 3
    return Workload(f"uneven-{count}x{lo}-{hi}", uniform_sizes(count, lo, hi, seed), seed, "mixed")


def large_clusters(count: int = 256, n: int = 1000) -> Workload:
    """256 candidates of N = 1000, 500-iteration cap, mixed precision, no polish."""
    return Workload(f"lj{n}-batch-{count}", np.full(count, n), SEED_BASE + 4, "mixed",
                    max_iter=500, polish=False)


def many_chains(chains: int = 512, lo: int = 38, hi: int = 75, steps: int = 1000) -> Workload:
    """512 adaptive BH chains, N uniform on 38..75, 8 candidates, 1000 steps."""
    seed = SEED_BASE + 5
    return Workload(f"chains-{chains}x8x{steps}-{lo}-{hi}", uniform_sizes(chains, lo, hi, seed),
                    seed, "mixed", chains=chains, cands=8, steps=steps)


def morse38_batch(count: int = 1024, rho: float = 6.0) -> Workload:
    """1024 independent 38-atom Morse clusters (range rho) from random cube
    starts, one launch: the LJ38 batch with the Morse pair."""
    return Workload(f"morse38-rho{rho:g}-batch-{count}", np.full(count, 38), SEED_BASE + 6,
                    "mixed", extra={"pair": "morse", "rho": rho})


def lj13_batch(count: int = 16384) -> Workload:
    """16384 independent LJ13 candidates from random cube starts, one launch:
    the small-cluster end of the batched minimiser (the paper's LJ13 candidate
    shape at many chains' worth of candidates)."""
    return Workload(f"lj13-batch-{count}", np.full(count, 13), SEED_BASE + 7, "fp64")
