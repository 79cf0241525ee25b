"""Seeded synthetic workloads for HE matrix multiplication.

This module only draws inputs: ring/modulus sizes, matrix shapes, matrix
entries and request arrival times.  It holds none of the homomorphic
arithmetic (no primes, no roots, no sampling of keys or noise); both the CPU
oracle and the GPU library derive those themselves from the sizes given here.

The paper evaluates on synthetic matrices only (Section IV-A: random pairs
with row and column counts uniform in [1, 64]; the entry distribution is not
stated).  The configurations below keep that spirit at the sizes the GPU
build is measured on:

* ``tiny``     N=1024,  t=12289,  3+1 primes, A 4x3, B 3x5, entries in [0,16)
* ``headline`` N=8192,  t=65537,  4+1 primes, A 64x32, B 32x48, entries in [-8,8]
* ``batched``  N=8192,  t=65537,  4+1 primes, 256 shapes from {8,...,64}^3
* ``large``    N=32768, t=786433, 8+2 primes, A 128x96, B 96x128, entries in [-4,4]
* ``serving``  N=16384, t=65537,  6+2 primes, Poisson arrivals at 200 req/s,
  shapes from {16,...,128}^3 with m*l, l*n, m*n <= N/2
"""
from __future__ import annotations

import dataclasses
from typing import List, Tuple

import numpy as np

MASTER_SEED_BASE = 240502238


@dataclasses.dataclass(frozen=True)
class RingConfig:
    """Sizes of one BGV parameter set (no derived constants)."""
    name: str
    N: int          # ring degree, power of two
    t: int          # plaintext modulus, prime, t = 1 (mod 2N)
    L: int          # number of ciphertext primes
    alpha: int      # number of special (key-switching) primes
    index: int      # 1-based configuration index; master seed = base + index

    @property
    def seed(self) -> int:
        return MASTER_SEED_BASE + self.index

    @property
    def slots(self) -> int:
        return self.N // 2


TINY = RingConfig("tiny", 1024, 12289, 3, 1, 1)
HEADLINE = RingConfig("headline", 8192, 65537, 4, 1, 2)
BATCHED = RingConfig("batched", 8192, 65537, 4, 1, 3)
LARGE = RingConfig("large", 32768, 786433, 8, 2, 4)
SERVING = RingConfig("serving", 16384, 65537, 6, 2, 5)
CONFIGS = {c.name: c for c in (TINY, HEADLINE, BATCHED, LARGE, SERVING)}


def small_ring(N: int, t: int, L: int, alpha: int) -> RingConfig:
    """A toy parameter set for tests (seeded from index 0)."""
    return RingConfig(f"toy{N}", N, t, L, alpha, 0)


def matrix(rng: np.random.Generator, rows: int, cols: int, lo: int, hi: int) -> np.ndarray:
    """Uniform integer matrix with entries in [lo, hi] (inclusive), int64, row-major."""
    return rng.integers(lo, hi + 1, size=(rows, cols), dtype=np.int64)


def operands(cfg: RingConfig, m: int, l: int, n: int, lo: int, hi: int,
             seed_offset: int = 0) -> Tuple[np.ndarray, np.ndarray]:
    """Draw A (m x l) and B (l x n) from default_rng(seed + seed_offset)."""
    rng = np.random.default_rng(cfg.seed + seed_offset)
    a = matrix(rng, m, l, lo, hi)
    b = matrix(rng, l, n, lo, hi)
    return a, b


def tiny_operands() -> Tuple[np.ndarray, np.ndarray]:
    return operands(TINY, 4, 3, 5, 0, 15)


def headline_operands() -> Tuple[np.ndarray, np.ndarray]:
    return operands(HEADLINE, 64, 32, 48, -8, 8)


def large_operands() -> Tuple[np.ndarray, np.ndarray]:
    return operands(LARGE, 128, 96, 128, -4, 4)


# Blocked 100 x 100 product (the partitions of the paper's large-matrix
# experiment, Section IV-D): the row blocks of A and the column blocks of B.
# P1: 50 + 50 each way; P2: 64 + 36 each way.  On the headline ring.
BLOCKED_DIM = 100
PARTITIONS = {"P1": ((50, 50), (50, 50)), "P2": ((64, 36), (64, 36))}


def blocked_operands() -> Tuple[np.ndarray, np.ndarray]:
    """A and B, 100 x 100, entries in [-8, 8]."""
    return operands(HEADLINE, BLOCKED_DIM, BLOCKED_DIM, BLOCKED_DIM, -8, 8, seed_offset=100)


def batched_shapes(count: int = 256, seed_offset: int = 0) -> List[Tuple[int, int, int]]:
    """(m, l, n) i.i.d. uniform over {8, 16, ..., 64}^3 (the products never exceed 4096)."""
    rng = np.random.default_rng(BATCHED.seed + seed_offset)
    grid = np.arange(8, 65, 8)
    out = []
    for _ in range(count):
        m, l, n = (int(x) for x in rng.choice(grid, size=3))
        out.append((m, l, n))
    return out


def batched_requests(count: int = 256, seed_offset: int = 0):
    """Shapes plus operands for the batched workload: list of (m, l, n, A, B)."""
    shapes = batched_shapes(count, seed_offset)
    rng = np.random.default_rng(BATCHED.seed + 1000 + seed_offset)
    reqs = []
    for (m, l, n) in shapes:
        a = matrix(rng, m, l, -8, 8)
        b = matrix(rng, l, n, -8, 8)
        reqs.append((m, l, n, a, b))
    return reqs


def serving_requests(count: int = 512, rate_per_s: float = 200.0, seed_offset: int = 0):
    """Poisson arrivals: list of (arrival_s, m, l, n, A, B).

    Shapes are uniform over {16, 32, ..., 128}^3, redrawn until every pairwise
    product m*l, l*n, m*n is at most the slot count N/2 = 8192.
    """
    rng = np.random.default_rng(SERVING.seed + seed_offset)
    grid = np.arange(16, 129, 16)
    cap = SERVING.slots
    out = []
    t_now = 0.0
    for _ in range(count):
        t_now += float(rng.exponential(1.0 / rate_per_s))
        while True:
            m, l, n = (int(x) for x in rng.choice(grid, size=3))
            if m * l <= cap and l * n <= cap and m * n <= cap:
                break
        a = matrix(rng, m, l, -8, 8)
        b = matrix(rng, l, n, -8, 8)
        out.append((t_now, m, l, n, a, b))
    return out


def random_shapes(rng: np.random.Generator, count: int, lo: int, hi: int) -> List[Tuple[int, int, int]]:
    """Shapes with each dimension uniform in [lo, hi] (the paper's random-pair recipe)."""
    return [tuple(int(x) for x in rng.integers(lo, hi + 1, size=3)) for _ in range(count)]


def plain_matmul_mod(a: np.ndarray, b: np.ndarray, t: int) -> np.ndarray:
    """Brute-force integer product reduced into [0, t): the ground truth C = A.B mod t."""
    a = [[int(x) for x in row] for row in a]
    b = [[int(x) for x in row] for row in b]
    m, l, n = len(a), len(b), len(b[0]) if b else 0
    c = np.zeros((m, n), dtype=np.int64)
    for i in range(m):
        for j in range(n):
            s = 0
            for k in range(l):
                s += a[i][k] * b[k][j]
            c[i, j] = s % t
    return c
