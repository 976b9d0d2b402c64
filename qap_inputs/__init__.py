"""Seeded synthetic QAP instances shaped like the paper's workloads.

This module holds only input generation (numpy PCG64 streams); it contains
none of the method's arithmetic and is shared by the tests, the benchmark and
the smoke check.  The paper measures on QAPLIB instances (n = 12 .. 150,
Table 1 and Table 2), which are not reproduced here; these generators stand in
for them with the sizes and value ranges of the workloads below.
"""
from __future__ import annotations

import numpy as np


def symmetric_uniform(n: int, lo: int, hi: int, rng: np.random.Generator, zero_diag: bool = True) -> np.ndarray:
    """Symmetric integer matrix, upper triangle uniform in [lo, hi], mirrored."""
    A = rng.integers(lo, hi + 1, size=(n, n), dtype=np.int64)
    A = np.triu(A, 1)
    A = A + A.T
    if not zero_diag:
        A[np.arange(n), np.arange(n)] = rng.integers(lo, hi + 1, size=n)
    return A.astype(np.int32)


def uniform_instance(n: int, lo: int, hi: int, seed: int, *, d_hi: int | None = None):
    """F and D symmetric, uniform integers, zero diagonal (the paper's common case)."""
    rng = np.random.default_rng(seed)
    F = symmetric_uniform(n, lo, hi, rng)
    D = symmetric_uniform(n, lo, hi if d_hi is None else d_hi, rng)
    return F, D


def general_instance(n: int, lo: int, hi: int, seed: int):
    """Asymmetric F and D with non-zero diagonals (and negative entries if lo < 0)."""
    rng = np.random.default_rng(seed)
    F = rng.integers(lo, hi + 1, size=(n, n)).astype(np.int32)
    D = rng.integers(lo, hi + 1, size=(n, n)).astype(np.int32)
    return F, D


def euclid_sparse_instance(n: int, seed: int, density: float = 0.3):
    """D = rounded Euclidean distances of n points uniform in a 100x100 square;
    F symmetric, each off-diagonal pair non-zero with probability `density`,
    value floor(exp(U[0, 8))) (a heavy-tailed flow)."""
    rng = np.random.default_rng(seed)
    pts = rng.uniform(0.0, 100.0, size=(n, 2))
    dist = np.sqrt(((pts[:, None, :] - pts[None, :, :]) ** 2).sum(-1))
    D = np.floor(dist + 0.5).astype(np.int32)
    mask = np.triu(rng.random((n, n)) < density, 1)
    vals = np.floor(np.exp(rng.uniform(0.0, 8.0, size=(n, n)))).astype(np.int64)
    F = np.where(mask, vals, 0)
    F = (F + F.T).astype(np.int32)
    return F, D


def linear_sum_instance(n: int, seed: int, hi: int = 20):
    """D[k][l] = a_k + a_l (non-zero diagonal): the QAP collapses to a linear
    assignment solved exactly by sorting (rearrangement inequality)."""
    rng = np.random.default_rng(seed)
    F = rng.integers(0, hi + 1, size=(n, n)).astype(np.int32)
    a = rng.integers(0, hi + 1, size=n).astype(np.int64)
    D = (a[:, None] + a[None, :]).astype(np.int32)
    return F, D, a


# Workloads (the paper's sizes; seeds fixed here).
WORKLOADS = {
    # n = 12, symmetric U{0..10}; 1 swarm x 64 particles, 100 iterations
    "n12": dict(gen=lambda: uniform_instance(12, 0, 10, 101), num_swarms=1, particles_per_swarm=64,
                iterations=100, migration=False),
    # n = 50 dense symmetric U{0..99}; 10 x 1000, 1000 iterations, int32 path
    "n50": dict(gen=lambda: uniform_instance(50, 0, 99, 102), num_swarms=10, particles_per_swarm=1000,
                iterations=1000, migration=False),
    # n = 100 Euclidean D (at most 121 at this seed), sparse heavy-tailed F (outside int8); 20 x 500, migration every 50 iterations
    "n100mig": dict(gen=lambda: euclid_sparse_instance(100, 103), num_swarms=20, particles_per_swarm=500,
                    iterations=2000, migration=True, migration_factor=0.33, migration_period=50),
    # n = 128 symmetric U{0..127} (int8-representable); 8 x 512
    "n128": dict(gen=lambda: uniform_instance(128, 0, 127, 104), num_swarms=8, particles_per_swarm=512,
                 iterations=200, migration=False),
    # same with D in U{0..1000}: outside int8 (byte-split MFMA on the fused engine, int32 on the per-stage one)
    "n128wide": dict(gen=lambda: uniform_instance(128, 0, 127, 1041, d_hi=1000), num_swarms=8,
                     particles_per_swarm=512, iterations=200, migration=False),
    # headline: n = 128 instance above with 200 swarms x 50 particles = 10,000 particles
    "n128x10k": dict(gen=lambda: uniform_instance(128, 0, 127, 104), num_swarms=200, particles_per_swarm=50,
                     iterations=200, migration=False),
}


def mixed_batch(count: int = 64, seed: int = 105, lo_n: int = 20, hi_n: int = 150):
    """`count` independent instances, n uniform in [lo_n, hi_n], F, D U{0..99} symmetric."""
    rng = np.random.default_rng(seed)
    ns = rng.integers(lo_n, hi_n + 1, size=count)
    return [uniform_instance(int(n), 0, 99, seed * 1000 + i) for i, n in enumerate(ns)]


def random_perms(count: int, n: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return np.stack([rng.permutation(n) for _ in range(count)]).astype(np.int32)
