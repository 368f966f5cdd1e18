"""Seeded synthetic two-table workloads.

This module only draws random inputs; it holds none of the method's arithmetic
and is shared by the GPU path's tests/bench and by the oracle's tests.

The paper's experiments use two synthetic relations whose columns are drawn
uniformly from (0, 1) and whose join is the Cartesian product (Experiments
section).  The workloads below keep that shape family and add the natural-join,
batched and wide cases the hot path must also serve.  Every table is returned
sorted (stably) by its join key, which is the paper's precondition on inputs
(Experiments section: relations sorted by the join attribute).

Seeds: ``numpy.random.Generator(PCG64(SeedSequence([250323385, k])))`` for
workload ``k``; draw order A, B, keys_A, keys_B, column scales.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np

SEED_BASE = 250323385


@dataclasses.dataclass
class Instance:
    """One two-table problem: row-major A (m1 x n1), B (m2 x n2), optional keys."""

    A: np.ndarray
    B: np.ndarray
    keys_A: Optional[np.ndarray] = None
    keys_B: Optional[np.ndarray] = None

    @property
    def shape(self):
        return (self.A.shape[0], self.A.shape[1], self.B.shape[0], self.B.shape[1])


def rng_for(k: int, extra: int = 0) -> np.random.Generator:
    if extra:
        return np.random.Generator(np.random.PCG64(np.random.SeedSequence([SEED_BASE, k, extra])))
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([SEED_BASE, k])))


def _sort_by_key(X: np.ndarray, keys: np.ndarray):
    order = np.argsort(keys, kind="stable")
    return np.ascontiguousarray(X[order]), np.ascontiguousarray(keys[order].astype(np.int32))


def zipf_keys(rng: np.random.Generator, m: int, n_values: int, s: float) -> np.ndarray:
    """Keys k-1 for ranks k in 1..n_values drawn with probability proportional to k^-s."""
    ranks = np.arange(1, n_values + 1, dtype=np.float64)
    p = ranks ** (-s)
    p /= p.sum()
    return rng.choice(n_values, size=m, p=p).astype(np.int32)


def cartesian_uniform(m: int, n: int, seed_k: int = 1, extra: int = 0, dtype=np.float64) -> Instance:
    """The paper's own synthetic family: two m x n relations, columns U(0,1), Cartesian join."""
    rng = rng_for(seed_k, extra)
    A = rng.random((m, n)).astype(dtype)
    B = rng.random((m, n)).astype(dtype)
    return Instance(A, B)


def config1() -> Instance:
    """Cartesian product of two 1000 x 4 FP64 U[0,1) tables (join 1e6 x 8)."""
    rng = rng_for(1)
    A = rng.random((1000, 4))
    B = rng.random((1000, 4))
    return Instance(A, B)


def config2(m: int = 100_000, n: int = 32) -> Instance:
    """Cartesian product of two 1e5 x 32 FP64 N(0,1) tables (join 1e10 x 64)."""
    rng = rng_for(2)
    A = rng.standard_normal((m, n))
    B = rng.standard_normal((m, n))
    return Instance(A, B)


def config3(m: int = 1 << 20, n: int = 64, n_values: int = 10_000, s: float = 1.1) -> Instance:
    """Natural join on one int32 key: two 2^20 x 64 FP64 N(0,1) tables, keys Zipf(1.1) over 1e4 values."""
    rng = rng_for(3)
    A = rng.standard_normal((m, n))
    B = rng.standard_normal((m, n))
    kA = zipf_keys(rng, m, n_values, s)
    kB = zipf_keys(rng, m, n_values, s)
    A, kA = _sort_by_key(A, kA)
    B, kB = _sort_by_key(B, kB)
    return Instance(A, B, kA, kB)


def config4(count: int = 256, lo: float = 3.0, hi: float = 5.0,
            widths=(8, 16, 32, 64)) -> List[Instance]:
    """Batch of independent Cartesian instances: m1, m2 = floor(10^U(lo,hi)), n1 = n2 from widths, FP32 U(-1,1)."""
    rng = rng_for(4)
    m1 = np.floor(10.0 ** rng.uniform(lo, hi, size=count)).astype(np.int64)
    m2 = np.floor(10.0 ** rng.uniform(lo, hi, size=count)).astype(np.int64)
    nn = rng.choice(np.asarray(widths), size=count)
    out = []
    for i in range(count):
        A = rng.uniform(-1.0, 1.0, size=(int(m1[i]), int(nn[i]))).astype(np.float32)
        B = rng.uniform(-1.0, 1.0, size=(int(m2[i]), int(nn[i]))).astype(np.float32)
        out.append(Instance(A, B))
    return out


def config5(m: int = 1 << 18, n: int = 256, n_values: int = 4096) -> Instance:
    """Wide natural join: two 2^18 x 256 FP32 N(0,1) tables, each column scaled by 10^U(-3,0),
    int32 keys uniform over 4096 values."""
    rng = rng_for(5)
    A = rng.standard_normal((m, n))
    B = rng.standard_normal((m, n))
    kA = rng.integers(0, n_values, size=m).astype(np.int32)
    kB = rng.integers(0, n_values, size=m).astype(np.int32)
    sA = 10.0 ** rng.uniform(-3.0, 0.0, size=n)
    sB = 10.0 ** rng.uniform(-3.0, 0.0, size=n)
    A = (A * sA[None, :]).astype(np.float32)
    B = (B * sB[None, :]).astype(np.float32)
    A, kA = _sort_by_key(A, kA)
    B, kB = _sort_by_key(B, kB)
    return Instance(A, B, kA, kB)


def random_instance(rng: np.random.Generator, m1: int, n1: int, m2: int, n2: int,
                    n_values: Optional[int] = None, dtype=np.float64, dist: str = "normal",
                    key_skew: Optional[float] = None) -> Instance:
    """Small random instance for tests. n_values=None gives a Cartesian product."""
    if dist == "normal":
        A = rng.standard_normal((m1, n1))
        B = rng.standard_normal((m2, n2))
    else:
        A = rng.random((m1, n1))
        B = rng.random((m2, n2))
    A = A.astype(dtype)
    B = B.astype(dtype)
    if n_values is None:
        return Instance(np.ascontiguousarray(A), np.ascontiguousarray(B))
    if key_skew is None:
        kA = rng.integers(0, n_values, size=m1).astype(np.int32)
        kB = rng.integers(0, n_values, size=m2).astype(np.int32)
    else:
        kA = zipf_keys(rng, m1, n_values, key_skew)
        kB = zipf_keys(rng, m2, n_values, key_skew)
    A, kA = _sort_by_key(A, kA)
    B, kB = _sort_by_key(B, kB)
    return Instance(A, B, kA, kB)


CONFIGS = {1: config1, 2: config2, 3: config3, 5: config5}
