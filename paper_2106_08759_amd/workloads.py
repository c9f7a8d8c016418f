"""Seeded synthetic workloads: the master seed, the benchmark configurations and
random ring elements for the single-operation checks.

This module holds no arithmetic of the method; tests, the oracle-backed
checks and bench.py all draw their inputs from here.  Every key is a pure
function of (seed, p, index), so a configuration is fully described by the
seed, the parameter set and the index range.
"""
from __future__ import annotations

import numpy as np

# master seed: bytes 0x00 .. 0x1f
SEED = bytes(range(32))

# parameter sets (p, q, w) -- Section 2.1 of the paper for 653/761/857,
# round-3 values for 1277
PQW = {653: (653, 4621, 288), 761: (761, 4591, 286), 857: (857, 5167, 322), 1277: (1277, 7879, 492)}

# Benchmark configurations (sntrup761 unless stated): key index ranges
CONFIGS = {
    "plain32": dict(p=761, first_index=0, n=32, group_size=1, plain=True),
    "batched1024": dict(p=761, first_index=0, n=1024, group_size=32),
    "persistent65536": dict(p=761, first_index=0, n=65536),
    "mixed4x16384": dict(jobs=[(653, 0, 16384), (761, 0, 16384), (857, 0, 16384), (1277, 0, 16384)]),
}


def rng(tag: int) -> np.random.Generator:
    return np.random.default_rng(0x5EED0000 + tag)


def random_rq(p: int, n: int, tag: int = 0) -> np.ndarray:
    """n uniform elements of R/q, centered int16 [n, p]."""
    q = PQW[p][1]
    h = (q - 1) // 2
    return rng(tag).integers(-h, h + 1, size=(n, p), dtype=np.int64).astype(np.int16)


def random_small(p: int, n: int, tag: int = 0, bound: int = 1) -> np.ndarray:
    """n elements with coefficients uniform in [-bound, bound], int8/int16 [n, p]."""
    return rng(tag).integers(-bound, bound + 1, size=(n, p), dtype=np.int64).astype(np.int8)


def extreme_rq(p: int) -> np.ndarray:
    """Elements with every coefficient at +-(q-1)/2 (the largest products)."""
    q = PQW[p][1]
    h = (q - 1) // 2
    alt = np.where(np.arange(p) % 2 == 0, h, -h)
    return np.stack([np.full(p, h), np.full(p, -h), alt, -alt]).astype(np.int16)
