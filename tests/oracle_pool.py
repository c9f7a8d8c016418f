"""Run the CPU oracle over many keys in parallel processes (test helper)."""
from __future__ import annotations

import multiprocessing as mp
import os

import numpy as np

import oracle


def _worker(args):
    seed, p, indices = args
    _, q, w = oracle.PARAMS[p]
    out = []
    for i in indices:
        k = oracle.keygen(seed, p, int(i))
        out.append((int(i), oracle.encode_pk(k["h"], p, q), oracle.encode_sk(k["f"], k["ginv"], p),
                    k["h"], k["f"], k["ginv"], k["attempts"]))
    return out


def workers() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def oracle_keys(seed: bytes, p: int, indices) -> dict:
    """index -> (pk bytes, sk bytes, h, f, ginv, attempts) from the oracle."""
    indices = list(indices)
    nw = workers()
    chunks = [indices[i::nw] for i in range(nw) if indices[i::nw]]
    oracle.build()
    with mp.get_context("fork").Pool(len(chunks)) as pool:
        res = pool.map(_worker, [(seed, p, c) for c in chunks])
    return {r[0]: r[1:] for part in res for r in part}


def pk_sk_arrays(keys: dict, indices):
    pk = np.stack([np.frombuffer(keys[i][0], dtype=np.uint8) for i in indices])
    sk = np.stack([np.frombuffer(keys[i][1], dtype=np.uint8) for i in indices])
    return pk, sk
