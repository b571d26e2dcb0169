"""Host-core timing of the FP64 oracle on a sample of orbital pairs.

TEST INFRASTRUCTURE ONLY (the benchmark's CPU-baseline leg).  A process pool
with one worker per requested core runs the oracle's own pair Poisson solve
(ace_oracle.pair_potential) and W updates on contiguous chunks of the sampled
pairs, one FFT thread per worker.
"""
from __future__ import annotations

import multiprocessing as mp
import os
import time
from typing import List, Tuple

import numpy as np

from . import ace_oracle as O

_PHI = None
_K = None
_ALPHA = None


def _init(phi, K, alpha):
    global _PHI, _K, _ALPHA
    _PHI, _K, _ALPHA = phi, K, alpha


def _work(chunk: List[Tuple[int, int]]) -> int:
    W = {}
    for i, j in chunk:
        v = O.pair_potential(_PHI[i] * _PHI[j], _K, workers=1)
        W.setdefault(i, np.zeros_like(_PHI[i]))
        W[i] -= _ALPHA * v * _PHI[j]
        if i != j:
            W.setdefault(j, np.zeros_like(_PHI[j]))
            W[j] -= _ALPHA * v * _PHI[i]
    return len(chunk)


def time_pair_sample(phi: np.ndarray, cell: np.ndarray, alpha: float,
                     pairs: List[Tuple[int, int]], processes: int):
    """Wall time of the oracle's pair loop over `pairs` on `processes` cores.

    Returns (pairs per second, seconds, processes used).
    """
    K = O.coulomb_kernel(phi.shape[1:], cell)
    processes = max(1, min(processes, len(pairs)))
    chunks = [pairs[k::processes] for k in range(processes)]
    ctx = mp.get_context("fork")
    with ctx.Pool(processes, initializer=_init, initargs=(phi, K, alpha)) as pool:
        pool.map(_work, [[pairs[0]]] * processes)  # warm the workers
        t0 = time.perf_counter()
        done = sum(pool.map(_work, chunks))
        dt = time.perf_counter() - t0
    return done / dt, dt, processes


def default_processes() -> int:
    n = os.cpu_count() or 1
    return max(1, min(n, 16))


def _row_chunk(args):
    i, js = args
    w = np.zeros_like(_PHI[i])
    for j in js:
        w -= _ALPHA * O.pair_potential(_PHI[i] * _PHI[j], _K, workers=1) * _PHI[j]
    return i, w


def apply_vx_rows_parallel(phi: np.ndarray, cell: np.ndarray, alpha: float, rows,
                           processes: int):
    """W_i = -alpha sum_j v_ij phi_j for the given rows, the j sum split over processes
    and added back in a fixed order."""
    K = O.coulomb_kernel(phi.shape[1:], cell)
    k = phi.shape[0]
    processes = max(1, processes)
    jobs = [(i, list(range(c, k, processes))) for i in rows for c in range(processes)]
    ctx = mp.get_context("fork")
    with ctx.Pool(processes, initializer=_init, initargs=(phi, K, alpha)) as pool:
        parts = pool.map(_row_chunk, jobs)
    out = {i: np.zeros_like(phi[0]) for i in rows}
    for i, w in parts:
        out[i] += w
    return out
