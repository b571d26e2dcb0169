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
    """Host processes for the timed sample: every core the process may use,
    capped at 16 (the CPU share a one-GPU host gives a job)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(n, 16))
