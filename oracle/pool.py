"""Process pools over the FP64 oracle's rows of Eq. (2).

TEST INFRASTRUCTURE ONLY: called by the committed reference scripts under
tests/golden/ and by the oracle job the GPU test session starts in a separate
process.  Workers are forked, so call these only from a process that has not
initialised a GPU (the reference scripts and the oracle job are such fresh
processes; a test process that has touched the GPU must not call them).

Each worker evaluates ``ace_oracle.apply_vx_rows`` itself: whole rows when
there are at least as many rows as workers (row i = -alpha sum_j v_ij phi_j),
otherwise each row's sum over j split into residue classes of j and added
back in a fixed order.  No arithmetic of the method lives here.
"""
from __future__ import annotations

import multiprocessing as mp
from typing import Dict, Optional, Sequence

import numpy as np

from . import ace_oracle as O

_S = {}


def _init(phi, cell, alpha, mask):
    _S.update(phi=phi, cell=cell, alpha=alpha, mask=mask)


def _rows_job(args):
    rows, cols = args
    w = O.apply_vx_rows(_S["phi"], _S["cell"], _S["alpha"], rows, pair_mask=_S["mask"],
                        cols=cols)
    return rows, cols, w


def apply_vx_rows_pool(phi: np.ndarray, cell: np.ndarray, alpha: float, rows: Sequence[int],
                       processes: int, pair_mask: Optional[np.ndarray] = None
                       ) -> Dict[int, np.ndarray]:
    """{i: W_i} for i in rows (Eq. (2), optionally restricted to the kept pairs)."""
    rows = [int(i) for i in rows]
    k = phi.shape[0]
    processes = max(1, int(processes))
    if len(rows) >= processes:
        jobs = [([i], None) for i in rows]
    else:
        jobs = [([i], list(range(c, k, processes))) for i in rows for c in range(processes)]
    out = {i: np.zeros(phi.shape[1:]) for i in rows}
    ctx = mp.get_context("fork")
    with ctx.Pool(processes, initializer=_init, initargs=(phi, cell, alpha, pair_mask)) as pool:
        parts = pool.map(_rows_job, jobs, chunksize=1)
    # map keeps the job order: residue classes c = 0, 1, ... are added in turn
    for rr, _, w in parts:
        out[rr[0]] += w[0]
    return out


def apply_vx_pool(phi: np.ndarray, cell: np.ndarray, alpha: float, processes: int,
                  out: Optional[np.ndarray] = None,
                  pair_mask: Optional[np.ndarray] = None) -> np.ndarray:
    """All rows of Eq. (2), one row per task (every ordered pair solved once)."""
    k = phi.shape[0]
    W = np.zeros_like(phi) if out is None else out
    ctx = mp.get_context("fork")
    with ctx.Pool(max(1, int(processes)), initializer=_init,
                  initargs=(phi, cell, alpha, pair_mask)) as pool:
        for rr, _, w in pool.imap_unordered(_rows_job, [([i], None) for i in range(k)]):
            W[rr[0]] = w[0]
    return W
