"""Launch-shape tuner for ace_build.

For one (grid n, precision, orbital count) it times ace_build on the GPU for
candidate launch shapes and keeps the fastest in a JSON cache:

  block   : orbital block of the pair tiles (16 or 8),
  chunk   : packed transforms per forward / inverse launch (0 = whole tile),
  pencils : x-pass pencils per workgroup (8, 16 or 32 dividing n; 0 = default).

The search is coordinate-wise: (block, chunk) at the default pencils first,
then the pencils at the best (block, chunk).  Timing inputs are random
orbitals drawn on the device: the kernels' work does not depend on the values,
and any full-rank real orbital set gives a negative definite M, so the
Cholesky branch is the production one.
"""
from __future__ import annotations

import json
import os
from typing import Dict, List, Optional, Tuple

from . import _lib

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "paper_2110_07670_amd",
                             "autotune.json")

Shape = Tuple[int, int, int]


def key(n: int, precision: str, n_orb: int) -> str:
    return "n%d/%s/k%d" % (int(n), precision, int(n_orb))


def _valid_pencils(n: int) -> List[int]:
    return [c for c in (8, 16, 32) if n % c == 0]


def tile_candidates(n_orb: int) -> List[Tuple[int, int]]:
    """(block, chunk) pairs worth timing for n_orb orbitals."""
    out = [(16, 0)]
    if n_orb > 8:
        out.append((8, 0))
    if n_orb > 16:
        out.append((16, 32))
    return out


def pencil_candidates(n: int) -> List[int]:
    """x-pass shapes other than the default (which the first sweep times)."""
    default = 16 if n % 16 == 0 else 8
    return [c for c in _valid_pencils(n) if c != default]


def load_cache(path: Optional[str] = None) -> Dict[str, dict]:
    path = path or DEFAULT_CACHE
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        data = json.load(f)
    return data if isinstance(data, dict) else {}


def save_cache(cache: Dict[str, dict], path: Optional[str] = None):
    path = path or DEFAULT_CACHE
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def time_shape(n: int, precision: str, n_orb: int, shape: Shape, phi, reps: int = 2) -> float:
    """Milliseconds of one ace_build with the given launch shape (best of reps).
    The cell size does not change the work; any positive one will do."""
    import torch
    plan = _lib.Plan(n, (10.0, 10.0, 10.0), n_orb, precision, 0.25)
    plan.set_tiling(*shape)
    ws = _lib.workspace(plan.workspace_bytes(), phi.device)
    out = _lib.ace_build(plan, phi, ws=ws)              # warm-up, also allocates outputs
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    best = float("inf")
    for _ in range(reps):
        ev0.record()
        _lib.build_into(plan, phi, out["W"], out["M"], out["xi"], out["ex"], out["info"], ws)
        ev1.record()
        ev1.synchronize()
        best = min(best, ev0.elapsed_time(ev1))
    del ws, out
    return best


def tune(n: int, precision: str, n_orb: int, cache_path: Optional[str] = None,
         device: str = "cuda:0", reps: int = 2, force: bool = False, log=None) -> dict:
    """Best launch shape for the key, from the cache or by timing."""
    import torch
    cache = load_cache(cache_path)
    k = key(n, precision, n_orb)
    if not force and k in cache:
        return cache[k]
    g = torch.Generator(device=device)
    g.manual_seed(1234 + n + 7 * n_orb)
    phi = torch.randn((n_orb, n, n, n), dtype=torch.float64, device=device, generator=g)
    phi *= (1.0 / n ** 1.5)
    results = []
    for block, chunk in tile_candidates(n_orb):
        ms = time_shape(n, precision, n_orb, (block, chunk, 0), phi, reps)
        results.append(((block, chunk, 0), ms))
    (block, chunk, _), _ms = min(results, key=lambda r: r[1])
    for c in pencil_candidates(n):
        ms = time_shape(n, precision, n_orb, (block, chunk, c), phi, reps)
        results.append(((block, chunk, c), ms))
    shape, ms = min(results, key=lambda r: r[1])
    entry = {"block": shape[0], "chunk": shape[1], "pencils": shape[2], "ms": round(ms, 4),
             "tried": [[list(s), round(t, 4)] for s, t in results]}
    if log:
        log("tuned %s -> %s (%.3f ms over %d shapes)" % (k, shape, ms, len(results)))
    cache = load_cache(cache_path)
    cache[k] = entry
    save_cache(cache, cache_path)
    del phi
    torch.cuda.empty_cache()
    return entry


def apply(plan: "_lib.Plan", precision: str, cache_path: Optional[str] = None,
          tune_missing: bool = True, log=None) -> Shape:
    """Set the plan's launch shape from the cache (tuning the key if absent)."""
    k = key(plan.n, precision, plan.n_orb)
    cache = load_cache(cache_path)
    if k in cache:
        e = cache[k]
    elif tune_missing:
        e = tune(plan.n, precision, plan.n_orb, cache_path, log=log)
    else:
        return plan.tiling
    plan.set_tiling(int(e["block"]), int(e["chunk"]), int(e["pencils"]))
    return plan.tiling
