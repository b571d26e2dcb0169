"""Launch-shape tuner for ace_build and for batches.

For one (grid n, precision, orbital count) it times ace_build on the GPU for
candidate launch shapes and keeps the fastest in a JSON cache:

  block    : orbital block of the pair tiles (16 or 8),
  chunk    : packed transforms per forward / inverse launch (0 = whole tile;
             16, 32 or 64 where smaller than a full tile's count),
  schedule : three passes where the kernels fit (auto) or four everywhere,
  pencils  : x-pass pencils per workgroup (8, 16 or 32 dividing n; 0 = default).

The search is coordinate-wise: (block, chunk) at the automatic schedule and
default pencils, then the schedule, then the pencils at the best of those.

For a batch, tune_batch times the whole batch graph: every instance on its
own tuned shape, every instance on block 16, every instance on block 8, then,
from the best of those, each grid size's block flipped in turn (instances of
one grid, precision and block share the persistent pass launches, so the best
shape of an instance alone need not be the best inside the batch), and
finally the same shapes with every instance on its own launches instead of
the lanes' shared ones (ACE_BATCH_NO_LANES); the faster mode is kept.

Timing inputs are random orbitals drawn on the device: the kernels' work
does not depend on the values, and any full-rank real orbital set gives a
negative definite M, so the Cholesky branch is the production one.
"""
from __future__ import annotations

import json
import os
from typing import Dict, List, Optional, Tuple

from . import _lib

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "paper_2110_07670_amd",
                             "autotune.json")

Shape = Tuple[int, int, int]
Full = Tuple[int, int, int, bool]  # block, chunk, pencils, four_pass


def key(n: int, precision: str, n_orb: int) -> str:
    return "n%d/%s/k%d" % (int(n), precision, int(n_orb))


def _valid_pencils(n: int) -> List[int]:
    return [c for c in (8, 16, 32) if n % c == 0]


def tile_candidates(n_orb: int) -> List[Tuple[int, int]]:
    """(block, chunk) pairs worth timing for n_orb orbitals: a chunk only
    where it splits a full tile (block^2 / 2 transforms off the diagonal)."""
    out = []
    for block in (16, 8):
        if block == 8 and n_orb <= 8:
            continue
        out.append((block, 0))
        full = block * block // 2
        for chunk in (16, 32, 64):
            if chunk < full and n_orb > block:
                out.append((block, chunk))
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


def time_shape(n: int, precision: str, n_orb: int, shape, phi, reps: int = 2) -> float:
    """Milliseconds of one ace_build with the given launch shape (block,
    chunk, pencils[, four_pass]), best of reps.  The cell size does not
    change the work; any positive one will do."""
    import torch
    plan = _lib.Plan(n, (10.0, 10.0, 10.0), n_orb, precision, 0.25)
    plan.set_tiling(*shape[:3])
    if len(shape) > 3 and shape[3]:
        plan.set_schedule(True)
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
        ms = time_shape(n, precision, n_orb, (block, chunk, 0, False), phi, reps)
        results.append(((block, chunk, 0, False), ms))
    (block, chunk, _, _), _ms = min(results, key=lambda r: r[1])
    ms = time_shape(n, precision, n_orb, (block, chunk, 0, True), phi, reps)
    results.append(((block, chunk, 0, True), ms))
    (block, chunk, _, four), _ms = min(results, key=lambda r: r[1])
    for c in pencil_candidates(n):
        ms = time_shape(n, precision, n_orb, (block, chunk, c, four), phi, reps)
        results.append(((block, chunk, c, four), ms))
    shape, ms = min(results, key=lambda r: r[1])
    entry = {"block": shape[0], "chunk": shape[1], "pencils": shape[2],
             "four_pass": bool(shape[3]), "ms": round(ms, 4),
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
    set_shape(plan, (int(e["block"]), int(e["chunk"]), int(e["pencils"]),
                     bool(e.get("four_pass", False))))
    return plan.tiling


def set_shape(plan: "_lib.Plan", shape) -> None:
    plan.set_tiling(*shape[:3])
    plan.set_schedule(bool(shape[3]) if len(shape) > 3 else False)


def batch_key(sizes, precision: str) -> str:
    """Cache key of a batch: its (grid, orbitals) list in order."""
    return "batch/%s/" % precision + ",".join("%dx%d" % (int(n), int(k)) for n, k in sizes)


def time_batch(plans, phis, shapes, reps: int = 2, lanes: bool = True) -> float:
    """Milliseconds of one batch graph launch with the given per-instance
    shapes (best of reps, after the recording launch)."""
    import torch
    for p, sh in zip(plans, shapes):
        set_shape(p, sh)
    batch = _lib.Batch(plans)
    ws = _lib.workspace(batch.workspace_bytes(), phis[0].device)
    out = batch.outputs(phis)
    batch.build_into(phis, out, ws, lanes=lanes)  # records the graph
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    best = float("inf")
    for _ in range(reps):
        ev0.record()
        batch.build_into(phis, out, ws, lanes=lanes)
        ev1.record()
        ev1.synchronize()
        best = min(best, ev0.elapsed_time(ev1))
    del batch, ws, out
    torch.cuda.empty_cache()
    return best


def tune_batch(plans, precision: str, cache_path: Optional[str] = None, device: str = "cuda:0",
               reps: int = 2, force: bool = False, log=None) -> dict:
    """Per-instance shapes for a batch (see the module notes), from the cache
    or by timing; the plans are left on the chosen shapes."""
    import torch
    sizes = [(p.n, p.n_orb) for p in plans]
    k = batch_key(sizes, precision)
    cache = load_cache(cache_path)
    if not force and k in cache:
        e = cache[k]
        for p, sh in zip(plans, e["shapes"]):
            set_shape(p, sh)
        e.setdefault("lanes", True)
        return e
    own = []
    for p in plans:
        e1 = tune(p.n, precision, p.n_orb, cache_path, device, reps, log=log)
        own.append((int(e1["block"]), int(e1["chunk"]), int(e1["pencils"]),
                    bool(e1.get("four_pass", False))))
    g = torch.Generator(device=device)
    g.manual_seed(4321)
    phis = []
    for p in plans:
        f = torch.randn((p.n_orb, p.n, p.n, p.n), dtype=torch.float64, device=device, generator=g)
        phis.append(f * (1.0 / p.n ** 1.5))
    tried = []

    def run(label, shapes, lanes=True):
        ms = time_batch(plans, phis, shapes, reps, lanes)
        tried.append([label, [list(s) for s in shapes], round(ms, 4)])
        if log:
            log("batch shapes %s: %.3f ms" % (label, ms))
        return ms

    cands = [("own", own),
             ("block16", [(16, 0, 0, False)] * len(plans)),
             ("block8", [(8, 0, 0, False)] * len(plans))]
    best_ms, best = float("inf"), None
    for label, shapes in cands:
        ms = run(label, shapes)
        if ms < best_ms:
            best_ms, best = ms, list(shapes)
    for n in sorted({p.n for p in plans}):
        trial = [((8 if sh[0] == 16 else 16), 0, sh[2], False) if p.n == n else sh
                 for p, sh in zip(plans, best)]
        ms = run("flip n=%d" % n, trial)
        if ms < best_ms:
            best_ms, best = ms, trial
    # the lanes' shared pass launches against every instance on its own
    # launches, on the chosen shapes
    lanes = True
    ms = run("without lanes", best, lanes=False)
    if ms < best_ms:
        best_ms, lanes = ms, False
    for p, sh in zip(plans, best):
        set_shape(p, sh)
    entry = {"shapes": [list(s) for s in best], "lanes": lanes, "ms": round(best_ms, 4),
             "tried": tried}
    cache = load_cache(cache_path)
    cache[k] = entry
    save_cache(cache, cache_path)
    del phis
    torch.cuda.empty_cache()
    return entry
