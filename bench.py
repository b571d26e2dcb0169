#!/usr/bin/env python3
"""ACE-build throughput on one MI355X: orbital-pair Poisson solves per second.

One step = one ace_build (pair densities, forward transforms, Coulomb
multiply, inverse transforms, W accumulation, M = dV Phi^T W, Cholesky,
projectors xi, E_x = tr(M)) followed by one ace_apply of the projectors to
the orbitals, on the 32-water-shaped workload (128 orbitals, 96^3 grid,
L = 18.6 bohr, all 8256 pairs, FP64).  Inputs are resident in HBM before the
timed region starts.

Prints one JSON line (rank 0, one GPU).  `value` comes from the timed steps,
run without any stage events.  The same number of steps is then run again
with HIP events around every launch on the library's stream: `roofline`
reports the kernel that takes the largest share of the step, its algorithmic
bytes per launch over its average launch time from those events, against the
8 TB/s HBM peak, with the whole pair loop (all transform passes) beside it;
`hbm_ceilings_GBps` holds what plain streaming kernels of the passes' access
kinds reach on the same device (read + write in place, read only, write
only), and each stage is reported against both.  `traffic` is the
counter-measured HBM bytes per launch of that kernel from the committed
rocprofv3 summary, or null when the kernel source changed since.
`cpu_baseline` times the FP64 oracle's pair loop on a bounded sample of the
same workload on the host cores.
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
FP64_MFMA_PEAK_TFLOPS = 78.6
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_water32_n96.md")
KERNEL_SOURCE = os.path.join(ROOT, "paper_2110_07670_amd", "csrc", "poisson.hip")


def tile_plan(n_orb, block, full_kind="three_pass"):
    """(bi, bj, diag, npack, kind) for every tile of the unmasked schedule;
    kind: the passes the tile takes ("three_pass", "rows_fused" or
    "four_pass"; full tiles take the plan's full-tile schedule, the library's
    ace_plan_schedule, the others four passes)."""
    out = []
    nb = (n_orb + block - 1) // block
    for I in range(nb):
        for J in range(I, nb):
            bi = min(block, n_orb - I * block)
            bj = min(block, n_orb - J * block)
            # two pairs of one row share a transform; a row's odd leftover is alone
            rows = [bi - a for a in range(bi)] if I == J else [bj] * bi
            kind = full_kind if bi == block and bj == block else "four_pass"
            out.append((bi, bj, I == J, sum((r + 1) // 2 for r in rows), kind))
    return out


def plan_tiles(plan):
    kind, plane = plan.schedule()
    return tile_plan(plan.n_orb, plan.tiling[0], kind), plane


def algorithmic_bytes(stage, tiles, npts, bulk, plane=True):
    """Compulsory HBM bytes of one step's launches of `stage` in this design.

    Per packed transform (two pairs) and grid point, c = one complex value:
    yz_fwd writes c (a plane, or slab by slab where a plane does not fit
    LDS); x_poisson (the middle pass: x, and on three-pass tiles the inverse
    y too) reads and writes c; yz_inv reads and writes c on four-pass tiles
    (twice where a plane does not fit: inverse y lines, then z rows) and on
    row-fused tiles (the inverse y lines); w_accumulate reads c.
    Orbital traffic is counted once per tile: yz_fwd reads the tile's
    orbitals (8 B/pt each); w_accumulate reads them and reads + writes their
    W rows (24 B/pt each).
    """
    c = 2 * bulk
    tot = 0
    for bi, bj, diag, npack, kind in tiles:
        orbs = bi if diag else bi + bj
        if stage == "yz_fwd":
            tot += (npack * c + orbs * 8) * npts
        elif stage == "yz_inv":
            if kind == "rows_fused":
                tot += npack * 2 * c * npts
            elif kind == "four_pass":
                tot += npack * (2 * c if plane else 4 * c) * npts
        elif stage == "x_poisson":
            tot += npack * 2 * c * npts
        elif stage == "w_accumulate":
            tot += (npack * c + orbs * 24) * npts
    return tot


def read_traffic(stage):
    """Counter-measured bytes per launch from the committed summary, or None."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    text = open(TRAFFIC_FILE).read()
    m = re.search(r"<!-- traffic-json\s*(\{.*?\})\s*-->", text, re.S)
    if not m:
        return None
    rec = json.loads(m.group(1))
    src = hashlib.sha256(open(KERNEL_SOURCE, "rb").read()).hexdigest()
    if rec.get("source_sha256") != src:
        return None
    k = rec.get("kernels", {}).get(stage)
    return None if k is None else k.get("bytes_per_launch")


def workload_text(spec, precision):
    if spec.name == "water32_n96" and precision == "fp64":
        return ("water32_n96: 128 Loewdin-orthonormal sum-of-Gaussian orbitals on 32 random "
                "rigid waters, L=18.6 bohr, 96^3 grid, all 8256 pairs, alpha=0.25, FP64; "
                "step = ace_build + ace_apply(xi, phi)")
    return ("%s: %d orbitals, %d^3 grid, L=%.1f bohr, all %d pairs, alpha=%.2f, %s; "
            "step = ace_build + ace_apply(xi, phi)"
            % (spec.name, spec.n_orb, spec.n, spec.L, spec.n_pairs, spec.alpha,
               "FP64" if precision == "fp64" else "FP32 transforms with FP64 W/M/Cholesky/E"))


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(system, spec, n_pairs_sample):
    from oracle import timing
    k = spec.n_orb
    pairs = [(i, j) for i in range(k) for j in range(i, k)]
    step = max(1, len(pairs) // n_pairs_sample)
    sample = pairs[::step][:n_pairs_sample]
    procs = timing.default_processes()
    rate, secs, used = timing.time_pair_sample(system.phi, spec.cell, spec.alpha, sample, procs)
    return {"value": rate, "unit": "pair-solves/s", "cores": used, "kind": "oracle",
            "host_cpu_count": os.cpu_count(), "cpu_model": cpu_model(),
            "sample": "%d of %d pairs (every %d-th in i<=j order) of the same %d^3 / %d-orbital "
                      "workload, oracle FFT pair loop with W updates, %.1f s wall on %d processes "
                      "(one per usable host core, capped at the 16-core share of a one-GPU host; "
                      "os.cpu_count() = %s)"
                      % (len(sample), len(pairs), step, spec.n, k, secs, used, os.cpu_count())}


def measure_ceilings(torch, dev, gib=2, reps=5):
    """Achievable HBM rates of plain streaming kernels (include/ace_probe.h) on
    a buffer far larger than the caches: read + write in place, read only,
    write only.  GB/s counts the bytes moved (read + written)."""
    from paper_2110_07670_amd import _lib
    buf = torch.empty(gib << 30, dtype=torch.uint8, device=dev)
    blocks = 256 * 16
    out = {}
    for kind, factor in (("write", 1), ("read_write", 2), ("read", 1)):
        _lib.bandwidth_probe(kind, buf, blocks)  # warm
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record()
        for _ in range(reps):
            _lib.bandwidth_probe(kind, buf, blocks)
        ev[1].record()
        torch.cuda.synchronize()
        ms = ev[0].elapsed_time(ev[1]) / reps
        out[kind] = factor * buf.numel() / (ms * 1e-3) / 1e9
    del buf
    return out


# the probe whose access kind matches each transform pass's traffic
STAGE_ACCESS = {"yz_fwd": "write", "x_poisson": "read_write", "yz_inv": "read_write",
                "w_accumulate": "read"}


RHO_CUT = {2: 2.5e-2, 3: 1e-2, 5: 2e-3}  # the paper's Table 3 by system size


def run_screened(args):
    """Screened build vs all-pairs builds on one workload (default config 5).

    A screened step = the library's screening decision (ace_screen_mask:
    overlap integrals, or Wannier moments + MLP pair predictions, on the GPU,
    then the mask on the host, with the all-pairs fallback) + ace_build(mask)
    + ace_apply.  The MLP is trained beforehand (not timed) on pair energies
    the GPU build produces for the training systems.  Timed beside it, on the
    same inputs: the all-pairs build in the screened run's bulk precision and
    the plain FP64 all-pairs build (the reference form); E_x errors are
    judged against the FP64 all-pairs build."""
    import numpy as np
    import torch

    from paper_2110_07670_amd import _lib, screening, synth

    cfg = args.config if args.config != 2 else 5
    spec = synth.config(cfg)
    system = synth.build_system(spec)
    dev = torch.device("cuda:0")
    wts = None
    t_train = 0.0
    if args.screen == "mlp":
        t0 = time.perf_counter()
        X, y = screening.training_data()
        params = screening.train_pair_mlp(X, y)
        t_train = time.perf_counter() - t0
        wts = torch.from_numpy(screening.weights_to_array(params)).to(dev)
    phi = torch.from_numpy(system.phi).to(dev)
    budget = 1e-6 * spec.n_atoms
    rho_cut = RHO_CUT.get(cfg, 2e-3)

    def make(precision):
        plan = _lib.Plan(spec.n, (spec.L,) * 3, spec.n_orb, precision, spec.alpha)
        if args.tiling:
            plan.set_tiling(*[int(v) for v in args.tiling.split(",")])
        return plan

    def timed(fn, steps):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps

    plan = make(args.precision)
    ws = _lib.workspace(plan.workspace_bytes(), dev)
    ws_apply = _lib.workspace(plan.apply_workspace_bytes(spec.n_orb), dev)
    W = torch.empty_like(phi)
    xi = torch.empty_like(phi)
    out = torch.empty_like(phi)
    M = torch.empty((spec.n_orb, spec.n_orb), dtype=torch.float64, device=dev)
    ex = torch.zeros(1, dtype=torch.float64, device=dev)
    info = torch.zeros(1, dtype=torch.int32, device=dev)
    state = {}

    def full_step(pl=plan, w=ws):
        _lib.build_into(pl, phi, W, M, xi, ex, info, w)
        _lib.apply_into(pl, xi, phi, out, ws_apply)

    def screened_step():
        mask, rep = _lib.screen_mask(plan, phi, args.screen, rho_cut=rho_cut, budget=budget,
                                     weights=wts, ws=ws)
        _lib.build_into(plan, phi, W, M, xi, ex, info, ws, pair_mask=mask)
        _lib.apply_into(plan, xi, phi, out, ws_apply)
        state["mask"], state["rep"] = mask, rep

    t_full = timed(full_step, args.steps)
    e_full = float(ex.item())
    t_scr = timed(screened_step, args.steps)
    e_scr = float(ex.item())
    stages = {}
    for label, fn in (("screened", screened_step), ("all_pairs", full_step)):
        plan.set_profiling(True)
        fn()
        torch.cuda.synchronize()
        stages[label] = {k: [round(ms, 3), c] for k, (ms, c) in plan.profile_read().items() if c}
        plan.set_profiling(False)
    t_fp64, e_fp64 = None, None
    if args.precision != "fp64" and not args.no_fp64_reference:
        del ws
        torch.cuda.empty_cache()
        plan64 = make("fp64")
        ws64 = _lib.workspace(plan64.workspace_bytes(), dev)
        t_fp64 = timed(lambda: full_step(plan64, ws64), max(1, min(args.steps, 2)))
        e_fp64 = float(ex.item())
        del ws64
    elif args.precision == "fp64":
        t_fp64, e_fp64 = t_full, e_full
    kept = int(state["mask"].sum())
    e_ref = e_fp64 if e_fp64 is not None else e_full
    result = {
        "metric": "screened ACE build vs all-pairs builds (%s screen)" % args.screen,
        "value": spec.n_pairs / t_scr, "unit": "pairs covered/s",
        "solves_per_s": kept / t_scr, "all_pairs_value": spec.n_pairs / t_full,
        "speedup_vs_all_pairs_same_precision": t_full / t_scr,
        "speedup_vs_fp64_all_pairs": (t_fp64 / t_scr) if t_fp64 else None,
        "ms_per_step": 1000 * t_scr, "all_pairs_ms": 1000 * t_full,
        "fp64_all_pairs_ms": 1000 * t_fp64 if t_fp64 else None,
        "pairs_kept": kept, "pairs_total": spec.n_pairs, "screen_report": state["rep"],
        "ex_fp64_all_pairs": e_fp64, "ex_all_pairs": e_full, "ex_screened": e_scr,
        "ex_error_Ha_per_atom_vs_fp64": abs(e_scr - e_ref) / spec.n_atoms,
        "ex_error_Ha_per_atom_all_pairs_same_precision_vs_fp64": abs(e_full - e_ref) / spec.n_atoms,
        "budget_Ha": budget, "train_s": t_train, "steps": args.steps, "n_gpus": 1,
        "stages_ms_launches": stages,
        "dtype": "f64" if args.precision == "fp64" else "f32 transforms, f64 W/M/Cholesky/E",
        "config": {"workload": workload_text(spec, args.precision), "n_orb": spec.n_orb,
                   "grid": spec.n, "rho_cut": rho_cut if args.screen == "overlap" else None},
    }
    print(json.dumps(result), flush=True)


def run_batch(args):
    """Sixteen uneven systems (grids 48-96, 32-128 orbitals, liquid-water
    density) built together: one recorded HIP graph per step, every instance
    on launch shapes from the tuner.  Compared in the same run with the same
    builds issued one after another on one stream, and with the graph's
    branches launched directly (no graph)."""
    import numpy as np
    import torch

    from paper_2110_07670_amd import _lib, autotune, synth

    def say(*a):
        print("[bench]", *a, file=sys.stderr, flush=True)

    specs = synth.batch_config4()
    systems = []
    for sp in specs:
        systems.append(synth.build_system(sp))
        say("built %s n=%d orbitals=%d" % (sp.name, sp.n, sp.n_orb))
    assert torch.cuda.is_available(), "bench needs a GPU"
    dev = torch.device("cuda:0")
    plans = [_lib.Plan(sp.n, (sp.L,) * 3, sp.n_orb, args.precision, sp.alpha) for sp in specs]
    tuned = None
    use_lanes = True
    if not args.no_tune:
        t0 = time.perf_counter()
        tuned = autotune.tune_batch(plans, args.precision, cache_path=args.tune_cache, log=say)
        use_lanes = bool(tuned.get("lanes", True))
        tuned = {"batch_ms": tuned["ms"], "lanes": use_lanes,
                 "trials": [t[0] for t in tuned["tried"]],
                 "tune_s": round(time.perf_counter() - t0, 1)}
    phis = [torch.from_numpy(s.phi).to(dev) for s in systems]
    batch = _lib.Batch(plans)
    lanes, whole_tiles, other_tiles = batch.lanes()
    ws = _lib.workspace(batch.workspace_bytes(), dev)
    out = batch.outputs(phis)
    total_pairs = sum(sp.n_pairs for sp in specs)

    def timed(fn):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / args.steps

    t_graph = timed(lambda: batch.build_into(phis, out, ws, lanes=use_lanes))
    ex_graph = out["ex"].cpu().numpy().copy()
    info = out["info"].cpu().numpy()
    assert (info == 0).all(), "Cholesky of -M failed in %s" % np.nonzero(info)[0]
    t_eager = timed(lambda: batch.build_into(phis, out, ws, eager=True, lanes=use_lanes))
    t_lanes = timed(lambda: batch.build_into(phis, out, ws, lanes=True))
    t_alone = timed(lambda: batch.build_into(phis, out, ws, lanes=False))
    seq_ws = [_lib.workspace(p.workspace_bytes(), dev) for p in plans]
    seq_out = [_lib.ace_build(p, f, ws=w) for p, f, w in zip(plans, phis, seq_ws)]

    def sequential():
        for p, f, w, o in zip(plans, phis, seq_ws, seq_out):
            _lib.build_into(p, f, o["W"], o["M"], o["xi"], o["ex"], o["info"], w)

    t_seq = timed(sequential)
    ex_seq = np.array([float(o["ex"].item()) for o in seq_out])
    # per-stage times from one profiled sequential pass (events cannot sit in a graph)
    mem_stages = ["yz_fwd", "x_poisson", "yz_inv", "w_accumulate"]
    bulk = 8 if args.precision == "fp64" else 4
    agg = {s: [0.0, 0, 0.0] for s in mem_stages}
    for p in plans:
        p.set_profiling(True)
    sequential()
    torch.cuda.synchronize()
    for p, sp in zip(plans, specs):
        prof = p.profile_read()
        p.set_profiling(False)
        tiles, plane = plan_tiles(p)
        for s in mem_stages:
            ms, cnt = prof[s]
            agg[s][0] += ms
            agg[s][1] += cnt
            agg[s][2] += algorithmic_bytes(s, tiles, sp.n ** 3, bulk, plane)
    stages = {s: {"ms": round(v[0], 3), "launches": v[1],
                  "alg_GBps": v[2] / (v[0] * 1e-3) / 1e9 if v[0] else None}
              for s, v in agg.items()}
    dom = max(mem_stages, key=lambda s: agg[s][0])
    achieved = agg[dom][2] / (agg[dom][0] * 1e-3) / 1e9
    # the whole pair loop of the batch graph: algorithmic bytes of every
    # transform and W pass of every instance over the graph's wall time
    # (which also holds the dense tails)
    loop_bytes = sum(v[2] for v in agg.values())
    result = {
        "metric": "orbital-pair Poisson solves/s over 16 uneven systems in one graph launch",
        "value": total_pairs / t_graph, "unit": "pair-solves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1000 * t_graph,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32 transforms, f64 W/M/Cholesky/E",
        "data": "synthetic",
        "config": {"workload": "16 single-Gaussian water-density systems, grids %s, orbitals %s, "
                               "%d pairs in all; step = one batch build"
                               % ([sp.n for sp in specs], [sp.n_orb for sp in specs], total_pairs),
                   "shapes": [list(p.tiling) + [p.four_pass] for p in plans]},
        "tuner": tuned,
        "lanes": lanes, "tiles_in_shared_passes": whole_tiles, "tiles_other": other_tiles,
        "graph_ms": 1000 * t_graph, "eager_branches_ms": 1000 * t_eager,
        "lanes_used": use_lanes, "graph_with_lanes_ms": 1000 * t_lanes,
        "graph_without_lanes_ms": 1000 * t_alone,
        "sequential_ms": 1000 * t_seq, "speedup_vs_sequential": t_seq / t_graph,
        "ex_bitwise_equal_to_sequential": bool(np.array_equal(ex_graph, ex_seq)),
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBPS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBPS, "traffic": None,
                     "note": "all launches of the kernel over the batch, sequential profiled pass",
                     "batch_graph": {"alg_bytes": loop_bytes,
                                     "achieved": loop_bytes / t_graph / 1e9,
                                     "frac": loop_bytes / t_graph / 1e9 / HBM_PEAK_GBPS}},
        "stages_sequential": stages,
    }
    print(json.dumps(result), flush=True)


def run_scdm(args):
    """SCDM localisation of one workload's orbitals: s' preselection, pivoted
    QR over the kept points, polar orthonormalisation and the rotation of the
    orbitals; the oracle's same steps timed on the host first."""
    import numpy as np
    import torch

    from paper_2110_07670_amd import _lib, synth

    spec = synth.config(args.config)
    system = synth.build_system(spec)
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import scdm_oracle as SO
        t0 = time.perf_counter()
        pts_ref, _, _ = SO.preselect(system.phi, spec.cell)
        t1 = time.perf_counter()
        SO.scdm(system.phi, pts_ref)
        t2 = time.perf_counter()
        cpu = {"preselect_s": t1 - t0, "localize_s": t2 - t1, "kept_points": int(len(pts_ref)),
               "kind": "oracle", "cores": 1,
               "sample": "the whole workload, numpy with its default BLAS threads"}
    dev = torch.device("cuda:0")
    phi = torch.from_numpy(system.phi).to(dev)
    plan = _lib.Plan(spec.n, (spec.L,) * 3, spec.n_orb, "fp64", spec.alpha)
    pts = _lib.scdm_preselect(plan, phi)
    m = int(pts.numel())
    ws = _lib.workspace(int(_lib.load().scdm_workspace_bytes(plan.handle, m)), dev)
    for _ in range(args.warmup):
        _lib.scdm_localize(plan, phi, pts, ws=ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        pts = _lib.scdm_preselect(plan, phi, ws=ws)
    torch.cuda.synchronize()
    t_pre = (time.perf_counter() - t0) / args.steps
    t0 = time.perf_counter()
    for _ in range(args.steps):
        piv, loc, info = _lib.scdm_localize(plan, phi, pts, ws=ws)
    torch.cuda.synchronize()
    t_loc = (time.perf_counter() - t0) / args.steps
    f = loc.reshape(spec.n_orb, -1)
    defect = float((spec.L ** 3 / spec.n ** 3 * (f @ f.T) -
                    torch.eye(spec.n_orb, dtype=torch.float64, device=dev)).abs().max())
    result = {
        "metric": "SCDM localisation time (s' preselection + pivoted QR + polar + rotation)",
        "value": 1000 * (t_pre + t_loc), "unit": "ms", "higher_is_better": False,
        "preselect_ms": 1000 * t_pre, "localize_ms": 1000 * t_loc, "kept_points": m,
        "grid_points": spec.n ** 3, "info": int(info.item()), "orthonormality_defect": defect,
        "steps": args.steps, "n_gpus": 1, "dtype": "f64",
        "config": {"workload": workload_text(spec, "fp64").split(";")[0], "n_orb": spec.n_orb,
                   "grid": spec.n},
    }
    if cpu is not None:
        result["cpu_baseline"] = cpu
    print(json.dumps(result), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-pairs", type=int, default=640)
    ap.add_argument("--config", type=int, default=2,
                    help="workload: 2 (default, the headline), 1, 3, 5, or 4 (uneven batch)")
    ap.add_argument("--tune-cache", default=None,
                    help="launch-shape tuner cache for --config 4 (default: user cache)")
    ap.add_argument("--tiling", default=None,
                    help="launch shape BLOCK,CHUNK,PENCILS (ace_plan_set_tiling)")
    ap.add_argument("--scdm", action="store_true",
                    help="time SCDM localisation of the workload's orbitals instead")
    ap.add_argument("--four-pass", action="store_true",
                    help="four transform passes on every tile (ace_plan_set_schedule)")
    ap.add_argument("--no-tune", action="store_true",
                    help="--config 4 with the default launch shapes")
    ap.add_argument("--precision", default=None, choices=["fp64", "fp32"],
                    help="bulk precision (default: FP64 for configs 1-2 and SCDM, FP32 for "
                         "configs 3-5, as the workloads are specified)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one 1 GiB in-place streaming pass (counter calibration runs)")
    ap.add_argument("--no-ceilings", action="store_true",
                    help="skip the streaming-probe measurement of the achievable HBM rates")
    ap.add_argument("--screen", choices=["mlp", "overlap"], default=None,
                    help="measure a screened build against the all-pairs builds instead")
    ap.add_argument("--no-fp64-reference", action="store_true",
                    help="--screen: skip timing the plain FP64 all-pairs build")
    args = ap.parse_args()
    if args.precision is None:
        cfg = 5 if args.screen and args.config == 2 else args.config  # the screened default
        args.precision = "fp32" if cfg in (3, 4, 5) and not args.scdm else "fp64"
    if args.gpus != 1:
        sys.exit("bench.py measures one GPU: the ACE build here runs on a single MI355X "
                 "(--gpus %d requested; multi-GPU sharding is described, not built)" % args.gpus)
    if args.screen:
        return run_screened(args)
    if args.config == 4:
        return run_batch(args)
    if args.scdm:
        return run_scdm(args)

    import numpy as np
    import torch

    from paper_2110_07670_amd import _lib, synth

    spec = synth.config(args.config)
    system = synth.build_system(spec)
    # the host-core oracle runs before this process touches the GPU
    cpu = None if args.no_cpu_baseline else cpu_baseline(system, spec, args.cpu_pairs)
    assert torch.cuda.is_available(), "bench needs a GPU"
    dev = torch.device("cuda:0")
    phi = torch.from_numpy(system.phi).to(dev)
    plan = _lib.Plan(spec.n, (spec.L,) * 3, spec.n_orb, args.precision, spec.alpha)
    if args.tiling:
        plan.set_tiling(*[int(v) for v in args.tiling.split(",")])
    if args.four_pass:
        plan.set_schedule(True)
    ws = _lib.workspace(plan.workspace_bytes(), dev)
    ws_apply = _lib.workspace(plan.apply_workspace_bytes(spec.n_orb), dev)
    W = torch.empty_like(phi)
    xi = torch.empty_like(phi)
    out = torch.empty_like(phi)
    M = torch.empty((spec.n_orb, spec.n_orb), dtype=torch.float64, device=dev)
    ex = torch.zeros(1, dtype=torch.float64, device=dev)
    info = torch.zeros(1, dtype=torch.int32, device=dev)

    def step():
        _lib.build_into(plan, phi, W, M, xi, ex, info, ws)
        _lib.apply_into(plan, xi, phi, out, ws_apply)

    if args.copy_calibration:
        # a known-size in-place streaming pass (1 GiB read + 1 GiB written)
        # for scaling the FETCH_SIZE / WRITE_SIZE counters of the same run
        cal = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
        _lib.bandwidth_probe("read_write", cal, 256 * 16)
        torch.cuda.synchronize()
        del cal

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # the timed steps run without stage events (value); the same number of
    # steps is then run again with HIP events around every launch on the
    # library's stream for the per-stage and per-kernel times
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    assert int(info.item()) == 0, "Cholesky of -M failed"
    elapsed = t1 - t0
    value = spec.n_pairs * args.steps / elapsed
    ms_per_step = 1000.0 * elapsed / args.steps
    plan.set_profiling(True)
    torch.cuda.synchronize()
    tp0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    tp1 = time.perf_counter()
    prof = plan.profile_read()
    plan.set_profiling(False)
    ceilings = None if args.no_ceilings else measure_ceilings(torch, dev)

    bulk = 8 if args.precision == "fp64" else 4
    tiles, plane = plan_tiles(plan)
    npts = spec.n ** 3
    mem_stages = ["yz_fwd", "x_poisson", "yz_inv", "w_accumulate"]
    stages = {}
    for name, (ms, cnt) in prof.items():
        if cnt:
            stages[name] = {"ms_per_step": ms / args.steps, "launches_per_step": cnt // args.steps}
    for name in mem_stages:
        if name in stages:
            ab = algorithmic_bytes(name, tiles, npts, bulk, plane)
            launch_ms = stages[name]["ms_per_step"] / stages[name]["launches_per_step"]
            gbps = ab / (stages[name]["ms_per_step"] * 1e-3) / 1e9
            stages[name]["alg_GBps"] = gbps
            stages[name]["frac_of_peak"] = gbps / HBM_PEAK_GBPS
            if ceilings:
                acc = STAGE_ACCESS[name]
                stages[name]["ceiling_kind"] = acc
                stages[name]["frac_of_ceiling"] = gbps / ceilings[acc]
            stages[name]["alg_bytes_per_launch"] = ab / stages[name]["launches_per_step"]
            stages[name]["avg_launch_ms"] = launch_ms
    # FP64 MFMA products: M = dV Phi^T W and xi = W L^-T (2 n^2 N flops each),
    # the apply (dV xi^T psi, then -xi C: 4 n n_vec N flops, n_vec = n here)
    for name, fl in (("m_product", 2.0 * spec.n_orb ** 2 * npts),
                     ("xi_product", 2.0 * spec.n_orb ** 2 * npts),
                     ("apply_products", 4.0 * spec.n_orb ** 2 * npts)):
        if name in stages:
            tf = fl / (stages[name]["ms_per_step"] * 1e-3) / 1e12
            stages[name]["TFLOPs"] = tf
            stages[name]["mfma_frac"] = tf / FP64_MFMA_PEAK_TFLOPS
    dom = max((s for s in mem_stages if s in stages), key=lambda s: stages[s]["ms_per_step"])
    d = stages[dom]
    achieved = d["alg_bytes_per_launch"] / (d["avg_launch_ms"] * 1e-3) / 1e9
    traffic = read_traffic(dom) if (args.config, args.precision) == (2, "fp64") else None
    pair_loop_ms = sum(stages[s]["ms_per_step"] for s in mem_stages if s in stages)
    # the survey's algorithmic bytes: 32 B (FP64) or 16 B (FP32) per point per pair
    loop_bytes = spec.n_pairs * 4.0 * bulk * npts
    loop_gbps = loop_bytes / (pair_loop_ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBPS,
                "unit": "GB/s", "frac": achieved / HBM_PEAK_GBPS, "traffic": traffic,
                "pair_loop": {"ms": pair_loop_ms, "alg_bytes": loop_bytes,
                              "achieved": loop_gbps, "frac": loop_gbps / HBM_PEAK_GBPS}}
    if ceilings:
        roofline["frac_of_ceiling"] = achieved / ceilings[STAGE_ACCESS[dom]]
        roofline["pair_loop"]["frac_of_copy_ceiling"] = loop_gbps / ceilings["read_write"]

    result = {
        "metric": "orbital-pair Poisson solves/s in ACE build (128 orb, 96^3) + % HBM roofline",
        "value": value,
        "unit": "pair-solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32 transforms, f64 W/M/Cholesky/E",
        "data": "synthetic",
        "config": {"workload": workload_text(spec, args.precision),
                   "n_orb": spec.n_orb, "grid": spec.n, "pairs": spec.n_pairs,
                   "tiling": list(plan.tiling), "full_tiles": plan.schedule()[0]},
        "roofline": roofline,
        "pair_loop_ms": pair_loop_ms,
        "profiled_ms_per_step": 1000.0 * (tp1 - tp0) / args.steps,
        "hbm_ceilings_GBps": ceilings,
        "stages": stages,
        "ex": float(ex.item()),
    }
    if cpu is not None:
        result["cpu_baseline"] = cpu
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
