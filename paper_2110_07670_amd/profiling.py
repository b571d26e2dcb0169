"""Summaries of rocprofv3 runs of bench.py for the profiles/ folder.

Reads the rocpd SQLite databases of three runs of the same command:
a kernel trace with --stats, a --pmc FETCH_SIZE run and a --pmc WRITE_SIZE
run.  HBM bytes per dispatch are the counters (KiB) scaled by what the same
counters read for a known streaming pass in the same process
(bench.py --copy-calibration: one in-place read + write launch over 1 GiB,
k_probe_rw, whose true traffic is 1 GiB read + 1 GiB written).

Usage: python -m paper_2110_07670_amd.profiling TRACE_DB FETCH_DB WRITE_DB OUT.md "COMMAND"
       python -m paper_2110_07670_amd.profiling --trace-only TRACE_DB OUT.md "TITLE" "COMMAND"
(the second form: kernel times per kernel and per stage from a trace alone)
"""
from __future__ import annotations

import collections
import hashlib
import json
import os
import sqlite3
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCE = os.path.join(HERE, "csrc", "poisson.hip")

STAGE_OF = [
    ("k_plane_fwd", "yz_fwd"), ("k_rows_fwd", "yz_fwd"), ("k_plane_inv", "yz_inv"),
    ("k_rows_inv", "yz_inv"), ("k_accumulate", "w_accumulate"), ("k_zinv_acc", "w_accumulate"),
    ("k_plane_mid", "x_poisson"), ("k_gemm_abt", "abt_product"),
    ("k_reduce_splits", "abt_product"), ("k_gemm_ab", "ab_product"), ("k_chol_left", "cholesky_inv"),
    ("k_tri_inv", "cholesky_inv"),
]


def stage_of(name: str) -> str:
    if "k_lines" in name:
        # third template argument MODE: 0 Poisson (x), 1 energy, 2 y forward, 3 y inverse
        mode = name.split("k_lines<")[1].split(">")[0].split(",")[2].strip()
        return {"0": "x_poisson", "1": "x_energy", "2": "yz_fwd", "3": "yz_inv"}.get(mode, "lines")
    for key, st in STAGE_OF:
        if key in name:
            return st
    return "other"


def _short(name: str) -> str:
    return name.split("(")[0].replace("void ", "")


def kernel_stats(trace_db: str):
    db = sqlite3.connect(trace_db)
    rows = db.execute("select name, duration from kernels").fetchall()
    agg = collections.OrderedDict()
    for name, dur in rows:
        k = _short(name)
        a = agg.setdefault(k, [0, 0.0])
        a[0] += 1
        a[1] += dur
    return agg


def counters(db_path: str, counter: str):
    db = sqlite3.connect(db_path)
    rows = db.execute("select dispatch_id, kernel_name, value, duration from counters_collection "
                      "where counter_name = ?", (counter,)).fetchall()
    return [(d, _short(k), float(v), float(dur)) for d, k, v, dur in rows]


CALIBRATION_KERNEL = "k_probe_rw"


def calibration(fetch, write):
    """(fetch factor, write factor): true KiB / counter KiB for the 1 GiB
    in-place streaming pass."""
    true_kib = float(1 << 20)
    cf = [v for _, k, v, _ in fetch if CALIBRATION_KERNEL in k]
    cw = [v for _, k, v, _ in write if CALIBRATION_KERNEL in k]
    if not cf or not cw:
        raise SystemExit("no %s dispatch in the counter runs (bench.py --copy-calibration)"
                         % CALIBRATION_KERNEL)
    return true_kib / max(cf), true_kib / max(cw)


def summarize(trace_db, fetch_db, write_db, out_md, command):
    stats = kernel_stats(trace_db)
    fetch = counters(fetch_db, "FETCH_SIZE")
    write = counters(write_db, "WRITE_SIZE")
    ff, fw = calibration(fetch, write)
    per = collections.defaultdict(lambda: {"fetch": [], "write": []})
    for _, k, v, _ in fetch:
        per[k]["fetch"].append(v)
    for _, k, v, _ in write:
        per[k]["write"].append(v)
    stage_bytes = collections.defaultdict(list)
    lines = ["# rocprofv3 summary: ACE build, water32_n96 (128 orbitals, 96^3, FP64)", "",
             "Commands (run from the repository root on one MI355X):", "", "```", command, "```", "",
             "Counter calibration (one in-place read + write launch over 1 GiB in the same "
             "process, %s): FETCH_SIZE x %.3f, WRITE_SIZE x %.3f give true bytes."
             % (CALIBRATION_KERNEL, ff, fw), "",
             "| kernel | calls | avg us | total ms | HBM read MB/launch | HBM write MB/launch |",
             "|---|---|---|---|---|---|"]
    for k, (calls, tot) in stats.items():
        c = per.get(k)
        rd = wr = float("nan")
        if c and c["fetch"] and c["write"]:
            rd = sum(c["fetch"]) / len(c["fetch"]) * ff * 1024 / 1e6
            wr = sum(c["write"]) / len(c["write"]) * fw * 1024 / 1e6
            stage_bytes[stage_of(k)].append(((rd + wr) * 1e6, calls))
        lines.append("| %s | %d | %.1f | %.3f | %.1f | %.1f |" % (k[:70], calls, tot / calls / 1e3,
                                                                tot / 1e6, rd, wr))
    kern = {}
    for st, vals in stage_bytes.items():
        tot_calls = sum(c for _, c in vals)
        kern[st] = {"bytes_per_launch": sum(b * c for b, c in vals) / tot_calls}
    rec = {"source_sha256": hashlib.sha256(open(KERNEL_SOURCE, "rb").read()).hexdigest(),
           "calibration": {"fetch_factor": ff, "write_factor": fw}, "kernels": kern}
    lines += ["", "Per-stage HBM bytes per launch (calibrated counters), keyed to the kernel "
              "source they were measured on:", "", "<!-- traffic-json", json.dumps(rec), "-->", ""]
    with open(out_md, "w") as f:
        f.write("\n".join(lines))
    return rec


def summarize_trace(trace_db, out_md, title, command):
    """Kernel-trace summary only (no counters): calls, average and total time
    per kernel and the time per stage."""
    stats = kernel_stats(trace_db)
    lines = ["# rocprofv3 summary: %s" % title, "",
             "Command (run from the repository root on one MI355X):", "", "```", command, "```",
             "", "| kernel | stage | calls | avg us | total ms |", "|---|---|---|---|---|"]
    per_stage = collections.OrderedDict()
    for k, (calls, tot) in stats.items():
        st = stage_of(k)
        lines.append("| %s | %s | %d | %.1f | %.3f |" % (k[:70], st, calls, tot / calls / 1e3,
                                                        tot / 1e6))
        a = per_stage.setdefault(st, [0, 0.0])
        a[0] += calls
        a[1] += tot
    lines += ["", "| stage | launches | total ms |", "|---|---|---|"]
    for st, (calls, tot) in per_stage.items():
        lines.append("| %s | %d | %.3f |" % (st, calls, tot / 1e6))
    with open(out_md, "w") as f:
        f.write("\n".join(lines) + "\n")
    return {st: tot / 1e6 for st, (_, tot) in per_stage.items()}


if __name__ == "__main__":
    if len(sys.argv) == 6 and sys.argv[1] == "--trace-only":
        print(json.dumps(summarize_trace(*sys.argv[2:6]), indent=1))
    elif len(sys.argv) == 6:
        print(json.dumps(summarize(*sys.argv[1:6]), indent=1))
    else:
        sys.exit(__doc__)
