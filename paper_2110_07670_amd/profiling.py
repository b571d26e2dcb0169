"""Summaries of rocprofv3 runs of bench.py for the profiles/ folder.

Reads the rocpd SQLite databases of three runs of the same command:
a kernel trace with --stats, a --pmc FETCH_SIZE run and a --pmc WRITE_SIZE
run.  HBM bytes per dispatch are the counters (KiB) scaled by what the same
counters read for a known streaming pass in the same process
(bench.py --copy-calibration: one in-place read + write launch over 1 GiB,
k_probe_rw, whose true traffic is 1 GiB read + 1 GiB written).

Usage: python -m paper_2110_07670_amd.profiling TRACE_DB FETCH_DB WRITE_DB OUT.md "COMMAND" ["TITLE"]
       python -m paper_2110_07670_amd.profiling --trace-only TRACE_DB OUT.md "TITLE" "COMMAND"
       python -m paper_2110_07670_amd.profiling --counters OUT.md "TITLE" "COMMAND" DB [DB ...]
(the second form: kernel times per kernel and per stage from a trace alone;
the third: per-kernel averages of the hardware counters of one or more
--pmc runs, with the MFMA busy fraction and FP64 matrix rate, and the VALU,
LDS and wait fractions where those counters were collected)
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
    ("k_plane_fwd", "yz_fwd"), ("k_rows_fwd", "yz_fwd"), ("k_slab_fwd", "yz_fwd"),
    ("k_slab_mid", "x_poisson"), ("k_plane_inv", "yz_inv"), ("k_slab_inv", "yz_inv"),
    ("k_rows_inv", "yz_inv"), ("k_accumulate", "w_accumulate"), ("k_zinv_acc", "w_accumulate"),
    ("k_plane_mid", "x_poisson"), ("k_gemm_abt", "abt_product"),
    ("k_reduce_splits", "abt_product"), ("k_gemm_ab", "ab_product"), ("k_chol_left", "cholesky_inv"),
    ("k_tri_inv", "cholesky_inv"),
]


def stage_of(name: str) -> str:
    if "k_batch_pass<" in name:
        # second template argument: the pass (0 forward, 1 middle, 2 inverse z + W)
        p = name.split("k_batch_pass<")[1].split(">")[0].split(",")[1].strip()
        return {"0": "yz_fwd", "1": "x_poisson", "2": "w_accumulate"}.get(p, "other")
    if "k_lines" in name:
        # third template argument MODE: 0 Poisson (x), 1 energy, 2 y forward, 3 y inverse
        mode = name.split("k_lines<")[1].split(">")[0].split(",")[2].strip()
        return {"0": "x_poisson", "1": "x_energy", "2": "yz_fwd", "3": "yz_inv"}.get(mode, "lines")
    for key, st in STAGE_OF:
        if key in name:
            return st
    return "other"


def _short(name: str) -> str:
    name = name.replace("(anonymous namespace)::", "")
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
    in-place streaming pass (the first k_probe_rw dispatch of the run: the
    HBM-ceiling probes that bench.py runs later use larger buffers)."""
    true_kib = float(1 << 20)
    cf = sorted((d, v) for d, k, v, _ in fetch if CALIBRATION_KERNEL in k)
    cw = sorted((d, v) for d, k, v, _ in write if CALIBRATION_KERNEL in k)
    if not cf or not cw:
        raise SystemExit("no %s dispatch in the counter runs (bench.py --copy-calibration)"
                         % CALIBRATION_KERNEL)
    return true_kib / cf[0][1], true_kib / cw[0][1]


DEFAULT_TITLE = "ACE build, water32_n96 (128 orbitals, 96^3, FP64)"


def summarize(trace_db, fetch_db, write_db, out_md, command, title=DEFAULT_TITLE):
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
    lines = ["# rocprofv3 summary: %s" % title, "",
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


# MI355X: 8 XCDs, 256 CUs, 4 SIMDs each; GRBM_GUI_ACTIVE sums the XCDs' cycles
N_XCD, N_CU, N_SIMD = 8, 256, 1024


def counter_table(dbs):
    """{kernel: {counter: mean per dispatch}, '_dur_us': mean duration}."""
    out = collections.OrderedDict()
    for path in dbs:
        db = sqlite3.connect(path)
        rows = db.execute("select dispatch_id, kernel_name, counter_name, value, duration "
                          "from counters_collection").fetchall()
        per = collections.defaultdict(lambda: collections.defaultdict(dict))
        for d, k, c, v, dur in rows:
            per[_short(k)][d][c] = float(v)
            per[_short(k)][d]["_dur"] = float(dur)
        for k, disp in per.items():
            rec = out.setdefault(k, {})
            cnt = collections.defaultdict(list)
            for d, cs in disp.items():
                for c, v in cs.items():
                    cnt[c].append(v)
            for c, vs in cnt.items():
                if c == "_dur":
                    rec["_dur_us"] = sum(vs) / len(vs) / 1e3
                    rec["_n"] = len(vs)
                else:
                    rec[c] = sum(vs) / len(vs)
    return out


def derived(rec):
    """Fractions from the raw counters a record holds."""
    d = {}
    g = rec.get("GRBM_GUI_ACTIVE")
    if g:
        cyc = g / N_XCD  # cycles of the dispatch
        if "SQ_VALU_MFMA_BUSY_CYCLES" in rec:
            d["mfma_busy"] = rec["SQ_VALU_MFMA_BUSY_CYCLES"] / (cyc * N_SIMD)
        if "SQ_INSTS_VALU_MFMA_MOPS_F64" in rec and rec.get("_dur_us"):
            d["f64_mfma_tflops"] = rec["SQ_INSTS_VALU_MFMA_MOPS_F64"] * 512 / (rec["_dur_us"] * 1e-6) / 1e12
    w = rec.get("SQ_WAVE_CYCLES")
    if w:
        for c, name in (("SQ_WAIT_INST_ANY", "wait_any"), ("SQ_WAIT_INST_LDS", "wait_lds"),
                        ("SQ_ACTIVE_INST_VALU", "valu_active"), ("SQ_ACTIVE_INST_LDS", "lds_active")):
            if c in rec:
                d[name + "_per_wave_cycle"] = rec[c] / w
    return d


def summarize_counters(out_md, title, command, dbs):
    """One row per library kernel: dispatches, mean duration and the derived
    fractions of the collected counters."""
    tab = counter_table(dbs)
    cols = [("mfma_busy", "MFMA busy"), ("f64_mfma_tflops", "FP64 MFMA TFLOP/s"),
            ("wait_any", "wait any / wave-cycle"), ("wait_lds", "wait LDS / wave-cycle"),
            ("valu_active", "VALU active / wave-cycle"), ("lds_active", "LDS active / wave-cycle")]
    lines = ["# rocprofv3 counters: %s" % title, "",
             "Commands (run from the repository root on one MI355X):", "", "```", command, "```", "",
             "Per library kernel, means per dispatch.  MFMA busy = SQ_VALU_MFMA_BUSY_CYCLES / "
             "(GRBM_GUI_ACTIVE per XCD x 1024 SIMDs); FP64 MFMA TFLOP/s = "
             "SQ_INSTS_VALU_MFMA_MOPS_F64 x 512 / duration; the per-wave-cycle fractions are "
             "SQ_WAIT_INST_ANY, SQ_WAIT_INST_LDS, SQ_ACTIVE_INST_VALU and SQ_ACTIVE_INST_LDS over "
             "SQ_WAVE_CYCLES.", "",
             "| kernel | dispatches | mean us | LDS bank conflicts | " +
             " | ".join(h for _, h in cols) + " |",
             "|---|---|---|---|" + "---|" * len(cols)]
    out = {}
    for k, rec in tab.items():
        if not k.startswith("acex::"):
            continue
        d = derived(rec)
        out[k] = d
        vals = []
        for key, _ in cols:
            hit = [v for name, v in d.items() if name.startswith(key)]
            vals.append("%.3f" % hit[0] if hit else "")
        lines.append("| %s | %d | %.1f | %.3g | %s |" % (
            k.replace("acex::", ""), rec.get("_n", 0), rec.get("_dur_us", 0.0),
            rec.get("SQ_LDS_BANK_CONFLICT", 0.0), " | ".join(vals)))
    lines.append("")
    with open(out_md, "w") as f:
        f.write("\n".join(lines))
    return out


if __name__ == "__main__":
    if len(sys.argv) >= 6 and sys.argv[1] == "--counters":
        print(json.dumps(summarize_counters(sys.argv[2], sys.argv[3], sys.argv[4], sys.argv[5:]),
                         indent=1))
    elif len(sys.argv) == 6 and sys.argv[1] == "--trace-only":
        print(json.dumps(summarize_trace(*sys.argv[2:6]), indent=1))
    elif len(sys.argv) in (6, 7):
        print(json.dumps(summarize(*sys.argv[1:]), indent=1))
    else:
        sys.exit(__doc__)
