"""FP64 oracle references for the full-size GPU tests, computed in a process of
their own.

The GPU test session starts this script (tests/conftest.py) as soon as it has
collected its tests, before any test touches the GPU, so the oracle's process
pool forks from a process that never initialises a GPU and runs while the
first GPU tests do.  Every task regenerates its seeded inputs with the shared
generator and calls only the oracle (oracle.pool over ace_oracle.apply_vx_rows,
pinned to ace_oracle.apply_vx on the CPU), then writes <task>.npy and
<task>.done into the output folder.

Usage: python tests/oracle_job.py OUTDIR PROCESSES TASK [TASK ...]
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, ROOT)

from oracle import pool  # noqa: E402
from paper_2110_07670_amd import synth  # noqa: E402

# task -> (system spec, rows of Eq. (2); None = every row)
TASKS = {
    "config2_all_rows": (lambda: synth.config(2), None),
    "config3_row77": (lambda: synth.config(3), [77]),
    "config5_row255": (lambda: synth.config(5), [255]),
    "batch13_rows": (lambda: synth.batch_config4()[13], [0, 57, 127]),
}


def run(task, outdir, processes):
    make_spec, rows = TASKS[task]
    spec = make_spec()
    t0 = time.time()
    s = synth.build_system(spec)
    print("[oracle-job] %s: inputs in %.1fs" % (task, time.time() - t0), flush=True)
    if rows is None:
        path = os.path.join(outdir, task + ".npy")
        W = np.lib.format.open_memmap(path + ".tmp", mode="w+", dtype=np.float64,
                                      shape=s.phi.shape)
        pool.apply_vx_pool(s.phi, spec.cell, spec.alpha, processes, out=W)
        W.flush()
        del W
        os.replace(path + ".tmp", path)
    else:
        got = pool.apply_vx_rows_pool(s.phi, spec.cell, spec.alpha, rows, processes)
        np.save(os.path.join(outdir, task + ".npy"), np.stack([got[i] for i in rows]))
    with open(os.path.join(outdir, task + ".done"), "w") as f:
        json.dump({"rows": rows, "seconds": time.time() - t0, "subseed": s.subseed}, f)
    print("[oracle-job] %s: done in %.1fs" % (task, time.time() - t0), flush=True)


def main():
    outdir, processes = sys.argv[1], int(sys.argv[2])
    for task in sys.argv[3:]:
        run(task, outdir, processes)


if __name__ == "__main__":
    main()
