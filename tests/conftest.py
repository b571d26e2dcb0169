import json
import os
import shutil
import subprocess
import sys
import tempfile
import time

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# test module -> oracle tasks it reads (tests/oracle_job.py)
_JOB_TASKS = {
    "test_gpu_config2.py": ["config2_all_rows"],
    "test_gpu_batch_full.py": ["batch13_rows"],
    "test_gpu_config3.py": ["config3_row77"],
    "test_gpu_config5.py": ["config5_row255"],
}
_JOB = {}


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU test")


def _job_processes():
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(n, 16))


def pytest_collection_finish(session):
    """Start the oracle references the selected full-size GPU tests need, in a
    separate process, before any test initialises the GPU."""
    if session.config.option.collectonly:
        return
    tasks = []
    for item in session.items:
        for t in _JOB_TASKS.get(os.path.basename(str(item.fspath)), []):
            if t not in tasks:
                tasks.append(t)
    if not tasks:
        return
    out = tempfile.mkdtemp(prefix="acex_oracle_")
    log = open(os.path.join(out, "job.log"), "w")
    proc = subprocess.Popen([sys.executable, "-u", os.path.join(ROOT, "tests", "oracle_job.py"),
                             out, str(_job_processes())] + tasks,
                            stdout=log, stderr=subprocess.STDOUT, cwd=ROOT)
    _JOB.update(proc=proc, out=out, log=log, tasks=tasks)
    print("[oracle-job] started pid %d for %s" % (proc.pid, ", ".join(tasks)), flush=True)


def pytest_sessionfinish(session, exitstatus):
    proc = _JOB.get("proc")
    if proc is not None:
        if proc.poll() is None:
            proc.kill()
            proc.wait()
        _JOB["log"].close()
        shutil.rmtree(_JOB["out"], ignore_errors=True)
        _JOB.clear()


class OracleJob:
    """Results of tests/oracle_job.py: W rows of Eq. (2) from the FP64 oracle."""

    def result(self, task, timeout=900.0):
        if task not in _JOB.get("tasks", []):
            pytest.fail("oracle task %s was not started for this session" % task)
        out, proc = _JOB["out"], _JOB["proc"]
        done = os.path.join(out, task + ".done")
        t0 = time.time()
        while not os.path.exists(done):
            if proc.poll() is not None and not os.path.exists(done):
                _JOB["log"].flush()
                pytest.fail("oracle job ended (rc %s) without %s:\n%s"
                            % (proc.returncode, task,
                               open(os.path.join(out, "job.log")).read()[-2000:]))
            if time.time() - t0 > timeout:
                pytest.fail("oracle task %s still running after %.0f s" % (task, timeout))
            time.sleep(0.5)
        meta = json.load(open(done))
        return meta["rows"], np.load(os.path.join(out, task + ".npy"), mmap_mode="r")


@pytest.fixture(scope="session")
def oracle_job():
    return OracleJob()
