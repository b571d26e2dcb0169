"""The uneven batch at full size: sixteen water-density systems (grids 48-96,
32-128 orbitals, FP32 bulk) built together through ace_batch_build.

- Every instance equals, bit for bit, a separate ace_build with the same plan.
- Instance 13 (96^3, 128 orbitals) against the FP64 oracle: E_x against the
  sum of all 8256 oracle pair energies, the full M against the oracle's M
  (both committed by tests/golden/make_reference.py), and three W rows of
  Eq. (2) and their ACE apply against oracle rows computed in a separate
  process (tests/oracle_job.py), within the stated FP32 bounds.
"""
import json
import os
import sys

import numpy as np
import pytest

from oracle import ace_oracle as O
from paper_2110_07670_amd import synth

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))
REF = os.path.join(HERE, "golden", "reference_batch13.json")
M_FULL = os.path.join(HERE, "golden", "M_full_batch13.npz")
CHECK = 13


def _say(*a):
    print("[gpu-case]", *a, flush=True)


@pytest.fixture(scope="module")
def batch_run(oracle_job):
    import torch
    from paper_2110_07670_amd import _lib
    assert torch.cuda.is_available()
    specs = synth.batch_config4()
    systems = [synth.build_system(sp) for sp in specs]
    ref = json.load(open(REF))
    sys.path.insert(0, os.path.join(HERE, "golden"))
    from make_reference import fingerprint_matches
    assert fingerprint_matches(systems[CHECK].phi, ref["phi_fingerprint"]), "generator drift"
    dev = torch.device("cuda:0")
    plans = [_lib.Plan(sp.n, (sp.L,) * 3, sp.n_orb, "fp32", sp.alpha) for sp in specs]
    phis = [torch.from_numpy(s.phi).to(dev) for s in systems]
    batch = _lib.Batch(plans)
    _say("batch of 16 at full size: graph build")
    out = batch.build(phis)
    torch.cuda.synchronize()
    rows, w = oracle_job.result("batch13_rows")
    return dict(specs=specs, systems=systems, plans=plans, phis=phis, out=out, lib=_lib,
                ref=ref, M_full=np.load(M_FULL)["M"], rows=rows, w_rows=np.array(w))


def test_batch_full_instances_bitwise_equal_separate_builds(batch_run):
    import torch
    lib, out = batch_run["lib"], batch_run["out"]
    info = out["info"].cpu().numpy()
    assert (info == 0).all()
    for k, (p, phi) in enumerate(zip(batch_run["plans"], batch_run["phis"])):
        _say("batch full: separate build of instance %d" % k)
        sep = lib.ace_build(p, phi)
        torch.cuda.synchronize()
        assert float(sep["ex"].item()) == float(out["ex"][k].item()), k
        assert torch.equal(sep["M"], out["M"][k]), k
        assert torch.equal(sep["W"], out["W"][k]), k
        del sep


def test_batch_full_instance13_against_oracle(batch_run):
    import torch
    st = batch_run
    spec, s = st["specs"][CHECK], st["systems"][CHECK]
    out, lib, plan = st["out"], st["lib"], st["plans"][CHECK]
    ex = float(out["ex"][CHECK].item())
    ex_err = abs(ex - st["ref"]["ex"]) / spec.n_atoms
    M = out["M"][CHECK].cpu().numpy()
    m_err = O.rel_err(M, st["M_full"])
    W = out["W"][CHECK]
    rows = st["rows"]
    w_err = max(O.rel_err(W[i].cpu().numpy(), st["w_rows"][a]) for a, i in enumerate(rows))
    psi = st["phis"][CHECK][rows].contiguous()
    back = lib.ace_apply(plan, out["xi"][CHECK], psi).cpu().numpy()
    torch.cuda.synchronize()
    a_err = max(O.rel_err(back[a], st["w_rows"][a]) for a in range(len(rows)))
    print("batch instance 13 (96^3, 128 orbitals, FP32 bulk): E_x %.12f (oracle %.12f), "
          "%.2e Ha/atom; M %.2e; W rows %.2e; ACE rows %.2e"
          % (ex, st["ref"]["ex"], ex_err, m_err, w_err, a_err), flush=True)
    assert ex_err < 1e-6
    assert m_err < 1e-6 and w_err < 1e-6 and a_err < 1e-6
