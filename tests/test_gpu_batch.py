"""Batches of uneven systems in one recorded HIP graph, through the C-ABI.

Every instance of a batch must equal, bit for bit, a separate ace_build with
the same plan and mask (the graph only reorders independent launches across
streams); graph replays, with unrelated eager work and output poisoning
between them, must reproduce the first result.  One instance per batch is
also held against the FP64 oracle at 1e-10.
"""
import sys

import numpy as np
import pytest

from oracle import ace_oracle as O
from paper_2110_07670_amd import synth

pytestmark = pytest.mark.gpu
TOL = 1e-10

# (n, orbitals, precision, (block, chunk, pencils), mask: None, "random" or
# "tail" (pairs of the first 16 orbitals all kept, the rest random))
# From the sixth on they take the persistent batch passes for their whole
# tiles: a lane of two instances with unequal tile counts (48 FP32), one
# instance with a mask whose leading tiles are complete, and the partial
# tiles of all of them between the passes.  The last five complete the
# grid sizes and precisions of the lanes: there the system's own forward
# pass takes each plane as two slabs and the lane's items whole planes, with
# the same operations per element, so the bits must agree.
INSTANCES = [
    (16, 4, "fp64", (16, 0, 0), None),
    (24, 13, "fp64", (8, 0, 8), None),
    (32, 9, "fp64", (16, 5, 32), "random"),
    (40, 6, "fp32", (16, 0, 0), None),
    (48, 20, "fp64", (8, 7, 16), None),
    (48, 20, "fp32", (8, 0, 0), None),
    (64, 17, "fp64", (16, 0, 0), None),
    (48, 9, "fp32", (8, 0, 0), None),
    (64, 22, "fp64", (8, 0, 0), "tail"),
    (80, 8, "fp32", (8, 0, 16), None),
    (48, 8, "fp64", (8, 0, 0), None),
    (64, 8, "fp32", (8, 0, 0), None),
    (80, 8, "fp64", (8, 0, 0), None),
    (96, 8, "fp64", (8, 0, 0), None),
    (96, 8, "fp32", (8, 0, 0), None),
]


def _say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def lib():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2110_07670_amd import _lib
    _lib.load()
    return _lib


def _dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")


def _host(t):
    return t.detach().cpu().numpy()


def _mask(k, seed, kind="random"):
    rng = np.random.default_rng(seed)
    m = rng.random((k, k)) < 0.6
    if kind == "tail":
        m[:16, :16] = True
    m = m | m.T
    np.fill_diagonal(m, True)
    return m.astype(np.uint8)


@pytest.fixture(scope="module")
def systems():
    out = []
    for idx, (n, k, prec, shape, masked) in enumerate(INSTANCES):
        L = 0.11 * n + 5.0
        spec = synth.SystemSpec("b%d" % idx, L, n, k, "random", 0, (1.0, 1.4), 0.25, 70 + idx)
        s = synth.build_system(spec)
        out.append((spec, s, prec, shape, _mask(k, 90 + idx, masked) if masked else None))
    return out


def _plans(lib, systems):
    plans = []
    for spec, s, prec, shape, _ in systems:
        p = lib.Plan(spec.n, (spec.L,) * 3, spec.n_orb, prec, spec.alpha)
        p.set_tiling(*shape)
        plans.append(p)
    return plans


def _separate(lib, plans, systems, phis):
    import torch
    refs = []
    for p, (spec, s, prec, shape, mask), phi in zip(plans, systems, phis):
        out = lib.ace_build(p, phi, pair_mask=mask)
        refs.append(out)
    torch.cuda.synchronize()
    return [{k: _host(v) for k, v in r.items()} for r in refs]


def _assert_same(out, refs):
    for i, r in enumerate(refs):
        assert np.array_equal(_host(out["W"][i]), r["W"]), "W of instance %d" % i
        assert np.array_equal(_host(out["M"][i]), r["M"]), "M of instance %d" % i
        assert np.array_equal(_host(out["xi"][i]), r["xi"]), "xi of instance %d" % i
        assert _host(out["ex"])[i] == r["ex"][0], "ex of instance %d" % i
        assert _host(out["info"])[i] == r["info"][0], "info of instance %d" % i


def test_batch_graph_matches_separate_builds_and_replays(lib, systems):
    import torch
    _say("batch graph: %d uneven instances n=16..96" % len(systems))
    plans = _plans(lib, systems)
    phis = [_dev(s.phi) for _, s, _, _, _ in systems]
    refs = _separate(lib, plans, systems, phis)
    batch = lib.Batch(plans, [m for *_, m in systems])
    # lanes: 48^3 FP32 block 8 (two instances), 64^3 FP64 block 16 and
    # block 8 (one each), 80^3 FP32 block 8 (one), and one each of 48^3
    # FP64, 64^3 FP32, 80^3 FP64, 96^3 FP64 and FP32, block 8
    lanes, whole, other = batch.lanes()
    assert lanes == 9 and whole > 0 and other > 0
    ws = lib.workspace(batch.workspace_bytes())
    out = batch.outputs(phis)
    batch.build_into(phis, out, ws)
    torch.cuda.synchronize()
    _assert_same(out, refs)
    # replays: poison the outputs and run unrelated eager work in between
    for rep in range(3):
        _say("batch graph replay", rep)
        for key in ("W", "M", "xi"):
            for t in out[key]:
                t.fill_(float("nan"))
        out["ex"].fill_(float("nan"))
        out["info"].fill_(-7)
        junk = torch.randn(1 << 20, device="cuda:0", dtype=torch.float64)
        junk = (junk * junk).sum()
        torch.cuda.synchronize()
        batch.build_into(phis, out, ws)
        torch.cuda.synchronize()
        _assert_same(out, refs)
    # the oracle on two instances: plain all pairs, and the masked one
    spec0, s0, _, _, _ = systems[0]
    assert O.rel_err(_host(out["W"][0]), O.apply_vx(s0.phi, spec0.cell, spec0.alpha)) < TOL
    spec2, s2, _, _, m2 = systems[2]
    ref2 = O.apply_vx(s2.phi, spec2.cell, spec2.alpha, pair_mask=m2.astype(bool), workers=4)
    assert O.rel_err(_host(out["W"][2]), ref2) < TOL


def test_batch_eager_and_new_pointers(lib, systems):
    import torch
    _say("batch eager branches and re-record on new pointers")
    plans = _plans(lib, systems)
    phis = [_dev(s.phi) for _, s, _, _, _ in systems]
    refs = _separate(lib, plans, systems, phis)
    batch = lib.Batch(plans, [m for *_, m in systems])
    ws = lib.workspace(batch.workspace_bytes())
    out = batch.build(phis, ws=ws, eager=True)
    torch.cuda.synchronize()
    _assert_same(out, refs)
    out1 = batch.build(phis, ws=ws)          # records the graph
    out2 = batch.build(phis, ws=ws)          # new outputs: records again
    torch.cuda.synchronize()
    _assert_same(out1, refs)
    _assert_same(out2, refs)
    # every instance on its own launches instead of the lanes: same bits
    out3 = batch.build(phis, ws=ws, lanes=False)
    out4 = batch.build(phis, ws=ws, eager=True, lanes=False)
    torch.cuda.synchronize()
    _assert_same(out3, refs)
    _assert_same(out4, refs)


def test_batch_singular_instance_reports_its_own_info(lib, systems):
    """A zero orbital in one instance: its info is set, the others are clean."""
    import torch
    _say("batch with one singular instance")
    plans = _plans(lib, systems[:3])
    phis = [_dev(s.phi) for _, s, _, _, _ in systems[:3]]
    bad = phis[1].clone()
    bad[2].zero_()
    phis[1] = bad
    batch = lib.Batch(plans, [m for *_, m in systems[:3]])
    out = batch.build(phis)
    torch.cuda.synchronize()
    info = _host(out["info"])
    assert info[0] == 0 and info[2] == 0
    assert info[1] == 3


@pytest.mark.parametrize("n", [64, 96])
def test_pencil_shapes_change_no_bit(lib, n):
    import torch
    _say("x-pass pencil shapes n=%d" % n)
    spec = synth.SystemSpec("pen", 0.11 * n + 4.0, n, 5, "random", 0, (1.0, 1.4), 0.25, 150 + n)
    s = synth.build_system(spec)
    phi = _dev(s.phi)
    outs = []
    for c in (0, 8, 16, 32):
        if c and n % c:
            continue
        p = lib.Plan(n, (spec.L,) * 3, 5, "fp64", spec.alpha)
        p.set_tiling(16, 0, c)
        outs.append(_host(lib.ace_build(p, phi)["W"]))
    torch.cuda.synchronize()
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])


def test_autotune_cache_and_parity(lib, tmp_path):
    from paper_2110_07670_amd import autotune
    _say("autotune n=32 orbitals=12")
    cache = str(tmp_path / "tune.json")
    e = autotune.tune(32, "fp64", 12, cache_path=cache, reps=1)
    assert e["block"] in (8, 16) and e["chunk"] >= 0 and e["pencils"] in (0, 8, 16, 32)
    assert len(e["tried"]) >= 3 and e["ms"] > 0
    assert autotune.load_cache(cache)[autotune.key(32, "fp64", 12)]["ms"] == e["ms"]
    spec = synth.SystemSpec("tune", 9.0, 32, 12, "random", 0, (1.0, 1.4), 0.25, 333)
    s = synth.build_system(spec)
    p = lib.Plan(32, (spec.L,) * 3, 12, "fp64", spec.alpha)
    shape = autotune.apply(p, "fp64", cache_path=cache, tune_missing=False)
    assert shape == (e["block"], e["chunk"], e["pencils"])
    W = _host(lib.ace_build(p, _dev(s.phi))["W"])
    assert O.rel_err(W, O.apply_vx(s.phi, spec.cell, spec.alpha)) < TOL
