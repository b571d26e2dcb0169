"""The three-pass schedule (inverse z transform fused into the W update) on
full off-diagonal tiles, against the FP64 oracle and against the four-pass
schedule, through the C-ABI.  Tolerance as in the other parity tests: 1e-10
normwise relative in FP64."""
import sys

import numpy as np
import pytest

from oracle import ace_oracle as O
from paper_2110_07670_amd import synth

pytestmark = pytest.mark.gpu
TOL = 1e-10


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


def _host(out):
    import torch
    torch.cuda.synchronize()
    return {k: v.detach().cpu().numpy() for k, v in out.items()}


def _both(lib, spec, phi, precision, block, chunk=0):
    res = []
    for four in (False, True):
        p = lib.Plan(spec.n, (spec.L,) * 3, phi.shape[0], precision, spec.alpha)
        p.set_tiling(block, chunk)
        p.set_schedule(four)
        res.append(_host(lib.ace_build(p, _dev(phi))))
    return res


@pytest.mark.parametrize("n", [16, 24, 32, 40, 48, 64, 80, 96])
def test_three_pass_every_plane_grid_fp64(lib, n):
    """16 orbitals in blocks of 8: one full off-diagonal tile (three passes)
    between two diagonal tiles (four passes)."""
    _say("three-pass grid", n, "orbitals 16 block 8")
    L = 0.11 * n + 5.0
    spec = synth.SystemSpec("t3", L, n, 16, "random", 0, (1.0, 1.4), 0.25, 300 + n)
    s = synth.build_system(spec)
    three, four = _both(lib, spec, s.phi, "fp64", 8)
    ref = O.ace_build(s.phi, spec.cell, spec.alpha, workers=8)
    assert three["info"][0] == 0
    for key in ("W", "M", "xi"):
        assert O.rel_err(three[key], ref[key]) < TOL, key
        assert O.rel_err(three[key], four[key]) < 1e-13, key
    assert abs(three["ex"][0] - ref["ex"]) < TOL * abs(ref["ex"])


def test_three_pass_block16_ragged_chunks(lib):
    """Block 16 at 40 orbitals: full tile (0,1), ragged tiles (0,2), (1,2);
    chunked forward / middle launches."""
    _say("three-pass block 16, 40 orbitals, n=32, chunk 24")
    spec = synth.SystemSpec("t3b", 11.0, 32, 40, "random", 0, (1.0, 1.4), 0.25, 411)
    s = synth.build_system(spec)
    three, four = _both(lib, spec, s.phi, "fp64", 16, chunk=24)
    W_ref = O.apply_vx(s.phi, spec.cell, spec.alpha, workers=8)
    assert O.rel_err(three["W"], W_ref) < TOL
    assert O.rel_err(three["W"], four["W"]) < 1e-13


def test_three_pass_repeatable(lib):
    _say("three-pass bitwise repeatability n=48")
    spec = synth.SystemSpec("t3r", 10.0, 48, 32, "random", 0, (1.0, 1.4), 0.25, 412)
    s = synth.build_system(spec)
    p = lib.Plan(spec.n, (spec.L,) * 3, 32, "fp64", spec.alpha)
    phi = _dev(s.phi)
    a = _host(lib.ace_build(p, phi))
    b = _host(lib.ace_build(p, phi))
    assert np.array_equal(a["W"], b["W"]) and np.array_equal(a["xi"], b["xi"])


@pytest.mark.parametrize("n", [96, 120, 128, 160])
def test_three_pass_fp32_matches_four_pass(lib, n):
    """FP32 bulk, block 16: the two schedules agree to FP32 rounding; both
    stay within the FP32 bound against the FP64 build (at 120^3 and 128^3 the
    four-pass inverse y/z works slab by slab; at 160^3 the automatic
    schedule is the large-grid one: slab forward pass, row-form inverse z)."""
    _say("three-pass fp32 n=%d orbitals 32" % n)
    spec = synth.SystemSpec("t3f", 0.11 * n + 5.0, n, 32, "random", 0, (1.0, 1.4), 0.25, 500 + n)
    s = synth.build_system(spec)
    three, four = _both(lib, spec, s.phi, "fp32", 16)
    p64 = lib.Plan(spec.n, (spec.L,) * 3, 32, "fp64", spec.alpha)
    ref = _host(lib.ace_build(p64, _dev(s.phi)))
    assert O.rel_err(three["W"], four["W"]) < 1e-6
    assert O.rel_err(three["W"], ref["W"]) < 1e-6
    assert abs(three["ex"][0] - ref["ex"][0]) < 1e-6 * abs(ref["ex"][0])


@pytest.mark.parametrize("n", [16, 24, 32, 40, 48, 64, 80, 96, 120, 128, 144, 160])
def test_three_pass_every_plane_grid_fp32_against_oracle(lib, n):
    """FP32 bulk, 16 orbitals in blocks of 8 (three full tiles), on every
    grid whose FP32 plane fits LDS (the three-pass schedule) and on 144^3 and
    160^3 (slab forward pass, row-form inverse z): W and E_x within the FP32
    bounds of the FP64 oracle.  Covers the inverse-z workgroup order on grids
    that whole 128-byte scratch segments do not tile (24, 40, 120)."""
    _say("three-pass fp32 n=%d orbitals 16 block 8 vs oracle" % n)
    spec = synth.SystemSpec("t3o", 0.11 * n + 5.0, n, 16, "random", 0, (1.0, 1.4), 0.25, 700 + n)
    s = synth.build_system(spec)
    ref = O.ace_build(s.phi, spec.cell, spec.alpha, workers=8)
    p = lib.Plan(spec.n, (spec.L,) * 3, 16, "fp32", spec.alpha)
    p.set_tiling(8)
    out = _host(lib.ace_build(p, _dev(s.phi)))
    assert out["info"][0] == 0
    assert O.rel_err(out["W"], ref["W"]) < 1e-6
    assert abs(out["ex"][0] - ref["ex"]) < 1e-6 * abs(ref["ex"])


@pytest.mark.parametrize("n", [120, 128, 144])
def test_fused_rows_large_grids_fp64(lib, n):
    """Grids whose plane does not fit LDS, full tiles in blocks of 8: 120^3
    and 128^3 take the slab three-pass schedule (forward and middle passes a
    slab of the plane at a time, the plane-form inverse z with W); 144^3
    the large-grid schedule that fuses the inverse z rows with the W update."""
    _say("large-grid fused schedule fp64 n=%d orbitals 16 block 8" % n)
    L = 0.11 * n + 5.0
    spec = synth.SystemSpec("t3L", L, n, 16, "random", 0, (1.0, 1.4), 0.25, 600 + n)
    s = synth.build_system(spec)
    fused, four = _both(lib, spec, s.phi, "fp64", 8)
    W_ref = O.apply_vx(s.phi, spec.cell, spec.alpha, workers=8)
    assert fused["info"][0] == 0
    assert O.rel_err(fused["W"], W_ref) < TOL
    assert O.rel_err(fused["W"], four["W"]) < 1e-13
    assert O.rel_err(fused["xi"], four["xi"]) < 1e-12


@pytest.mark.parametrize("n", [144, 160, 192])
def test_fused_rows_large_grids_fp32(lib, n):
    _say("large-grid fused schedule fp32 n=%d orbitals 32" % n)
    spec = synth.SystemSpec("t3Lf", 0.11 * n + 5.0, n, 32, "random", 0, (1.0, 1.4), 0.25, 700 + n)
    s = synth.build_system(spec)
    fused, four = _both(lib, spec, s.phi, "fp32", 16)
    p64 = lib.Plan(spec.n, (spec.L,) * 3, 32, "fp64", spec.alpha)
    ref = _host(lib.ace_build(p64, _dev(s.phi)))
    assert O.rel_err(fused["W"], four["W"]) < 1e-6
    assert O.rel_err(fused["W"], ref["W"]) < 1e-6
    assert abs(fused["ex"][0] - ref["ex"][0]) < 1e-6 * abs(ref["ex"][0])


@pytest.mark.parametrize("n", [48, 120])
def test_masked_build_fuses_complete_tiles(lib, n):
    """A mask that drops two pairs: the tiles holding them take the masked
    four-pass path, every other (complete) tile the fused one."""
    _say("masked build with complete tiles n=%d orbitals 24 block 8" % n)
    spec = synth.SystemSpec("t3m", 0.11 * n + 5.0, n, 24, "random", 0, (1.0, 1.4), 0.25, 800 + n)
    s = synth.build_system(spec)
    mask = np.ones((24, 24), dtype=np.uint8)
    mask[2, 13] = mask[13, 2] = 0     # tile (0, 1)
    mask[17, 17] = 0                  # tile (2, 2), a diagonal pair
    p = lib.Plan(spec.n, (spec.L,) * 3, 24, "fp64", spec.alpha)
    p.set_tiling(8)
    got = _host(lib.ace_build(p, _dev(s.phi), pair_mask=mask))
    W_ref = O.apply_vx(s.phi, spec.cell, spec.alpha, pair_mask=mask.astype(bool), workers=8)
    assert O.rel_err(got["W"], W_ref) < TOL
