"""Host side of bench.py: the pass schedule the library reports and the
algorithmic-byte model built on it (no GPU)."""
import pytest

import bench
from paper_2110_07670_amd import _lib


@pytest.mark.parametrize("n,prec,four,kind,plane", [
    (96, "fp64", False, "three_pass", True),
    (96, "fp64", True, "four_pass", True),
    (128, "fp32", False, "three_pass", True),
    (128, "fp64", False, "three_pass", False),   # slab grid, block 8 by default
    (160, "fp32", False, "rows_fused", False),
    (144, "fp64", False, "rows_fused", False),
])
def test_plan_schedule(n, prec, four, kind, plane):
    p = _lib.Plan(n, (10.0,) * 3, 32, prec, 0.25)
    p.set_schedule(four)
    assert p.schedule() == (kind, plane)


def test_slab_grid_block16_is_not_three_pass():
    p = _lib.Plan(128, (10.0,) * 3, 32, "fp64", 0.25)
    p.set_tiling(16)
    assert p.schedule() == ("rows_fused", False)


def test_tile_plan_counts_every_pair_once():
    for n_orb in (8, 9, 31, 128):
        for block in (8, 16):
            tiles = bench.tile_plan(n_orb, block)
            pairs = sum(bi * (bi + 1) // 2 if diag else bi * bj for bi, bj, diag, _, _ in tiles)
            assert pairs == n_orb * (n_orb + 1) // 2
            # two pairs per transform, a row's odd leftover alone
            for bi, bj, diag, npack, kind in tiles:
                rows = [bi - a for a in range(bi)] if diag else [bj] * bi
                assert npack == sum((r + 1) // 2 for r in rows)
                assert kind == ("three_pass" if (bi, bj) == (block, block) else "four_pass")


def test_headline_bytes_per_point_per_pack():
    """Config 2, FP64, three passes: 16 B written forward, 32 B through the
    middle pass, 16 B read by the inverse-z/W pass, per packed transform and
    point, plus the orbital and W rows once per tile."""
    n_orb, npts, c = 128, 96 ** 3, 16
    tiles = bench.tile_plan(n_orb, 16, "three_pass")
    packs = sum(t[3] for t in tiles)
    orbs = sum(t[0] if t[2] else t[0] + t[1] for t in tiles)
    assert packs == 4160
    assert bench.algorithmic_bytes("yz_fwd", tiles, npts, 8) == (packs * c + orbs * 8) * npts
    assert bench.algorithmic_bytes("x_poisson", tiles, npts, 8) == packs * 2 * c * npts
    assert bench.algorithmic_bytes("yz_inv", tiles, npts, 8) == 0
    assert bench.algorithmic_bytes("w_accumulate", tiles, npts, 8) == (packs * c + orbs * 24) * npts


def test_large_grid_inverse_bytes():
    """Where a plane does not fit: row-fused full tiles read and write the
    grid once in the inverse y lines; four-pass tiles twice (lines, rows)."""
    npts, c = 160 ** 3, 8
    fused = bench.tile_plan(32, 16, "rows_fused")
    four = bench.tile_plan(32, 16, "four_pass")
    packs = sum(t[3] for t in fused)
    assert bench.algorithmic_bytes("yz_inv", fused, npts, 4, plane=False) == packs * 2 * c * npts
    assert bench.algorithmic_bytes("yz_inv", four, npts, 4, plane=False) == packs * 4 * c * npts
    assert bench.algorithmic_bytes("yz_inv", four, npts, 4, plane=True) == packs * 2 * c * npts
