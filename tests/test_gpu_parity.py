"""GPU parity: the HIP ACE build against the FP64 oracle, through the C-ABI.

Tolerance: 1e-10 normwise relative error per array in FP64 (||x - ref|| /
||ref||), |dE| / |E| for energies.  FP32-bulk results are held to stated
bounds instead.
"""
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


def _host(t):
    return t.detach().cpu().numpy()


def _build(lib, spec, phi, precision="fp64", mask=None, block=None, chunk=0):
    plan = lib.Plan(spec.n, (spec.L,) * 3, phi.shape[0], precision, spec.alpha)
    if block is not None:
        plan.set_tiling(block, chunk)
    out = lib.ace_build(plan, _dev(phi), pair_mask=mask)
    import torch
    torch.cuda.synchronize()
    return plan, {k: _host(v) for k, v in out.items()}


@pytest.mark.parametrize("n", [16, 24, 32, 40, 48, 64, 80, 96, 120, 128, 144, 160, 192])
def test_poisson_every_grid_fp64(lib, n):
    """Two orbitals: three pair solves through every kernel shape of this grid."""
    _say("poisson grid", n)
    L = 0.11 * n + 4.0
    spec = synth.SystemSpec("g", L, n, 2, "random", 0, (1.0, 1.4), 0.25, 50 + n)
    s = synth.build_system(spec)
    plan, out = _build(lib, spec, s.phi)
    W_ref = O.apply_vx(s.phi, spec.cell, spec.alpha, workers=8)
    assert O.rel_err(out["W"], W_ref) < TOL


def test_config1_full_parity(lib):
    spec = synth.config(1)
    _say("config1 n=32 orbitals=8")
    s = synth.build_system(spec)
    ref = O.ace_build(s.phi, spec.cell, spec.alpha)
    plan, out = _build(lib, spec, s.phi)
    assert out["info"][0] == 0
    assert O.rel_err(out["W"], ref["W"]) < TOL
    assert O.rel_err(out["M"], ref["M"]) < TOL
    assert O.rel_err(out["xi"], ref["xi"]) < TOL
    assert abs(out["ex"][0] - ref["ex"]) < TOL * abs(ref["ex"])
    # the operator: apply to the orbitals and to random vectors
    import torch
    psi = synth.random_field((5,) + s.phi.shape[1:], 77)
    got = _host(lib.ace_apply(plan, _dev(out["xi"]), _dev(psi)))
    assert O.rel_err(got, O.ace_apply(out["xi"], psi, s.dV)) < TOL
    back = _host(lib.ace_apply(plan, _dev(out["xi"]), _dev(s.phi)))
    assert O.rel_err(back, ref["W"]) < TOL
    ex, pe = lib.exx_energy(plan, _dev(s.phi), pair_energies=True)
    e_ref = O.pair_energies(s.phi, spec.cell, spec.alpha)
    torch.cuda.synchronize()
    assert abs(_host(ex)[0] - ref["ex"]) < TOL * abs(ref["ex"])
    assert O.rel_err(np.triu(_host(pe)), e_ref) < TOL
    ex2, _ = lib.exx_energy(plan, _dev(s.phi))
    assert abs(_host(ex2)[0] - ref["ex"]) < TOL * abs(ref["ex"])


@pytest.mark.parametrize("block,chunk", [(16, 0), (8, 0), (16, 5), (8, 3)])
def test_ragged_tiles_and_chunks(lib, block, chunk):
    """37 orbitals: partial blocks, diagonal and off-diagonal tiles, odd pair counts."""
    _say("ragged n=24 orbitals=37 block", block, "chunk", chunk)
    spec = synth.SystemSpec("r", 12.0, 24, 37, "random", 0, (1.0, 1.4), 0.25, 9)
    s = synth.build_system(spec)
    ref = O.ace_build(s.phi, spec.cell, spec.alpha, workers=8)
    plan, out = _build(lib, spec, s.phi, block=block, chunk=chunk)
    assert out["info"][0] == 0
    assert O.rel_err(out["W"], ref["W"]) < TOL
    assert O.rel_err(out["M"], ref["M"]) < TOL
    assert O.rel_err(out["xi"], ref["xi"]) < TOL
    assert abs(out["ex"][0] - ref["ex"]) < TOL * abs(ref["ex"])


@pytest.mark.parametrize("block", [8, 16])
def test_mask_clustered_tiles(lib, block):
    """45 orbitals, a sparse random mask: the kept pairs are re-blocked into
    clusters, tiles are partial, some rows hold a single pair."""
    _say("mask clusters n=24 orbitals=45 block", block)
    spec = synth.SystemSpec("mc", 13.0, 24, 45, "random", 0, (1.0, 1.4), 0.25, 14)
    s = synth.build_system(spec)
    k = spec.n_orb
    rng = np.random.default_rng(5)
    mask = np.triu(rng.random((k, k)) < 0.3)
    np.fill_diagonal(mask, rng.random(k) < 0.8)
    ref = O.apply_vx(s.phi, spec.cell, spec.alpha, pair_mask=mask, workers=8)
    for four_pass in (False, True):
        plan = lib.Plan(spec.n, (spec.L,) * 3, k, "fp64", spec.alpha)
        plan.set_tiling(block)
        plan.set_schedule(four_pass)
        out = lib.ace_build(plan, _dev(s.phi), pair_mask=mask)
        import torch
        torch.cuda.synchronize()
        assert O.rel_err(_host(out["W"]), ref) < TOL


def test_single_orbital(lib):
    """One doubly occupied orbital: the 1 x 1 tile, E_X = -(11|11) (the paper's
    Eq. (4) with a single pair), against the oracle."""
    _say("single orbital n=24")
    spec = synth.SystemSpec("one", 9.0, 24, 1, "random", 0, (1.0, 1.4), 0.25, 19)
    s = synth.build_system(spec)
    ref = O.ace_build(s.phi, spec.cell, spec.alpha, workers=4)
    for precision, tol in (("fp64", TOL), ("fp32", 1e-6)):
        plan, out = _build(lib, spec, s.phi, precision)
        assert out["info"][0] == 0
        assert O.rel_err(out["W"], ref["W"]) < tol
        assert abs(out["ex"][0] - ref["ex"]) < tol * abs(ref["ex"])


def test_empty_and_diagonal_masks(lib):
    """No kept pair: W = 0 exactly, -M = 0 is not positive definite (info = 1),
    E_x = 0; only the diagonal kept: W against the oracle's masked sum."""
    _say("empty and diagonal-only masks n=24 orbitals=12")
    import torch
    spec = synth.SystemSpec("em", 10.0, 24, 12, "random", 0, (1.0, 1.4), 0.25, 23)
    s = synth.build_system(spec)
    k = spec.n_orb
    plan = lib.Plan(spec.n, (spec.L,) * 3, k, "fp64", spec.alpha)
    empty = np.zeros((k, k), bool)
    out = lib.ace_build(plan, _dev(s.phi), pair_mask=empty)
    torch.cuda.synchronize()
    assert not np.any(_host(out["W"]))
    assert int(_host(out["info"])[0]) == 1
    assert _host(out["ex"])[0] == 0.0
    ex, _ = lib.exx_energy(plan, _dev(s.phi), pair_mask=empty)
    assert _host(ex)[0] == 0.0
    diag = np.eye(k, dtype=bool)
    ref = O.apply_vx(s.phi, spec.cell, spec.alpha, pair_mask=diag, workers=8)
    out = lib.ace_build(plan, _dev(s.phi), pair_mask=diag)
    torch.cuda.synchronize()
    assert O.rel_err(_host(out["W"]), ref) < TOL


def test_mask_parity_and_shard_sum(lib):
    """Screened pairs match the oracle; disjoint masks sum to the full W
    (the group sum over pair subsets that CP groups rely on)."""
    _say("masks n=24 orbitals=20")
    spec = synth.SystemSpec("m", 11.0, 24, 20, "random", 0, (1.0, 1.4), 0.25, 12)
    s = synth.build_system(spec)
    k = spec.n_orb
    rng = np.random.default_rng(3)
    mask = np.triu(rng.random((k, k)) < 0.6)
    ref = O.apply_vx(s.phi, spec.cell, spec.alpha, pair_mask=mask, workers=8)
    import torch
    plan = lib.Plan(spec.n, (spec.L,) * 3, k, "fp64", spec.alpha)
    out = lib.ace_build(plan, _dev(s.phi), pair_mask=mask)
    torch.cuda.synchronize()
    assert O.rel_err(_host(out["W"]), ref) < TOL
    iu = np.argwhere(np.triu(np.ones((k, k), bool)))
    total = np.zeros_like(s.phi)
    for part in range(4):
        m = np.zeros((k, k), bool)
        for (i, j) in iu[part::4]:
            m[i, j] = True
        o = lib.ace_build(plan, _dev(s.phi), pair_mask=m)
        total += _host(o["W"])
    full = _host(lib.ace_build(plan, _dev(s.phi))["W"])
    assert O.rel_err(total, full) < 1e-12
    ex, _ = lib.exx_energy(plan, _dev(s.phi), pair_mask=mask)
    e_ref = O.exchange_energy_parseval(s.phi, spec.cell, spec.alpha, pair_mask=mask)
    assert abs(_host(ex)[0] - e_ref) < TOL * abs(e_ref)


def test_deterministic_bitwise(lib):
    _say("determinism config1")
    spec = synth.config(1)
    s = synth.build_system(spec)
    a = _build(lib, spec, s.phi)[1]
    b = _build(lib, spec, s.phi)[1]
    for key in ("W", "M", "xi", "ex"):
        assert np.array_equal(a[key], b[key]), key


def test_non_positive_overlap_sets_info(lib):
    """-M not positive definite: the failing leading minor is reported, xi untouched.

    A zero orbital gives an exactly zero third pivot; a negative exchange
    fraction makes -M negative definite, failing at the first pivot.
    """
    _say("non-positive M")
    import torch
    spec = synth.small_spec(n=16, n_orb=3, L=8.0, seed=4)
    s = synth.build_system(spec)
    phi = s.phi.copy()
    phi[2] = 0.0
    with pytest.raises(O.OracleError):
        O.ace_build(phi, spec.cell, spec.alpha)
    plan = lib.Plan(spec.n, (spec.L,) * 3, 3, "fp64", spec.alpha)
    out = lib.ace_build(plan, _dev(phi))
    torch.cuda.synchronize()
    assert _host(out["info"])[0] == 3
    neg = lib.Plan(spec.n, (spec.L,) * 3, 3, "fp64", -0.25)
    xi_before = torch.full_like(_dev(s.phi), 7.0)
    W = torch.empty_like(xi_before)
    M = torch.empty((3, 3), dtype=torch.float64, device="cuda:0")
    ex = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    info = torch.zeros(1, dtype=torch.int32, device="cuda:0")
    ws = lib.workspace(neg.workspace_bytes())
    lib.build_into(neg, _dev(s.phi), W, M, xi_before, ex, info, ws)
    torch.cuda.synchronize()
    assert _host(info)[0] == 1
    assert bool((xi_before == 7.0).all())


def test_fp32_bulk_error_bounds(lib):
    """FP32 transforms with FP64 M/Cholesky/energy: errors stated, not 1e-10."""
    spec = synth.config(1)
    _say("fp32 config1")
    s = synth.build_system(spec)
    ref = O.ace_build(s.phi, spec.cell, spec.alpha)
    plan, out = _build(lib, spec, s.phi, precision="fp32")
    assert out["info"][0] == 0
    assert O.rel_err(out["W"], ref["W"]) < 1e-5
    assert O.rel_err(out["M"], ref["M"]) < 1e-5
    assert abs(out["ex"][0] - ref["ex"]) < 1e-5 * abs(ref["ex"])
    for n in (96, 128, 160):
        _say("fp32 poisson grid", n)
        sp = synth.SystemSpec("g", 0.11 * n + 4.0, n, 2, "random", 0, (1.0, 1.4), 0.25, 60 + n)
        sy = synth.build_system(sp)
        _, o = _build(lib, sp, sy.phi, precision="fp32")
        assert O.rel_err(o["W"], O.apply_vx(sy.phi, sp.cell, sp.alpha, workers=8)) < 1e-5
