"""SCDM localisation on the GPU against the FP64 oracle, through the C-ABI.

Preselection: the kept point sets must agree except at points whose density
or gradient norm ties the average to rounding (the averages are sums in
different orders).  Pivoted QR: where the two pivot sequences agree the
localised orbitals must match the oracle to 1e-10; every GPU pivot must be a
valid Businger-Golub choice (its residual norm the largest to 1e-10 relative,
checked by replaying the QR with the GPU's pivots).
"""
import sys

import numpy as np
import pytest

from oracle import ace_oracle as O
from oracle import scdm_oracle as SO
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


def _replay_valid(A, order):
    """Replay Householder QR on A (rows x cols) with the given column order;
    at each step the chosen column must have the largest residual norm."""
    A = A.copy()
    k = A.shape[0]
    chosen = np.zeros(A.shape[1], dtype=bool)
    for s in range(k):
        norms = np.sum(A[s:, :] ** 2, axis=0)
        norms[chosen] = -1.0
        j = order[s]
        assert not chosen[j] and norms[j] >= norms.max() * (1 - 1e-10), ("step", s)
        chosen[j] = True
        x = A[s:, j].copy()
        nx = np.sqrt(np.sum(x * x))
        beta = -nx if x[0] >= 0 else nx
        v = x / (x[0] - beta)
        v[0] = 1.0
        tau = (beta - x[0]) / beta
        A[s:, :] -= tau * np.outer(v, v @ A[s:, :])
    return True


def _check_system(lib, spec, s, preselect=True):
    import torch
    plan = lib.Plan(spec.n, (spec.L,) * 3, spec.n_orb, "fp64", spec.alpha)
    phi = _dev(s.phi)
    out = lib.scdm(plan, phi, preselect=preselect)
    torch.cuda.synchronize()
    assert int(out["info"].item()) == 0
    piv = out["pivots"].cpu().numpy().astype(np.int64)
    loc = out["phi_loc"].cpu().numpy()
    flat = s.phi.reshape(spec.n_orb, -1)
    if preselect:
        pts_ref, rho, g = SO.preselect(s.phi, spec.cell)
        pts = out["points"].cpu().numpy().astype(np.int64)
        diff = np.setxor1d(pts, pts_ref)
        r, gg = rho.ravel(), g.ravel()
        for d in diff:   # only ties of the averages may differ
            assert (abs(r[d] - r.mean()) <= 1e-12 * r.mean()
                    or abs(gg[d] - gg.mean()) <= 1e-12 * gg.mean()), d
    else:
        pts = pts_ref = np.arange(spec.n ** 3)
    # pivots: valid choices on the GPU's own point set
    pos = {p: i for i, p in enumerate(pts.tolist())}
    _replay_valid(flat[:, pts], [pos[p] for p in piv.tolist()])
    piv_ref, U_ref, loc_ref = SO.scdm(s.phi, pts_ref)
    if np.array_equal(pts, pts_ref) and np.array_equal(piv, piv_ref):
        assert O.rel_err(loc, loc_ref) < TOL
    else:
        _say("pivot sequences differ at a tie; comparing at the GPU's pivots")
        U = SO.polar_factor(flat[:, piv])
        assert O.rel_err(loc, (U.T @ flat).reshape(loc.shape)) < TOL
    f = loc.reshape(spec.n_orb, -1)
    assert np.abs(s.dV * f @ f.T - np.eye(spec.n_orb)).max() < 1e-11
    return piv, piv_ref


@pytest.mark.parametrize("n,k,seed,L", [(24, 9, 62, 10.2), (24, 6, 61, 9.0), (32, 8, 63, 10.0),
                                        (32, 12, 66, 11.0)])
def test_scdm_small_systems(lib, n, k, seed, L):
    _say("scdm n=%d orbitals=%d" % (n, k))
    spec = synth.SystemSpec("scdm", L, n, k, "random", 0, (1.0, 1.4), 0.25, seed)
    s = synth.build_system(spec)
    piv, piv_ref = _check_system(lib, spec, s)
    assert np.array_equal(piv, piv_ref)


def test_scdm_all_points(lib):
    _say("scdm without preselection n=16 orbitals=6")
    spec = synth.SystemSpec("scdm_all", 7.0, 16, 6, "random", 0, (1.0, 1.4), 0.25, 64)
    s = synth.build_system(spec)
    _check_system(lib, spec, s, preselect=False)


def test_scdm_config1(lib):
    _say("scdm config1")
    spec = synth.config(1)
    _check_system(lib, spec, synth.build_system(spec))


def test_scdm_water32(lib):
    _say("scdm water32 n=96 orbitals=128")
    spec = synth.config(2)
    _check_system(lib, spec, synth.build_system(spec))


def test_scdm_rank_deficient_reports_info(lib):
    import torch
    _say("scdm with a zero orbital")
    spec = synth.SystemSpec("scdm_def", 8.0, 16, 5, "random", 0, (1.0, 1.4), 0.25, 65)
    s = synth.build_system(spec)
    phi = s.phi.copy()
    phi[3] = 0.0
    plan = lib.Plan(spec.n, (spec.L,) * 3, 5, "fp64", spec.alpha)
    out = lib.scdm(plan, _dev(phi), preselect=False)
    torch.cuda.synchronize()
    assert int(out["info"].item()) == 5     # the last step meets a zero residual
