"""Pair screening on the GPU: Wannier moments/features, overlap integrals and the
MLP inference kernel against the oracle's plain definitions; then a learned
screen end to end, judged by the all-pairs build."""
import numpy as np
import pytest

from oracle import ace_oracle as O
from paper_2110_07670_amd import screening, synth

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu-case]", *a, flush=True)


@pytest.fixture(scope="module")
def lib():
    import torch
    assert torch.cuda.is_available()
    from paper_2110_07670_amd import _lib
    _lib.load()
    return _lib


@pytest.fixture(scope="module")
def small():
    spec = synth.SystemSpec("scr", 14.0, 40, 20, "water1", 5, (1.0, 2.0), 0.25, 31)
    return spec, synth.build_system(spec)


def _dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")


def test_wannier_matches_oracle(lib, small):
    _say("wannier n=40 orbitals=20")
    spec, s = small
    plan = lib.Plan(spec.n, (spec.L,) * 3, spec.n_orb, "fp64", spec.alpha)
    z, feat = lib.wannier(plan, _dev(s.phi))
    z = z.cpu().numpy()
    feat = feat.cpu().numpy()
    z_ref = O.wannier_moments(s.phi, spec.cell)
    f_ref = O.wannier_features(z_ref, spec.cell)
    zc = z[:, 0::2] + 1j * z[:, 1::2]
    assert np.abs(zc - z_ref).max() < 1e-12
    # centres compared modulo the cell
    d = feat[:, :3] - f_ref[:, :3]
    d -= spec.L * np.rint(d / spec.L)
    assert np.abs(d).max() < 1e-10
    assert np.abs(feat[:, 3] - f_ref[:, 3]).max() < 1e-10


def test_overlap_integrals_match_oracle(lib, small):
    _say("overlap integrals n=40 orbitals=20")
    spec, s = small
    plan = lib.Plan(spec.n, (spec.L,) * 3, spec.n_orb, "fp64", spec.alpha)
    S = lib.overlap_integrals(plan, _dev(s.phi)).cpu().numpy()
    _, S_ref = O.overlap_screen(s.phi, s.dV, 1e-2)
    assert O.rel_err(S, S_ref) < 1e-12


def test_mlp_kernel_matches_oracle_forward(lib, small):
    _say("mlp inference orbitals=20")
    spec, s = small
    rng = np.random.default_rng(5)
    H = screening.HIDDEN
    p = {"mean": np.array([8.0, 1.2, 1.6]), "std": np.array([4.0, 0.3, 0.4]),
         "W1": rng.standard_normal((H, 3)) * 0.6, "b1": rng.standard_normal(H) * 0.1,
         "W2": rng.standard_normal((H, H)) * 0.2, "b2": rng.standard_normal(H) * 0.1,
         "w3": rng.standard_normal(H) * 0.3, "b3": -4.0}
    w = screening.weights_to_array(p)
    assert w.size == lib.mlp_weight_count()
    plan = lib.Plan(spec.n, (spec.L,) * 3, spec.n_orb, "fp64", spec.alpha)
    _, feat = lib.wannier(plan, _dev(s.phi))
    pred = lib.mlp_screen(plan, feat, w).cpu().numpy()
    f_ref = O.wannier_features(O.wannier_moments(s.phi, spec.cell), spec.cell)
    iu, ju, X = O.pair_features(f_ref, spec.cell)
    p32 = {k: (np.asarray(v, dtype=np.float32).astype(np.float64) if k != "b3" else float(np.float32(v)))
           for k, v in p.items()}
    y_ref = O.mlp_forward(X, p32)
    got = pred[iu, ju]
    assert np.abs(got - y_ref).max() < 1e-4 * max(1.0, np.abs(y_ref).max())
    assert np.isnan(pred[1, 0])


def test_learned_screen_end_to_end(lib):
    """Train on the method's own pair energies, screen a held-out system, and
    judge the skipped energy against the all-pairs build."""
    import torch
    _say("learned screen: training")
    specs = screening.training_specs()[:3]
    X, y = screening.training_data(specs)
    # the three inputs leave about one decade of spread in log10 |e| at a given
    # distance (orbital orientation is not among them), so the fit is judged
    # by its mean error and the calibrated upper bound by its coverage
    p_mean = screening.train_pair_mlp(X, y, epochs=60, calibration=None)
    rmse = float(np.sqrt(np.mean((screening.forward(X, p_mean) - y) ** 2)))
    p_up = screening.train_pair_mlp(X, y, epochs=60, calibration="upper")
    under = float(np.mean(screening.forward(X, p_up) < y))
    print("training rmse (log10 |e|): %.3f, upper-bound under-prediction %.3f, samples %d"
          % (rmse, under, len(y)), flush=True)
    assert rmse < 1.3 and under < 0.07
    # the screen itself uses the expected-value calibration
    p = screening.train_pair_mlp(X, y, epochs=60)
    spec = synth.SystemSpec("held_out", 28.0, 64, 160, "water1", 40, (1.0, 2.0), 0.25, 77)
    s = synth.build_system(spec)
    _say("learned screen: held-out n=64 orbitals=160")
    plan = lib.Plan(spec.n, (spec.L,) * 3, spec.n_orb, "fp64", spec.alpha)
    phi = _dev(s.phi)
    budget = 1e-6 * spec.n_atoms
    wts = _dev(screening.weights_to_array(p))
    mask, rep = lib.screen_mask(plan, phi, "mlp", budget=budget, weights=wts)
    # the library's decision equals the plain rule on its own predictions
    _, feat = lib.wannier(plan, phi)
    pred = lib.mlp_screen(plan, feat, wts).cpu().numpy()
    assert np.array_equal(mask, screening.mask_by_budget(pred, budget).astype(np.uint8))
    assert not rep["fallback"] and rep["pairs_kept"] == int(mask.sum())
    full = lib.ace_build(plan, phi)
    scr = lib.ace_build(plan, phi, pair_mask=mask)
    torch.cuda.synchronize()
    e_full, e_scr = float(full["ex"].item()), float(scr["ex"].item())
    kept = int(mask.sum())
    print("pairs kept %d of %d; E_x error %.3e Ha (budget %.3e)"
          % (kept, spec.n_pairs, abs(e_scr - e_full), budget), flush=True)
    assert int(scr["info"].item()) == 0
    assert kept < 0.7 * spec.n_pairs
    assert abs(e_scr - e_full) <= budget
    # the screened W equals the oracle's W over the same pairs (exactness of the
    # masked build itself, independent of the predictor)
    small_mask = mask[:24, :24]
    W_ref = O.apply_vx(s.phi[:24], spec.cell, spec.alpha, pair_mask=small_mask, workers=8)
    plan24 = lib.Plan(spec.n, (spec.L,) * 3, 24, "fp64", spec.alpha)
    W24 = lib.ace_build(plan24, _dev(s.phi[:24]), pair_mask=small_mask)["W"].cpu().numpy()
    assert O.rel_err(W24, W_ref) < 1e-10
