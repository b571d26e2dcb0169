"""Host-side screening logic: weight layout, the numpy forward pass against the
oracle's definition, budget-based mask selection, MLP training on a known
function."""
import numpy as np

from oracle import ace_oracle as O
from paper_2110_07670_amd import screening


def _params(seed=1):
    rng = np.random.default_rng(seed)
    H = screening.HIDDEN
    return {"mean": rng.standard_normal(3), "std": rng.random(3) + 0.5,
            "W1": rng.standard_normal((H, 3)), "b1": rng.standard_normal(H),
            "W2": rng.standard_normal((H, H)) * 0.1, "b2": rng.standard_normal(H),
            "w3": rng.standard_normal(H), "b3": 0.3}


def test_weight_layout_and_forward():
    p = _params()
    w = screening.weights_to_array(p)
    H = screening.HIDDEN
    assert w.dtype == np.float32
    assert w.size == 6 + 3 * H + H + H * H + H + H + 1
    assert np.allclose(w[:3], p["mean"]) and np.allclose(w[3:6], p["std"])
    assert np.allclose(w[6:6 + 3 * H].reshape(H, 3), p["W1"])
    assert np.isclose(w[-1], p["b3"])
    x = np.random.default_rng(2).standard_normal((50, 3))
    assert np.allclose(screening.forward(x, p), O.mlp_forward(x, p))


def test_pair_features_host_matches_oracle():
    rng = np.random.default_rng(3)
    feat = np.concatenate([rng.random((9, 3)) * 11.0, rng.random((9, 1)) + 1.0], axis=1)
    L = 11.0
    iu, ju, X = screening.pair_features_host(feat, (L, L, L))
    iu2, ju2, X2 = O.pair_features(feat, np.eye(3) * L)
    assert np.array_equal(iu, iu2) and np.array_equal(ju, ju2)
    assert np.allclose(X, X2)


def test_mask_by_budget_skips_smallest_within_budget():
    k = 6
    pred = np.full((k, k), np.nan)
    vals = {}
    rng = np.random.default_rng(4)
    for i in range(k):
        for j in range(i, k):
            pred[i, j] = rng.uniform(-9, -2)
            vals[(i, j)] = 10 ** pred[i, j]
    budget = 1e-6
    m = screening.mask_by_budget(pred, budget, safety=1.0)
    skipped = [v for (i, j), v in vals.items() if not m[i, j]]
    kept_off = [v for (i, j), v in vals.items() if m[i, j] and i != j]
    assert all(m[i, i] for i in range(k))
    assert sum(skipped) <= budget
    if kept_off:
        assert min(kept_off) >= max(skipped, default=0.0)
        assert sum(skipped) + min(kept_off) > budget
    assert not m[np.tril_indices(k, -1)].any()


def test_overlap_mask():
    S = np.array([[1.0, 0.05, 0.001], [0.05, 1.0, 0.2], [0.001, 0.2, 1.0]])
    m = screening.overlap_mask(S, 0.01)
    assert m[0, 1] and m[1, 2] and not m[0, 2] and not m[1, 0]


def test_training_fits_a_smooth_decay():
    rng = np.random.default_rng(6)
    X = np.stack([rng.uniform(0, 15, 3000), rng.uniform(1, 2, 3000), rng.uniform(1, 2, 3000)], 1)
    X[:, 1], X[:, 2] = np.minimum(X[:, 1], X[:, 2]), np.maximum(X[:, 1], X[:, 2])
    y = -1.0 - 0.35 * X[:, 0] ** 2 / (X[:, 1] ** 2 + X[:, 2] ** 2)
    p = screening.train_pair_mlp(X, y, epochs=60, seed=1, upper_quantile=None)
    rmse = float(np.sqrt(np.mean((screening.forward(X, p) - y) ** 2)))
    assert rmse < 0.25 * y.std()
    # calibrated: the output is raised until 95% of the training pairs lie below it
    q = screening.train_pair_mlp(X, y, epochs=60, seed=1, upper_quantile=0.95)
    under = float(np.mean(screening.forward(X, q) < y))
    assert 0.03 < under < 0.07
