"""Pair screening for the ACE build (the s-MTACE idea: skip orbital pairs whose
exchange contribution is negligible).

Two screens produce the host `pair_mask` that ace_build takes:

* overlap screen (the paper's criterion): keep (i, j) when
  dV sum_r |phi_i phi_j| >= rho_cut, the integrals from ace_overlap_integrals;
* learned screen: a 3-64-64-1 ReLU network predicts log10 of the expected
  |e_ij| of the pair energy e_ij = -alpha (2 - delta_ij) (ij|ji) from the
  minimum-image distance of the two orbitals' Wannier centres and their
  spreads (ace_wannier + ace_mlp_screen run on the GPU); pairs are skipped
  smallest-predicted first while the predicted skipped energy stays within a
  budget.

Both decisions are made by the library (ace_screen_mask, through
_lib.screen_mask), which also falls back to all pairs when the predicted
energy of the skipped pairs exceeds the budget.  The network is trained
here, in numpy, on pair energies and features that the GPU build itself
produces (exx_energy with per-pair output, ace_wannier) for systems drawn by
the seeded generators.  The all-pairs build stays the judge of the screened
result.
"""
from __future__ import annotations

import math
from typing import Dict, List, Sequence

import numpy as np

from . import synth

HIDDEN = 64


# ------------------------------------------------------------------ weights

def weights_to_array(p: Dict[str, np.ndarray]) -> np.ndarray:
    """Flatten into the kernel layout: mean[3] std[3] W1[H][3] b1[H] W2[H][H] b2[H] w3[H] b3."""
    parts = [p["mean"], p["std"], p["W1"].ravel(), p["b1"], p["W2"].ravel(), p["b2"], p["w3"],
             np.array([p["b3"]])]
    return np.concatenate([np.asarray(a, dtype=np.float64).ravel() for a in parts]).astype(np.float32)


def forward(x: np.ndarray, p: Dict[str, np.ndarray]) -> np.ndarray:
    xs = (x - p["mean"]) / p["std"]
    h1 = np.maximum(xs @ p["W1"].T + p["b1"], 0.0)
    h2 = np.maximum(h1 @ p["W2"].T + p["b2"], 0.0)
    return h2 @ p["w3"] + p["b3"]


def train_pair_mlp(X: np.ndarray, y: np.ndarray, hidden: int = HIDDEN, epochs: int = 150,
                   batch: int = 2048, lr: float = 2e-3, seed: int = 0,
                   calibration: str = "sum", upper_quantile: float = 0.95,
                   tails=(0.02, 0.05, 0.1, 0.2, 0.35, 0.5)) -> Dict[str, np.ndarray]:
    """Mean-squared error on log10 |e| with Adam (He-initialised ReLU network),
    then the output bias is calibrated:

    * "sum" (default): the bias gains the smallest c for which, on the
      training pairs, sum 10^(f + c) is at least sum 10^y over every tail of
      smallest predictions (the lowest 2, 5, 10, 20, 35 and 50 % of f): the
      screen skips such a tail and needs its total, which a mean fit of
      log10 |e| underestimates by the scatter (the sum is dominated by the
      pairs that lie above the fit);
    * "upper": the bias gains the `upper_quantile` of the residuals, so the
      prediction bounds log10 |e| from above for that share of pairs (a
      per-pair bound; far more conservative for the sum);
    * None: the mean fit of log10 |e|.
    """
    rng = np.random.default_rng(seed)
    mean = X.mean(axis=0)
    std = X.std(axis=0) + 1e-12
    p = {"mean": mean, "std": std,
         "W1": rng.standard_normal((hidden, 3)) * math.sqrt(2.0 / 3),
         "b1": np.zeros(hidden),
         "W2": rng.standard_normal((hidden, hidden)) * math.sqrt(2.0 / hidden),
         "b2": np.zeros(hidden),
         "w3": rng.standard_normal(hidden) * math.sqrt(1.0 / hidden),
         "b3": float(y.mean())}
    keys = ["W1", "b1", "W2", "b2", "w3", "b3"]
    m = {k: np.zeros_like(np.asarray(p[k], dtype=np.float64)) for k in keys}
    v = {k: np.zeros_like(np.asarray(p[k], dtype=np.float64)) for k in keys}
    b1_, b2_, eps = 0.9, 0.999, 1e-8
    t = 0
    n = X.shape[0]
    Xs = (X - mean) / std
    for ep in range(epochs):
        order = rng.permutation(n)
        step_lr = lr * (0.5 * (1 + math.cos(math.pi * ep / epochs)) + 0.02)
        for s0 in range(0, n, batch):
            idx = order[s0:s0 + batch]
            xb, yb = Xs[idx], y[idx]
            a1 = xb @ p["W1"].T + p["b1"]
            h1 = np.maximum(a1, 0.0)
            a2 = h1 @ p["W2"].T + p["b2"]
            h2 = np.maximum(a2, 0.0)
            out = h2 @ p["w3"] + p["b3"]
            g = 2.0 * (out - yb) / len(idx)
            grads = {"w3": h2.T @ g, "b3": np.sum(g)}
            gh2 = np.outer(g, p["w3"]) * (a2 > 0)
            grads["W2"] = gh2.T @ h1
            grads["b2"] = gh2.sum(axis=0)
            gh1 = (gh2 @ p["W2"]) * (a1 > 0)
            grads["W1"] = gh1.T @ xb
            grads["b1"] = gh1.sum(axis=0)
            t += 1
            for k in keys:
                m[k] = b1_ * m[k] + (1 - b1_) * grads[k]
                v[k] = b2_ * v[k] + (1 - b2_) * grads[k] ** 2
                mh = m[k] / (1 - b1_ ** t)
                vh = v[k] / (1 - b2_ ** t)
                p[k] = p[k] - step_lr * mh / (np.sqrt(vh) + eps)
    p["b3"] = float(p["b3"])
    res = y - forward(X, p)
    if calibration == "sum":
        f = y - res
        c = -np.inf
        for t in tails:
            tail = f <= np.quantile(f, t)
            c = max(c, float(np.log10(np.sum(10.0 ** y[tail]) / np.sum(10.0 ** f[tail]))))
        p["b3"] += c
        p["calibration"] = {"kind": "sum", "shift": c}
    elif calibration == "upper":
        p["b3"] += float(np.quantile(res, upper_quantile))
        p["calibration"] = {"kind": "upper", "quantile": upper_quantile}
    return p


# ------------------------------------------------------------------ features / targets

def pair_features_host(feat: np.ndarray, L: Sequence[float]):
    """(iu, ju, X[n_pairs, 3]) for i <= j from per-orbital (centre xyz, spread)."""
    L = np.asarray(L, dtype=np.float64)
    k = feat.shape[0]
    iu, ju = np.triu_indices(k)
    d = feat[iu, :3] - feat[ju, :3]
    d -= L * np.rint(d / L)
    dist = np.sqrt(np.sum(d * d, axis=1))
    s_i, s_j = feat[iu, 3], feat[ju, 3]
    return iu, ju, np.stack([dist, np.minimum(s_i, s_j), np.maximum(s_i, s_j)], axis=1)


def training_specs() -> List[synth.SystemSpec]:
    """Systems from the random-centre and water generators, several densities and widths."""
    return [
        synth.SystemSpec("train_waterK", 18.6, 64, 128, "waterK", 32, (0.8, 1.6), 0.25, 21),
        synth.SystemSpec("train_random", 20.0, 64, 96, "random", 0, (1.0, 2.0), 0.25, 22),
        synth.SystemSpec("train_water1", 26.0, 64, 144, "water1", 36, (1.0, 2.0), 0.25, 23),
        synth.SystemSpec("train_water1b", 30.0, 80, 192, "water1", 48, (1.0, 2.0), 0.25, 24),
    ]


def training_data(specs=None, device="cuda:0", floor: float = 1e-12):
    """Features and log10 |e_ij| from the GPU method (exx_energy per-pair, ace_wannier)."""
    import torch

    from . import _lib
    Xs, ys = [], []
    for spec in specs or training_specs():
        s = synth.build_system(spec)
        plan = _lib.Plan(spec.n, (spec.L,) * 3, spec.n_orb, "fp64", spec.alpha)
        phi = torch.from_numpy(s.phi).to(device)
        _, pe = _lib.exx_energy(plan, phi, pair_energies=True)
        _, feat = _lib.wannier(plan, phi)
        torch.cuda.synchronize()
        e = pe.cpu().numpy()
        iu, ju, X = pair_features_host(feat.cpu().numpy(), (spec.L,) * 3)
        Xs.append(X)
        ys.append(np.log10(np.maximum(np.abs(e[iu, ju]), floor)))
        del phi, pe, feat, plan
    return np.concatenate(Xs), np.concatenate(ys)


# ------------------------------------------------------------------ masks

def mask_by_budget(pred_log10: np.ndarray, budget: float, safety: float = 2.0) -> np.ndarray:
    """The learned screen's decision on host predictions (the library's
    ace_screen_mask_host): skip the smallest predicted |e_ij| while their
    predicted sum stays <= budget / safety; diagonal pairs always kept."""
    from . import _lib
    mask, _ = _lib.screen_mask_host("mlp", pred=pred_log10, budget=budget, safety=safety)
    return mask.astype(bool)


def overlap_mask(S: np.ndarray, rho_cut: float) -> np.ndarray:
    """The s-MTACE screen on host integrals (the library's ace_screen_mask_host):
    keep (i, j), i <= j, when dV sum |phi_i phi_j| >= rho_cut."""
    from . import _lib
    mask, _ = _lib.screen_mask_host("overlap", S=S, rho_cut=rho_cut, budget=float("inf"))
    return mask.astype(bool)
