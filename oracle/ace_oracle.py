"""FP64 CPU oracle for the adaptively compressed exchange (ACE) build.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports this module:
only the tests, the smoke check and the benchmark's CPU-baseline leg do.  It
shares no code with the HIP library and imports nothing from the package.

What it computes (arXiv 2110.07670, section "HF Exchange Operator" and
section "ACE Operator"), for Gamma-point real orbitals phi_i sampled on a
periodic n1 x n2 x n3 grid of a cell with volume Omega, dV = Omega / N:

* Eq. (3): v_ij(r) = int phi_i(r') phi_j(r') / |r - r'| dr', evaluated in
  reciprocal space (text after Eq. (4)): rho = phi_i phi_j, rho^ = FFT(rho),
  v^ = K rho^ with K(G) = 4 pi / |G|^2 and K(0) = 0, v = Re IFFT(v^).
* Eq. (2): W_i = alpha * V_X phi_i = -alpha * sum_j v_ij phi_j.  Pairs are
  evaluated once each for i <= j (v_ij = v_ji for real orbitals): both
  W_i -= alpha v_ij phi_j and, for i != j, W_j -= alpha v_ij phi_i.
* ACE form and application: M = dV Phi^T W (symmetric, negative definite),
  -M = L L^T (Cholesky, lower), xi = W L^{-T}; the projectors xi_k play the
  role of the paper's P_k and V_ACE psi = -xi (dV xi^T psi).
* Eq. (4): E_x = alpha * E_X^HF = -alpha sum_{i,j} <phi_i| v_ij |phi_j>
  = tr(M); also the forward-only Parseval form
  (ij|ji) = dV sum_r rho_ij v_ij = (Omega / N^2) sum_m K(m) |rho^_ij(m)|^2.

Readings where the paper is silent (each is listed with the design notes):
alpha multiplies W, M, xi and E_x; closed shell with no factor 1/2 in
Eq. (4); K(0) = 0 with no finite-size correction; full real-space grid box;
numpy FFT conventions (unnormalised forward, 1/N inverse); the Nyquist plane
is kept; the Cholesky factor is lower with a positive diagonal.

Every routine is a plain transcription of a definition; no blocking, packing
or fusion.  Array layout: orbitals are (k, n1, n2, n3) float64 in C order.
"""
from __future__ import annotations

import math
from typing import Optional, Tuple

import numpy as np
import scipy.fft as sfft
import scipy.linalg as sla


class OracleError(RuntimeError):
    """Raised when -M is not positive definite (Cholesky fails)."""


# ----------------------------------------------------------------- grid geometry

def cell_volume(cell: np.ndarray) -> float:
    """Omega = |det(a1, a2, a3)|, lattice vectors as rows (bohr)."""
    return float(abs(np.linalg.det(np.asarray(cell, dtype=np.float64))))


def reciprocal_vectors(cell: np.ndarray) -> np.ndarray:
    """Rows b_a with a_i . b_j = 2 pi delta_ij."""
    A = np.asarray(cell, dtype=np.float64)
    return 2.0 * math.pi * np.linalg.inv(A).T


def integer_frequencies(n: int) -> np.ndarray:
    """Integer m for each FFT index in numpy order: 0..n/2-1, -n/2..-1 (even n)."""
    return np.rint(np.fft.fftfreq(n) * n).astype(np.int64)


def g_squared(shape: Tuple[int, int, int], cell: np.ndarray) -> np.ndarray:
    """|G(m)|^2 with G = m1 b1 + m2 b2 + m3 b3 on the FFT index grid."""
    B = reciprocal_vectors(cell)
    m1, m2, m3 = (integer_frequencies(s) for s in shape)
    M1, M2, M3 = np.meshgrid(m1, m2, m3, indexing="ij")
    G = (M1[..., None] * B[0] + M2[..., None] * B[1] + M3[..., None] * B[2])
    return np.einsum("...a,...a->...", G, G)


def coulomb_kernel(shape: Tuple[int, int, int], cell: np.ndarray) -> np.ndarray:
    """K(m) = 4 pi / |G|^2, K(0) = 0 (Coulomb Green's function in reciprocal space)."""
    g2 = g_squared(shape, cell)
    K = np.zeros_like(g2)
    nz = g2 > 0
    K[nz] = 4.0 * math.pi / g2[nz]
    return K


# ----------------------------------------------------------------- Eq. (3)

def pair_potential(rho: np.ndarray, K: np.ndarray, workers: int = 1) -> np.ndarray:
    """v = Re IFFT(K * FFT(rho)): the periodic Poisson solve of a real pair density."""
    rho_hat = sfft.fftn(rho, workers=workers)
    return sfft.ifftn(K * rho_hat, workers=workers).real


def pair_coulomb(rho: np.ndarray, K: np.ndarray, omega: float, workers: int = 1) -> float:
    """(ij|ji) = (Omega / N^2) sum_m K(m) |rho^(m)|^2 (forward transform only)."""
    N = rho.size
    rho_hat = sfft.fftn(rho, workers=workers)
    return float(omega / (N * N) * np.sum(K * (rho_hat.real ** 2 + rho_hat.imag ** 2)))


def _pairs(n_orb: int, pair_mask: Optional[np.ndarray]):
    for i in range(n_orb):
        for j in range(i, n_orb):
            if pair_mask is None or pair_mask[i, j]:
                yield i, j


# ----------------------------------------------------------------- Eq. (2)

def apply_vx(phi: np.ndarray, cell: np.ndarray, alpha: float,
             pair_mask: Optional[np.ndarray] = None, all_ordered: bool = False,
             workers: int = 1) -> np.ndarray:
    """W = alpha V_X Phi, i.e. W_i = -alpha sum_j v_ij phi_j  (Eq. (2)).

    Default: each unordered pair i <= j once, updating both W_i and W_j.
    ``all_ordered``: every ordered pair (i, j) on its own (N_orb^2 solves),
    updating only W_i; used to pin the pair bookkeeping.
    ``pair_mask``: (n_orb, n_orb) boolean, upper triangle read; a skipped
    pair contributes nothing to either orbital.
    """
    phi = np.asarray(phi, dtype=np.float64)
    n_orb = phi.shape[0]
    K = coulomb_kernel(phi.shape[1:], cell)
    W = np.zeros_like(phi)
    if all_ordered:
        for i in range(n_orb):
            for j in range(n_orb):
                if pair_mask is not None and not pair_mask[min(i, j), max(i, j)]:
                    continue
                v = pair_potential(phi[i] * phi[j], K, workers)
                W[i] -= alpha * v * phi[j]
        return W
    for i, j in _pairs(n_orb, pair_mask):
        v = pair_potential(phi[i] * phi[j], K, workers)
        W[i] -= alpha * v * phi[j]
        if i != j:
            W[j] -= alpha * v * phi[i]
    return W


def apply_vx_rows(phi: np.ndarray, cell: np.ndarray, alpha: float, rows,
                  pair_mask: Optional[np.ndarray] = None, cols=None,
                  workers: int = 1) -> np.ndarray:
    """Selected rows of Eq. (2): W_i = -alpha sum_j v_ij phi_j for i in ``rows``.

    The sum runs over j in ``cols`` (default: every orbital, in increasing
    order), skipping pairs whose upper-triangle ``pair_mask`` entry
    (min(i, j), max(i, j)) is zero.  Summing the results of disjoint ``cols``
    gives the full row, so a row can be split over processes.  For a row i
    the unordered-pair loop of apply_vx adds the same terms in the same
    order (j = 0, 1, ...), so the two agree to rounding.
    """
    phi = np.asarray(phi, dtype=np.float64)
    K = coulomb_kernel(phi.shape[1:], cell)
    js = range(phi.shape[0]) if cols is None else cols
    out = np.zeros((len(rows),) + phi.shape[1:])
    for a, i in enumerate(rows):
        for j in js:
            if pair_mask is not None and not pair_mask[min(i, j), max(i, j)]:
                continue
            v = pair_potential(phi[i] * phi[j], K, workers)
            out[a] -= alpha * v * phi[j]
    return out


# ----------------------------------------------------------------- ACE

def overlap_matrix(phi: np.ndarray, W: np.ndarray, dV: float) -> np.ndarray:
    """M = dV Phi^T W, M[i, j] = dV sum_r phi_i(r) W_j(r)."""
    k = phi.shape[0]
    return dV * (phi.reshape(k, -1) @ W.reshape(W.shape[0], -1).T)


def cholesky_neg(M: np.ndarray) -> np.ndarray:
    """Lower L with positive diagonal and L L^T = -M (lower triangle of -M read)."""
    try:
        return np.linalg.cholesky(-M)
    except np.linalg.LinAlgError as e:
        raise OracleError("-M is not positive definite") from e


def ace_projectors(W: np.ndarray, L: np.ndarray) -> np.ndarray:
    """xi = W L^{-T}: in orbital-major layout xi_k = sum_i (L^{-1})_{k i} W_i."""
    k = W.shape[0]
    Wf = W.reshape(k, -1)
    # Solve L X = W (forward substitution); X = L^{-1} W has rows xi_k.
    X = sla.solve_triangular(L, Wf, lower=True)
    return X.reshape(W.shape)


def ace_apply(xi: np.ndarray, psi: np.ndarray, dV: float) -> np.ndarray:
    """V_ACE psi = -sum_k xi_k <xi_k, psi>, with <f, g> = dV sum_r f g."""
    k = xi.shape[0]
    nv = psi.shape[0]
    X = xi.reshape(k, -1)
    P = psi.reshape(nv, -1)
    C = dV * (X @ P.T)            # (k, nv)
    return (-(C.T @ X)).reshape(psi.shape)


def exchange_energy_trace(M: np.ndarray) -> float:
    """E_x = tr(M) = -alpha sum_ij (ij|ji)  (Eq. (4), alpha included)."""
    return float(np.trace(M))


def pair_energies(phi: np.ndarray, cell: np.ndarray, alpha: float,
                  pair_mask: Optional[np.ndarray] = None, workers: int = 1) -> np.ndarray:
    """e[i, j] (i <= j) = -alpha (2 - delta_ij) (ij|ji): each unordered pair's share of E_x."""
    phi = np.asarray(phi, dtype=np.float64)
    n_orb = phi.shape[0]
    K = coulomb_kernel(phi.shape[1:], cell)
    omega = cell_volume(cell)
    e = np.zeros((n_orb, n_orb))
    for i, j in _pairs(n_orb, pair_mask):
        c = pair_coulomb(phi[i] * phi[j], K, omega, workers)
        e[i, j] = -alpha * (1.0 if i == j else 2.0) * c
    return e


def exchange_energy_parseval(phi: np.ndarray, cell: np.ndarray, alpha: float,
                             pair_mask: Optional[np.ndarray] = None,
                             workers: int = 1) -> float:
    """E_x via forward transforms only: sum of the pair energies."""
    return float(pair_energies(phi, cell, alpha, pair_mask, workers).sum())


# ----------------------------------------------------------------- the whole build

def ace_build(phi: np.ndarray, cell: np.ndarray, alpha: float,
              pair_mask: Optional[np.ndarray] = None, workers: int = 1):
    """W, M, L, xi, E_x for one set of occupied orbitals (the ACE build)."""
    phi = np.asarray(phi, dtype=np.float64)
    N = int(np.prod(phi.shape[1:]))
    dV = cell_volume(cell) / N
    W = apply_vx(phi, cell, alpha, pair_mask, workers=workers)
    M = overlap_matrix(phi, W, dV)
    L = cholesky_neg(M)
    xi = ace_projectors(W, L)
    return {"W": W, "M": M, "L": L, "xi": xi, "ex": exchange_energy_trace(M), "dV": dV}


def orthonormality_defect(phi: np.ndarray, dV: float) -> float:
    """max |dV Phi Phi^T - I| (inputs are the caller's to orthonormalise)."""
    k = phi.shape[0]
    S = dV * (phi.reshape(k, -1) @ phi.reshape(k, -1).T)
    return float(np.abs(S - np.eye(k)).max())


# ----------------------------------------------------------------- screening (s-MTACE)

def overlap_screen(phi: np.ndarray, dV: float, rho_cut: float) -> np.ndarray:
    """Keep pair (i, j) when dV sum_r |phi_i phi_j| >= rho_cut (s-MTACE section).

    Returns the boolean upper-triangle mask and, as a second value, the
    integrals themselves.
    """
    k = phi.shape[0]
    A = np.abs(phi.reshape(k, -1))
    S = dV * (A @ A.T)
    mask = np.triu(S >= rho_cut)
    return mask, S


def rel_err(x: np.ndarray, ref: np.ndarray) -> float:
    """Normwise relative error ||x - ref||_F / ||ref||_F."""
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = np.linalg.norm(ref.ravel())
    return float(np.linalg.norm((x - ref).ravel()) / (den if den > 0 else 1.0))


# ----------------------------------------------------------------- learned screening inputs

def wannier_moments(phi: np.ndarray, cell: np.ndarray) -> np.ndarray:
    """z[i, a] = dV sum_r phi_i(r)^2 exp(2 pi i p_a / n_a): Berry-phase moments of
    each orbital density on the periodic cell (orthorhombic, r_a / L_a = p_a / n_a)."""
    phi = np.asarray(phi, dtype=np.float64)
    k = phi.shape[0]
    shape = phi.shape[1:]
    dV = cell_volume(cell) / float(np.prod(shape))
    z = np.zeros((k, 3), dtype=np.complex128)
    for a in range(3):
        n = shape[a]
        ph = np.exp(2j * math.pi * np.arange(n) / n)
        dens = phi ** 2
        axes = tuple(b + 1 for b in range(3) if b != a)
        prof = dens.sum(axis=axes)          # (k, n_a)
        z[:, a] = dV * (prof @ ph)
    return z


def wannier_features(z: np.ndarray, cell: np.ndarray) -> np.ndarray:
    """(centre_x, centre_y, centre_z, spread) per orbital from the moments:
    centre_a = L_a/(2 pi) arg z_a in [0, L_a), spread^2 = sum_a (L_a/2pi)^2 (-ln|z_a|^2)."""
    L = np.diag(np.asarray(cell, dtype=np.float64))
    scale = L / (2 * math.pi)
    centre = np.mod(scale * np.angle(z), L)
    spread = np.sqrt(np.sum(scale ** 2 * (-np.log(np.abs(z) ** 2)), axis=1))
    return np.concatenate([centre, spread[:, None]], axis=1)


def pair_features(feat: np.ndarray, cell: np.ndarray):
    """For i <= j: (minimum-image centre distance, smaller spread, larger spread)."""
    L = np.diag(np.asarray(cell, dtype=np.float64))
    k = feat.shape[0]
    iu, ju = np.triu_indices(k)
    d = feat[iu, :3] - feat[ju, :3]
    d -= L * np.rint(d / L)
    dist = np.sqrt(np.sum(d * d, axis=1))
    s_i, s_j = feat[iu, 3], feat[ju, 3]
    return iu, ju, np.stack([dist, np.minimum(s_i, s_j), np.maximum(s_i, s_j)], axis=1)


def mlp_forward(x: np.ndarray, params: dict) -> np.ndarray:
    """y = w3 . relu(W2 relu(W1 xs + b1) + b2) + b3 with xs = (x - mean) / std."""
    xs = (np.asarray(x, dtype=np.float64) - params["mean"]) / params["std"]
    h1 = np.maximum(xs @ params["W1"].T + params["b1"], 0.0)
    h2 = np.maximum(h1 @ params["W2"].T + params["b2"], 0.0)
    return h2 @ params["w3"] + params["b3"]
