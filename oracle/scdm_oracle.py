"""FP64 CPU oracle for SCDM localisation with s' grid preselection.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py): imported by the tests only.
It shares no code with the HIP library and imports nothing from the package.

What it computes (arXiv 2110.07670, section "s-MTACE Method" and section
"s'-MTACE Method"), for Gamma-point real orbitals phi_i (rows of Phi, so the
paper's Psi^* is Phi restricted to grid points, an n_orb x m matrix):

* preselection (s' section): keep grid point r when rho(r) > <rho> and
  |grad rho(r)| < <|grad rho|>, the averages taken over all grid points,
  rho = sum_i phi_i^2;
* SCDM (s-MTACE section): a rank-revealing QR factorisation with column
  pivoting of Psi^* restricted to the kept points picks n_orb columns C;
  the selected density-matrix columns Gamma(:, C) = Phi^T Psi^*(:, C) are
  orthonormalised.

Readings where the paper is silent (listed with the design notes):
* the density gradient is taken by second-order central differences on the
  periodic grid, and "grad rho < <grad rho>" compares its Euclidean norm;
* the rank-revealing QR is Businger-Golub column pivoting (at every step the
  remaining column of largest residual norm; the first one on a tie);
* the selected columns are orthonormalised symmetrically (Loewdin): with
  A = Psi^*(:, C) the localised orbitals are U^T Phi with U the orthogonal
  polar factor of A, U = A (A^T A)^{-1/2}.  For orthonormal Phi (dV Phi Phi^T
  = I) this is exactly the Loewdin orthonormalisation of Gamma(:, C).
"""
from __future__ import annotations

from typing import Tuple

import numpy as np


def density(phi: np.ndarray) -> np.ndarray:
    """rho(r) = sum_i phi_i(r)^2, summed over i in order."""
    phi = np.asarray(phi, dtype=np.float64)
    rho = np.zeros(phi.shape[1:])
    for i in range(phi.shape[0]):
        rho = rho + phi[i] * phi[i]
    return rho


def gradient_norm(rho: np.ndarray, cell) -> np.ndarray:
    """|grad rho| by second-order central differences on the periodic grid:
    d_a rho(r) = (rho(r + h_a e_a) - rho(r - h_a e_a)) / (2 h_a), h_a = L_a / n_a."""
    L = np.diag(np.asarray(cell, dtype=np.float64)) if np.ndim(cell) == 2 else np.asarray(cell)
    g2 = np.zeros_like(rho)
    for a in range(3):
        h = L[a] / rho.shape[a]
        d = (np.roll(rho, -1, axis=a) - np.roll(rho, 1, axis=a)) / (2.0 * h)
        g2 = g2 + d * d
    return np.sqrt(g2)


def preselect(phi: np.ndarray, cell) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """(indices of the kept points in C order, rho, |grad rho|)."""
    rho = density(phi)
    g = gradient_norm(rho, cell)
    keep = (rho > rho.mean()) & (g < g.mean())
    return np.flatnonzero(keep.ravel()), rho, g


def qrcp(A: np.ndarray, steps: int):
    """Householder QR with column pivoting of A (rows x cols), `steps` steps.

    Returns (perm, R_diag): perm[s] is the original column chosen at step s
    (the first `steps` entries; the rest is the order left behind), R_diag[s]
    the diagonal of R.  The residual column norms are recomputed at every
    step rather than downdated.
    """
    A = np.array(A, dtype=np.float64, copy=True)
    rows, cols = A.shape
    perm = np.arange(cols)
    rdiag = np.zeros(steps)
    for s in range(steps):
        norms = np.sum(A[s:, s:] ** 2, axis=0)
        p = s + int(np.argmax(norms))        # first maximum on a tie
        if p != s:
            A[:, [s, p]] = A[:, [p, s]]
            perm[[s, p]] = perm[[p, s]]
        x = A[s:, s].copy()
        nx = np.sqrt(np.sum(x * x))
        if nx == 0.0:
            rdiag[s] = 0.0
            continue
        beta = -nx if x[0] >= 0 else nx
        v = x.copy()
        v[0] = x[0] - beta
        tau = (beta - x[0]) / beta
        v = v / v[0]
        # A[s:, s:] <- (I - tau v v^T) A[s:, s:]
        w = v @ A[s:, s:]
        A[s:, s:] -= tau * np.outer(v, w)
        rdiag[s] = A[s, s]
    return perm, rdiag


def polar_factor(A: np.ndarray) -> np.ndarray:
    """Orthogonal polar factor U = A (A^T A)^{-1/2} of a square nonsingular A,
    from the singular value decomposition A = X S Y^T: U = X Y^T (forming
    A^T A would square the condition number)."""
    X, _, Yt = np.linalg.svd(A)
    return X @ Yt


def scdm(phi: np.ndarray, points: np.ndarray):
    """Localised orbitals from the kept points.

    Returns (pivot_points, U, phi_loc): the grid points (flat C-order indices)
    the pivoted QR selects, in selection order; the polar factor U of
    A = Psi^*(:, C); and phi_loc = U^T Phi, row j localised at pivot j.
    """
    phi = np.asarray(phi, dtype=np.float64)
    k = phi.shape[0]
    flat = phi.reshape(k, -1)
    points = np.asarray(points)
    A = flat[:, points]
    perm, _ = qrcp(A, k)
    piv = points[perm[:k]]
    U = polar_factor(flat[:, piv])
    phi_loc = (U.T @ flat).reshape(phi.shape)
    return piv, U, phi_loc
