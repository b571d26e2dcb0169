"""Pins of the SCDM oracle (pivoted QR, polar factor, density gradient,
preselection) against library routines, closed forms and invariants."""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import scdm_oracle as SO
from paper_2110_07670_amd import synth


def _scaled_random(rows, cols, seed):
    rng = np.random.default_rng(seed)
    # distinct column scales keep the pivot choices far from ties
    return rng.standard_normal((rows, cols)) * rng.uniform(0.2, 3.0, size=cols)


@pytest.mark.parametrize("rows,cols,seed", [(6, 6, 1), (12, 50, 2), (20, 33, 3), (8, 200, 4)])
def test_qrcp_matches_lapack_geqp3(rows, cols, seed):
    A = _scaled_random(rows, cols, seed)
    steps = min(rows, cols)
    perm, rdiag = SO.qrcp(A, steps)
    _, R, P = sla.qr(A, pivoting=True, mode="economic")
    assert np.array_equal(perm[:steps], P[:steps])
    assert np.allclose(np.abs(rdiag), np.abs(np.diag(R)[:steps]), rtol=1e-12, atol=0)


def test_qrcp_properties():
    A = _scaled_random(10, 10, 7)
    perm, rdiag = SO.qrcp(A, 10)
    # a permutation; |R_ss| non-increasing; prod |R_ss| = |det A|
    assert sorted(perm.tolist()) == list(range(10))
    assert np.all(np.diff(np.abs(rdiag)) <= 1e-12)
    assert np.isclose(np.prod(np.abs(rdiag)), abs(np.linalg.det(A)), rtol=1e-11)
    # the first pivot is the column of largest norm
    assert perm[0] == int(np.argmax(np.sum(A * A, axis=0)))


def test_polar_factor_matches_scipy_and_definition():
    A = _scaled_random(9, 9, 11)
    U = SO.polar_factor(A)
    Us, H = sla.polar(A)
    assert np.abs(U - Us).max() < 1e-12
    assert np.abs(U.T @ U - np.eye(9)).max() < 1e-13
    Hm = U.T @ A
    assert np.abs(Hm - Hm.T).max() < 1e-12 and np.linalg.eigvalsh(0.5 * (Hm + Hm.T)).min() > 0


def test_gradient_central_difference_closed_form():
    n, L = (12, 10, 8), np.array([6.0, 5.0, 4.0])
    x = np.arange(n[0]) * L[0] / n[0]
    y = np.arange(n[1]) * L[1] / n[1]
    X, Y, _ = np.meshgrid(x, y, np.arange(n[2]), indexing="ij")
    kx, ky = 2 * np.pi / L[0], 2 * 2 * np.pi / L[1]
    rho = np.sin(kx * X) + 0.3 * np.cos(ky * Y)
    g = SO.gradient_norm(rho, L)
    hx, hy = L[0] / n[0], L[1] / n[1]
    # the central difference of sin/cos is exact: sin(k h)/h times the derivative's shape
    dx = np.cos(kx * X) * np.sin(kx * hx) / hx
    dy = -0.3 * np.sin(ky * Y) * np.sin(ky * hy) / hy
    assert np.abs(g - np.sqrt(dx * dx + dy * dy)).max() < 1e-13


def test_density_sums_to_orbital_count_and_is_rotation_invariant():
    spec = synth.small_spec(n=16, n_orb=5, L=8.0, seed=21)
    s = synth.build_system(spec)
    rho = SO.density(s.phi)
    assert abs(rho.sum() * s.dV - 5.0) < 1e-12
    O = synth.random_orthogonal(5, 3)
    rho2 = SO.density(np.tensordot(O, s.phi, axes=1))
    assert np.abs(rho2 - rho).max() < 1e-13 * rho.max()


def test_preselection_rule_on_a_plane_wave_density():
    """rho = 1 + 0.5 cos(2 pi x / L): mean 1 exactly; kept points are those
    with cos > 0 and |sin| below its grid average (central differences)."""
    n, L = 24, 9.0
    x = np.arange(n) * L / n
    prof = 1.0 + 0.5 * np.cos(2 * np.pi * x / L)
    phi = np.sqrt(np.broadcast_to(prof[:, None, None], (n, n, n)))[None].copy()
    idx, rho, g = SO.preselect(phi, [L, L, L])
    s = np.abs(np.sin(2 * np.pi * x / L))
    keep_x = (np.cos(2 * np.pi * x / L) > 1e-12) & (s < s.mean() - 1e-12)
    expect = np.flatnonzero(np.broadcast_to(keep_x[:, None, None], (n, n, n)).ravel())
    assert np.array_equal(idx, expect)


def test_scdm_orthonormal_same_span_and_rotation_invariant():
    spec = synth.SystemSpec("scdm", 10.0, 24, 6, "random", 0, (1.0, 1.4), 0.25, 41)
    s = synth.build_system(spec)
    pts, _, _ = SO.preselect(s.phi, spec.cell)
    piv, U, loc = SO.scdm(s.phi, pts)
    k = 6
    f = loc.reshape(k, -1)
    assert np.abs(s.dV * f @ f.T - np.eye(k)).max() < 1e-12
    P0 = s.phi.reshape(k, -1)
    # same occupied space: the projections of loc onto Phi reproduce loc
    back = (s.dV * f @ P0.T) @ P0
    assert np.abs(back - f).max() < 1e-12 * np.abs(f).max()
    # rotating the input orbitals changes neither the pivots nor the result
    O = synth.random_orthogonal(k, 9)
    piv2, _, loc2 = SO.scdm(np.tensordot(O, s.phi, axes=1), pts)
    assert np.array_equal(piv, piv2)
    assert np.abs(loc2 - loc).max() < 1e-11 * np.abs(loc).max()


def test_scdm_recovers_separated_gaussians():
    """Orbitals that barely overlap are already local: SCDM returns them (up
    to order and sign), each pivot at the peak of one orbital."""
    n, L, k = 32, 16.0, 4
    centres = np.array([[3.0, 3.0, 3.0], [11.0, 3.5, 4.0], [4.0, 11.0, 12.0], [12.0, 12.0, 10.0]])
    x = np.arange(n) * L / n
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    phi = []
    for c in centres:
        d2 = sum((np.remainder(G - ci + L / 2, L) - L / 2) ** 2 for G, ci in zip((X, Y, Z), c))
        g = np.exp(-d2 / (2 * 0.8 ** 2))
        phi.append(g / np.sqrt(np.sum(g * g) * (L / n) ** 3))
    phi = np.array(phi)
    piv, U, loc = SO.scdm(phi, np.arange(n ** 3))
    flat = phi.reshape(k, -1)
    for j in range(k):
        i = int(np.argmax(np.abs(flat[:, piv[j]])))
        assert np.abs(np.abs(loc[j]) - np.abs(phi[i])).max() < 1e-6
        assert piv[j] == int(np.argmax(flat[i] ** 2))
