"""The seeded generators: deterministic bytes, orthonormal output, water geometry."""
import math

import numpy as np

from paper_2110_07670_amd import synth


def test_same_seed_same_bytes_and_orthonormal():
    spec = synth.small_spec(n=16, n_orb=6, L=9.0, seed=5)
    a = synth.build_system(spec)
    b = synth.build_system(spec)
    assert a.sha256() == b.sha256()
    k = spec.n_orb
    S = a.dV * a.phi.reshape(k, -1) @ a.phi.reshape(k, -1).T
    assert np.abs(S - np.eye(k)).max() < 1e-13
    c = synth.build_system(synth.small_spec(n=16, n_orb=6, L=9.0, seed=6))
    assert c.sha256() != a.sha256()


def test_water_geometry_and_spacing():
    rng = np.random.default_rng(0)
    atoms, sites = synth.water_sites(rng, 8, 12.0)
    for m in range(8):
        o, h1, h2 = atoms[m]
        assert abs(np.linalg.norm(h1 - o) - synth.OH_BOHR) < 1e-12
        cosang = np.dot(h1 - o, h2 - o) / synth.OH_BOHR ** 2
        assert abs(math.degrees(math.acos(cosang)) - synth.HOH_DEG) < 1e-9
    o = atoms[:, 0]
    d = o[:, None, :] - o[None, :, :]
    d -= 12.0 * np.round(d / 12.0)
    r = np.linalg.norm(d, axis=-1) + np.eye(8) * 100
    assert r.min() >= synth.OO_MIN_BOHR


def test_water_system_small_grid():
    spec = synth.SystemSpec("w2", 9.0, 24, 8, "waterK", 2, (0.8, 1.6), 0.25, 9)
    s = synth.build_system(spec)
    assert s.phi.shape == (8, 24, 24, 24)
    assert s.lambda_min >= synth.LAMBDA_MIN_GUARD


def test_periodic_gaussian_is_periodic():
    g = synth.periodic_gaussian_1d(20, 5.0, 4.9, 1.3)
    h = synth.periodic_gaussian_1d(20, 5.0, 4.9 - 5.0, 1.3)
    assert np.abs(g - h).max() < 1e-15


def test_config_shapes():
    assert synth.config(1).n_pairs == 36
    assert synth.config(2).n_pairs == 8256
    assert synth.config(3).n_pairs == 32896
    b = synth.batch_config4()
    assert len(b) == 16 and all(s.n in (48, 64, 80, 96) for s in b)
    assert all(32 <= s.n_orb <= 128 and s.n_orb % 4 == 0 for s in b)
