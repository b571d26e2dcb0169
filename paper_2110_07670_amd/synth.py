"""Seeded synthetic inputs: water-box-shaped Gaussian orbitals on a periodic grid.

This module builds inputs only.  It holds none of the exchange arithmetic
(no pair densities, no Poisson solve, no ACE algebra) and is shared by the
FP64 oracle tests, the GPU tests and the benchmark.

The paper benchmarks liquid water boxes of 32, 64 and 128 molecules
(Table 1: 4 doubly occupied orbitals per molecule, cells of 9.85, 12.41 and
15.64 Angstrom).  No snapshots or Kohn-Sham orbitals exist here, so these
generators stand in: rigid water molecules placed at random in a cubic cell,
four Wannier-like orbital sites per molecule, one or a few periodised
Gaussians per orbital, then Loewdin orthonormalisation under the grid inner
product  <f, g> = dV * sum_r f(r) g(r).

All randomness is drawn from numpy's PCG64 (``numpy.random.default_rng``) in a
fixed order, so a (config, seed) pair always gives the same bytes.
"""
from __future__ import annotations

import dataclasses
import hashlib
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

# Rigid water geometry (bohr, degrees).
OH_BOHR = 1.8088
HOH_DEG = 104.52
# Minimum image O-O distance kept by the rejection sampler (bohr).
OO_MIN_BOHR = 4.5
# Loewdin guard: regenerate with the next sub-seed below this overlap eigenvalue.
LAMBDA_MIN_GUARD = 1e-2
# Image sums are cut where exp(-d^2 / (2 sigma^2)) < 1e-20.
IMAGE_CUT = math.sqrt(2.0 * math.log(1e20))


@dataclasses.dataclass(frozen=True)
class SystemSpec:
    """One synthetic system: a cubic cell of side L on an n^3 grid."""

    name: str
    L: float                 # cubic cell edge (bohr)
    n: int                   # grid points per axis
    n_orb: int               # occupied orbitals
    kind: str                # "random" (centres uniform in cell) | "water1" | "waterK"
    n_mol: int = 0           # molecules for the water kinds
    sigma: Tuple[float, float] = (1.0, 1.5)
    alpha: float = 0.25      # exact-exchange fraction (PBE0)
    seed: int = 1

    @property
    def cell(self) -> np.ndarray:
        return np.eye(3) * self.L

    @property
    def n_pairs(self) -> int:
        return self.n_orb * (self.n_orb + 1) // 2

    @property
    def n_atoms(self) -> int:
        return 3 * self.n_mol


def config(idx: int) -> SystemSpec:
    """The five benchmark shapes (1-based), with the seeds fixed per config."""
    if idx == 1:
        return SystemSpec("gauss8_n32", 10.0, 32, 8, "random", 0, (1.0, 1.5), 0.25, 1)
    if idx == 2:
        return SystemSpec("water32_n96", 18.6, 96, 128, "waterK", 32, (0.8, 1.6), 0.25, 2)
    if idx == 3:
        return SystemSpec("water64_n128", 23.5, 128, 256, "water1", 64, (1.0, 1.5), 0.25, 3)
    if idx == 5:
        return SystemSpec("water128_n160", 37.2, 160, 512, "water1", 128, (1.0, 2.0), 0.25, 5)
    raise ValueError("config %d has no single-system spec (config 4 is a batch)" % idx)


def batch_config4(seed: int = 4, count: int = 16) -> List[SystemSpec]:
    """Sixteen uneven instances: grid from {48,64,80,96}, 32..128 orbitals.

    The cell follows liquid density, about 201.5 bohr^3 per molecule.
    """
    rng = np.random.default_rng(seed)
    grids = rng.choice(np.array([48, 64, 80, 96]), size=count)
    norbs = 4 * rng.integers(8, 33, size=count)
    out = []
    for k in range(count):
        n_orb = int(norbs[k])
        n_mol = n_orb // 4
        L = (201.5 * n_mol) ** (1.0 / 3.0)
        out.append(SystemSpec("batch%02d" % k, L, int(grids[k]), n_orb, "water1",
                              n_mol, (1.0, 1.5), 0.25, 400 + k))
    return out


def small_spec(n: int = 16, n_orb: int = 4, L: float = 8.0, seed: int = 11,
               sigma: Tuple[float, float] = (1.0, 1.4)) -> SystemSpec:
    """A tiny random-centre system for fast tests."""
    return SystemSpec("small_n%d_o%d" % (n, n_orb), L, n, n_orb, "random", 0, sigma, 0.25, seed)


# --------------------------------------------------------------------------- geometry

def _quat_to_rot(q: np.ndarray) -> np.ndarray:
    w, x, y, z = q / np.linalg.norm(q)
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
        [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
        [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)],
    ])


def _min_image(d: np.ndarray, L: float) -> np.ndarray:
    return d - L * np.round(d / L)


def place_oxygens(rng: np.random.Generator, n_mol: int, L: float,
                  dmin: float = OO_MIN_BOHR, max_tries: int = 200000) -> np.ndarray:
    """Random sequential addition of O positions with a minimum-image distance."""
    pos = np.zeros((0, 3))
    tries = 0
    while pos.shape[0] < n_mol:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("could not place %d molecules in L=%g" % (n_mol, L))
        c = rng.uniform(0.0, L, size=3)
        if pos.shape[0]:
            d = np.linalg.norm(_min_image(pos - c, L), axis=1)
            if d.min() < dmin:
                continue
        pos = np.vstack([pos, c])
    return pos


def water_sites(rng: np.random.Generator, n_mol: int, L: float):
    """Atoms (O, H1, H2) and the four orbital sites of every molecule.

    Returns (atoms[n_mol, 3, 3], sites[n_mol, 4, 3]).  Sites: the two bond
    midpoints and two lone-pair points O - 0.5 b +- 0.7 n, with b the unit
    bisector towards the hydrogens and n the unit normal of the molecular plane.
    """
    oxy = place_oxygens(rng, n_mol, L)
    half = math.radians(HOH_DEG) / 2.0
    h1b = np.array([OH_BOHR * math.sin(half), 0.0, OH_BOHR * math.cos(half)])
    h2b = np.array([-OH_BOHR * math.sin(half), 0.0, OH_BOHR * math.cos(half)])
    bis = np.array([0.0, 0.0, 1.0])
    nrm = np.array([0.0, 1.0, 0.0])
    atoms = np.zeros((n_mol, 3, 3))
    sites = np.zeros((n_mol, 4, 3))
    for m in range(n_mol):
        R = _quat_to_rot(rng.standard_normal(4))
        o = oxy[m]
        h1, h2 = o + R @ h1b, o + R @ h2b
        b, nn = R @ bis, R @ nrm
        atoms[m] = [o, h1, h2]
        sites[m] = [o + 0.5 * (h1 - o), o + 0.5 * (h2 - o),
                    o - 0.5 * b + 0.7 * nn, o - 0.5 * b - 0.7 * nn]
    return atoms, sites


# --------------------------------------------------------------------------- orbitals

def periodic_gaussian_1d(n: int, L: float, c: float, sigma: float) -> np.ndarray:
    """sum_t exp(-(x - c - t L)^2 / (2 sigma^2)) on x = L p / n, p = 0..n-1."""
    x = L * np.arange(n) / n
    reach = int(math.ceil(IMAGE_CUT * sigma / L)) + 1
    g = np.zeros(n)
    for t in range(-reach, reach + 1):
        g += np.exp(-((x - c - t * L) ** 2) / (2.0 * sigma * sigma))
    return g


def gaussian_on_grid(n: int, L: float, centre: Sequence[float], sigma: float) -> np.ndarray:
    """Periodised isotropic Gaussian (unnormalised) on an n^3 grid of a cubic cell."""
    gx = periodic_gaussian_1d(n, L, centre[0], sigma)
    gy = periodic_gaussian_1d(n, L, centre[1], sigma)
    gz = periodic_gaussian_1d(n, L, centre[2], sigma)
    return gx[:, None, None] * gy[None, :, None] * gz[None, None, :]


def loewdin(phi: np.ndarray, dV: float) -> Tuple[np.ndarray, float]:
    """Phi <- Phi S^{-1/2} with S = dV Phi Phi^T; returns (phi, lambda_min(S))."""
    k = phi.shape[0]
    flat = phi.reshape(k, -1)
    S = dV * (flat @ flat.T)
    lam, U = np.linalg.eigh(S)
    if lam.min() <= 0:
        return phi, float(lam.min())
    X = (U / np.sqrt(lam)) @ U.T
    out = (X @ flat).reshape(phi.shape)
    return out, float(lam.min())


@dataclasses.dataclass
class System:
    spec: SystemSpec
    phi: np.ndarray              # (n_orb, n, n, n) float64, orthonormal under dV
    centres: np.ndarray          # (n_orb, 3) primary Gaussian centres
    sigmas: np.ndarray           # (n_orb,) primary widths
    atoms: Optional[np.ndarray]  # (n_mol, 3, 3) or None
    subseed: int
    lambda_min: float

    @property
    def dV(self) -> float:
        return self.spec.L ** 3 / self.spec.n ** 3

    def sha256(self) -> str:
        return hashlib.sha256(np.ascontiguousarray(self.phi).tobytes()).hexdigest()


def _draw(spec: SystemSpec, subseed: int):
    rng = np.random.default_rng([spec.seed, subseed])
    n, L = spec.n, spec.L
    phi = np.zeros((spec.n_orb, n, n, n))
    centres = np.zeros((spec.n_orb, 3))
    sigmas = np.zeros(spec.n_orb)
    atoms = None
    lo, hi = spec.sigma
    if spec.kind == "random":
        for k in range(spec.n_orb):
            c = rng.uniform(0.0, L, size=3)
            s = rng.uniform(lo, hi)
            phi[k] = gaussian_on_grid(n, L, c, s)
            centres[k], sigmas[k] = c, s
    elif spec.kind in ("water1", "waterK"):
        if spec.n_orb != 4 * spec.n_mol:
            raise ValueError("water kinds need 4 orbitals per molecule")
        atoms, sites = water_sites(rng, spec.n_mol, L)
        for m in range(spec.n_mol):
            for s_i in range(4):
                k = 4 * m + s_i
                c = sites[m, s_i] % L
                s = rng.uniform(lo, hi)
                orb = gaussian_on_grid(n, L, c, s)
                if spec.kind == "waterK":
                    n_extra = int(rng.integers(0, 4))
                    picks = rng.permutation(3)[:n_extra]
                    for a in picks:
                        coef = rng.uniform(0.2, 0.6)
                        s2 = rng.uniform(lo, hi)
                        orb += coef * gaussian_on_grid(n, L, atoms[m, a] % L, s2)
                phi[k] = orb
                centres[k], sigmas[k] = c, s
    else:
        raise ValueError("unknown kind %r" % spec.kind)
    return phi, centres, sigmas, atoms


def build_system(spec: SystemSpec, max_subseed: int = 16) -> System:
    """Generate and Loewdin-orthonormalise; bump the sub-seed on a near-singular overlap."""
    dV = spec.L ** 3 / spec.n ** 3
    for sub in range(max_subseed):
        phi, centres, sigmas, atoms = _draw(spec, sub)
        out, lam = loewdin(phi, dV)
        if lam >= LAMBDA_MIN_GUARD:
            return System(spec, np.ascontiguousarray(out), centres, sigmas, atoms, sub, lam)
    raise RuntimeError("overlap stayed near-singular for %s" % spec.name)


def random_orthogonal(k: int, seed: int) -> np.ndarray:
    """A seeded random orthogonal k x k matrix (QR of a Gaussian matrix, sign-fixed)."""
    rng = np.random.default_rng(seed)
    Q, R = np.linalg.qr(rng.standard_normal((k, k)))
    return Q * np.sign(np.diag(R))


def random_field(shape, seed: int) -> np.ndarray:
    """Seeded standard-normal FP64 field, for FFT and apply tests."""
    return np.random.default_rng(seed).standard_normal(shape)
