"""Write FP64-oracle reference values for the large configurations.

Calls only the oracle (and the seeded input generator): E_x as the sum of
all pair energies (forward transforms only), the pair energies themselves
(compressed), and M rows for a few sampled orbitals (each from that
orbital's W row of Eq. (2), ace_oracle.apply_vx_rows); with --full-m, the
whole M = dV Phi^T W from every W row.  The results are committed next to
this script and read by the GPU tests; nothing here touches the GPU.

CONFIG is 1, 2, 3 or 5, or 4.K for instance K of the uneven batch.

Usage: python tests/golden/make_reference.py CONFIG [PROCESSES]
       python tests/golden/make_reference.py --full-m CONFIG [PROCESSES]
       python tests/golden/make_reference.py --refresh-fingerprint CONFIG
"""
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import ace_oracle as O  # noqa: E402
from oracle import pool  # noqa: E402
from paper_2110_07670_amd import synth  # noqa: E402

SAMPLE_ROWS = {"2": [0, 63, 127], "3": [0, 77, 200], "5": [0, 255, 511],
               "4.13": [0, 57, 127]}
_S = {}


def spec_of(cfg):
    """The system of CONFIG: a single config, or 4.K = instance K of the batch."""
    if cfg.startswith("4."):
        return synth.batch_config4()[int(cfg[2:])]
    return synth.config(int(cfg))


def tag_of(cfg):
    return "batch%02d" % int(cfg[2:]) if cfg.startswith("4.") else "config" + cfg


def _init(phi, K, omega, alpha):
    _S.update(phi=phi, K=K, omega=omega, alpha=alpha)


def _pair_e(chunk):
    phi, K, omega, alpha = _S["phi"], _S["K"], _S["omega"], _S["alpha"]
    out = []
    for i, j in chunk:
        c = O.pair_coulomb(phi[i] * phi[j], K, omega)
        out.append((i, j, -alpha * (1.0 if i == j else 2.0) * c))
    return out


def fingerprint(phi):
    """Platform-robust input check: orbital norms and a few sampled values.

    Loewdin's BLAS rounding differs between CPUs, so inputs are compared to a
    tolerance (1e-12 relative) rather than by a byte hash."""
    k = phi.shape[0]
    flat = phi.reshape(k, -1)
    rng = np.random.default_rng(1234)
    idx = rng.integers(0, flat.shape[1], size=8)
    rows = [0, k // 3, k - 1]
    return {"norms": [float(np.linalg.norm(flat[i])) for i in rows],
            "rows": rows, "idx": [int(v) for v in idx],
            "values": [[float(flat[i, j]) for j in idx] for i in rows]}


def fingerprint_matches(phi, fp, tol=1e-12):
    k = phi.shape[0]
    flat = phi.reshape(k, -1)
    for a, i in enumerate(fp["rows"]):
        if abs(np.linalg.norm(flat[i]) - fp["norms"][a]) > tol * fp["norms"][a]:
            return False
        scale = np.abs(flat[i]).max()
        for b, j in enumerate(fp["idx"]):
            if abs(flat[i, j] - fp["values"][a][b]) > tol * scale:
                return False
    return True


def full_m(cfg, procs):
    """M = dV Phi^T W from every oracle W row, written as M_full_<tag>.npz."""
    spec = spec_of(cfg)
    t0 = time.time()
    s = synth.build_system(spec)
    print("generated %s in %.1fs" % (spec.name, time.time() - t0), flush=True)
    W = pool.apply_vx_pool(s.phi, spec.cell, spec.alpha, procs)
    print("all W rows in %.1fs" % (time.time() - t0), flush=True)
    M = O.overlap_matrix(s.phi, W, s.dV)
    np.savez_compressed(os.path.join(HERE, "M_full_%s.npz" % tag_of(cfg)), M=M,
                        ex_trace=np.trace(M))
    print("tr(M) = %.12f  (%.1fs)" % (np.trace(M), time.time() - t0), flush=True)


def main():
    if sys.argv[1] == "--refresh-fingerprint":
        cfg = sys.argv[2]
        path = os.path.join(HERE, "reference_%s.json" % tag_of(cfg))
        rec = json.load(open(path))
        s = synth.build_system(spec_of(cfg))
        rec["phi_fingerprint"] = fingerprint(s.phi)
        json.dump(rec, open(path, "w"))
        return
    if sys.argv[1] == "--full-m":
        cfg = sys.argv[2]
        procs = int(sys.argv[3]) if len(sys.argv) > 3 else (os.cpu_count() or 1)
        return full_m(cfg, procs)
    cfg = sys.argv[1]
    procs = int(sys.argv[2]) if len(sys.argv) > 2 else (os.cpu_count() or 1)
    spec = spec_of(cfg)
    t0 = time.time()
    s = synth.build_system(spec)
    print("generated %s in %.1fs" % (spec.name, time.time() - t0), flush=True)
    K = O.coulomb_kernel(s.phi.shape[1:], spec.cell)
    omega = O.cell_volume(spec.cell)
    k = spec.n_orb
    pairs = [(i, j) for i in range(k) for j in range(i, k)]
    chunks = [pairs[c::procs * 8] for c in range(procs * 8)]
    ctx = mp.get_context("fork")
    e = np.zeros((k, k))
    with ctx.Pool(procs, initializer=_init, initargs=(s.phi, K, omega, spec.alpha)) as p:
        for res in p.imap_unordered(_pair_e, chunks):
            for i, j, v in res:
                e[i, j] = v
    print("pair energies done in %.1fs" % (time.time() - t0), flush=True)
    rows = pool.apply_vx_rows_pool(s.phi, spec.cell, spec.alpha, SAMPLE_ROWS[cfg], procs)
    print("rows done in %.1fs" % (time.time() - t0), flush=True)
    # M[i][j] = dV phi_j . W_i (M is symmetric)
    flat = s.phi.reshape(k, -1)
    mrows = {str(i): (s.dV * (flat @ rows[i].ravel())).tolist() for i in rows}
    wnorm = {str(i): float(np.linalg.norm(rows[i])) for i in rows}
    out = {"config": cfg, "name": spec.name, "phi_sha256": s.sha256(),
           "phi_fingerprint": fingerprint(s.phi), "subseed": s.subseed,
           "alpha": spec.alpha, "ex": float(e.sum()), "M_rows": mrows, "W_row_norms": wnorm,
           "note": "E_x = sum of oracle pair energies -alpha (2 - delta_ij) (ij|ji); "
                   "M rows from oracle W rows (all pairs)."}
    with open(os.path.join(HERE, "reference_%s.json" % tag_of(cfg)), "w") as f:
        json.dump(out, f)
    np.savez_compressed(os.path.join(HERE, "pair_energies_%s.npz" % tag_of(cfg)),
                        e=np.triu(e).astype(np.float64))
    print("E_x = %.12f  (%.1fs)" % (out["ex"], time.time() - t0), flush=True)


if __name__ == "__main__":
    main()
