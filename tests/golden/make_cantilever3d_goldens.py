"""Write the oracle's reference values for the 96 x 48 x 48 cantilever.

    python tests/golden/make_cantilever3d_goldens.py

Calls only ``oracle/`` and ``inputs/``.  For the 3D workload (96 x 48 x 48
H8 elements, 698,691 DOFs, S = 6, one overlap layer, kmax 16, Emin 1e-6)
it records, from the plain CPU FP64 implementation of M_EH+Rot:

* per coarse node: the heat modes selected by the eigenvalue threshold
  (Section 4.1), their eigenvalues, the first eigenvalue the threshold
  rejected (or the cap cut), and whether the kmax cap was hit;
* the coarse dimension N_c, the cap hits and the rank the pseudo-inverse
  of K_0 kept;
* the oracle's PCG run (Section 2, Fletcher-Reeves, x0 = 0, relres 1e-8):
  iterations, the Lanczos condition estimate (Section 5), true relative
  residual and compliance f^T u;
* for one seeded r (standard normal on the free DOFs): the coarse
  correction R_0^T K_0^+ R_0 r and M^{-1} r at a seeded sample of DOFs,
  with their max-abs over all free DOFs.

Output: ``cantilever3d_golden.json`` and ``cantilever3d_probe.npz``.  About
half an hour of one CPU core and 20 GB of memory.
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import inputs  # noqa: E402
import oracle  # noqa: E402
from oracle import dd  # noqa: E402

PROBE_SEED = 31
SAMPLE_SEED = 32
NSAMPLE = 16384


def main():
    p = inputs.config(2, precision=0)
    t0 = time.perf_counter()
    h = dd.build_preconditioner(p.desc, p.rho, p.fixed)
    t1 = time.perf_counter()
    print(f"setup {t1 - t0:.1f} s", flush=True)
    cs = h.coarse
    H2 = dd.coarse_H(p.desc) ** 2
    lim = p.desc["eig_tau"] / H2
    nodes = []
    for l, c in enumerate(cs.coarse_nodes):
        lam = np.asarray(cs.eigvals[l][0])
        seen = np.asarray(cs.lam_seen[l][0])
        rejected = seen[len(lam):]
        nodes.append({
            "node": [int(v) for v in c],
            "n_modes": int(cs.n_modes[l, 0]),
            "eigvals": [float(v) for v in lam],
            "first_rejected": float(rejected[0]) if len(rejected) else None,
            "cap_hit": bool(np.sum(seen < lim) > p.desc["eig_kmax"]),
        })
    r = inputs.probe_vector(p.fixed, PROBE_SEED)
    zc = np.zeros(len(p.fixed))
    zc[h.free] = h.M.coarse(r[h.free])
    zp = np.zeros(len(p.fixed))
    zp[h.free] = h.M(r[h.free])
    free = np.nonzero(p.fixed == 0)[0]
    idx = np.sort(np.random.default_rng(SAMPLE_SEED).choice(free, size=NSAMPLE, replace=False))
    t2 = time.perf_counter()
    u, info, _ = oracle.solve(p.desc, p.rho, p.fixed, p.f, tol=1e-8, hierarchy=h)
    t3 = time.perf_counter()
    print(f"pcg {t3 - t2:.1f} s: iters {info.iters} cond {info.cond_est:.5g}", flush=True)
    out = {
        "source": "oracle/ (CPU FP64 M_EH+Rot) on inputs.config(2); written by "
                  "tests/golden/make_cantilever3d_goldens.py",
        "workload": "cantilever3d_96x48x48",
        "Emin": p.desc["Emin"], "kmax": p.desc["eig_kmax"], "tau": p.desc["eig_tau"],
        "probe_seed": PROBE_SEED, "sample_seed": SAMPLE_SEED,
        "n_coarse": int(cs.Phi.shape[1]),
        "cap_hits": int(cs.cap_hits),
        "coarse_rank": int(h.M.K0_rank),
        "nodes": nodes,
        "pcg": {"iters": int(info.iters), "cond": float(info.cond_est),
                "relres_true": float(info.relres_true),
                "compliance": float(info.compliance)},
        "probe": {"coarse_zmax": float(np.abs(zc).max()),
                  "prec_zmax": float(np.abs(zp).max())},
        "seconds": {"setup": t1 - t0, "pcg": t3 - t2},
    }
    with open(os.path.join(HERE, "cantilever3d_golden.json"), "w") as fh:
        json.dump(out, fh, indent=1)
    np.savez_compressed(os.path.join(HERE, "cantilever3d_probe.npz"),
                        idx=idx.astype(np.int64), z_coarse=zc[idx], z_prec=zp[idx])


if __name__ == "__main__":
    main()
