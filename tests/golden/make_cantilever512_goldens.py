"""Write the oracle's reference values for the 512 x 256 cantilever.

    python tests/golden/make_cantilever512_goldens.py

Calls only ``oracle/`` and ``inputs/``.  For the benchmark workload (the
512 x 256 cantilever, kmax 16) at each contrast Emin in {1e-3, 1e-6, 1e-9}
it records, from the plain CPU FP64 implementation of M_EH+Rot:

* per coarse node: the heat modes selected by the eigenvalue threshold
  (Section 4.1), their eigenvalues, the first eigenvalue the threshold
  rejected (or the cap cut), and whether the kmax cap was hit;
* the coarse dimension N_c and the number of cap hits;
* the oracle's PCG run (Section 2, Fletcher-Reeves, x0 = 0, relres 1e-8):
  iterations, the Lanczos condition estimate (Section 5), true relative
  residual and compliance f^T u;
* the coarse correction z = R_0^T K_0^+ R_0 r for one seeded r (standard
  normal on the free DOFs), at a seeded sample of DOFs, with its max-abs
  and 2-norm over all free DOFs.

Output: ``cantilever512_emin.json`` (scalars, counts, eigenvalues) and
``cantilever512_coarse_probe.npz`` (the sampled coarse correction).
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

EMINS = (1e-3, 1e-6, 1e-9)
PROBE_SEED = 21          # r of the coarse-correction probe
SAMPLE_SEED = 22         # sampled DOFs
NSAMPLE = 16384


def sample_dofs(p):
    free = np.nonzero(p.fixed == 0)[0]
    rng = np.random.default_rng(SAMPLE_SEED)
    return np.sort(rng.choice(free, size=min(NSAMPLE, len(free)), replace=False))


def one_contrast(Emin):
    p = inputs.config(1, Emin=Emin)
    t0 = time.perf_counter()
    h = dd.build_preconditioner(p.desc, p.rho, p.fixed)
    t1 = time.perf_counter()
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
    u, info, _ = oracle.solve(p.desc, p.rho, p.fixed, p.f, tol=1e-8, hierarchy=h)
    t2 = time.perf_counter()
    r = inputs.probe_vector(p.fixed, PROBE_SEED)
    zc = np.zeros(len(p.fixed))
    zc[h.free] = h.M.coarse(r[h.free])
    idx = sample_dofs(p)
    out = {
        "Emin": Emin,
        "n_coarse": int(cs.Phi.shape[1]),
        "cap_hits": int(cs.cap_hits),
        "coarse_rank": int(h.M.K0_rank),
        "nodes": nodes,
        "pcg": {"iters": int(info.iters), "cond": float(info.cond_est),
                "relres_true": float(info.relres_true),
                "compliance": float(info.compliance)},
        "coarse_probe": {"zmax": float(np.abs(zc).max()),
                         "znorm": float(np.linalg.norm(zc))},
        "seconds": {"setup": t1 - t0, "pcg": t2 - t1},
    }
    print(f"Emin={Emin:g}: Nc={out['n_coarse']} cap={out['cap_hits']} "
          f"iters={info.iters} cond={info.cond_est:.4g} "
          f"setup={t1 - t0:.1f}s pcg={t2 - t1:.1f}s", flush=True)
    return out, idx, zc[idx]


def main():
    res = {
        "source": "oracle/ (CPU FP64 M_EH+Rot) on inputs.config(1) at each Emin; "
                  "written by tests/golden/make_cantilever512_goldens.py",
        "workload": "cantilever2d_512x256",
        "kmax": inputs.KMAX_FRAGMENTED,
        "tau": 2.0,
        "probe_seed": PROBE_SEED,
        "sample_seed": SAMPLE_SEED,
        "contrasts": {},
    }
    arrays = {}
    for Emin in EMINS:
        out, idx, zs = one_contrast(Emin)
        key = f"{Emin:.0e}"
        res["contrasts"][key] = out
        arrays["idx"] = idx.astype(np.int64)
        arrays[f"z_{key}"] = zs
    with open(os.path.join(HERE, "cantilever512_emin.json"), "w") as fh:
        json.dump(res, fh, indent=1)
    np.savez_compressed(os.path.join(HERE, "cantilever512_coarse_probe.npz"), **arrays)


if __name__ == "__main__":
    main()
