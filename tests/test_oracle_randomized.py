"""Pins of the oracle's randomized heat eigen setup (Section 3, the
randomized algorithm; Section 4.3 and Table 1, M_EH+Rot;Rand).

* the random numbers: SplitMix64 against its published first outputs;
* the reduced pencil: Ritz values never fall below the exact eigenvalues
  (Poincare separation), equal them when the snapshots span the whole space,
  and the constant function in the snapshot space gives the exact zero
  eigenvalue of a floating neighbourhood;
* the forcings have zero M-mean;
* Table 2 (contrast 1): with 15 snapshots the coarse dimension is the
  paper's 243 and the iteration count lies between the exact setup's and
  the paper's randomized count (the paper's random draws are not known, so
  the count is pinned to that band only; with 10 snapshots one
  neighbourhood's first Ritz value crosses the threshold here and N_c is
  240 against the paper's 243).
"""
import numpy as np
import scipy.linalg as sla

import inputs
import oracle
from oracle import dd


def test_splitmix64_published_outputs():
    # the first two outputs of SplitMix64 seeded with 0
    assert int(dd.splitmix64(np.uint64(0))) == 0xE220A8397B1DCDAF
    assert int(dd.splitmix64(np.uint64(0x9E3779B97F4A7C15))) == 0x6E789E6AA1B965F4
    u = dd.forcing_uniform(3, 5, 2, np.arange(4096))
    assert np.all((u >= -1.0) & (u < 1.0))
    assert abs(u.mean()) < 0.05 and abs(u.var() - 1.0 / 3.0) < 0.03


def _pencil(floating=True, seed=11):
    desc = inputs.problem_desc(2, (32, 32), sub_nel=8, overlap=1, Emin=1e-4)
    rng = np.random.default_rng(seed)
    rho = inputs.threshold(inputs.grf((32, 32), 4, rng), 0.5)
    E = oracle.simp_modulus(inputs._to_element_order(rho), 1.0, 1e-4, 3.0)
    c = (2, 2)
    dn = None if floating else np.array([0])
    _, nbox = dd.neighbourhood(desc, c)
    ids, _ = dd._node_ids_of_box(desc, nbox)
    if not floating:
        dn = ids[:17]                       # the box's first node row
    A, M, kept = dd.heat_pencil(desc, E, c, dn)
    return desc, A, M, np.searchsorted(ids, kept)


def test_ritz_values_bound_the_eigenvalues_from_above():
    for floating in (True, False):
        desc, A, M, pos = _pencil(floating)
        H = dd.coarse_H(desc)
        lam = sla.eigh(A.toarray(), M.toarray(), eigvals_only=True)
        hm = dd.heat_modes_randomized(A, M, 1e9, H, 10, 8, 7, 3, pos)
        r = hm.lam_seen
        assert len(r) == 9
        assert np.all(r >= lam[:9] - 1e-10 * lam[-1])
        # M-orthonormal approximate eigenvectors
        G = hm.vecs.T @ (M @ hm.vecs)
        assert np.allclose(G, np.eye(G.shape[0]), atol=1e-9)
        if floating:
            assert abs(r[0]) <= 1e-10 * lam[-1]     # the constant is in W


def test_full_snapshot_space_gives_the_exact_eigenvalues():
    desc = inputs.problem_desc(2, (8, 8), sub_nel=2, overlap=1, Emin=1e-3)
    rng = np.random.default_rng(2)
    rho = rng.uniform(0.0, 1.0, 64)
    E = oracle.simp_modulus(rho, 1.0, 1e-3, 3.0)
    c = (2, 2)
    A, M, kept = dd.heat_pencil(desc, E, c)
    _, nbox = dd.neighbourhood(desc, c)
    ids, _ = dd._node_ids_of_box(desc, nbox)
    n = A.shape[0]
    hm = dd.heat_modes_randomized(A, M, 1e9, dd.coarse_H(desc), n, n + 4, 1, 0,
                                  np.searchsorted(ids, kept))
    lam = sla.eigh(A.toarray(), M.toarray(), eigvals_only=True)
    assert len(hm.lam_seen) == n
    assert np.allclose(hm.lam_seen, lam, rtol=1e-8, atol=1e-10 * lam[-1])


def test_forcings_have_zero_mass_mean():
    desc, A, M, pos = _pencil(True)
    one = np.ones(A.shape[0])
    w = M @ one
    F = np.stack([dd.forcing_uniform(9, 3, j, pos) for j in range(6)], axis=1)
    F = F - np.outer(one, (w @ F) / (w @ one))
    assert np.all(np.abs(w @ F) <= 1e-12 * np.abs(w) @ np.abs(F))


def test_table2_randomized_rows():
    p = inputs.config_p()
    _, exact, _ = oracle.solve(p.desc, p.rho, p.fixed, p.f, tol=p.tol)
    d15 = dict(p.desc, eig_random=15, eig_seed=1)
    _, r15, _ = oracle.solve(d15, p.rho, p.fixed, p.f, tol=p.tol)
    assert r15.n_coarse == 243                    # Table 2, M_EH+Rot;Rand
    assert exact.iters <= r15.iters <= 25         # paper: 25 with 15 snapshots
    d10 = dict(p.desc, eig_random=10, eig_seed=1)
    _, r10, _ = oracle.solve(d10, p.rho, p.fixed, p.f, tol=p.tol)
    assert 236 <= r10.n_coarse <= 243
    assert exact.iters <= r10.iters <= 24         # paper: 24 with 10 snapshots
