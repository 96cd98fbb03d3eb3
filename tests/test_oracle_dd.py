"""Pins of the oracle's domain-decomposition layer: subdomain geometry,
partition of unity, heat eigenproblems against closed forms and a second
eigensolver, the automatic threshold on homogeneous material (including the
coarse dimension 243 that the paper prints), coarse projector identities and
symmetry of the preconditioner."""
import numpy as np
import pytest
import scipy.linalg as sla

import inputs
from oracle import dd, fem


def _mu_1d(N, h, kind):
    """Eigenvalues of the uniform linear-element pencil on N elements:
    (6/h^2)(1 - cos t)/(2 + cos t) with t = k pi/N (Neumann-Neumann, k=0..N),
    t = (k + 1/2) pi/N (Dirichlet-Neumann, k=0..N-1), t = k pi/N
    (Dirichlet-Dirichlet, k=1..N-1)."""
    if kind == "NN":
        t = np.arange(N + 1) * np.pi / N
    elif kind == "DN":
        t = (np.arange(N) + 0.5) * np.pi / N
    else:
        t = np.arange(1, N) * np.pi / N
    return 6.0 / h ** 2 * (1 - np.cos(t)) / (2 + np.cos(t))


def test_subdomain_sizes_and_cover_config0():
    p = inputs.config(0)
    boxes = dd.subdomain_node_boxes(p.desc, p.fixed)
    assert len(boxes) == 8
    idx = dd.subdomain_free_indices(p.desc, p.fixed, boxes)
    sizes = [len(i) for i in idx]
    assert max(sizes) == 684      # 19 x 18 nodes, 2 DOFs each
    # interior block (1, 0): x nodes 15..33, y nodes 0..17
    assert boxes[1] == ((15, 33), (0, 17))


def test_subdomain_sizes_config1_geometry():
    desc = inputs.problem_desc(2, (512, 256), sub_nel=32, overlap=2)
    fixed = inputs.clamp_face_mask(desc)
    boxes = dd.subdomain_node_boxes(desc, fixed)
    assert len(boxes) == 128
    widths = {(b[0][1] - b[0][0] + 1, b[1][1] - b[1][0] + 1) for b in boxes}
    assert (35, 35) in widths and max(max(w) for w in widths) == 35


def test_vertex_mode_skips_clamped_coarse_nodes():
    p = inputs.config_p()
    boxes = dd.subdomain_node_boxes(p.desc, p.fixed)
    assert len(boxes) == 81
    idx = dd.subdomain_free_indices(p.desc, p.fixed, boxes)
    assert len(idx[0]) == 2 * 19 * 19


@pytest.mark.parametrize("dim,nel,S", [(2, (8, 6), (4, 3)), (3, (4, 4, 2), (2, 2, 1))])
def test_partition_of_unity(dim, nel, S):
    desc = inputs.problem_desc(dim, nel, sub_nel=S, overlap=0)
    X = np.rint(fem.node_coords(desc)).astype(int)
    total = np.zeros(len(X))
    for c in dd.coarse_node_grid(desc):
        total += dd.partition_of_unity(desc, c, [X[:, d] for d in range(dim)])
    assert np.allclose(total, 1.0, atol=1e-15)


def test_heat_pencil_homogeneous_neumann_spectrum():
    # interior omega of a 4x4-block mesh: (2S) x (2S) elements, Neumann all
    # round; spectrum = all sums of the 1D Neumann pencil eigenvalues
    S = 6
    desc = inputs.problem_desc(2, (4 * S, 4 * S), sub_nel=S, overlap=0)
    E = np.ones(inputs.n_elems(desc))
    A, M, ids = dd.heat_pencil(desc, E, (2, 2))
    w = sla.eigh(A.toarray(), M.toarray(), eigvals_only=True)
    mu = _mu_1d(2 * S, 1.0, "NN")
    ref = np.sort((mu[:, None] + mu[None, :]).ravel())
    assert np.allclose(w, ref, rtol=1e-10, atol=1e-12)
    assert abs(w[0]) < 1e-12


def test_heat_pencil_dirichlet_side_spectrum():
    # omega of coarse node (1, 1) on a mesh clamped on x = 0: 2S x 2S
    # elements, Dirichlet on the x = 0 side only
    S = 5
    desc = inputs.problem_desc(2, (4 * S, 2 * S), sub_nel=S, overlap=0)
    fixed = inputs.clamp_face_mask(desc)
    E = np.ones(inputs.n_elems(desc))
    node_ids = np.nonzero(fixed[0::2])[0]
    A, M, ids = dd.heat_pencil(desc, E, (1, 1), node_ids)
    w = sla.eigh(A.toarray(), M.toarray(), eigvals_only=True)
    mux = _mu_1d(2 * S, 1.0, "DN")
    muy = _mu_1d(2 * S, 1.0, "NN")
    ref = np.sort((mux[:, None] + muy[None, :]).ravel())
    assert np.allclose(w, ref, rtol=1e-10, atol=1e-12)
    # the lowest eigenvalue of the continuous problem: (pi / 4H)^2
    assert abs(w[0] * (S ** 2) - (np.pi / 4) ** 2) < 0.01


def test_heat_pencil_floating_constant_mode_heterogeneous():
    rng = np.random.default_rng(5)
    desc = inputs.problem_desc(2, (16, 16), sub_nel=4, overlap=0)
    E = 10.0 ** rng.uniform(-6, 0, inputs.n_elems(desc))
    A, M, ids = dd.heat_pencil(desc, E, (2, 2))
    one = np.ones(A.shape[0])
    assert np.abs(A @ one).max() < 1e-14
    hm = dd.heat_modes(A, M, 2.0, 4.0, 6)
    assert abs(hm.lam[0]) < 1e-12
    v = hm.vecs[:, 0]
    assert np.allclose(v / v[0], 1.0, atol=1e-8)


def test_heat_modes_dense_and_arpack_agree(monkeypatch):
    rng = np.random.default_rng(11)
    desc = inputs.problem_desc(2, (48, 48), sub_nel=12, overlap=0)
    g = inputs.grf((48, 48), 4, rng)
    rho = inputs._to_element_order(inputs.threshold(g, 0.4))
    E = fem.simp_modulus(rho, 1.0, 1e-6, 3.0)
    A, M, ids = dd.heat_pencil(desc, E, (2, 2))
    dense = dd.heat_modes(A, M, 2.0, 12.0, 6)
    monkeypatch.setattr(dd, "DENSE_EIG_MAX", 10)
    arp = dd.heat_modes(A, M, 2.0, 12.0, 6)
    assert len(dense.lam) == len(arp.lam) > 0
    assert np.allclose(dense.lam, arp.lam, rtol=1e-9, atol=1e-14)
    # same spans: M-orthonormal bases with all principal cosines 1
    G = dense.vecs.T @ (M @ arp.vecs)
    s = np.linalg.svd(G, compute_uv=False)
    assert np.allclose(s, 1.0, atol=1e-7)


def test_threshold_homogeneous_counts_config0_and_configP():
    # homogeneous material: one heat mode per coarse node that is not
    # clamped, plus one rotation (2D) -> 3 columns per such node
    p = inputs.config(0)
    E = np.ones(inputs.n_elems(p.desc))
    cs = dd.build_coarse_basis(p.desc, E, p.fixed)
    assert cs.Phi.shape[1] == 36
    assert cs.cap_hits == 0
    pp = inputs.config_p()
    cs = dd.build_coarse_basis(pp.desc, np.ones(10000), pp.fixed)
    assert cs.Phi.shape[1] == 243     # Table 2, M_EH+Rot coarse dimension
    cs0 = dd.build_coarse_basis(pp.desc, np.ones(10000), pp.fixed, rot=0)
    assert cs0.Phi.shape[1] == 162


def test_threshold_eigenvalue_bands_homogeneous():
    # lambda_1 H^2 for the three omega types of the clamped square:
    # one Dirichlet side ~ (pi/4)^2, two sides ~ 2 (pi/4)^2, interior 0,
    # coarse node on the clamped edge: no mode below tau = 2
    pp = inputs.config_p()
    E = np.ones(10000)
    cs = dd.build_coarse_basis(pp.desc, E, pp.fixed)
    H2 = 100.0
    lam = {}
    for c, ev in zip(cs.coarse_nodes, cs.eigvals):
        lam[c] = ev[0] * H2
    assert len(lam[(0, 5)]) == 0
    assert abs(lam[(1, 1)][0] - 2 * (np.pi / 4) ** 2) < 0.02
    assert abs(lam[(1, 5)][0] - (np.pi / 4) ** 2) < 0.02
    assert abs(lam[(5, 5)][0]) < 1e-10


def _small_problem(Emin=1e-4, seed=2):
    rng = np.random.default_rng(seed)
    desc = inputs.problem_desc(2, (24, 16), sub_nel=8, overlap=1, Emin=Emin)
    rho = inputs.threshold(inputs.grf((24, 16), 4, rng), 0.45)
    rho = inputs._to_element_order(inputs.fill_hinges(rho))
    fixed = inputs.clamp_face_mask(desc)
    return desc, rho, fixed


def test_coarse_projector_identities():
    desc, rho, fixed = _small_problem()
    h = dd.build_preconditioner(desc, rho, fixed)
    K = h.K_FF.toarray()
    Phi = h.coarse.Phi[h.free].toarray()
    assert Phi.shape[1] > 0
    P0 = Phi @ h.M.K0_pinv @ Phi.T @ K
    assert np.allclose(P0 @ P0, P0, atol=1e-9 * np.abs(P0).max())
    assert np.allclose(P0 @ Phi, Phi, atol=1e-9 * np.abs(Phi).max())


def test_coarse_pseudo_inverse_handles_dependent_rotations():
    # every coarse node carries a rotation: the rotations sum to zero
    desc = inputs.problem_desc(2, (8, 8), sub_nel=4, overlap=1, Emin=1e-6)
    E = np.ones(64)
    fixed = np.zeros(inputs.n_dofs(desc), np.uint8)
    fixed[:2] = 1      # pin one node so K_FF is positive definite... plus
    fixed[2 * 8] = 1   # one more DOF to remove the rotation null mode
    cs = dd.build_coarse_basis(desc, E, fixed)
    rot_cols = []
    col = 0
    for l in range(len(cs.coarse_nodes)):
        col += int(cs.n_modes[l].sum())
        for k in range(int(cs.n_rot[l])):
            rot_cols.append(col)
            col += 1
    assert len(rot_cols) == 9
    s = np.asarray(cs.Phi[:, rot_cols].sum(axis=1)).ravel()
    assert np.abs(s).max() < 1e-14
    K = fem.assemble_stiffness(desc, E)
    free = np.nonzero(fixed == 0)[0]
    Phi = cs.Phi[free].toarray()
    K0 = Phi.T @ K[free][:, free] @ Phi
    P, rank = dd.coarse_pseudo_inverse(K0)
    assert rank == K0.shape[0] - 1
    assert np.allclose(K0 @ P @ K0, K0, atol=1e-10 * np.abs(K0).max())


def test_preconditioner_is_symmetric_positive_definite():
    desc, rho, fixed = _small_problem()
    h = dd.build_preconditioner(desc, rho, fixed)
    n = h.K_FF.shape[0]
    Minv = np.stack([h.M(e) for e in np.eye(n)], axis=1)
    assert np.allclose(Minv, Minv.T, atol=1e-10 * np.abs(Minv).max())
    assert np.linalg.eigvalsh(0.5 * (Minv + Minv.T))[0] > 0


def test_single_subdomain_level1_is_exact_inverse():
    desc, rho, fixed = _small_problem()
    desc = dict(desc, sub_nel=(24, 16), overlap=0)
    h = dd.build_preconditioner(desc, rho, fixed, level="one")
    rng = np.random.default_rng(0)
    r = rng.standard_normal(h.K_FF.shape[0])
    z = h.M(r)
    assert np.linalg.norm(h.K_FF @ z - r) < 1e-9 * np.linalg.norm(r)
