"""GPU parity of the 3D (H8) stiffness product (Section 1.1 discretisation
in three dimensions); the 3D first level and solve are in
test_gpu_3d_solve.py.

The reference is the oracle's assembled K(E) = sum_e E_e P_e^T K^_e P_e
with the trilinear element matrix by 2x2x2 Gauss quadrature, restricted to
the free DOFs: y = K_FF x_F, y = 0 at clamped DOFs.
"""
import numpy as np
import pytest

import inputs
import oracle

from _checks import assert_entrywise

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _msp():
    import paper_2006_13387_amd as msp
    return msp


def _dev(a):
    return torch.tensor(np.asarray(a, dtype=np.float64), device="cuda")


def _case(nel, seed):
    desc = inputs.problem_desc(3, nel, sub_nel=1, overlap=0, Emin=1e-6)
    rng = np.random.default_rng(seed)
    rho = rng.uniform(0.0, 1.0, inputs.n_elems(desc))
    rho[rng.uniform(size=rho.size) < 0.3] = 0.0     # void elements
    fixed = inputs.clamp_face_mask(desc, axis=0, side=0)
    return desc, rho, fixed


@pytest.mark.parametrize("nel,seed", [((7, 5, 4), 11), ((1, 1, 1), 12), ((33, 3, 2), 13)])
def test_matvec3d_parity(nel, seed):
    desc, rho, fixed = _case(nel, seed)
    print(f"[matvec3d] nel={nel} n={len(fixed)}", flush=True)
    msp = _msp()
    s = msp.Solver(desc, fixed)
    s.set_densities(_dev(rho))
    E = oracle.simp_modulus(rho, desc["E0"], desc["Emin"], desc["penal"])
    K = oracle.assemble_stiffness(desc, E)
    x = np.random.default_rng(seed + 100).standard_normal(len(fixed))
    y = s.apply_K(_dev(x)).cpu().numpy()
    xm = np.where(fixed == 1, 0.0, x)
    yref = np.where(fixed == 1, 0.0, K @ xm)
    # same terms in another order: per entry within 1e-13 (|K| |x|)_i
    assert_entrywise(y, yref, 1e-13, abs(K) @ np.abs(xm), "3D K x")
    assert np.all(y[fixed == 1] == 0.0)
    s.close()


def test_matvec3d_unclamped_rigid_motions():
    # no clamps: every rigid-body motion is in the null space of K
    desc, rho, _ = _case((6, 4, 5), 21)
    fixed = np.zeros(inputs.n_dofs(desc), dtype=np.uint8)
    msp = _msp()
    s = msp.Solver(desc, fixed)
    s.set_densities(_dev(rho))
    nn = inputs.n_nodes(desc)
    nx, ny, nz = (v + 1 for v in desc["nel"])
    i, j, k = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    X = np.stack([i.transpose(2, 1, 0).ravel(), j.transpose(2, 1, 0).ravel(),
                  k.transpose(2, 1, 0).ravel()], axis=1).astype(np.float64)
    assert X.shape == (nn, 3)
    rbms = []
    for c in range(3):
        u = np.zeros((nn, 3)); u[:, c] = 1.0; rbms.append(u)
    for a, b in ((0, 1), (1, 2), (2, 0)):
        u = np.zeros((nn, 3)); u[:, a] = -X[:, b]; u[:, b] = X[:, a]; rbms.append(u)
    for u in rbms:
        y = s.apply_K(_dev(u.ravel())).cpu().numpy()
        assert np.linalg.norm(y) <= 1e-11 * np.linalg.norm(u), np.linalg.norm(y)
    s.close()


def test_3d_coarse_space_refusals():
    """The 3D coarse space needs whole-node clamps (its heat pencils remove
    clamped nodes), takes the exact heat eigenpairs and the heat coarse
    space only."""
    msp = _msp()
    desc = inputs.problem_desc(3, (12, 6, 6), sub_nel=6, overlap=1, eig_kmax=6)
    rng = np.random.default_rng(32)
    rho = rng.uniform(0.0, 1.0, inputs.n_elems(desc))
    fixed = inputs.clamp_face_mask(desc, axis=0, side=0)
    part = fixed.copy()
    node = int(np.nonzero(fixed[0::3])[0][0])
    part[3 * node + 1] = 0          # a node clamped in x only
    s = msp.Solver(desc, part)
    s.set_densities(_dev(rho))
    with pytest.raises(Exception, match="all three components"):
        s.setup()
    s.close()
    with pytest.raises(Exception, match="randomized heat setup"):
        s = msp.Solver(dict(desc, eig_random=5), fixed)
        s.set_densities(_dev(rho))
        s.setup()
    with pytest.raises(Exception, match="heat coarse space"):
        msp.Solver(dict(desc, coarse_kind=1), fixed)
