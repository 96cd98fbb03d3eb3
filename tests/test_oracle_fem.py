"""Pins of the oracle's finite-element layer against facts fixed by the
mathematics: exact symbolic integration, a textbook closed form, the rigid
body null space, the patch test and tensor-product structure."""
import itertools
import math

import numpy as np
import pytest
import sympy

import inputs
from oracle import fem


def _exact_element(dim, nu, h=1):
    """Element stiffness by exact polynomial integration with sympy."""
    xs = sympy.symbols("x0:%d" % dim)
    nu = sympy.Rational(nu).limit_denominator(1000)
    h = sympy.Integer(h)
    nv = 2 ** dim
    N = []
    for a in range(nv):
        f = sympy.Integer(1)
        for d in range(dim):
            f *= xs[d] / h if (a >> d) & 1 else 1 - xs[d] / h
        N.append(sympy.expand(f))
    grads = [[sympy.diff(Na, x) for x in xs] for Na in N]
    if dim == 2:
        C = sympy.Matrix([[1, nu, 0], [nu, 1, 0], [0, 0, (1 - nu) / 2]]) / (1 - nu ** 2)
        B = sympy.zeros(3, 2 * nv)
        for a in range(nv):
            gx, gy = grads[a]
            B[0, 2 * a], B[1, 2 * a + 1] = gx, gy
            B[2, 2 * a], B[2, 2 * a + 1] = gy, gx
    else:
        lam = nu / ((1 + nu) * (1 - 2 * nu))
        mu = 1 / (2 * (1 + nu))
        C = sympy.zeros(6, 6)
        for i in range(3):
            for j in range(3):
                C[i, j] = lam + (2 * mu if i == j else 0)
        C[3, 3] = C[4, 4] = C[5, 5] = mu
        B = sympy.zeros(6, 3 * nv)
        for a in range(nv):
            gx, gy, gz = grads[a]
            B[0, 3 * a], B[1, 3 * a + 1], B[2, 3 * a + 2] = gx, gy, gz
            B[3, 3 * a], B[3, 3 * a + 1] = gy, gx
            B[4, 3 * a + 1], B[4, 3 * a + 2] = gz, gy
            B[5, 3 * a], B[5, 3 * a + 2] = gz, gx
    integrand = (B.T * C * B).applyfunc(sympy.expand)

    def integrate(expr):
        poly = sympy.Poly(expr, *xs)
        total = sympy.Integer(0)
        for monom, coeff in poly.terms():
            term = coeff
            for p in monom:
                term *= h ** (p + 1) / (p + 1)
            total += term
        return total

    nd = B.shape[1]
    out = np.zeros((nd, nd))
    for i in range(nd):
        for j in range(i, nd):
            v = float(integrate(integrand[i, j]))
            out[i, j] = out[j, i] = v
    return out


def test_simp_closed_form():
    rho = np.array([0.0, 0.5, 1.0, 0.25])
    E = fem.simp_modulus(rho, 1.0, 1e-9, 3.0)
    assert E[0] == 1e-9
    assert E[2] == 1.0
    assert math.isclose(E[1], 1e-9 + 0.125 * (1 - 1e-9), rel_tol=1e-15)
    assert math.isclose(E[3], 1e-9 + 0.015625 * (1 - 1e-9), rel_tol=1e-15)


@pytest.mark.parametrize("nu", [0.3, 0.25])
def test_q1_element_matches_exact_integration(nu):
    K = fem.elasticity_element(2, nu)
    assert np.allclose(K, _exact_element(2, nu), rtol=0, atol=1e-14)


def test_h8_element_matches_exact_integration():
    K = fem.elasticity_element(3, 0.3)
    assert np.allclose(K, _exact_element(3, 0.3), rtol=0, atol=1e-14)


def test_q1_element_matches_textbook_closed_form():
    # Unit-square plane-stress bilinear element in the closed form used by
    # the compact topology-optimisation codes (Andreassen et al. 2011),
    # vertices counter-clockwise from (0, 0).
    nu = 0.3
    k = np.array([1 / 2 - nu / 6, 1 / 8 + nu / 8, -1 / 4 - nu / 12,
                  -1 / 8 + 3 * nu / 8, -1 / 4 + nu / 12, -1 / 8 - nu / 8,
                  nu / 6, 1 / 8 - 3 * nu / 8])
    I = np.array([[1, 2, 3, 4, 5, 6, 7, 8], [2, 1, 8, 7, 6, 5, 4, 3],
                  [3, 8, 1, 6, 7, 4, 5, 2], [4, 7, 6, 1, 8, 3, 2, 5],
                  [5, 6, 7, 8, 1, 2, 3, 4], [6, 5, 4, 3, 2, 1, 8, 7],
                  [7, 4, 5, 2, 3, 8, 1, 6], [8, 3, 2, 5, 4, 7, 6, 1]]) - 1
    KE = k[I] / (1 - nu ** 2)
    ccw = [0, 1, 3, 2]
    idx = [2 * a + c for a in ccw for c in range(2)]
    K = fem.elasticity_element(2, nu)
    assert np.allclose(K[np.ix_(idx, idx)], KE, rtol=0, atol=1e-15)


@pytest.mark.parametrize("dim", [2, 3])
def test_element_null_space_is_rigid_body_modes(dim):
    K = fem.elasticity_element(dim, 0.3, h=1.0)
    assert np.allclose(K, K.T, atol=0)
    w = np.linalg.eigvalsh(K)
    nzero = 3 if dim == 2 else 6
    assert np.all(np.abs(w[:nzero]) < 1e-12)
    assert w[nzero] > 1e-2
    desc = inputs.problem_desc(dim, (1,) * dim, sub_nel=1, overlap=0)
    R = fem.rigid_body_modes(desc)
    assert R.shape[1] == nzero
    assert np.abs(K @ R).max() < 1e-13


def test_h_scaling_of_element_matrices():
    # 2D stiffness is independent of h, 3D scales with h; mass scales h^d
    assert np.allclose(fem.elasticity_element(2, 0.3, 2.0),
                       fem.elasticity_element(2, 0.3, 1.0), atol=1e-14)
    assert np.allclose(fem.elasticity_element(3, 0.3, 2.0),
                       2.0 * fem.elasticity_element(3, 0.3, 1.0), atol=1e-13)
    A1, M1 = fem.heat_element(2, 1.0)
    A2, M2 = fem.heat_element(2, 0.5)
    assert np.allclose(A1, A2) and np.allclose(M2, 0.25 * M1)


@pytest.mark.parametrize("dim", [2, 3])
def test_heat_element_is_tensor_product(dim):
    h = 0.7
    A1 = np.array([[1.0, -1.0], [-1.0, 1.0]]) / h
    M1 = np.array([[2.0, 1.0], [1.0, 2.0]]) * h / 6.0
    # vertex a = ax + 2 ay (+ 4 az): x is the fastest index, i.e. the last
    # Kronecker factor
    if dim == 2:
        A = np.kron(M1, A1) + np.kron(A1, M1)
        M = np.kron(M1, M1)
    else:
        A = (np.kron(np.kron(M1, M1), A1) + np.kron(np.kron(M1, A1), M1)
             + np.kron(np.kron(A1, M1), M1))
        M = np.kron(np.kron(M1, M1), M1)
    Ae, Me = fem.heat_element(dim, h)
    assert np.allclose(Ae, A, atol=1e-15)
    assert np.allclose(Me, M, atol=1e-15)


@pytest.mark.parametrize("dim,nel", [(2, (5, 3)), (3, (3, 2, 2))])
def test_assembled_stiffness_annihilates_rigid_body_modes(dim, nel):
    rng = np.random.default_rng(7)
    desc = inputs.problem_desc(dim, nel, sub_nel=1, overlap=0)
    E = 10.0 ** rng.uniform(-9, 0, inputs.n_elems(desc))
    K = fem.assemble_stiffness(desc, E)
    assert abs(K - K.T).max() < 1e-15
    R = fem.rigid_body_modes(desc)
    assert np.abs(K @ R).max() < 1e-13
    w = np.linalg.eigvalsh(K.toarray())
    assert w[0] > -1e-13
    nzero = 3 if dim == 2 else 6
    assert np.sum(np.abs(w) < 1e-13) == nzero


@pytest.mark.parametrize("dim,nel", [(2, (6, 5)), (3, (3, 3, 4))])
def test_patch_test_linear_field(dim, nel):
    # A linear displacement field gives constant stress, hence zero net
    # nodal force at every interior node of a homogeneous mesh.
    desc = inputs.problem_desc(dim, nel, sub_nel=1, overlap=0)
    K = fem.assemble_stiffness(desc, np.full(inputs.n_elems(desc), 3.0))
    X = fem.node_coords(desc)
    rng = np.random.default_rng(3)
    G = rng.standard_normal((dim, dim))
    a = rng.standard_normal(dim)
    u = (X @ G.T + a).ravel()
    y = (K @ u).reshape(-1, dim)
    interior = np.ones(len(X), dtype=bool)
    for d in range(dim):
        interior &= (X[:, d] > 0) & (X[:, d] < nel[d])
    assert np.abs(y[interior]).max() < 1e-12
    assert np.abs(y[~interior]).max() > 1e-3   # boundary tractions exist


def test_element_node_ids_follow_numbering():
    desc = inputs.problem_desc(2, (3, 2), sub_nel=1, overlap=0)
    ids = fem.element_node_ids(desc)
    # element (1, 1) = id 4; its vertices (1,1),(2,1),(1,2),(2,2)
    assert list(ids[4]) == [1 + 4 * 1, 2 + 4 * 1, 1 + 4 * 2, 2 + 4 * 2]
