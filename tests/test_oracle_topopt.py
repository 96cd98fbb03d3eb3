"""Pins of the oracle's design-update pieces (Section 1): the gradient
formula against finite differences of the objective computed by direct
solves, and the optimality-criteria step against its defining properties
and an independent root finder."""
import numpy as np
import pytest
import scipy.optimize as sopt
import scipy.sparse.linalg as spla

import inputs
import oracle
from oracle import topopt


def _tiny(dim=2, seed=0):
    if dim == 2:
        desc = inputs.problem_desc(2, (6, 4), sub_nel=(3, 2), overlap=1, Emin=1e-3)
        f = inputs.point_load(desc, (6, 2), 1, -1.0)
    else:
        desc = inputs.problem_desc(3, (3, 2, 2), sub_nel=(3, 2, 2), overlap=1, Emin=1e-3)
        f = inputs.point_load(desc, (3, 1, 1), 1, -1.0)
    fixed = inputs.clamp_face_mask(desc)
    rng = np.random.default_rng(seed)
    rho = rng.uniform(0.3, 1.0, inputs.n_elems(desc))
    return desc, fixed, f, rho


def _solve(desc, fixed, rho, f):
    E = oracle.simp_modulus(rho, desc["E0"], desc["Emin"], desc["penal"])
    K = oracle.assemble_stiffness(desc, E)
    free = np.nonzero(fixed == 0)[0]
    u = np.zeros(len(f))
    u[free] = spla.spsolve(K[free][:, free].tocsc(), f[free])
    return u


@pytest.mark.parametrize("dim", [2, 3])
def test_compliance_gradient_against_finite_differences(dim):
    desc, fixed, f, rho = _tiny(dim)
    u = _solve(desc, fixed, rho, f)
    g = topopt.compliance_sensitivity(desc, rho, u)
    assert np.all(g <= 0.0)
    h = 1e-6
    for e in range(0, len(rho), max(1, len(rho) // 7)):
        rp, rm = rho.copy(), rho.copy()
        rp[e] += h
        rm[e] -= h
        fd = (f @ _solve(desc, fixed, rp, f) - f @ _solve(desc, fixed, rm, f)) / (2 * h)
        assert abs(g[e] - fd) <= 1e-6 * max(abs(fd), 1e-12 * abs(g).max()), (e, g[e], fd)


def test_adjoint_gradient_against_finite_differences():
    desc, fixed, f, rho = _tiny(2, seed=1)
    out = inputs.point_load(desc, (4, 3), 0, 1.0)        # objective l^T u
    u = _solve(desc, fixed, rho, f)
    lam = _solve(desc, fixed, rho, out)
    g = topopt.compliance_sensitivity(desc, rho, u, lam)
    h = 1e-6
    for e in range(0, len(rho), 3):
        rp, rm = rho.copy(), rho.copy()
        rp[e] += h
        rm[e] -= h
        fd = (out @ _solve(desc, fixed, rp, f) - out @ _solve(desc, fixed, rm, f)) / (2 * h)
        assert abs(g[e] - fd) <= 1e-6 * abs(g).max(), (e, g[e], fd)


def _oc_case(seed=2, n=500):
    rng = np.random.default_rng(seed)
    rho = rng.uniform(0.0, 1.0, n)
    dg = -rng.lognormal(0.0, 2.0, n)
    return rho, dg


def test_oc_meets_volume_and_bounds():
    rho, dg = _oc_case()
    # reachable within the move limit 0.2 from this design: volume 0.31 .. 0.68
    for vf in (0.35, 0.5, 0.65):
        new, lam = topopt.oc_update(rho, dg, vf, move=0.2)
        assert abs(new.sum() - vf * len(rho)) <= 1e-9 * len(rho)
        assert np.all(new >= np.maximum(0.0, rho - 0.2) - 1e-15)
        assert np.all(new <= np.minimum(1.0, rho + 0.2) + 1e-15)
        # strictly inside the bounds the update is rho sqrt(-dg / lam)
        inner = (new > np.maximum(0.0, rho - 0.2) + 1e-12) & (new < np.minimum(1.0, rho + 0.2) - 1e-12)
        assert inner.any()
        assert np.allclose(new[inner], rho[inner] * np.sqrt(-dg[inner] / lam), rtol=1e-12)


def test_oc_multiplier_matches_brent_root():
    rho, dg = _oc_case(seed=5)
    vf = 0.45
    _, lam = topopt.oc_update(rho, dg, vf, move=0.3)
    vol = lambda L: topopt.oc_candidate(rho, dg, np.ones_like(rho), L, 0.3).sum() - vf * len(rho)
    ref = sopt.brentq(vol, 1e-12, 1e12, xtol=1e-300, rtol=1e-14)
    assert abs(lam - ref) <= 1e-10 * ref


def test_oc_fixed_point_of_uniform_sensitivity():
    """B_e the same for every element and the volume already at the target:
    the design does not move and the multiplier is that B."""
    rng = np.random.default_rng(9)
    rho = rng.uniform(0.2, 0.8, 300)
    c = 3.7
    new, lam = topopt.oc_update(rho, -c * np.ones_like(rho), rho.mean(), move=0.2)
    assert np.allclose(new, rho, rtol=0, atol=1e-12)
    assert abs(lam - c) <= 1e-10 * c


def test_oc_out_of_reach_targets_stop_at_the_range_ends():
    rho, dg = _oc_case(seed=3)
    # below the smallest volume the move limit allows: every element at its
    # lower limit; above the largest: every element with a gradient at its
    # upper limit
    new, lam = topopt.oc_update(rho, dg, 0.01, move=0.1)
    assert lam == topopt.LAM_MAX
    assert np.allclose(new, np.maximum(0.0, rho - 0.1), atol=1e-8)
    new, lam = topopt.oc_update(rho, dg, 0.99, move=0.1)
    assert lam == topopt.LAM_MIN
    assert np.allclose(new, np.minimum(1.0, rho + 0.1), atol=1e-12)
