"""GPU parity: every step of the hot path through the C ABI against the CPU
FP64 oracle on the same seeded inputs.

Tolerances (stated here, derived in the design notes):
* K x                   : relative 2-norm 1e-13 (same sums, other order)
* FP64 local solves     : relative 1e-9 at Emin = 1e-3, 1e-6 at 1e-6
                          (two backward-stable solvers; forward error grows
                          with the conditioning of K_i)
* FP32 local solves     : relative 1e-3 (single precision inverse blocks)
* heat eigenvalues      : relative 1e-6 (selected eigenvalues)
* coarse correction     : relative 1e-6 (depends only on the coarse span)
* full solve            : true relative residual <= 1e-8, compliance and
                          displacement relative error <= 1e-6 against a
                          direct solve
"""
import math

import numpy as np
import pytest

import inputs
import oracle
from oracle import dd

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _msp():
    import paper_2006_13387_amd as msp
    msp.load_library()
    return msp


def _dev(a):
    return torch.tensor(np.asarray(a, dtype=np.float64), device="cuda")


def _host(t):
    return t.detach().cpu().numpy()


def _solver(p, **kw):
    msp = _msp()
    d = dict(p.desc, **kw)
    s = msp.Solver(d, p.fixed)
    s.set_densities(_dev(p.rho))
    return s


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(scope="module")
def cfg0():
    p = inputs.config(0)
    h = dd.build_preconditioner(p.desc, p.rho, p.fixed)
    return p, h


def _ragged():
    # 70 x 26 elements: x not a multiple of the 64-node tile, several tiles
    desc = inputs.problem_desc(2, (70, 26), sub_nel=(14, 13), overlap=2,
                               Emin=1e-4, eig_kmax=8)
    rng = np.random.default_rng(77)
    rho = inputs.threshold(inputs.grf((70, 26), 5, rng), 0.5)
    rho = inputs.fill_hinges(rho)
    rho = inputs.force_solid_disk(rho, (70, 13), 3.0)
    rho = inputs.connect_load_path(rho, (70, 13))
    fixed = inputs.clamp_face_mask(desc)
    f = inputs.point_load(desc, (70, 13), 1, -1.0)
    return inputs.Problem("ragged70x26", desc, inputs._to_element_order(rho),
                          fixed, f)


def test_vec_dot():
    msp = _msp()
    rng = np.random.default_rng(1)
    for n in (1, 255, 4097, 300001):
        x, y = rng.standard_normal(n), rng.standard_normal(n)
        v = msp.vec_dot(_dev(x), _dev(y))
        assert abs(v - x @ y) <= 1e-12 * np.abs(x * y).sum()


@pytest.mark.parametrize("which", ["config0", "ragged"])
def test_matvec_parity(which, cfg0):
    p = cfg0[0] if which == "config0" else _ragged()
    print(f"[matvec] {which} n={len(p.fixed)}", flush=True)
    s = _solver(p)
    E = oracle.simp_modulus(p.rho, p.desc["E0"], p.desc["Emin"], p.desc["penal"])
    K = oracle.assemble_stiffness(p.desc, E)
    rng = np.random.default_rng(3)
    x = rng.standard_normal(len(p.fixed))
    y = _host(s.apply_K(_dev(x)))
    xm = np.where(p.fixed == 1, 0.0, x)
    yref = np.where(p.fixed == 1, 0.0, K @ xm)
    assert _rel(y, yref) <= 1e-13
    assert np.all(y[p.fixed == 1] == 0.0)


@pytest.mark.parametrize("Emin,tol", [(1e-3, 1e-9), (1e-6, 1e-6)])
def test_level1_parity_fp64(Emin, tol):
    p = inputs.config(0, Emin=Emin)
    print(f"[level1] config0 Emin={Emin}", flush=True)
    h = dd.build_preconditioner(p.desc, p.rho, p.fixed, level="one")
    s = _solver(p)
    s.setup()
    rng = np.random.default_rng(5)
    r = rng.standard_normal(len(p.fixed))
    r[p.fixed == 1] = 0.0
    z = _host(s.apply_level1(_dev(r)))
    zref = h.M.level1(r[h.free])
    assert _rel(z[h.free], zref) <= tol
    assert np.all(z[p.fixed == 1] == 0.0)


def test_level1_parity_fp32(cfg0):
    p, h = cfg0
    s = _solver(p, precision=1)
    s.setup()
    rng = np.random.default_rng(6)
    r = rng.standard_normal(len(p.fixed))
    r[p.fixed == 1] = 0.0
    z = _host(s.apply_level1(_dev(r)))
    zref = h.M.level1(r[h.free])
    assert _rel(z[h.free], zref) <= 1e-3


def test_heat_modes_and_coarse_counts(cfg0):
    p, h = cfg0
    s = _solver(p)
    s.setup()
    ci = s.coarse_info()
    cs = h.coarse
    H2 = dd.coarse_H(p.desc) ** 2
    for l in range(len(cs.coarse_nodes)):
        seen = cs.lam_seen[l][0] * H2
        # skip neighbourhoods with an eigenvalue within 1% of the threshold
        if np.any(np.abs(seen - p.desc["eig_tau"]) < 0.01 * p.desc["eig_tau"]):
            continue
        assert ci["n_modes"][l] == cs.n_modes[l, 0], l
        ref = cs.eigvals[l][0]
        got = ci["eigvals"][l][: len(ref)]
        assert np.allclose(got, ref, rtol=1e-6, atol=1e-12 / H2), (l, got, ref)
    assert ci["n_coarse"] == cs.Phi.shape[1]
    assert ci["cap_hits"] == cs.cap_hits


def test_coarse_span_and_correction(cfg0):
    p, h = cfg0
    s = _solver(p)
    s.setup()
    phi = _host(s.coarse_basis())[h.free]
    ref = h.coarse.Phi[h.free].toarray()
    assert phi.shape == ref.shape
    qa, _ = np.linalg.qr(phi)
    qb, _ = np.linalg.qr(ref)
    sv = np.linalg.svd(qa.T @ qb, compute_uv=False)
    assert sv.min() > 1 - 1e-7
    rng = np.random.default_rng(8)
    r = rng.standard_normal(len(p.fixed))
    r[p.fixed == 1] = 0.0
    z = _host(s.apply_coarse(_dev(r)))
    zref = h.M.coarse(r[h.free])
    assert _rel(z[h.free], zref) <= 1e-6


def test_full_preconditioner_parity(cfg0):
    p, h = cfg0
    s = _solver(p)
    s.setup()
    rng = np.random.default_rng(9)
    r = rng.standard_normal(len(p.fixed))
    r[p.fixed == 1] = 0.0
    z = _host(s.apply_prec(_dev(r)))
    assert _rel(z[h.free], h.M(r[h.free])) <= 1e-6


def _check_solution(p, u, info, ud, tol=1e-8):
    assert info["relres_true"] <= tol, info
    assert _rel(u, ud) <= 1e-6, _rel(u, ud)
    c_ref = float(p.f @ ud)
    assert abs(info["compliance"] - c_ref) <= 1e-6 * abs(c_ref)
    assert abs(float(p.f @ u) - c_ref) <= 1e-6 * abs(c_ref)
    assert np.all(u[p.fixed == 1] == 0.0)


@pytest.mark.parametrize("precision", [0, 1])
def test_solve_config0(precision, cfg0):
    p, h = cfg0
    print(f"[solve] config0 precision={precision}", flush=True)
    u_o, info_o, _ = oracle.solve(p.desc, p.rho, p.fixed, p.f, hierarchy=h)
    ud = oracle.direct_solve(p.desc, p.rho, p.fixed, p.f)
    s = _solver(p, precision=precision)
    u, info = s.solve(_dev(p.f), rtol=1e-8)
    u = _host(u)
    print(f"  gpu iters={info['iters']} oracle iters={info_o.iters} "
          f"relres={info['relres_true']:.2e} cond={info['cond_est']:.3g} "
          f"oracle cond={info_o.cond_est:.3g}", flush=True)
    _check_solution(p, u, info, ud)
    assert info["n_coarse"] == info_o.n_coarse
    if precision == 0:
        assert abs(info["iters"] - info_o.iters) <= max(2, 0.1 * info_o.iters)
        assert abs(info["cond_est"] - info_o.cond_est) <= 0.05 * info_o.cond_est


def test_solve_ragged():
    p = _ragged()
    ud = oracle.direct_solve(p.desc, p.rho, p.fixed, p.f)
    u_o, info_o, _ = oracle.solve(p.desc, p.rho, p.fixed, p.f)
    s = _solver(p)
    u, info = s.solve(_dev(p.f))
    _check_solution(p, _host(u), info, ud)
    assert abs(info["iters"] - info_o.iters) <= max(2, 0.1 * info_o.iters)


def test_config_p_table2_row():
    p = inputs.config_p()
    u_o, info_o, _ = oracle.solve(p.desc, p.rho, p.fixed, p.f, tol=p.tol)
    s = _solver(p)
    u, info = s.solve(_dev(p.f), rtol=p.tol)
    assert info["n_coarse"] == 243
    assert abs(info["iters"] - info_o.iters) <= 1
    assert abs(info["cond_est"] - info_o.cond_est) <= 0.05 * info_o.cond_est


def test_warm_start_and_status_codes(cfg0):
    p, h = cfg0
    msp = _msp()
    s = _solver(p)
    f = _dev(p.f)
    u, info = s.solve(f)
    # warm start from the solution: converges at once
    u2, info2 = s.solve(f, u=u.clone(), warm=True)
    assert info2["iters"] <= 1
    # maxit = 1 -> not converged, valid output
    u3, info3 = s.solve(f, maxit=1)
    assert info3["status"] == msp.binding.MSP_NOT_CONVERGED
    # invalid densities
    bad = _dev(np.where(np.arange(len(p.rho)) == 5, 1.5, p.rho))
    with pytest.raises(msp.MspError):
        s.set_densities(bad)
    nan = _dev(np.where(np.arange(len(p.rho)) == 7, np.nan, p.rho))
    with pytest.raises(msp.MspError):
        s.set_densities(nan)


def test_deterministic_repeat(cfg0):
    p, h = cfg0
    s = _solver(p)
    f = _dev(p.f)
    u1, i1 = s.solve(f)
    u2, i2 = s.solve(f)
    assert torch.equal(u1, u2)
    assert i1["iters"] == i2["iters"]


def test_solve_config1_full_size_properties():
    """The benchmark workload at full size (263,682 DOFs), Emin = 1e-6,
    FP64 and FP32 local solves: true residual, compliance identity and the
    displacement against a sparse direct solve."""
    p = inputs.config(1, Emin=1e-6)
    ud = oracle.direct_solve(p.desc, p.rho, p.fixed, p.f)
    E = oracle.simp_modulus(p.rho, 1.0, 1e-6, 3.0)
    K = oracle.assemble_stiffness(p.desc, E)
    free = p.fixed == 0
    for precision in (0, 1):
        print(f"[config1] precision={precision}", flush=True)
        s = _solver(p, precision=precision)
        u, info = s.solve(_dev(p.f))
        u = _host(u)
        print(f"  iters={info['iters']} relres={info['relres_true']:.2e} "
              f"Nc={info['n_coarse']} setup={info['t_setup_ms']:.1f}ms "
              f"solve={info['t_solve_ms']:.1f}ms", flush=True)
        r = (p.f - K @ u)[free]
        assert np.linalg.norm(r) <= 1e-8 * np.linalg.norm(p.f[free])
        _check_solution(p, u, info, ud)
