"""GPU parity: every step of the hot path through the C ABI against the CPU
FP64 oracle on the same seeded inputs, compared entry by entry.

Tolerances (stated here, derived in the design notes):
* K x                   : |y_i - y_ref_i| <= 1e-13 (|K| |x|)_i (same terms,
                          other summation order)
* FP64 local solves     : |z_i - z_ref_i| <= tol * (largest max-abs of the
                          local solutions holding entry i); tol 1e-10 at
                          Emin = 1e-3, 1e-8 at 1e-6 (two backward-stable
                          solvers; forward error grows with cond(K_i))
* FP32 local solves     : the same with tol 1e-4 (single-precision blocks)
* heat eigenvalues      : relative 1e-6 (selected eigenvalues)
* coarse correction     : |z_i - z_ref_i| <= 1e-6 max|z_ref| (depends only on
                          the coarse span)
* full solve            : true relative residual <= 1e-8; displacement
                          (2-norm, energy norm, scaled max-abs) and
                          compliance relative error <= 1e-6 against a direct
                          solve
"""
import math

import numpy as np
import pytest

import inputs
import oracle
from oracle import dd

from _checks import assert_entrywise, local_scales, max_abs_scaled

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
    scale = abs(K) @ np.abs(xm)
    assert_entrywise(y, yref, 1e-13, scale, "K x")
    assert np.all(y[p.fixed == 1] == 0.0)


def _level1_ref(h, r):
    """The oracle's first level and the per-entry local scales."""
    rF = r[h.free]
    parts = [(idx, lu.solve(rF[idx])) for idx, lu in zip(h.sub_idx, h.M.factors)]
    zref = np.zeros(len(h.free))
    for idx, v in parts:
        zref[idx] += v
    return zref, local_scales(len(h.free), parts)


@pytest.mark.parametrize("Emin,tol", [(1e-3, 1e-10), (1e-6, 1e-8)])
def test_level1_parity_fp64(Emin, tol):
    p = inputs.config(0, Emin=Emin)
    print(f"[level1] config0 Emin={Emin}", flush=True)
    h = dd.build_preconditioner(p.desc, p.rho, p.fixed, level="one")
    s = _solver(p)
    s.setup()
    r = inputs.probe_vector(p.fixed, 5)
    z = _host(s.apply_level1(_dev(r)))
    zref, scale = _level1_ref(h, r)
    print(f"  local-scaled error {np.max(np.abs(z[h.free] - zref) / scale):.3e}", flush=True)
    assert_entrywise(z[h.free], zref, tol, scale, "level1 fp64")
    assert np.all(z[p.fixed == 1] == 0.0)


def test_level1_parity_fp32(cfg0):
    p, h = cfg0
    s = _solver(p, precision=1)
    s.setup()
    r = inputs.probe_vector(p.fixed, 6)
    z = _host(s.apply_level1(_dev(r)))
    zref, scale = _level1_ref(h, r)
    print(f"  local-scaled error {np.max(np.abs(z[h.free] - zref) / scale):.3e}", flush=True)
    assert_entrywise(z[h.free], zref, 1e-4, scale, "level1 fp32")


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
    # the library counts neighbourhoods, the oracle pencils per component
    assert ci["cap_hits"] * p.desc["dim"] == cs.cap_hits


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
    r = inputs.probe_vector(p.fixed, 8)
    z = _host(s.apply_coarse(_dev(r)))
    zref = h.M.coarse(r[h.free])
    assert_entrywise(z[h.free], zref, 1e-6, np.max(np.abs(zref)), "coarse")


def test_full_preconditioner_parity(cfg0):
    p, h = cfg0
    s = _solver(p)
    s.setup()
    r = inputs.probe_vector(p.fixed, 9)
    z = _host(s.apply_prec(_dev(r)))
    z1, scale = _level1_ref(h, r)
    zc = h.M.coarse(r[h.free])
    # the level-1 part to 1e-8 of its local scales, the coarse part to 1e-6
    # of its max-abs
    bound = 1e-8 * scale + 1e-6 * np.max(np.abs(zc))
    assert_entrywise(z[h.free], z1 + zc, 1.0, bound, "M^-1 r")


def _check_solution(p, u, info, ud, tol=1e-8):
    """relres, then u against the direct solve in the 2-norm, the energy
    norm and entry by entry (scaled max-abs), and the compliance."""
    assert info["relres_true"] <= tol, info
    E = oracle.simp_modulus(p.rho, p.desc["E0"], p.desc["Emin"], p.desc["penal"])
    K = oracle.assemble_stiffness(p.desc, E)
    d = np.where(p.fixed == 0, u - ud, 0.0)
    eK = float(np.sqrt(d @ (K @ d)) / np.sqrt(ud @ (K @ ud)))
    e2 = float(np.linalg.norm(d) / np.linalg.norm(ud))
    assert e2 <= 1e-6 and eK <= 1e-6, (e2, eK)
    assert_entrywise(u, ud, 1e-6, np.max(np.abs(ud)), "u")
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


@pytest.mark.parametrize("which", ["config0", "config_p"])
def test_meh_without_rotations(which):
    """M_EH (rot_enrich = 0, Table 1): the coarse space of heat modes alone.
    The GPU's coarse dimension, iterations and condition estimate against
    the oracle's M_EH; on the paper's 100 x 100 example the coarse
    dimension is 2 x 81 = 162 (one heat mode per component and coarse node
    that is not clamped) and the paper's Table 2 row gives 15 iterations."""
    p = inputs.config(0) if which == "config0" else inputs.config_p()
    tol = p.tol
    print(f"[meh] {which} rot_enrich=0", flush=True)
    h = dd.build_preconditioner(p.desc, p.rho, p.fixed, rot=0)
    u_o, info_o, _ = oracle.solve(p.desc, p.rho, p.fixed, p.f, tol=tol, hierarchy=h)
    s = _solver(p, rot_enrich=0)
    u, info = s.solve(_dev(p.f), rtol=tol)
    u = _host(u)
    print(f"  gpu Nc={info['n_coarse']} iters={info['iters']} cond={info['cond_est']:.4g}"
          f" | oracle Nc={info_o.n_coarse} iters={info_o.iters} cond={info_o.cond_est:.4g}",
          flush=True)
    assert info["status"] == 0
    assert info["n_coarse"] == info_o.n_coarse
    assert abs(info["iters"] - info_o.iters) <= max(1, 0.1 * info_o.iters)
    assert abs(info["cond_est"] - info_o.cond_est) <= 0.05 * info_o.cond_est
    if which == "config_p":
        assert info["n_coarse"] == 162
        ud = oracle.direct_solve(p.desc, p.rho, p.fixed, p.f)
        assert np.linalg.norm(u - ud) <= 1e-5 * np.linalg.norm(ud)
    else:
        ud = oracle.direct_solve(p.desc, p.rho, p.fixed, p.f)
        _check_solution(p, u, info, ud)


def test_kmax_cap_branch(cfg0):
    """The mode cap of the threshold rule (at most kmax modes per
    neighbourhood, Section 4.1): with kmax = 2 three neighbourhoods of the
    64 x 32 cantilever have more eigenvalues below the threshold than the
    cap.  Counts, eigenvalues, cap hits and the solve against the oracle."""
    p0, _ = cfg0
    p = p0.with_(eig_kmax=2)
    h = dd.build_preconditioner(p.desc, p.rho, p.fixed)
    cs = h.coarse
    assert cs.cap_hits > 0
    s = _solver(p)
    s.setup()
    ci = s.coarse_info()
    H2 = dd.coarse_H(p.desc) ** 2
    print(f"[cap] gpu cap={ci['cap_hits']} Nc={ci['n_coarse']} | oracle "
          f"cap={cs.cap_hits} Nc={cs.Phi.shape[1]}", flush=True)
    assert ci["cap_hits"] * p.desc["dim"] == cs.cap_hits
    assert ci["n_coarse"] == cs.Phi.shape[1]
    for l in range(len(cs.coarse_nodes)):
        assert ci["n_modes"][l] == cs.n_modes[l, 0], l
        ref = cs.eigvals[l][0]
        assert np.allclose(ci["eigvals"][l][: len(ref)], ref, rtol=1e-6,
                           atol=1e-12 / H2), l
    u_o, info_o, _ = oracle.solve(p.desc, p.rho, p.fixed, p.f, hierarchy=h)
    u, info = s.solve(_dev(p.f))
    u = _host(u)
    ud = oracle.direct_solve(p.desc, p.rho, p.fixed, p.f)
    _check_solution(p, u, info, ud)
    assert info["cap_hits"] == ci["cap_hits"]
    assert abs(info["iters"] - info_o.iters) <= max(2, 0.1 * info_o.iters)
    assert abs(info["cond_est"] - info_o.cond_est) <= 0.05 * info_o.cond_est
