"""GPU parity of the 3D (H8) coarse space M_EH+Rot through the C ABI:
heat eigenproblems on the coarse neighbourhoods with the eigenvalue
threshold (Section 4.1), three rotations per coarse node (Section 4.2), the
coarse term R_0^T K_0^+ R_0 (Section 2) and the two-level solve.

The GPU factors each neighbourhood's A + sigma M by node planes and finds
the low eigenpairs by shift-invert subspace iteration; the oracle solves
each pencil with LAPACK or ARPACK.  Tolerances:
- mode counts exact (neighbourhoods with an eigenvalue within 1% of the
  threshold skipped), eigenvalues to 1e-6 relative;
- coarse spans: every column within 1e-7 (relative) of the other basis's
  span (eigenvectors are unique only up to sign and within degenerate
  eigenspaces);
- coarse correction and M^{-1} r per entry, 1e-6 of max |z|;
- solves: true relres <= 1e-8, u per entry 1e-6 of max |u| against a sparse
  direct solve, compliance 1e-6, iterations within 10% and the condition
  estimate within 5% of the oracle's two-level PCG.
"""
import numpy as np
import pytest

import inputs
import oracle
from oracle import dd

from _checks import assert_entrywise

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


def _case(nel, seed, Emin=1e-6, kmax=16, rot=1, precision=0):
    """A 3D cantilever: random densities with 30% void, the x = 0 face
    clamped, a unit downward load spread over the x = nx face; S = 6,
    one overlap layer."""
    desc = inputs.problem_desc(3, nel, sub_nel=6, overlap=1, Emin=Emin,
                               eig_kmax=kmax, rot_enrich=rot, precision=precision)
    rng = np.random.default_rng(seed)
    rho = rng.uniform(0.0, 1.0, inputs.n_elems(desc))
    rho[rng.uniform(size=rho.size) < 0.3] = 0.0
    fixed = inputs.clamp_face_mask(desc, axis=0, side=0)
    ny = nel[1]
    f = inputs.face_patch_load(desc, max(0, ny // 2 - 1), ny // 2 + 1, 1, -1.0)
    f[fixed == 1] = 0.0
    return desc, rho, fixed, f


CASES = [((18, 12, 12), 51), ((12, 6, 18), 52)]

_HIER = {}


def _hier(nel, seed, **kw):
    key = (nel, seed, tuple(sorted(kw.items())))
    if key not in _HIER:
        desc, rho, fixed, f = _case(nel, seed, **kw)
        _HIER[key] = (desc, rho, fixed, f,
                      dd.build_preconditioner(desc, rho, fixed, level="both"))
    return _HIER[key]


def _solver(desc, rho, fixed):
    msp = _msp()
    s = msp.Solver(desc, fixed)
    s.set_densities(_dev(rho))
    s.setup()
    return s


def _check_modes(desc, ci, cs):
    H2 = dd.coarse_H(desc) ** 2
    tau = desc["eig_tau"]
    checked = 0
    for l in range(len(cs.coarse_nodes)):
        seen = np.asarray(cs.lam_seen[l][0]) * H2
        if np.any(np.abs(seen - tau) < 0.01 * tau):
            continue
        assert ci["n_modes"][l] == cs.n_modes[l, 0], (l, ci["n_modes"][l], cs.n_modes[l])
        ref = cs.eigvals[l][0]
        got = ci["eigvals"][l][: len(ref)]
        assert np.allclose(got, ref, rtol=1e-6, atol=1e-12 / H2), (l, got, ref)
        checked += 1
    assert checked >= len(cs.coarse_nodes) // 2
    return checked


@pytest.mark.parametrize("nel,seed", CASES)
def test_heat3_modes_counts_and_coarse_dimension(nel, seed):
    desc, rho, fixed, _, h = _hier(nel, seed)
    print(f"[3d coarse] modes nel={nel}", flush=True)
    s = _solver(desc, rho, fixed)
    ci = s.coarse_info()
    cs = h.coarse
    n = _check_modes(desc, ci, cs)
    print(f"  {n} of {len(cs.coarse_nodes)} neighbourhoods compared, N_c gpu "
          f"{ci['n_coarse']} oracle {cs.Phi.shape[1]}", flush=True)
    assert ci["n_coarse"] == cs.Phi.shape[1]
    # the library counts neighbourhoods, the oracle pencils per component
    assert ci["cap_hits"] * 3 == cs.cap_hits
    s.close()


@pytest.mark.parametrize("nel,seed", CASES)
def test_coarse3_span_correction_and_prec(nel, seed):
    desc, rho, fixed, _, h = _hier(nel, seed)
    print(f"[3d coarse] span nel={nel}", flush=True)
    s = _solver(desc, rho, fixed)
    phi = _host(s.coarse_basis())[h.free]
    ref = h.coarse.Phi[h.free].toarray()
    assert phi.shape == ref.shape
    # every column of each basis lies in the other's span (orthonormal
    # bases by SVD with a rank cut: when every coarse node carries its
    # rotations, sum_l chi_l r_l = 0 makes three columns dependent)
    def span(a):
        u, sv, _ = np.linalg.svd(a, full_matrices=False)
        return u[:, sv > 1e-10 * sv[0]]
    qa, qb = span(phi), span(ref)
    assert qa.shape[1] == qb.shape[1]
    worst = 0.0
    for a, q in ((phi, qb), (ref, qa)):
        res = a - q @ (q.T @ a)
        worst = max(worst, float(np.max(np.linalg.norm(res, axis=0) /
                                        np.linalg.norm(a, axis=0))))
    print(f"  rank {qa.shape[1]} of {phi.shape[1]}, largest relative distance of a "
          f"column from the other span {worst:.3e}", flush=True)
    assert worst <= 1e-7
    r = inputs.probe_vector(fixed, 8)
    z = _host(s.apply_coarse(_dev(r)))
    zref = np.zeros(len(fixed))
    zref[h.free] = h.M.coarse(r[h.free])
    assert np.all(z[fixed == 1] == 0.0)
    assert_entrywise(z, zref, 1e-6, np.max(np.abs(zref)), "3D coarse correction")
    # M^-1 r = first level + coarse level
    zp = _host(s.apply_prec(_dev(r)))
    z1 = np.zeros(len(fixed))
    z1[h.free] = h.M.level1(r[h.free])
    assert_entrywise(zp, z1 + zref, 1e-6, np.max(np.abs(z1 + zref)), "3D M^-1 r")
    s.close()


@pytest.mark.parametrize("nel,seed", CASES)
@pytest.mark.parametrize("precision", [0, 1])
def test_solve3_two_level_against_direct_and_oracle(nel, seed, precision):
    desc, rho, fixed, f, h = _hier(nel, seed)
    print(f"[3d coarse] solve nel={nel} precision={precision}", flush=True)
    msp = _msp()
    s = msp.Solver(dict(desc, precision=precision), fixed)
    s.set_densities(_dev(rho))
    u, info = s.solve(_dev(f), rtol=1e-8)
    u = _host(u)
    ud = oracle.direct_solve(desc, rho, fixed, f)
    _, info_o, _ = oracle.solve(desc, rho, fixed, f, hierarchy=h)
    print(f"  iters gpu {info['iters']} oracle {info_o.iters}, cond gpu "
          f"{info['cond_est']:.4g} oracle {info_o.cond_est:.4g}, N_c "
          f"{info['n_coarse']}, relres {info['relres_true']:.2e}", flush=True)
    assert info["status"] == 0 and info["relres_true"] <= 1e-8
    assert np.all(u[fixed == 1] == 0.0)
    assert_entrywise(u, ud, 1e-6, np.max(np.abs(ud)), "u")
    c_ref = float(f @ ud)
    assert abs(info["compliance"] - c_ref) <= 1e-6 * abs(c_ref)
    assert info["n_coarse"] == h.coarse.Phi.shape[1]
    assert info["eig_unconverged"] == 0
    if precision == 0:
        assert abs(info["iters"] - info_o.iters) <= max(2, 0.1 * info_o.iters)
        assert abs(info["cond_est"] - info_o.cond_est) <= 0.05 * info_o.cond_est
    else:
        # flexible PR with FP32 first-level inverses: a few iterations more
        assert info["iters"] <= 1.2 * info_o.iters + 2
    s.close()


def test_coarse3_cap_and_no_rotations():
    """kmax = 1 forces the cap on neighbourhoods with two or more modes
    below the threshold; rot_enrich = 0 (M_EH alone) drops the rotation
    columns: counts against the oracle in both."""
    nel, seed = (18, 12, 12), 53
    desc, rho, fixed, _ = _case(nel, seed, kmax=1)
    print("[3d coarse] cap", flush=True)
    cs = dd.build_coarse_basis(desc, oracle.simp_modulus(rho, desc["E0"], desc["Emin"],
                                                         desc["penal"]), fixed)
    s = _solver(desc, rho, fixed)
    ci = s.coarse_info()
    assert cs.cap_hits > 0
    assert ci["cap_hits"] * 3 == cs.cap_hits
    assert np.array_equal(ci["n_modes"], cs.n_modes[:, 0])
    assert ci["n_coarse"] == cs.Phi.shape[1]
    s.close()
    desc0, rho0, fixed0, f0 = _case(nel, seed, rot=0)
    print("[3d coarse] M_EH", flush=True)
    h0 = dd.build_preconditioner(desc0, rho0, fixed0, level="both")
    s = _solver(desc0, rho0, fixed0)
    ci = s.coarse_info()
    assert ci["n_coarse"] == h0.coarse.Phi.shape[1] == 3 * int(h0.coarse.n_modes[:, 0].sum())
    r = inputs.probe_vector(fixed0, 5)
    z = _host(s.apply_coarse(_dev(r)))
    zref = np.zeros(len(fixed0))
    zref[h0.free] = h0.M.coarse(r[h0.free])
    assert_entrywise(z, zref, 1e-6, np.max(np.abs(zref)), "M_EH coarse correction")
    s.close()


def test_config2_two_level_against_goldens():
    """The 96 x 48 x 48 workload (698,691 DOFs, 1,377 coarse nodes, kmax 16)
    against the oracle's values written by
    tests/golden/make_cantilever3d_goldens.py: every neighbourhood's mode
    count and eigenvalues, N_c, the pseudo-inverse's rank, the coarse
    correction and M^{-1} r at 16,384 sampled DOFs, and the PCG run
    (iterations within 10%, condition estimate within 5%, compliance 1e-6)
    on the FP64 path; the FP32-local path to relres 1e-8 with at most 20%
    more iterations."""
    import json
    import os
    gdir = os.path.join(os.path.dirname(__file__), "golden")
    with open(os.path.join(gdir, "cantilever3d_golden.json")) as fh:
        gold = json.load(fh)
    probe = np.load(os.path.join(gdir, "cantilever3d_probe.npz"))
    p = inputs.config(2, precision=0)
    msp = _msp()
    H2 = dd.coarse_H(p.desc) ** 2
    tau = p.desc["eig_tau"]
    rho = _dev(p.rho)
    f = _dev(p.f)
    for prec in (0, 1):
        print(f"[3d config2] precision {prec}", flush=True)
        s = msp.Solver(dict(p.desc, precision=prec), p.fixed)
        s.set_densities(rho)
        s.setup()
        ci = s.coarse_info()
        assert ci["n_coarse"] == gold["n_coarse"]
        assert ci["cap_hits"] * 3 == gold["cap_hits"]
        compared = 0
        for l, node in enumerate(gold["nodes"]):
            lam = np.asarray(node["eigvals"])
            near = list(lam * H2) + ([node["first_rejected"] * H2]
                                     if node["first_rejected"] is not None else [])
            if np.any(np.abs(np.asarray(near) - tau) < 0.01 * tau):
                continue
            assert ci["n_modes"][l] == node["n_modes"], (l, ci["n_modes"][l], node)
            got = ci["eigvals"][l][: len(lam)]
            assert np.allclose(got, lam, rtol=1e-6, atol=1e-12 / H2), (l, got, lam)
            compared += 1
        print(f"  {compared} of {len(gold['nodes'])} neighbourhoods compared", flush=True)
        assert compared >= 0.9 * len(gold["nodes"])
        r = _dev(inputs.probe_vector(p.fixed, gold["probe_seed"]))
        idx = probe["idx"]
        zc = _host(s.apply_coarse(r))[idx]
        assert_entrywise(zc, probe["z_coarse"], 1e-6, gold["probe"]["coarse_zmax"],
                         "config-2 coarse correction")
        if prec == 0:
            zp = _host(s.apply_prec(r))[idx]
            assert_entrywise(zp, probe["z_prec"], 1e-6, gold["probe"]["prec_zmax"],
                             "config-2 M^-1 r")
        u, info = s.solve(f, rtol=1e-8, maxit=5000)
        g = gold["pcg"]
        print(f"  iters {info['iters']} (oracle {g['iters']}), cond {info['cond_est']:.5g} "
              f"(oracle {g['cond']:.5g}), rank {info['coarse_rank']} (oracle "
              f"{gold['coarse_rank']}), relres {info['relres_true']:.2e}", flush=True)
        assert info["status"] == 0 and info["relres_true"] <= 1e-8
        assert info["eig_unconverged"] == 0
        assert info["coarse_rank"] == gold["coarse_rank"]
        assert abs(info["compliance"] - g["compliance"]) <= 1e-6 * abs(g["compliance"])
        if prec == 0:
            assert abs(info["iters"] - g["iters"]) <= max(2, 0.1 * g["iters"])
            assert abs(info["cond_est"] - g["cond"]) <= 0.05 * g["cond"]
        else:
            assert info["iters"] <= 1.2 * g["iters"] + 2
        s.close()
