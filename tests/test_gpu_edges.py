"""Edge cases of the GPU path through the C ABI.

* A zero load (Section 2's system with f = 0, or a load only on clamped
  DOFs, which the problem statement of Section 1.1 ignores): u = 0 exactly,
  no iteration, from a cold or a warm start.
* Homogeneous material (Section 1.1's SIMP law at rho = 1 and rho = 0):
  K(0) = Emin K(1), and the two-level preconditioner built from K(0)
  (exact local solves, heat modes of the same pencil up to the factor
  Emin) is Emin^-1 times the one built from K(1), so PCG takes the same
  iterations and u(0) = u(1) / Emin, the coarse dimension is identical.
* The largest node row the first-level kernels take (36 nodes, 72 DOFs:
  70 x 70 elements, S = 35, overlap 1) and its 71-node coarse
  neighbourhood rows; level-1, heat-mode and coarse-correction parity
  against the oracle and full solves against a sparse direct solve.
* The first row size refused (37 nodes): MSP_E_INVALID, no launch.
"""
import numpy as np
import pytest

import inputs
import oracle
from oracle import dd

from _checks import assert_entrywise, local_scales

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
    s = msp.Solver(dict(p.desc, **kw), p.fixed)
    s.set_densities(_dev(p.rho))
    return s


def _close_u(u, ud, what):
    """Displacement against the direct solve: 2-norm and entry by entry
    (scaled max-abs), both 1e-6."""
    assert np.linalg.norm(u - ud) <= 1e-6 * np.linalg.norm(ud), what
    assert_entrywise(u, ud, 1e-6, np.max(np.abs(ud)), what)


def _square(nel, sub, overlap, seed):
    desc = inputs.problem_desc(2, (nel, nel), sub_nel=(sub, sub), overlap=overlap,
                               Emin=1e-4, eig_kmax=8)
    rng = np.random.default_rng(seed)
    rho = inputs.threshold(inputs.grf((nel, nel), 6, rng), 0.5)
    rho = inputs.fill_hinges(rho)
    rho = inputs.force_solid_disk(rho, (nel, nel // 2), 3.0)
    rho = inputs.connect_load_path(rho, (nel, nel // 2))
    fixed = inputs.clamp_face_mask(desc)
    f = inputs.point_load(desc, (nel, nel // 2), 1, -1.0)
    return inputs.Problem(f"square{nel}_S{sub}_d{overlap}", desc,
                          inputs._to_element_order(rho), fixed, f)


def _max_row_nodes(p):
    boxes = dd.subdomain_node_boxes(p.desc, p.fixed)
    return max(b[0][1] - b[0][0] + 1 for b in boxes)


@pytest.mark.parametrize("precision", [0, 1])
def test_zero_load(precision):
    p = inputs.config(0)
    print(f"[edges] zero load precision={precision}", flush=True)
    s = _solver(p, precision=precision)
    n = len(p.fixed)
    u, info = s.solve(torch.zeros(n, dtype=torch.float64, device="cuda"))
    assert info["status"] == 0 and info["iters"] == 0
    assert int(torch.count_nonzero(u)) == 0
    assert info["relres_true"] == 0.0 and info["compliance"] == 0.0
    # warm start from a nonzero vector: the zero load still gives u = 0
    u0 = _dev(np.random.default_rng(3).standard_normal(n))
    u, info = s.solve(torch.zeros_like(u0), u=u0, warm=True)
    assert info["status"] == 0 and info["iters"] == 0
    assert int(torch.count_nonzero(u)) == 0
    # a load only on clamped DOFs is no load
    f = np.where(p.fixed == 1, 1.0, 0.0)
    assert f.any()
    u, info = s.solve(_dev(f))
    assert info["status"] == 0 and info["iters"] == 0
    assert int(torch.count_nonzero(u)) == 0


@pytest.mark.parametrize("precision", [0, 1])
def test_homogeneous_scaling(precision):
    p0 = inputs.config(0)
    Emin = p0.desc["Emin"]
    print(f"[edges] homogeneous precision={precision} Emin={Emin}", flush=True)
    solid = inputs.Problem("solid", p0.desc, np.ones_like(p0.rho), p0.fixed, p0.f)
    void = inputs.Problem("void", p0.desc, np.zeros_like(p0.rho), p0.fixed, p0.f)
    u1, i1 = _solver(solid, precision=precision).solve(_dev(p0.f))
    u0, i0 = _solver(void, precision=precision).solve(_dev(p0.f))
    u1, u0 = _host(u1), _host(u0)
    ud = oracle.direct_solve(solid.desc, solid.rho, solid.fixed, solid.f)
    assert i1["relres_true"] <= 1e-8 and i0["relres_true"] <= 1e-8
    _close_u(u1, ud, "rho = 1")
    _close_u(u0 * Emin, ud, "Emin u(rho = 0)")
    assert i0["n_coarse"] == i1["n_coarse"]
    assert abs(i0["iters"] - i1["iters"]) <= 1
    assert abs(i0["compliance"] * Emin - i1["compliance"]) <= 1e-6 * i1["compliance"]
    if precision == 0:
        _, info_o, _ = oracle.solve(solid.desc, solid.rho, solid.fixed, solid.f)
        assert i1["n_coarse"] == info_o.n_coarse
        assert abs(i1["iters"] - info_o.iters) <= max(2, 0.1 * info_o.iters)


def test_largest_row_level1_and_solve():
    p = _square(70, 35, 1, seed=91)
    assert _max_row_nodes(p) == 36                 # 72 DOFs per node row
    assert 2 * 35 + 1 <= 72                        # neighbourhood rows of 71 nodes
    print(f"[edges] {p.name}: level-1, heat-mode and coarse parity", flush=True)
    h = dd.build_preconditioner(p.desc, p.rho, p.fixed)
    s = _solver(p)
    s.setup()
    r = inputs.probe_vector(p.fixed, 8)
    z = _host(s.apply_level1(_dev(r)))
    rF = r[h.free]
    parts = [(idx, lu.solve(rF[idx])) for idx, lu in zip(h.sub_idx, h.M.factors)]
    zref = np.zeros(len(h.free))
    for idx, v in parts:
        zref[idx] += v
    assert_entrywise(z[h.free], zref, 1e-8, local_scales(len(h.free), parts), "level1")
    assert np.all(z[p.fixed == 1] == 0.0)
    # heat modes of every neighbourhood, the 71 x 71 one included.  A
    # neighbourhood without clamped nodes has the eigenvalue 0 (constants);
    # both solvers fix it only to rounding of the pencil's largest
    # eigenvalue (order 10 at h = 1), so its absolute tolerance is 1e-13,
    # far below the smallest nonzero selected eigenvalue (about 2e-6).
    ci = s.coarse_info()
    cs = h.coarse
    H2 = dd.coarse_H(p.desc) ** 2
    for l in range(len(cs.coarse_nodes)):
        seen = cs.lam_seen[l][0] * H2
        if np.any(np.abs(seen - p.desc["eig_tau"]) < 0.01 * p.desc["eig_tau"]):
            continue
        assert ci["n_modes"][l] == cs.n_modes[l, 0], l
        ref = cs.eigvals[l][0]
        assert np.allclose(ci["eigvals"][l][: len(ref)], ref, rtol=1e-6, atol=1e-13), l
    assert ci["n_coarse"] == cs.Phi.shape[1]
    zc = _host(s.apply_coarse(_dev(r)))
    zcref = h.M.coarse(r[h.free])
    assert_entrywise(zc[h.free], zcref, 1e-6, np.max(np.abs(zcref)), "coarse")
    ud = oracle.direct_solve(p.desc, p.rho, p.fixed, p.f)
    for precision in (0, 1):
        print(f"[edges] {p.name}: solve precision={precision}", flush=True)
        u, info = _solver(p, precision=precision).solve(_dev(p.f))
        u = _host(u)
        assert info["relres_true"] <= 1e-8, info
        _close_u(u, ud, f"u precision={precision}")
        assert np.all(u[p.fixed == 1] == 0.0)


def test_row_too_large_is_refused():
    p = _square(72, 36, 1, seed=92)
    assert _max_row_nodes(p) == 37                 # 74 DOFs per node row
    msp = _msp()
    print(f"[edges] {p.name}: expect MSP_E_INVALID", flush=True)
    with pytest.raises(msp.MspError) as e:
        s = _solver(p)
        s.setup()
    assert e.value.status == msp.binding.MSP_E_INVALID
