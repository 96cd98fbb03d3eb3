"""GPU: lazy reuse of the preconditioner across density updates (Section 1:
the preconditioner is updated after a fixed number of design steps, or once
the solver's iteration count exceeds a threshold).

A setup built for older densities is still a symmetric positive definite
preconditioner for the new K(rho), so PCG converges to the new system's
solution: the reused solves must meet the true relative residual 1e-8 and
match the oracle's direct solve of the new system to 1e-6, and a handle
that was given the same setup and densities must give the same bits.
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


def _designs(p, n):
    """A sequence of density fields: the workload's, then smooth seeded
    perturbations of it (as between topology-optimisation steps)."""
    out = [p.rho]
    for t in range(1, n):
        out.append(inputs.perturb(out[-1], p.desc["nel"], inputs.perturb_seed(5000, t)))
    return out


@pytest.mark.parametrize("precision", [0, 1])
def test_reuse_by_age(precision):
    msp = _msp()
    p = inputs.config(0, precision=precision)
    rhos = _designs(p, 5)
    f = _dev(p.f)
    s = msp.Solver(p.desc, p.fixed)
    s.set_reuse(3)
    expect = [0, 1, 1, 1, 0]           # rebuilt at the 4th density change
    for t, rho in enumerate(rhos):
        s.set_densities(_dev(rho))
        u, info = s.solve(f)
        ud = oracle.direct_solve(p.desc, rho, p.fixed, p.f)
        u = u.cpu().numpy()
        print(f"[reuse] precision={precision} step {t}: reused={info['setup_reused']} "
              f"iters={info['iters']} relres={info['relres_true']:.2e} "
              f"setup_ms={info['t_setup_ms']:.2f}", flush=True)
        assert info["setup_reused"] == expect[t], (t, info)
        assert (info["t_setup_ms"] > 0) == (expect[t] == 0)
        assert info["status"] == 0 and info["relres_true"] <= 1e-8
        assert np.linalg.norm(u - ud) <= 1e-6 * np.linalg.norm(ud)
        assert_entrywise(u, ud, 1e-6, np.max(np.abs(ud)), f"u step {t}")
    s.close()


def test_reused_setup_is_bitwise_a_stale_setup():
    """Solving on a reused setup equals a handle that built its setup for
    the old densities explicitly and then received the new ones."""
    msp = _msp()
    p = inputs.config(0)
    rho0, rho1 = _designs(p, 2)
    f = _dev(p.f)
    a = msp.Solver(p.desc, p.fixed)
    a.set_reuse(2)
    a.set_densities(_dev(rho0))
    a.solve(f)
    a.set_densities(_dev(rho1))
    ua, ia = a.solve(f)
    b = msp.Solver(p.desc, p.fixed)
    b.set_reuse(2)
    b.set_densities(_dev(rho0))
    b.setup()
    b.set_densities(_dev(rho1))
    ub, ib = b.solve(f)
    assert ia["setup_reused"] == 1 and ib["setup_reused"] == 1
    assert torch.equal(ua, ub)
    assert ia["iters"] == ib["iters"]
    # a fresh setup for rho1 solves the same system
    c = msp.Solver(p.desc, p.fixed)
    c.set_densities(_dev(rho1))
    uc, ic = c.solve(f)
    print(f"[reuse] stale iters={ia['iters']} fresh iters={ic['iters']}", flush=True)
    assert ic["setup_reused"] == 0
    assert float(torch.linalg.norm(ua - uc) / torch.linalg.norm(uc)) <= 1e-6
    for s in (a, b, c):
        s.close()


def test_reuse_iteration_limit_rebuilds_and_continues():
    """A solve on a reused setup is stopped at iter_limit iterations, the
    setup is rebuilt for the current densities and the solve continues from
    the iterate it reached: the result meets 1e-8 and the direct solve, and
    the solve reports a setup built, not reused."""
    msp = _msp()
    p = inputs.config(0)
    rhos = _designs(p, 4)
    f = _dev(p.f)
    s = msp.Solver(p.desc, p.fixed)
    s.set_reuse(10, 5)                 # any reused solve exceeds 5 iterations
    for t, rho in enumerate(rhos):
        s.set_densities(_dev(rho))
        u, info = s.solve(f)
        ud = oracle.direct_solve(p.desc, rho, p.fixed, p.f)
        print(f"[reuse] limit step {t}: reused={info['setup_reused']} "
              f"iters={info['iters']} setup_ms={info['t_setup_ms']:.2f}", flush=True)
        assert info["status"] == 0 and info["relres_true"] <= 1e-8
        assert info["setup_reused"] == 0 and info["t_setup_ms"] > 0
        if t > 0:
            assert info["iters"] > 5          # the 5 stale iterations count
        u = u.cpu().numpy()
        assert_entrywise(u, ud, 1e-6, np.max(np.abs(ud)), f"u step {t}")
    s.close()
