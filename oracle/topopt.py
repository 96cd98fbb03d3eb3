"""The topology-optimisation consumer of the state solve: the compliance
sensitivity and one optimality-criteria density update.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section 1 states the minimum-compliance problem: minimise g_0 = f^T u
subject to K(rho) u = f, the volume constraint v_e^T rho <= V* and
0 <= rho <= 1, with the SIMP law E_e = Emin + rho_e^p (E0 - Emin).  Its
gradient is

    d g_0 / d rho_e = -u^T (dK / d rho_e) u
                    = -p rho_e^(p-1) (E0 - Emin) u_e^T K^_e u_e

(K^_e the unit-modulus element matrix, u_e the element's DOFs).  For an
objective l^T u with adjoint solution K lam = l the same formula holds with
lam_e^T on the left.  The densities are then updated by the optimality
criteria method, which Section 1 names (after Bendsoe and Sigmund,
Topology Optimization, 2003): the heuristic fixed-point update

    rho_e <- clamp(rho_e B_e^(1/2), max(0, rho_e - m), min(1, rho_e + m)),
    B_e = max(0, -dg/drho_e) / (Lam dV/drho_e),

with the multiplier Lam found by bisection so that the volume constraint is
met with equality.  Filters are not part of this step.
"""
from __future__ import annotations

import numpy as np

from .fem import elasticity_element, element_dof_ids


def element_energy_form(desc, a, b):
    """a_e^T K^_e b_e for every element (unit modulus)."""
    Ke = elasticity_element(desc["dim"], desc["nu"], desc["h"])
    dofs = element_dof_ids(desc)
    A = np.asarray(a, dtype=np.float64)[dofs]
    B = np.asarray(b, dtype=np.float64)[dofs]
    return np.einsum("ei,ij,ej->e", A, Ke, B)


def compliance_sensitivity(desc, rho, u, lam=None):
    """d g / d rho_e = -p rho_e^(p-1) (E0 - Emin) lam_e^T K^_e u_e, with
    lam = u for the compliance (Section 1, the gradient formula)."""
    rho = np.asarray(rho, dtype=np.float64)
    p = desc["penal"]
    q = element_energy_form(desc, u if lam is None else lam, u)
    return -p * rho ** (p - 1.0) * (desc["E0"] - desc["Emin"]) * q


def oc_candidate(rho, dg, dv, lam, move):
    """Densities of the optimality-criteria update for multiplier lam."""
    B = np.maximum(0.0, -dg) / (lam * dv)
    lo = np.maximum(0.0, rho - move)
    hi = np.minimum(1.0, rho + move)
    return np.clip(rho * np.sqrt(B), lo, hi)


# the multiplier is confined to [LAM_MIN, LAM_MAX]; a volume target out of
# reach within the move limits leaves it at the nearer end
LAM_MIN, LAM_MAX = 2.0 ** -80, 2.0 ** 75


def oc_update(rho, dg, volfrac, move=0.2, dv=None, rel_tol=1e-13):
    """One optimality-criteria step with the volume sum(dv rho) = volfrac *
    sum(dv).  The multiplier is bracketed by doubling or halving from 1
    (within [LAM_MIN, LAM_MAX]) and then bisected until the bracket is
    relatively narrower than rel_tol.  Returns (rho_new, lam)."""
    rho = np.asarray(rho, dtype=np.float64)
    dg = np.asarray(dg, dtype=np.float64)
    dv = np.ones_like(rho) if dv is None else np.asarray(dv, dtype=np.float64)
    target = volfrac * dv.sum()

    def volume(lam):
        return float(dv @ oc_candidate(rho, dg, dv, lam, move))

    if volume(LAM_MAX) > target:
        return oc_candidate(rho, dg, dv, LAM_MAX, move), LAM_MAX
    if volume(LAM_MIN) <= target:
        return oc_candidate(rho, dg, dv, LAM_MIN, move), LAM_MIN
    lo, hi = 1.0, 1.0
    if volume(hi) > target:
        while volume(hi) > target:
            lo, hi = hi, 2.0 * hi
    else:
        while volume(lo) <= target:
            lo, hi = 0.5 * lo, lo
    while (hi - lo) > rel_tol * hi:
        mid = 0.5 * (lo + hi)
        if volume(mid) > target:
            lo = mid
        else:
            hi = mid
    lam = 0.5 * (lo + hi)
    return oc_candidate(rho, dg, dv, lam, move), lam
