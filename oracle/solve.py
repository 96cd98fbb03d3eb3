"""Top-level oracle calls: the PCG state solve and direct reference solves.

TEST INFRASTRUCTURE ONLY (see the package docstring).
"""
from __future__ import annotations

import dataclasses
import time

import numpy as np
import scipy.sparse.linalg as spla

from .dd import build_preconditioner
from .fem import assemble_stiffness, simp_modulus
from .pcg import lanczos_condition, pcg


@dataclasses.dataclass
class SolveInfo:
    iters: int
    converged: bool
    relres_rec: float
    relres_true: float
    compliance: float
    n_coarse: int
    n_modes: np.ndarray
    cap_hits: int
    cond_est: float
    t_setup: float
    t_solve: float
    history: list


def solve(desc, rho, fixed, f, tol=1e-8, maxit=5000, x0=None, level="both",
          rot=None, hierarchy=None):
    """Solve K(rho) u = f by PCG with M_EH+Rot (rot=1) or M_EH (rot=0).

    Returns ``(u, info, hierarchy)``; u is a full-length vector, zero at
    clamped DOFs.  ``level`` 'none' runs plain CG.
    """
    fixed = np.asarray(fixed, dtype=np.uint8)
    t0 = time.perf_counter()
    if level == "none":
        E = simp_modulus(rho, desc["E0"], desc["Emin"], desc["penal"])
        K = assemble_stiffness(desc, E)
        free = np.nonzero(fixed == 0)[0]
        K_FF = K[free][:, free].tocsr()
        Minv = lambda r: r.copy()
        hier = None
        n_coarse, n_modes, cap = 0, np.zeros(0, np.int64), 0
    else:
        hier = hierarchy or build_preconditioner(desc, rho, fixed, level, rot)
        K_FF, free, Minv = hier.K_FF, hier.free, hier.M
        n_coarse = hier.coarse.Phi.shape[1]
        n_modes, cap = hier.coarse.n_modes, hier.coarse.cap_hits
    t1 = time.perf_counter()
    fF = np.asarray(f, dtype=np.float64)[free]
    xF0 = None if x0 is None else np.asarray(x0, dtype=np.float64)[free]
    res = pcg(K_FF, fF, Minv, tol, maxit, xF0)
    t2 = time.perf_counter()
    u = np.zeros(len(fixed))
    u[free] = res.x
    rt = fF - K_FF @ res.x
    fn = np.linalg.norm(fF)
    info = SolveInfo(res.iters, res.converged, res.relres,
                     float(np.linalg.norm(rt) / fn) if fn else 0.0,
                     float(fF @ res.x), n_coarse, n_modes, cap,
                     lanczos_condition(res.alphas, res.betas),
                     t1 - t0, t2 - t1, res.history)
    return u, info, hier


def direct_solve(desc, rho, fixed, f):
    """The plain definition: u_F = K_FF^{-1} f_F by a sparse direct solve."""
    fixed = np.asarray(fixed, dtype=np.uint8)
    E = simp_modulus(rho, desc["E0"], desc["Emin"], desc["penal"])
    K = assemble_stiffness(desc, E)
    free = np.nonzero(fixed == 0)[0]
    K_FF = K[free][:, free].tocsc()
    u = np.zeros(len(fixed))
    u[free] = spla.spsolve(K_FF, np.asarray(f, dtype=np.float64)[free])
    return u


def reference_solution(desc, rho, fixed, f, direct_max_dofs=300000):
    """Ground truth for parity: a direct solve where it fits, else the PCG
    oracle driven to a relative residual of 1e-12."""
    if len(fixed) <= direct_max_dofs:
        return direct_solve(desc, rho, fixed, f)
    u, _, _ = solve(desc, rho, fixed, f, tol=1e-12)
    return u
