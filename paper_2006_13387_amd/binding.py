"""ctypes binding of libmsp (include/msp.h).

Argument marshalling only: every step of the solve runs in the library's
HIP kernels.  Device arrays are torch tensors on the GPU; only their
data_ptr() crosses the boundary, with torch's current stream.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmsp.so")

MSP_OK = 0
MSP_NOT_CONVERGED = 1
MSP_E_INVALID = -1
MSP_E_NOMEM = -2
MSP_E_DEVICE = -3
MSP_E_NOT_SPD = -4
MSP_E_BREAKDOWN = -5
MSP_E_STATE = -7
STATUS_NAMES = {0: "MSP_OK", 1: "MSP_NOT_CONVERGED", -1: "MSP_E_INVALID",
                -2: "MSP_E_NOMEM", -3: "MSP_E_DEVICE", -4: "MSP_E_NOT_SPD",
                -5: "MSP_E_BREAKDOWN", -7: "MSP_E_STATE"}


class ProblemDesc(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("nel", ctypes.c_int32 * 3),
                ("h", ctypes.c_double), ("E0", ctypes.c_double),
                ("Emin", ctypes.c_double), ("nu", ctypes.c_double),
                ("penal", ctypes.c_double), ("sub_nel", ctypes.c_int32 * 3),
                ("overlap", ctypes.c_int32), ("sub_mode", ctypes.c_int32),
                ("eig_tau", ctypes.c_double), ("eig_kmax", ctypes.c_int32),
                ("rot_enrich", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("eig_random", ctypes.c_int32), ("eig_seed", ctypes.c_uint32),
                ("coarse_kind", ctypes.c_int32)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iters", ctypes.c_int32),
                ("converged", ctypes.c_int32), ("restarts", ctypes.c_int32),
                ("n_coarse", ctypes.c_int32), ("coarse_rank", ctypes.c_int32),
                ("cap_hits", ctypes.c_int32),
                ("fp64_subdomains", ctypes.c_int32),
                ("eig_unconverged", ctypes.c_int32),
                ("setup_reused", ctypes.c_int32),
                ("relres_true", ctypes.c_double),
                ("relres_rec", ctypes.c_double),
                ("compliance", ctypes.c_double), ("cond_est", ctypes.c_double),
                ("t_setup_ms", ctypes.c_double),
                ("t_solve_ms", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


EXPORTS = ["msp_create", "msp_destroy", "msp_last_error", "msp_set_densities",
           "msp_setup", "msp_solve", "msp_apply_K", "msp_apply_level1",
           "msp_apply_coarse", "msp_apply_prec", "msp_coarse_info",
           "msp_coarse_basis", "msp_vec_dot", "msp_query",
           "msp_kernel_timing", "msp_batch_create", "msp_batch_destroy",
           "msp_batch_last_error", "msp_batch_solve", "msp_batch_stats",
           "msp_batch_set_autotune", "msp_batch_tuning",
           "msp_server_create", "msp_server_destroy", "msp_server_last_error",
           "msp_server_add_run", "msp_server_submit", "msp_server_step",
           "msp_server_result", "msp_server_stats", "msp_set_reuse",
           "msp_server_set_reuse", "msp_vec_dot_noalloc",
           "msp_coarse_matrix", "msp_sensitivity", "msp_oc_update"]

KERNEL_NAMES = ["level1_apply", "cg_matvec", "heat_eigen", "combine",
                "coarse_restrict", "local_factor"]

_lib = None


def load_library(path=LIB_PATH):
    """Load libmsp.so; raises if it is missing (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(
            f"libmsp.so not found at {path}: build it with "
            "`python -m paper_2006_13387_amd.build` (no CPU fallback exists)")
    L = ctypes.CDLL(path)
    vp, i32, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
    L.msp_create.argtypes = [ctypes.POINTER(ProblemDesc), vp, ctypes.POINTER(vp)]
    L.msp_destroy.argtypes = [vp]
    L.msp_last_error.argtypes = [vp]
    L.msp_last_error.restype = ctypes.c_char_p
    L.msp_set_densities.argtypes = [vp, vp, vp]
    L.msp_setup.argtypes = [vp, vp]
    L.msp_solve.argtypes = [vp, vp, vp, i32, i32, dbl, i32, vp,
                            ctypes.POINTER(SolveInfo)]
    for name in ("msp_apply_K", "msp_apply_level1", "msp_apply_coarse",
                 "msp_apply_prec"):
        getattr(L, name).argtypes = [vp, vp, vp, vp]
    L.msp_coarse_info.argtypes = [vp, vp, vp, ctypes.POINTER(i32),
                                  ctypes.POINTER(i32), ctypes.POINTER(i32)]
    L.msp_coarse_basis.argtypes = [vp, vp, vp]
    L.msp_vec_dot.argtypes = [ctypes.c_int64, vp, vp, vp,
                              ctypes.POINTER(ctypes.c_double)]
    L.msp_coarse_matrix.argtypes = [vp, i32, vp, vp]
    L.msp_sensitivity.argtypes = [vp, vp, vp, vp, vp, vp]
    L.msp_oc_update.argtypes = [vp, vp, vp, dbl, dbl, vp,
                                ctypes.POINTER(ctypes.c_double), vp]
    L.msp_vec_dot_noalloc.argtypes = [ctypes.c_int64, vp, vp, vp, vp]
    L.msp_query.argtypes = [vp, ctypes.POINTER(ctypes.c_int64)]
    L.msp_kernel_timing.argtypes = [vp, i32, vp, vp, i32]
    L.msp_batch_create.argtypes = [ctypes.POINTER(vp)]
    L.msp_batch_destroy.argtypes = [vp]
    L.msp_batch_last_error.argtypes = [vp]
    L.msp_batch_last_error.restype = ctypes.c_char_p
    L.msp_batch_solve.argtypes = [vp, vp, vp, vp, vp, i32, dbl, i32, i32, vp,
                                  ctypes.POINTER(SolveInfo)]
    L.msp_batch_stats.argtypes = [vp, ctypes.POINTER(ctypes.c_int64),
                                  ctypes.POINTER(ctypes.c_int64)]
    L.msp_batch_set_autotune.argtypes = [vp, i32]
    L.msp_batch_tuning.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32),
                                   ctypes.POINTER(i32), vp]
    L.msp_server_create.argtypes = [ctypes.c_int64, i32, ctypes.POINTER(vp)]
    L.msp_server_destroy.argtypes = [vp]
    L.msp_server_last_error.argtypes = [vp]
    L.msp_server_last_error.restype = ctypes.c_char_p
    L.msp_server_add_run.argtypes = [vp, ctypes.POINTER(ProblemDesc), vp,
                                     ctypes.POINTER(i32)]
    L.msp_server_submit.argtypes = [vp, i32, vp, vp, vp, vp, vp, dbl, i32,
                                    ctypes.POINTER(i32)]
    L.msp_server_step.argtypes = [vp, vp, ctypes.POINTER(i32)]
    L.msp_server_result.argtypes = [vp, i32, ctypes.POINTER(SolveInfo),
                                    ctypes.POINTER(ctypes.c_double)]
    L.msp_server_stats.argtypes = [vp, ctypes.POINTER(ctypes.c_double), i32]
    L.msp_set_reuse.argtypes = [vp, i32, i32]
    L.msp_server_set_reuse.argtypes = [vp, i32, i32]
    for name in EXPORTS:
        if name not in ("msp_last_error", "msp_batch_last_error",
                        "msp_server_last_error"):
            getattr(L, name).restype = i32
    _lib = L
    return L


class MspError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a CUDA (HIP) torch tensor")
    if t.dtype != torch.float64 or not t.is_contiguous():
        raise TypeError("expected a contiguous float64 tensor")
    return ctypes.c_void_p(t.data_ptr())


def make_desc(d):
    pd = ProblemDesc()
    pd.dim = d["dim"]
    nel = list(d["nel"]) + [1] * (3 - len(d["nel"]))
    sub = list(d["sub_nel"]) + [1] * (3 - len(d["sub_nel"]))
    pd.nel = (ctypes.c_int32 * 3)(*nel)
    pd.sub_nel = (ctypes.c_int32 * 3)(*sub)
    pd.h, pd.E0, pd.Emin = d["h"], d["E0"], d["Emin"]
    pd.nu, pd.penal = d["nu"], d["penal"]
    pd.overlap, pd.sub_mode = d["overlap"], d["sub_mode"]
    pd.eig_tau, pd.eig_kmax = d["eig_tau"], d["eig_kmax"]
    pd.rot_enrich, pd.precision = d["rot_enrich"], d["precision"]
    pd.eig_random = d.get("eig_random", 0)
    pd.eig_seed = d.get("eig_seed", 0)
    pd.coarse_kind = d.get("coarse_kind", 0)
    return pd


class Solver:
    """One mesh, one set of boundary conditions (a msp_handle)."""

    def __init__(self, desc, fixed):
        self.L = load_library()
        self.desc = dict(desc)
        self._pd = make_desc(desc)
        mask = np.ascontiguousarray(np.asarray(fixed, dtype=np.uint8))
        self._mask = mask
        h = ctypes.c_void_p()
        st = self.L.msp_create(ctypes.byref(self._pd),
                               mask.ctypes.data_as(ctypes.c_void_p),
                               ctypes.byref(h))
        if st != 0:
            raise MspError(st, self.L.msp_last_error(None).decode())
        self.h = h
        q = (ctypes.c_int64 * 12)()
        self.L.msp_query(self.h, q)
        self.n = int(q[0])

    def _check(self, st, ok=(0,)):
        if st not in ok:
            raise MspError(st, self.L.msp_last_error(self.h).decode())
        return st

    def close(self):
        if getattr(self, "h", None):
            self.L.msp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_densities(self, rho):
        self._check(self.L.msp_set_densities(self.h, _ptr(rho), _stream()))

    def setup(self):
        self._check(self.L.msp_setup(self.h, _stream()))

    def set_reuse(self, max_age, iter_limit=0):
        self._check(self.L.msp_set_reuse(self.h, int(max_age), int(iter_limit)))

    def solve(self, f, u=None, warm=False, rtol=1e-8, maxit=5000):
        import torch
        nrhs = f.numel() // self.n
        if u is None:
            u = torch.zeros_like(f)
        info = SolveInfo()
        st = self.L.msp_solve(self.h, _ptr(f), _ptr(u), nrhs, int(bool(warm)),
                              float(rtol), int(maxit), _stream(),
                              ctypes.byref(info))
        self._check(st, ok=(0, 1))
        return u, info.as_dict()

    def _apply(self, fn, x):
        import torch
        y = torch.empty_like(x)
        self._check(fn(self.h, _ptr(x), _ptr(y), _stream()))
        return y

    def apply_K(self, x):
        return self._apply(self.L.msp_apply_K, x)

    def apply_level1(self, r):
        return self._apply(self.L.msp_apply_level1, r)

    def apply_coarse(self, r):
        return self._apply(self.L.msp_apply_coarse, r)

    def apply_prec(self, r):
        return self._apply(self.L.msp_apply_prec, r)

    def coarse_info(self):
        q = (ctypes.c_int64 * 12)()
        self.L.msp_query(self.h, q)
        ncn = int(q[3])
        kmax = self.desc["eig_kmax"]
        nm = np.zeros(ncn, np.int32)
        ev = np.zeros(ncn * kmax, np.float64)
        a, b, c = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        self._check(self.L.msp_coarse_info(
            self.h, nm.ctypes.data_as(ctypes.c_void_p),
            ev.ctypes.data_as(ctypes.c_void_p), ctypes.byref(a),
            ctypes.byref(b), ctypes.byref(c)))
        return {"n_modes": nm, "eigvals": ev.reshape(ncn, kmax),
                "n_coarse": b.value, "cap_hits": c.value}

    def coarse_basis(self):
        import torch
        nc = self.coarse_info()["n_coarse"]
        phi = torch.zeros((max(nc, 1), self.n), dtype=torch.float64,
                          device="cuda")
        self._check(self.L.msp_coarse_basis(self.h, _ptr(phi), _stream()))
        return phi[:nc].T

    def coarse_matrix(self, which):
        """K_0 (which=0) or the generalised inverse the coarse solve applies
        (which=1), N_c x N_c on the device."""
        import torch
        q = self.query()
        ldk, nc = q["ldk"], q["n_coarse"]
        out = torch.zeros((ldk, ldk), dtype=torch.float64, device="cuda")
        self._check(self.L.msp_coarse_matrix(self.h, int(which), _ptr(out),
                                             _stream()))
        return out[:nc, :nc]

    def sensitivity(self, rho, u, lam=None):
        """d g / d rho_e (compliance when lam is None), nel doubles."""
        import torch
        out = torch.empty_like(rho)
        self._check(self.L.msp_sensitivity(
            self.h, _ptr(rho), _ptr(u), None if lam is None else _ptr(lam),
            _ptr(out), _stream()))
        return out

    def oc_update(self, rho, dg, volfrac, move=0.2):
        """One optimality-criteria step; returns (rho_new, multiplier)."""
        import torch
        out = torch.empty_like(rho)
        lam = ctypes.c_double()
        self._check(self.L.msp_oc_update(self.h, _ptr(rho), _ptr(dg),
                                         float(volfrac), float(move), _ptr(out),
                                         ctypes.byref(lam), _stream()))
        return out, lam.value

    def kernel_timing(self, enable=-1):
        """Launch counts and summed event times (ms) of the tracked kernels
        since the last reset; enable (a bit mask over KERNEL_NAMES, or True
        for all) resets and switches timing, -1 only reads."""
        if enable is True:
            enable = (1 << len(KERNEL_NAMES)) - 1
        n = len(KERNEL_NAMES)
        cnt = np.zeros(n, np.int64)
        tot = np.zeros(n, np.float64)
        self._check(self.L.msp_kernel_timing(
            self.h, int(enable), cnt.ctypes.data_as(ctypes.c_void_p),
            tot.ctypes.data_as(ctypes.c_void_p), n))
        return {k: (int(c), float(t)) for k, c, t in zip(KERNEL_NAMES, cnt, tot)}

    def query(self):
        q = (ctypes.c_int64 * 12)()
        self._check(self.L.msp_query(self.h, q))
        keys = ["n_dofs", "n_elems", "n_subdomains", "n_coarse_nodes",
                "n_coarse", "max_local", "level1_record_bytes",
                "coarse_basis_bytes", "local_vec_entries",
                "omega_vec_entries", "omega_factor_bytes", "ldk"]
        return dict(zip(keys, [int(v) for v in q]))


class Batch:
    """A batch context: the PCG solves of several Solvers in lockstep."""

    def __init__(self):
        self.L = load_library()
        b = ctypes.c_void_p()
        st = self.L.msp_batch_create(ctypes.byref(b))
        if st != 0:
            raise MspError(st, self.L.msp_batch_last_error(None).decode())
        self.b = b

    def close(self):
        if getattr(self, "b", None):
            self.L.msp_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def solve(self, solvers, fs, us=None, warm=None, rtol=1e-8, maxit=5000,
              use_graph=True):
        """Solve solvers[e] with right-hand side fs[e] (device float64
        tensors); returns (us, infos) like Solver.solve per entry."""
        import torch
        n = len(solvers)
        if us is None:
            us = [torch.zeros_like(f) for f in fs]
        H = (ctypes.c_void_p * n)(*[s.h.value for s in solvers])
        F = (ctypes.c_void_p * n)(*[_ptr(f).value for f in fs])
        U = (ctypes.c_void_p * n)(*[_ptr(u).value for u in us])
        W = None
        if warm is not None:
            W = (ctypes.c_int32 * n)(*[int(bool(w)) for w in warm])
        infos = (SolveInfo * n)()
        st = self.L.msp_batch_solve(self.b, H, F, U, W, n, float(rtol),
                                    int(maxit), int(bool(use_graph)),
                                    _stream(), infos)
        if st not in (0, 1):
            raise MspError(st, self.L.msp_batch_last_error(self.b).decode())
        return us, [i.as_dict() for i in infos]

    def stats(self):
        c, g = ctypes.c_int64(), ctypes.c_int64()
        self.L.msp_batch_stats(self.b, ctypes.byref(c), ctypes.byref(g))
        return {"chunks": c.value, "graph_chunks": g.value}

    def set_autotune(self, on):
        st = self.L.msp_batch_set_autotune(self.b, 1 if on else 0)
        if st != 0:
            raise MspError(st, self.L.msp_batch_last_error(self.b).decode())

    def tuning(self):
        """The launch shape the autotuner chose (or is measuring) and the
        measured cost of each candidate."""
        ch, od, tu = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        cost = np.zeros(6)
        self.L.msp_batch_tuning(self.b, ctypes.byref(ch), ctypes.byref(od), ctypes.byref(tu),
                                cost.ctypes.data_as(ctypes.c_void_p))
        return {"chunk": ch.value, "largest_first": od.value, "tuned": bool(tu.value),
                "cost_ms_per_iter_dof": cost.tolist()}


class Server:
    """Continuous batching of state and adjoint solves of many runs."""

    def __init__(self, hbm_budget_bytes, max_active):
        self.L = load_library()
        sv = ctypes.c_void_p()
        st = self.L.msp_server_create(int(hbm_budget_bytes), int(max_active),
                                      ctypes.byref(sv))
        if st != 0:
            raise MspError(st, self.L.msp_server_last_error(None).decode())
        self.sv = sv
        self._keep = {}          # tensors the server reads or writes

    def _check(self, st, ok=(0,)):
        if st not in ok:
            raise MspError(st, self.L.msp_server_last_error(self.sv).decode())
        return st

    def close(self):
        if getattr(self, "sv", None):
            self.L.msp_server_destroy(self.sv)
            self.sv = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def add_run(self, desc, fixed):
        pd = make_desc(desc)
        mask = np.ascontiguousarray(np.asarray(fixed, dtype=np.uint8))
        rid = ctypes.c_int32()
        self._check(self.L.msp_server_add_run(
            self.sv, ctypes.byref(pd), mask.ctypes.data_as(ctypes.c_void_p),
            ctypes.byref(rid)))
        return rid.value

    def submit(self, run, rho, f_state, f_adj=None, rtol=1e-8, maxit=5000):
        """Queue a request; returns (ticket, u_state, u_adj) with the output
        tensors filled when the request completes."""
        import torch
        us = torch.zeros_like(f_state)
        ua = torch.zeros_like(f_adj) if f_adj is not None else None
        t = ctypes.c_int32()
        self._check(self.L.msp_server_submit(
            self.sv, int(run), _ptr(rho), _ptr(f_state),
            _ptr(f_adj) if f_adj is not None else None, _ptr(us),
            _ptr(ua) if ua is not None else None, float(rtol), int(maxit),
            ctypes.byref(t)))
        self._keep[t.value] = (rho, f_state, f_adj, us, ua)
        return t.value, us, ua

    def step(self):
        n = ctypes.c_int32()
        self._check(self.L.msp_server_step(self.sv, _stream(), ctypes.byref(n)))
        return n.value

    def result(self, ticket):
        """(state info, adjoint info, latency ms) or None while pending."""
        infos = (SolveInfo * 2)()
        lat = ctypes.c_double()
        st = self.L.msp_server_result(self.sv, int(ticket), infos,
                                      ctypes.byref(lat))
        if st == -7:
            return None
        self._check(st, ok=(0, 1))
        self._keep.pop(ticket, None)
        return infos[0].as_dict(), infos[1].as_dict(), lat.value

    def set_reuse(self, max_age, iter_limit=0):
        self._check(self.L.msp_server_set_reuse(self.sv, int(max_age),
                                                int(iter_limit)))

    def stats(self):
        v = (ctypes.c_double * 10)()
        self._check(self.L.msp_server_stats(self.sv, v, 10))
        keys = ["completed", "p50_ms", "p99_ms", "solves_per_s", "hbm_bytes",
                "queued", "active", "chunks", "setups_built", "setups_reused"]
        return dict(zip(keys, list(v)))


def vec_dot(x, y):
    L = load_library()
    out = ctypes.c_double()
    st = L.msp_vec_dot(x.numel(), _ptr(x), _ptr(y), _stream(),
                       ctypes.byref(out))
    if st != 0:
        raise MspError(st, L.msp_last_error(None).decode())
    return out.value


def vec_dot_noalloc(x, y, out):
    """out[0] = x . y through the entry point that allocates nothing; out is
    a one-element float64 device tensor, written on the current stream."""
    L = load_library()
    st = L.msp_vec_dot_noalloc(x.numel(), _ptr(x), _ptr(y), _ptr(out), _stream())
    if st != 0:
        raise MspError(st, L.msp_last_error(None).decode())
    return out
