"""Two-level overlapping Schwarz preconditioner M_EH+Rot (and M_EH).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Everything here works on the free degrees of freedom F (the complement of
the clamped set Gamma_D): the state system is K_FF u_F = f_F.

Readings taken where the paper is silent or garbled (each is listed with its
justification in the design notes of the repository):

* overlapping subdomains (Section 2): box mode extends each coarse block
  D_i by ``overlap`` element layers in the max-norm, clipped to the mesh;
  vertex mode uses the coarse neighbourhoods omega_l of the coarse nodes
  that are not clamped (the paper's experiments).  R_i selects the free DOFs
  of the nodes strictly inside D'_i, plus nodes on the physical boundary
  inside its closure, so K_i = R_i K R_i^T is the principal submatrix;
* partition of unity chi_l: the coarse bilinear / trilinear hat functions;
* heat eigenproblem (Section 4.1): -div(kappa grad psi) = lambda kappa psi
  on omega_l with kappa = E, Neumann on the boundary of omega_l except at
  clamped nodes, which are removed; consistent kappa-weighted mass matrix;
* automatic threshold: keep lambda with lambda * H^2 < tau in ascending
  order, at most kmax of them, H the coarse block edge (longest axis);
* rotation enrichment (Section 4.2): add chi_l times each infinitesimal
  rotation about the coarse node (1 in 2D, 3 in 3D, scaled by 1/H) when the
  neighbourhood selected at least one heat mode; clamped DOFs are zeroed.
"""
from __future__ import annotations

import dataclasses
import itertools

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .fem import (assemble_scalar, assemble_stiffness, elasticity_element,
                  heat_element, simp_modulus)

# omega with at most this many nodes is solved with a dense LAPACK eigh
DENSE_EIG_MAX = 1600


# --------------------------------------------------------------------------
# geometry
# --------------------------------------------------------------------------

def _blocks_per_axis(desc):
    nb = []
    for n, s in zip(desc["nel"], desc["sub_nel"]):
        if s <= 0 or n % s:
            raise ValueError("mesh size must be a multiple of the block size")
        nb.append(n // s)
    return nb


def coarse_node_grid(desc):
    """Multi-indices of the coarse nodes (block corners), x fastest."""
    nb = _blocks_per_axis(desc)
    ranges = [range(b + 1) for b in nb]
    return [tuple(reversed(t)) for t in itertools.product(*reversed(ranges))]


def _node_box_from_elements(e_lo, e_hi, nel):
    """Included node range [lo, hi] for the element range [e_lo, e_hi):
    strictly interior nodes plus nodes on the physical boundary."""
    lo = e_lo if e_lo == 0 else e_lo + 1
    hi = e_hi if e_hi == nel else e_hi - 1
    return lo, hi


def _node_ids_of_box(desc, box):
    nel = desc["nel"]
    axes = [np.arange(lo, hi + 1) for lo, hi in box]
    g = np.meshgrid(*axes, indexing="ij")
    flat = [np.ascontiguousarray(a.transpose()).ravel() for a in g]
    ids = np.zeros_like(flat[0])
    stride = 1
    for d in range(desc["dim"]):
        ids += flat[d] * stride
        stride *= nel[d] + 1
    return ids, flat


def _node_is_clamped(desc, fixed, ijk):
    dim = desc["dim"]
    nel = desc["nel"]
    p = 0
    stride = 1
    for d in range(dim):
        p += ijk[d] * stride
        stride *= nel[d] + 1
    return bool(np.all(fixed[dim * p:dim * p + dim] == 1))


def subdomain_node_boxes(desc, fixed):
    """Inclusive node boxes of the overlapping subdomains D'_i (Section 2)."""
    dim = desc["dim"]
    nel = desc["nel"]
    S = desc["sub_nel"]
    nb = _blocks_per_axis(desc)
    delta = desc["overlap"]
    boxes = []
    if desc["sub_mode"] == 0:
        for b in itertools.product(*[range(v) for v in reversed(nb)]):
            b = tuple(reversed(b))
            box = []
            for d in range(dim):
                e_lo = max(0, b[d] * S[d] - delta)
                e_hi = min(nel[d], (b[d] + 1) * S[d] + delta)
                box.append(_node_box_from_elements(e_lo, e_hi, nel[d]))
            boxes.append(tuple(box))
    else:
        for c in coarse_node_grid(desc):
            pos = tuple(c[d] * S[d] for d in range(dim))
            if _node_is_clamped(desc, fixed, pos):
                continue
            box = []
            for d in range(dim):
                e_lo = max(0, (c[d] - 1) * S[d])
                e_hi = min(nel[d], (c[d] + 1) * S[d])
                box.append(_node_box_from_elements(e_lo, e_hi, nel[d]))
            boxes.append(tuple(box))
    return boxes


def neighbourhood(desc, c):
    """omega_l of coarse node ``c``: (element box, closed node box)."""
    nel = desc["nel"]
    S = desc["sub_nel"]
    ebox, nbox = [], []
    for d in range(desc["dim"]):
        e_lo = max(0, (c[d] - 1) * S[d])
        e_hi = min(nel[d], (c[d] + 1) * S[d])
        ebox.append((e_lo, e_hi))
        nbox.append((e_lo, e_hi))
    return tuple(ebox), tuple(nbox)


def partition_of_unity(desc, c, node_xyz):
    """chi_l: coarse multilinear hat of coarse node ``c`` at integer node
    coordinates ``node_xyz`` (list of per-axis arrays)."""
    S = desc["sub_nel"]
    chi = np.ones_like(node_xyz[0], dtype=np.float64)
    for d in range(desc["dim"]):
        chi *= np.maximum(0.0, 1.0 - np.abs(node_xyz[d] - c[d] * S[d]) / S[d])
    return chi


def coarse_H(desc):
    return max(desc["sub_nel"]) * desc["h"]


# --------------------------------------------------------------------------
# heat eigenproblems and the automatic threshold
# --------------------------------------------------------------------------

def heat_pencil(desc, E, c, dirichlet_nodes=None):
    """(A_l, M_l, node ids) of the heat pencil on omega_l (Section 4.1).

    A_l = sum_e E_e int grad N grad N, M_l = sum_e E_e int N N over the
    elements of omega_l; nodes listed in ``dirichlet_nodes`` (global ids)
    are removed.  Returned node ids are global, in omega's x-fastest order.
    """
    dim = desc["dim"]
    nel = desc["nel"]
    ebox, nbox = neighbourhood(desc, c)
    Ae, Me = heat_element(dim, desc["h"])
    node_ids, _ = _node_ids_of_box(desc, nbox)
    shape = [hi - lo + 1 for lo, hi in nbox]
    # local element -> local node map
    eaxes = [np.arange(lo, hi) for lo, hi in ebox]
    g = np.meshgrid(*eaxes, indexing="ij")
    ecoord = [np.ascontiguousarray(a.transpose()).ravel() for a in g]
    estride = [1]
    for d in range(dim - 1):
        estride.append(estride[-1] * nel[d])
    eid = sum(ecoord[d] * estride[d] for d in range(dim))
    lstride = [1]
    for d in range(dim - 1):
        lstride.append(lstride[-1] * shape[d])
    lbase = sum((ecoord[d] - nbox[d][0]) * lstride[d] for d in range(dim))
    loc = np.empty((len(eid), 2 ** dim), dtype=np.int64)
    for a in range(2 ** dim):
        loc[:, a] = lbase + sum(((a >> d) & 1) * lstride[d] for d in range(dim))
    kappa = np.asarray(E)[eid]
    n = len(node_ids)
    A = assemble_scalar(loc, kappa, Ae, n)
    M = assemble_scalar(loc, kappa, Me, n)
    keep = np.ones(n, dtype=bool)
    if dirichlet_nodes is not None and len(dirichlet_nodes):
        keep &= ~np.isin(node_ids, dirichlet_nodes)
    idx = np.nonzero(keep)[0]
    return A[idx][:, idx].tocsc(), M[idx][:, idx].tocsc(), node_ids[idx]


@dataclasses.dataclass
class HeatModes:
    lam: np.ndarray        # selected eigenvalues, ascending
    vecs: np.ndarray       # (n, k) M-orthonormal eigenvectors
    lam_seen: np.ndarray   # all eigenvalues computed (ascending)
    cap_hit: bool          # more than kmax eigenvalues lie below threshold


def heat_modes(A, M, tau, H, kmax):
    """Eigenpairs of A psi = lambda M psi with lambda * H^2 < tau, ascending,
    at most kmax (the automatic threshold of Sections 2.1 and 4.1).

    Small pencils use LAPACK's dense symmetric-definite solver; larger ones
    use ARPACK in shift-invert mode about a point just below zero for the
    kmax + 1 eigenvalues of smallest magnitude, which is enough to decide
    both the selection and whether the cap was hit.
    """
    n = A.shape[0]
    if n == 0:
        return HeatModes(np.zeros(0), np.zeros((0, 0)), np.zeros(0), False)
    lim = tau / (H * H)
    if n <= DENSE_EIG_MAX:
        lam, vec = sla.eigh(A.toarray(), M.toarray())
    else:
        k = min(kmax + 1, n - 1)
        sigma = -1e-3 / (H * H)
        rng = np.random.default_rng(12345)
        lam, vec = spla.eigsh(A, k=k, M=M, sigma=sigma, which="LM", tol=0.0,
                              v0=rng.standard_normal(n), maxiter=100000)
        order = np.argsort(lam)
        lam, vec = lam[order], vec[:, order]
    below = np.nonzero(lam < lim)[0]
    cap_hit = len(below) > kmax
    sel = below[:kmax]
    vec = vec[:, sel]
    # M-orthonormalise (eigh / eigsh already are, up to rounding)
    if vec.shape[1]:
        G = vec.T @ (M @ vec)
        L = np.linalg.cholesky(0.5 * (G + G.T))
        vec = np.linalg.solve(L, vec.T).T
    return HeatModes(lam[sel], vec, lam, cap_hit)


# --------------------------------------------------------------------------
# the randomized approximation of the heat eigenproblems (Section 3, the
# randomized algorithm, applied to the heat pencil as in Section 4.3)
# --------------------------------------------------------------------------

# Reading: the paper's local solves K u = f with zero-mean forcings f are
# posed on the Neumann pencil's singular operator; here they use the
# regularised operator A + SHIFT/H^2 M (1/40 of the threshold tau/H^2 = 2/H^2),
# u = (A + sigma M)^{-1} M f, which samples the same low eigenspace (the
# pencil's eigenvectors with weights 1 / (lambda + sigma)).  The forcings
# keep zero M-mean, and the constant function (the heat operator's null
# space, its analogue of the rigid-body modes) is added to the snapshots.
RAND_SHIFT = 0.05

_SM_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_SM_C1 = np.uint64(0xBF58476D1CE4E5B9)
_SM_C2 = np.uint64(0x94D049BB133111EB)


def splitmix64(state):
    """The output of the SplitMix64 generator (Steele, Lea and Flood,
    "Fast splittable pseudorandom number generators", OOPSLA 2014) whose
    state is ``state`` before the step: z = state + gamma, then the
    variant-13 mix.  uint64 in, uint64 out (arithmetic mod 2^64)."""
    with np.errstate(over="ignore"):
        z = np.asarray(state, dtype=np.uint64) + _SM_GAMMA
        z = (z ^ (z >> np.uint64(30))) * _SM_C1
        z = (z ^ (z >> np.uint64(27))) * _SM_C2
    return z ^ (z >> np.uint64(31))


def forcing_uniform(seed, l, j, p):
    """Uniform forcing values in [-1, 1) for neighbourhood l, snapshot j and
    box-local node positions p: the SplitMix64 output at state
    key ^ (seed * gamma) with key = l * 2^40 + j * 2^24 + p, top 53 bits."""
    p = np.asarray(p, dtype=np.uint64)
    key = (np.uint64(l) << np.uint64(40)) | (np.uint64(j) << np.uint64(24)) | p
    with np.errstate(over="ignore"):
        z = splitmix64(key ^ (np.uint64(seed) * _SM_GAMMA))
    return (z >> np.uint64(11)).astype(np.float64) * (2.0 / 9007199254740992.0) - 1.0


def heat_modes_randomized(A, M, tau, H, kmax, nsnap, seed, l, pos):
    """Approximate eigenpairs of A psi = lambda M psi by the randomized
    algorithm of Section 3: nsnap zero-mean random forcings f_j on omega_l
    (uniform, positions ``pos`` in omega's node box), local solutions u_j,
    the space W = span{u_j} + span{1}, an M-orthonormal basis Q of W from the
    eigendecomposition of its Gram matrix (the SVD of the snapshots in the M
    inner product; directions below 1e-13 of the largest dropped), and the
    reduced pencil Q^T A Q.  The Ritz values below tau / H^2 are selected,
    ascending, at most kmax."""
    n = A.shape[0]
    if n == 0:
        return HeatModes(np.zeros(0), np.zeros((0, 0)), np.zeros(0), False)
    lim = tau / (H * H)
    one = np.ones(n)
    F = np.stack([forcing_uniform(seed, l, j, pos) for j in range(nsnap)], axis=1)
    w = M @ one
    F = F - np.outer(one, (w @ F) / (w @ one))          # 1^T M f_j = 0
    C = (A + (RAND_SHIFT / (H * H)) * M).tocsc()
    U = spla.splu(C).solve(np.asarray(M @ F))
    U = np.hstack([U, one[:, None]])
    G = U.T @ (M @ U)
    g, V = np.linalg.eigh(0.5 * (G + G.T))
    keep = g > 1e-13 * g[-1]
    Q = (U @ V[:, keep]) / np.sqrt(g[keep])[None, :]
    Ar = Q.T @ (A @ Q)
    lam, phi = np.linalg.eigh(0.5 * (Ar + Ar.T))
    vec = Q @ phi
    below = np.nonzero(lam < lim)[0]
    cap_hit = len(below) > kmax
    sel = below[:kmax]
    return HeatModes(lam[sel], vec[:, sel], lam, cap_hit)


def _rotations(desc, c, node_flat):
    """Infinitesimal rotations about coarse node ``c`` scaled by 1/H, as a
    list of (n_nodes, dim) arrays (rigid body rotations of Section 2.1)."""
    dim = desc["dim"]
    S = desc["sub_nel"]
    h = desc["h"]
    H = coarse_H(desc)
    rel = [(node_flat[d] - c[d] * S[d]) * h / H for d in range(dim)]
    z = np.zeros_like(rel[0])
    if dim == 2:
        return [np.stack([-rel[1], rel[0]], axis=1)]
    x, y, w = rel
    return [np.stack([z, -w, y], axis=1), np.stack([w, z, -x], axis=1),
            np.stack([-y, x, z], axis=1)]


@dataclasses.dataclass
class CoarseSpace:
    Phi: sp.csc_matrix            # (n, N_c) coarse basis on all DOFs
    n_modes: np.ndarray           # (n_coarse_nodes, dim) selected heat modes
    n_rot: np.ndarray             # (n_coarse_nodes,) rotation columns added
    eigvals: list                 # per coarse node: list over components
    lam_seen: list                # per coarse node: list over components
    cap_hits: int
    coarse_nodes: list


def build_coarse_basis(desc, E, fixed, rot=None):
    """R_0^T = [Phi_1 ... Phi_Nc] of M_EH(+Rot) (Sections 2.1, 4.1, 4.2);
    with desc["eig_random"] = M > 0 the heat eigenpairs are the randomized
    approximations of Section 3 from M snapshots (M_EH+Rot;Rand).

    Column order: coarse nodes x-fastest; per node, for each component c the
    selected heat modes chi_l psi_j e_c in ascending eigenvalue order, then
    the rotations chi_l r_k.
    """
    dim = desc["dim"]
    rot = desc["rot_enrich"] if rot is None else rot
    H = coarse_H(desc)
    tau, kmax = desc["eig_tau"], desc["eig_kmax"]
    n = len(fixed)
    nodes = coarse_node_grid(desc)
    rows, cols, vals = [], [], []
    n_modes = np.zeros((len(nodes), dim), dtype=np.int64)
    n_rot = np.zeros(len(nodes), dtype=np.int64)
    eigvals, seen = [], []
    cap_hits = 0
    col = 0
    fixed = np.asarray(fixed)
    for li, c in enumerate(nodes):
        _, nbox = neighbourhood(desc, c)
        node_ids, flat = _node_ids_of_box(desc, nbox)
        chi = partition_of_unity(desc, c, flat)
        cache = {}
        ev_l, seen_l, modes_l = [], [], []
        for comp in range(dim):
            dn = node_ids[fixed[dim * node_ids + comp] == 1]
            key = tuple(dn.tolist())
            if key not in cache:
                A, M, kept = heat_pencil(desc, E, c, dn)
                if desc.get("eig_random", 0) > 0:
                    pos = np.searchsorted(node_ids, kept)
                    hm = heat_modes_randomized(A, M, tau, H, kmax,
                                               desc["eig_random"],
                                               desc.get("eig_seed", 0), li, pos)
                else:
                    hm = heat_modes(A, M, tau, H, kmax)
                cache[key] = (hm, kept)
            hm, kept = cache[key]
            ev_l.append(hm.lam)
            seen_l.append(hm.lam_seen)
            modes_l.append((hm, kept))
            n_modes[li, comp] = len(hm.lam)
            cap_hits += int(hm.cap_hit)
        eigvals.append(ev_l)
        seen.append(seen_l)
        pos = {int(g): i for i, g in enumerate(node_ids)}
        for comp in range(dim):
            hm, kept = modes_l[comp]
            kidx = np.array([pos[int(g)] for g in kept], dtype=np.int64)
            for j in range(hm.vecs.shape[1]):
                v = chi[kidx] * hm.vecs[:, j]
                nz = v != 0.0
                rows.append(dim * kept[nz] + comp)
                cols.append(np.full(int(nz.sum()), col))
                vals.append(v[nz])
                col += 1
        if rot and n_modes[li].max() >= 1:
            for r in _rotations(desc, c, flat):
                v = (chi[:, None] * r)
                dofs = (dim * node_ids[:, None] + np.arange(dim)[None, :])
                v = v.ravel()
                dofs = dofs.ravel()
                keep = (fixed[dofs] == 0) & (v != 0.0)
                rows.append(dofs[keep])
                cols.append(np.full(int(keep.sum()), col))
                vals.append(v[keep])
                col += 1
                n_rot[li] += 1
    if col:
        Phi = sp.csc_matrix((np.concatenate(vals),
                             (np.concatenate(rows), np.concatenate(cols))),
                            shape=(n, col))
    else:
        Phi = sp.csc_matrix((n, 0))
    return CoarseSpace(Phi, n_modes, n_rot, eigvals, seen, cap_hits, nodes)


# --------------------------------------------------------------------------
# M_EE: the coarse space of local elasticity eigenproblems (Section 2.1)
# --------------------------------------------------------------------------

def elasticity_pencil(desc, E, c, fixed):
    """(K_l, M_l, DOF ids) of the elasticity pencil on omega_l (Section 2.1:
    -div sigma(psi) = lambda E psi, homogeneous Neumann on the boundary of
    omega_l, Dirichlet on its clamped part).

    K_l = sum_e E_e K^_e and M_l = sum_e E_e (M^_e on every displacement
    component) over the elements of omega_l; clamped DOFs are removed.
    Returned DOF ids are global (dim * node + component), in omega's
    x-fastest node order.
    """
    dim = desc["dim"]
    nel = desc["nel"]
    ebox, nbox = neighbourhood(desc, c)
    Ke = elasticity_element(dim, desc["nu"], desc["h"])
    _, Ms = heat_element(dim, desc["h"])
    nv = 2 ** dim
    Me = np.zeros((dim * nv, dim * nv))
    for comp in range(dim):
        Me[comp::dim, comp::dim] = Ms
    node_ids, _ = _node_ids_of_box(desc, nbox)
    shape = [hi - lo + 1 for lo, hi in nbox]
    eaxes = [np.arange(lo, hi) for lo, hi in ebox]
    g = np.meshgrid(*eaxes, indexing="ij")
    ecoord = [np.ascontiguousarray(a.transpose()).ravel() for a in g]
    estride = [1]
    for d in range(dim - 1):
        estride.append(estride[-1] * nel[d])
    eid = sum(ecoord[d] * estride[d] for d in range(dim))
    lstride = [1]
    for d in range(dim - 1):
        lstride.append(lstride[-1] * shape[d])
    lbase = sum((ecoord[d] - nbox[d][0]) * lstride[d] for d in range(dim))
    loc = np.empty((len(eid), dim * nv), dtype=np.int64)
    for a in range(nv):
        ln = lbase + sum(((a >> d) & 1) * lstride[d] for d in range(dim))
        for comp in range(dim):
            loc[:, dim * a + comp] = dim * ln + comp
    kappa = np.asarray(E)[eid]
    n = dim * len(node_ids)
    K = assemble_scalar(loc, kappa, Ke, n)
    M = assemble_scalar(loc, kappa, Me, n)
    dofs = (dim * node_ids[:, None] + np.arange(dim)[None, :]).ravel()
    idx = np.nonzero(np.asarray(fixed)[dofs] == 0)[0]
    return K[idx][:, idx].tocsc(), M[idx][:, idx].tocsc(), dofs[idx]


def elasticity_modes(K, M, count, H):
    """The ``count`` lowest eigenpairs of K psi = lambda M psi, ascending,
    M-orthonormal (LAPACK for small pencils, ARPACK shift-invert about a
    point just below zero otherwise); also returns the next eigenvalue."""
    n = K.shape[0]
    if count == 0 or n == 0:
        return np.zeros(0), np.zeros((n, 0)), np.zeros(0)
    if n <= DENSE_EIG_MAX:
        lam, vec = sla.eigh(K.toarray(), M.toarray())
    else:
        k = min(count + 1, n - 1)
        rng = np.random.default_rng(12345)
        lam, vec = spla.eigsh(K, k=k, M=M, sigma=-1e-3 / (H * H), which="LM", tol=0.0,
                              v0=rng.standard_normal(n), maxiter=100000)
        order = np.argsort(lam)
        lam, vec = lam[order], vec[:, order]
    sel = min(count, n)
    v = vec[:, :sel]
    G = v.T @ (M @ v)
    L = np.linalg.cholesky(0.5 * (G + G.T))
    v = np.linalg.solve(L, v.T).T
    return lam[:sel], v, lam[: sel + 1]


def _m_orthonormal(U, M):
    """An M-orthonormal basis of span(U) from the eigendecomposition of the
    Gram matrix U^T M U (directions below 1e-13 of the largest dropped)."""
    G = U.T @ (M @ U)
    g, V = np.linalg.eigh(0.5 * (G + G.T))
    keep = g > 1e-13 * g[-1]
    return (U @ V[:, keep]) / np.sqrt(g[keep])[None, :]


def elasticity_modes_randomized(K, M, count, H, nsnap, seed, l, pos, R):
    """The randomized algorithm of Section 3 on the elasticity pencil
    (M_EE;Rand): nsnap uniform random forcings f_j (values at the box-local
    DOF positions ``pos``), each made free of net force (zero M-weighted mean
    of every displacement component: f_j M-orthogonal to the translations,
    the first dim columns of R), local solutions u_j of the shifted pencil,
    the space W = span{u_j} + span{R} (R the rigid-body motions on the
    pencil's DOFs) with the basis Section 3 describes (the singular
    directions of the snapshot matrix, enriched with the rigid-body
    motions), the reduced pencil Q^T K Q, and its ``count`` lowest Ritz
    pairs, ascending; also returns the next Ritz value."""
    n = K.shape[0]
    if count == 0 or n == 0:
        return np.zeros(0), np.zeros((n, 0)), np.zeros(0)
    dim = 2 if R.shape[1] == 3 else 3       # R: 3 motions in 2D, 6 in 3D
    F = np.stack([forcing_uniform(seed, l, j, pos) for j in range(nsnap)], axis=1)
    T = R[:, :dim]
    MT = M @ T
    F = F - T @ np.linalg.solve(T.T @ MT, MT.T @ F)
    C = (K + (RAND_SHIFT / (H * H)) * M).tocsc()
    U = spla.splu(C).solve(np.asarray(M @ F))
    # the SVD of the snapshot matrix (in the M inner product): its
    # M-orthonormal left singular directions, those below 1e-13 of the
    # largest dropped; then enriched with the rigid-body motions (each of
    # unit M-norm) and orthonormalised once more
    Qs = _m_orthonormal(U, M)
    Rn = R / np.sqrt(np.einsum("ij,ij->j", R, M @ R))[None, :]
    Q = _m_orthonormal(np.hstack([Qs, Rn]), M)
    Kr = Q.T @ (K @ Q)
    lam, phi = np.linalg.eigh(0.5 * (Kr + Kr.T))
    vec = Q @ phi
    sel = min(count, len(lam))
    return lam[:sel], vec[:, :sel], lam[:sel + 1]


def rigid_body_motions(desc, c, node_flat, dofs, node_pos):
    """The rigid-body motions on the DOFs ``dofs`` (global ids dim * node +
    component) of omega_l: the dim translations, then the infinitesimal
    rotations about coarse node ``c`` scaled by 1/H; ``node_pos`` maps each
    DOF to its node's index in the box arrays ``node_flat``."""
    dim = desc["dim"]
    comp = np.asarray(dofs) % dim
    rows = np.asarray(node_pos)
    cols = [(comp == d).astype(np.float64) for d in range(dim)]
    for r in _rotations(desc, c, node_flat):
        cols.append(r[rows, comp])
    return np.stack(cols, axis=1)


def build_coarse_basis_ee(desc, E, fixed):
    """R_0^T of M_EE (Section 2.1): per coarse node the lowest eigenpairs of
    the elasticity pencil on omega_l times chi_l.

    Reading of the mode count: the paper selects, by hand, the rigid-body
    modes of each disconnected high-stiffness region of omega_l (d(d+1)/2
    per region); the number of such regions is what the heat threshold of
    Section 4.1 counts on the same neighbourhood, so n_l = d(d+1)/2 times
    the heat modes selected there (desc["coarse_kind"] = 2: twice that, the
    "twice many eigenvectors" rows of the tables).  With desc["eig_random"]
    = M > 0 the elasticity eigenpairs are the randomized approximations of
    Section 3 from M snapshots and the rigid-body motions (M_EE;Rand); the
    heat count stays exact.  Column order: coarse nodes x-fastest, per node
    its modes in ascending eigenvalue order.
    """
    dim = desc["dim"]
    H = coarse_H(desc)
    tau, kmax = desc["eig_tau"], desc["eig_kmax"]
    mult = 2 if desc.get("coarse_kind", 1) == 2 else 1
    per_region = dim * (dim + 1) // 2
    n = len(fixed)
    fixed = np.asarray(fixed)
    nodes = coarse_node_grid(desc)
    rows, cols, vals = [], [], []
    n_modes = np.zeros((len(nodes), dim), dtype=np.int64)
    eigvals, seen = [], []
    cap_hits = 0
    col = 0
    for li, c in enumerate(nodes):
        _, nbox = neighbourhood(desc, c)
        node_ids, flat = _node_ids_of_box(desc, nbox)
        chi = partition_of_unity(desc, c, flat)
        dn = node_ids[fixed[dim * node_ids] == 1]
        A, Mh, _ = heat_pencil(desc, E, c, dn)
        hm = heat_modes(A, Mh, tau, H, kmax)
        cap_hits += int(hm.cap_hit)
        count = mult * per_region * len(hm.lam)
        K, M, dofs = elasticity_pencil(desc, E, c, fixed)
        pos = {int(g): i for i, g in enumerate(node_ids)}
        if desc.get("eig_random", 0) > 0:
            npos = np.array([pos[int(d) // dim] for d in dofs], dtype=np.int64)
            R = rigid_body_motions(desc, c, flat, dofs, npos)
            lam, vec, lam_seen = elasticity_modes_randomized(
                K, M, count, H, desc["eig_random"], desc.get("eig_seed", 0), li,
                dim * npos + dofs % dim, R)
        else:
            lam, vec, lam_seen = elasticity_modes(K, M, count, H)
        n_modes[li, :] = len(lam)
        eigvals.append([lam] * dim)
        seen.append([lam_seen] * dim)
        chi_d = chi[np.array([pos[int(d) // dim] for d in dofs], dtype=np.int64)]
        for j in range(vec.shape[1]):
            v = chi_d * vec[:, j]
            nz = v != 0.0
            rows.append(dofs[nz])
            cols.append(np.full(int(nz.sum()), col))
            vals.append(v[nz])
            col += 1
    if col:
        Phi = sp.csc_matrix((np.concatenate(vals),
                             (np.concatenate(rows), np.concatenate(cols))),
                            shape=(n, col))
    else:
        Phi = sp.csc_matrix((n, 0))
    return CoarseSpace(Phi, n_modes, np.zeros(len(nodes), np.int64), eigvals, seen,
                       cap_hits, nodes)


# --------------------------------------------------------------------------
# the preconditioner
# --------------------------------------------------------------------------

# relative cut below which a scaled coarse eigenvalue counts as zero
K0_RCOND = 1e-12


def coarse_pseudo_inverse(K0):
    """Moore-Penrose inverse of K_0 = R_0 K R_0^T after symmetric scaling to
    unit diagonal, eigenvalues below K0_RCOND * lambda_max dropped.

    The coarse columns can be linearly dependent or vanish on the free
    DOFs: when every coarse node
    carries a rotation, sum_l chi_l r_l = 0 because the coarse hats reproduce
    linear functions.  R_0^T G R_0 is the same operator (the K-orthogonal
    projection onto span R_0^T composed with K^{-1}) for every generalized
    inverse G of K_0, so the pseudo-inverse is the natural reading of
    K_0^{-1} in Section 2.  Returns (pinv, numerical rank).
    """
    d = np.diag(K0).copy()
    if np.any(d < 0.0):
        raise np.linalg.LinAlgError("coarse matrix has a negative diagonal")
    # a column with zero energy (e.g. a mode living only where chi_l = 0)
    # spans nothing: its scale is set to zero, which drops it
    s = np.zeros_like(d)
    s[d > 0.0] = 1.0 / np.sqrt(d[d > 0.0])
    K0s = K0 * s[:, None] * s[None, :]
    w, V = np.linalg.eigh(K0s)
    if w[0] < -1e-8 * w[-1]:
        raise np.linalg.LinAlgError("coarse matrix is not positive semidefinite")
    keep = w > K0_RCOND * w[-1]
    Vk = V[:, keep]
    P = (Vk / w[keep][None, :]) @ Vk.T
    return P * s[:, None] * s[None, :], int(keep.sum())


class TwoLevelSchwarz:
    """M^{-1} r = sum_i R_i^T K_i^{-1} R_i r + R_0^T K_0^{-1} R_0 r on the
    free DOFs (Section 2, two-level additive Schwarz; Section 4.3 for the
    heat coarse space with rotations).  ``level`` selects 'both', 'one' or
    'coarse'."""

    def __init__(self, K_FF, sub_idx, Phi_F, level="both"):
        self.n = K_FF.shape[0]
        self.level = level
        self.sub_idx = sub_idx
        self.factors = []
        if level in ("both", "one"):
            for idx in sub_idx:
                Ki = K_FF[idx][:, idx].tocsc()
                self.factors.append(spla.splu(Ki))
        self.Phi = Phi_F
        self.K0 = None
        if level in ("both", "coarse") and Phi_F.shape[1] > 0:
            KPhi = K_FF @ Phi_F
            K0 = (Phi_F.T @ KPhi)
            K0 = K0.toarray() if sp.issparse(K0) else np.asarray(K0)
            self.K0 = 0.5 * (K0 + K0.T)
            self.K0_pinv, self.K0_rank = coarse_pseudo_inverse(self.K0)

    def level1(self, r):
        z = np.zeros(self.n)
        for idx, lu in zip(self.sub_idx, self.factors):
            z[idx] += lu.solve(r[idx])
        return z

    def coarse(self, r):
        if self.K0 is None:
            return np.zeros(self.n)
        c = self.Phi.T @ r
        return self.Phi @ (self.K0_pinv @ c)

    def __call__(self, r):
        z = np.zeros(self.n)
        if self.level in ("both", "one"):
            z += self.level1(r)
        if self.level in ("both", "coarse"):
            z += self.coarse(r)
        return z


@dataclasses.dataclass
class Hierarchy:
    desc: dict
    E: np.ndarray
    fixed: np.ndarray
    free: np.ndarray
    K: sp.csr_matrix
    K_FF: sp.csr_matrix
    sub_boxes: list
    sub_idx: list           # free-numbering indices per subdomain
    coarse: CoarseSpace
    M: TwoLevelSchwarz


def subdomain_free_indices(desc, fixed, boxes):
    dim = desc["dim"]
    n = len(fixed)
    fmap = -np.ones(n, dtype=np.int64)
    free = np.nonzero(np.asarray(fixed) == 0)[0]
    fmap[free] = np.arange(len(free))
    out = []
    covered = np.zeros(len(free), dtype=bool)
    for box in boxes:
        ids, _ = _node_ids_of_box(desc, box)
        dofs = (dim * ids[:, None] + np.arange(dim)[None, :]).ravel()
        loc = fmap[dofs]
        loc = loc[loc >= 0]
        out.append(loc)
        covered[loc] = True
    if not covered.all():
        raise ValueError("the overlapping subdomains do not cover every free DOF")
    return out


def build_preconditioner(desc, rho, fixed, level="both", rot=None):
    """Assemble K(rho) and build M_EH+Rot (rot=1) or M_EH (rot=0), or M_EE
    when desc["coarse_kind"] is 1 or 2."""
    fixed = np.asarray(fixed, dtype=np.uint8)
    E = simp_modulus(rho, desc["E0"], desc["Emin"], desc["penal"])
    K = assemble_stiffness(desc, E)
    free = np.nonzero(fixed == 0)[0]
    K_FF = K[free][:, free].tocsr()
    boxes = subdomain_node_boxes(desc, fixed)
    sub_idx = subdomain_free_indices(desc, fixed, boxes)
    if level in ("both", "coarse") and desc.get("coarse_kind", 0) in (1, 2):
        cs = build_coarse_basis_ee(desc, E, fixed)
    elif level in ("both", "coarse"):
        cs = build_coarse_basis(desc, E, fixed, rot)
    else:
        cs = CoarseSpace(sp.csc_matrix((len(fixed), 0)),
                         np.zeros((0, desc["dim"]), np.int64),
                         np.zeros(0, np.int64), [], [], 0, [])
    Phi_F = cs.Phi[free, :].tocsc()
    M = TwoLevelSchwarz(K_FF, sub_idx, Phi_F, level)
    return Hierarchy(desc, E, fixed, free, K, K_FF, boxes, sub_idx, cs, M)
