"""Seeded synthetic inputs for the high-contrast SIMP elasticity state solve.

This module is shared by the CPU reference, the tests and the benchmark.  It
builds problem *definitions* only: mesh sizes, densities, clamped degrees of
freedom and nodal loads.  It contains none of the solver's arithmetic (no
element matrices, no assembly, no preconditioner, no Krylov method).

Numbering used throughout (the same at the C boundary):

* node ``(i, j[, k])`` has id ``i + (nx+1)*(j + (ny+1)*k)``;
* degree of freedom ``c`` of node ``p`` is ``dim*p + c`` (interleaved);
* element ``(i, j[, k])`` has id ``i + nx*(j + ny*k)``.

Densities follow the paper's setting of a design field bounded in [0, 1]
with void = 0 and solid = 1 (Section 1, the SIMP interpolation law).  The material
maps of the paper's experiments exist only as figures that are not available,
so the fields here are stand-ins for their *structure*: stiff channels and
inclusions that cross coarse-block boundaries at high contrast, with loads
applied on solid material (Section 5, description of the experiments).
"""
from __future__ import annotations

import dataclasses
import hashlib
import math
from typing import Optional

import numpy as np
from scipy.ndimage import gaussian_filter

__all__ = [
    "Problem", "problem_desc", "n_nodes", "n_dofs", "n_elems",
    "grf", "two_scale_grf", "threshold", "stamp_bars", "fill_hinges", "clamp_face_mask",
    "clamp_all_mask", "point_load", "face_patch_load", "force_solid_disk",
    "connect_load_path",
    "config", "config_p", "batch_configs", "perturb", "perturb_seed",
    "output_dof_load", "probe_vector",
]


# --------------------------------------------------------------------------
# problem description (mirrors the C struct msp_problem_desc)
# --------------------------------------------------------------------------

def problem_desc(dim, nel, *, sub_nel, overlap, h=1.0, E0=1.0, Emin=1e-6,
                 nu=0.3, penal=3.0, sub_mode=0, eig_tau=2.0, eig_kmax=6,
                 rot_enrich=1, precision=0, eig_random=0, eig_seed=0,
                 coarse_kind=0):
    """Return a plain dict describing a problem.

    ``sub_nel`` is the coarse block edge S in elements, ``overlap`` the number
    of element layers delta added around each block, ``sub_mode`` 0 = boxes
    D_i extended by delta, 1 = coarse-vertex neighbourhoods.  ``eig_tau`` is
    the eigenvalue threshold (lambda * H^2 < tau) and ``eig_kmax`` the cap on
    modes per neighbourhood; ``rot_enrich`` 1 adds rotations; ``precision``
    0 = FP64 local solves, 1 = FP32 local solves inside the FP64 outer CG.
    ``eig_random`` > 0 approximates the heat eigenpairs by the randomized
    method from that many snapshots (M_EH+Rot;Rand), drawn with ``eig_seed``.
    ``coarse_kind`` 0 = heat coarse space, 1 = M_EE (elasticity pencils),
    2 = M_EE with twice as many modes.
    """
    nel = tuple(int(v) for v in nel)
    sub = (sub_nel,) * dim if np.isscalar(sub_nel) else tuple(int(v) for v in sub_nel)
    if len(nel) != dim or len(sub) != dim:
        raise ValueError("nel / sub_nel must have dim entries")
    return dict(dim=int(dim), nel=nel, h=float(h), E0=float(E0),
                Emin=float(Emin), nu=float(nu), penal=float(penal),
                sub_nel=sub, overlap=int(overlap), sub_mode=int(sub_mode),
                eig_tau=float(eig_tau), eig_kmax=int(eig_kmax),
                rot_enrich=int(rot_enrich), precision=int(precision),
                eig_random=int(eig_random), eig_seed=int(eig_seed),
                coarse_kind=int(coarse_kind))


def n_nodes(desc):
    return int(np.prod([n + 1 for n in desc["nel"]]))


def n_dofs(desc):
    return desc["dim"] * n_nodes(desc)


def n_elems(desc):
    return int(np.prod(desc["nel"]))


@dataclasses.dataclass
class Problem:
    """A complete state-solve input: description, densities, BCs, load."""
    name: str
    desc: dict
    rho: np.ndarray          # (nel,) float64 in [0, 1], element order
    fixed: np.ndarray        # (n,) uint8, 1 = displacement DOF clamped to 0
    f: np.ndarray            # (n,) float64 nodal load, zero at clamped DOFs
    tol: float = 1e-8

    def with_(self, **kw):
        d = dict(self.desc)
        d.update(kw)
        return dataclasses.replace(self, desc=d)


# --------------------------------------------------------------------------
# random fields and geometric features
# --------------------------------------------------------------------------

def grf(shape, ell, rng):
    """Standardised Gaussian random field on the element grid.

    White noise smoothed by a Gaussian kernel of sigma = ell / sqrt(2), which
    gives the field a covariance length ``ell`` (in elements).  ``shape`` is
    given in (x, y[, z]) order; the returned array is indexed [x, y(, z)].
    """
    w = rng.standard_normal(shape)
    g = gaussian_filter(w, sigma=ell / math.sqrt(2.0), mode="reflect")
    return (g - g.mean()) / g.std()


def two_scale_grf(shape, ell1, ell2, rng):
    return (grf(shape, ell1, rng) + grf(shape, ell2, rng)) / math.sqrt(2.0)


def threshold(g, vf):
    """1 where g lies in the top ``vf`` fraction of its values, else 0."""
    q = np.quantile(g, 1.0 - vf)
    return (g >= q).astype(np.float64)


def _element_centres(shape):
    axes = [np.arange(n) + 0.5 for n in shape]
    return np.meshgrid(*axes, indexing="ij")


def stamp_bars(rho, nbars, widths, rng):
    """Set to solid every element whose centre is within w/2 of a segment.

    Endpoints are uniform in the box, the width w is drawn uniformly from
    ``widths``.  Works in 2D (bars) and 3D (rods).
    """
    shape = rho.shape
    dim = len(shape)
    cent = np.stack([c.ravel() for c in _element_centres(shape)], axis=1)
    hi = np.array(shape, dtype=np.float64)
    out = rho.ravel().copy()
    for _ in range(nbars):
        a = rng.uniform(0.0, 1.0, dim) * hi
        b = rng.uniform(0.0, 1.0, dim) * hi
        w = float(rng.choice(np.asarray(widths)))
        ab = b - a
        L2 = float(ab @ ab)
        if L2 == 0.0:
            t = np.zeros(len(cent))
        else:
            t = np.clip((cent - a) @ ab / L2, 0.0, 1.0)
        d = cent - (a[None, :] + t[:, None] * ab[None, :])
        out[np.einsum("ij,ij->i", d, d) <= (0.5 * w) ** 2] = 1.0
    return out.reshape(shape)


def fill_hinges(rho):
    """Remove one-node (2D) and one-edge / one-node (3D) contacts.

    With bilinear / trilinear elements two solid elements that touch only
    at a node or an edge form a hinge: the stiff phase then has mechanisms
    whose energy scales with the soft modulus.  Filtered topology
    optimisation designs do not contain such contacts, so every 2x2 (2x2x2)
    window whose solid elements are not face-connected inside the window is
    filled until none remain.  Input is indexed [x, y(, z)].
    """
    s = rho > 0.5
    dim = s.ndim
    while True:
        changed = False
        if dim == 2:
            planes = [(0, 1)]
        else:
            planes = [(0, 1), (1, 2), (0, 2)]
        for (p, q) in planes:
            t = np.moveaxis(s, (p, q), (0, 1))
            a = t[:-1, :-1]
            b = t[1:, 1:]
            c = t[1:, :-1]
            d = t[:-1, 1:]
            bad1 = a & b & ~c & ~d
            bad2 = c & d & ~a & ~b
            if bad1.any() or bad2.any():
                c |= bad1
                a |= bad2
                changed = True
        if dim == 3:
            for sx in (0, 1):
                for sy in (0, 1):
                    sl = lambda v, sgn: slice(1, None) if v ^ sgn else slice(None, -1)
                    a = s[sl(0, sx), sl(0, sy), :-1]
                    b = s[sl(1, sx), sl(1, sy), 1:]
                    # other six cells of the window must all be void
                    o = []
                    for ox in (0, 1):
                        for oy in (0, 1):
                            for oz in (0, 1):
                                if (ox, oy, oz) in ((0, 0, 0), (1, 1, 1)):
                                    continue
                                o.append(s[sl(ox, sx), sl(oy, sy),
                                           slice(1, None) if oz else slice(None, -1)])
                    lone = a & b
                    for v in o:
                        lone = lone & ~v
                    if lone.any():
                        s[sl(1, sx), sl(0, sy), :-1] |= lone
                        s[sl(1, sx), sl(1, sy), :-1] |= lone
                        changed = True
        if not changed:
            break
    return np.where(s, 1.0, np.where(rho > 0.5, 1.0, rho))


def connect_load_path(rho, load_node, width=2):
    """Make the solid under the load reach the clamped face x = 0.

    A load carried only through void material is held by the soft phase,
    which no topology-optimisation design does and which drives the
    displacement up by the contrast.  If the face-connected solid component
    that contains the element next to ``load_node`` does not touch x = 0,
    a straight bar of the given width is drawn from the load node to the
    nearest solid element of a component that does; repeated until the load
    component touches the clamped face.  Input is indexed [x, y(, z)].
    """
    from scipy import ndimage

    dim = rho.ndim
    rho = rho.copy()
    cen = [min(int(v), n - 1) for v, n in zip(load_node, rho.shape)]
    for _ in range(8):
        lab, _ = ndimage.label(rho > 0.5)      # face connectivity
        here = lab[tuple(cen)]
        ground = set(np.unique(lab[0])) - {0}
        if here in ground:
            return rho
        cand = np.argwhere(np.isin(lab, list(ground)))
        if len(cand) == 0:
            cand = np.argwhere(np.zeros(rho.shape, bool) | True)[:1] * 0
        d2 = ((cand + 0.5 - np.asarray(load_node, float)) ** 2).sum(axis=1)
        tgt = cand[int(np.argmin(d2))] + 0.5
        a = np.asarray(load_node, float)
        ab = tgt - a
        cent = np.stack([c.ravel() for c in _element_centres(rho.shape)], axis=1)
        t = np.clip((cent - a) @ ab / max(float(ab @ ab), 1e-30), 0.0, 1.0)
        dd = cent - (a[None, :] + t[:, None] * ab[None, :])
        flat = rho.ravel()
        flat[np.einsum("ij,ij->i", dd, dd) <= (0.5 * width) ** 2] = 1.0
        rho = flat.reshape(rho.shape)
        rho = fill_hinges(rho)
    return rho


def force_solid_disk(rho, centre, radius):
    """Solid material within ``radius`` (elements) of a node position."""
    cen = _element_centres(rho.shape)
    d2 = sum((c - float(x)) ** 2 for c, x in zip(cen, centre))
    rho = rho.copy()
    rho[d2 <= radius * radius] = 1.0
    return rho


def _to_element_order(rho_xyz):
    """[x, y(, z)] indexed array -> flat element order (x fastest)."""
    return np.ascontiguousarray(rho_xyz.transpose()).ravel().astype(np.float64)


# --------------------------------------------------------------------------
# boundary conditions and loads
# --------------------------------------------------------------------------

def _node_grid(desc):
    """Integer node coordinates as arrays (x fastest flat order)."""
    nel = desc["nel"]
    axes = [np.arange(n + 1) for n in nel]
    g = np.meshgrid(*axes, indexing="ij")
    return [np.ascontiguousarray(a.transpose()).ravel() for a in g]


def clamp_face_mask(desc, axis=0, side=0):
    """Clamp every DOF of the nodes on one face (2D: one edge)."""
    dim = desc["dim"]
    coord = _node_grid(desc)[axis]
    target = 0 if side == 0 else desc["nel"][axis]
    on = coord == target
    m = np.zeros(dim * len(coord), dtype=np.uint8)
    for c in range(dim):
        m[dim * np.nonzero(on)[0] + c] = 1
    return m


def clamp_all_mask(desc):
    dim = desc["dim"]
    g = _node_grid(desc)
    on = np.zeros(len(g[0]), dtype=bool)
    for ax in range(dim):
        on |= (g[ax] == 0) | (g[ax] == desc["nel"][ax])
    m = np.zeros(dim * len(g[0]), dtype=np.uint8)
    for c in range(dim):
        m[dim * np.nonzero(on)[0] + c] = 1
    return m


def node_id(desc, ijk):
    nel = desc["nel"]
    idx, stride = 0, 1
    for d, v in enumerate(ijk):
        idx += int(v) * stride
        stride *= nel[d] + 1
    return idx


def point_load(desc, ijk, comp, value, f=None):
    if f is None:
        f = np.zeros(n_dofs(desc))
    f[desc["dim"] * node_id(desc, ijk) + comp] += value
    return f


def face_patch_load(desc, lo, hi, comp, total):
    """Uniform traction on the x = nx face over nodes j, k in [lo, hi].

    Each face element of the patch passes a quarter of its force to each of
    its corner nodes, so corner / edge / interior patch nodes carry weights
    1/4, 1/2, 1 before normalisation to the stated total force.
    """
    nx = desc["nel"][0]
    f = np.zeros(n_dofs(desc))
    nel_face = (hi - lo) ** 2
    for j in range(lo, hi):
        for k in range(lo, hi):
            for dj in (0, 1):
                for dk in (0, 1):
                    p = node_id(desc, (nx, j + dj, k + dk))
                    f[3 * p + comp] += total / (4.0 * nel_face)
    return f


# --------------------------------------------------------------------------
# the named workloads
# --------------------------------------------------------------------------

def _cantilever_2d(name, nel, seed, *, ells, vf, nbars, widths, sub, overlap,
                   Emin, precision=0):
    rng = np.random.default_rng(seed)
    nx, ny = nel
    if len(ells) == 1:
        g = grf((nx, ny), ells[0], rng)
    else:
        g = two_scale_grf((nx, ny), ells[0], ells[1], rng)
    rho = threshold(g, vf)
    rho = stamp_bars(rho, nbars, widths, rng)
    rho = fill_hinges(rho)
    load = (nx, ny // 2)
    rho = force_solid_disk(rho, load, 3.0)
    rho = connect_load_path(rho, load)
    desc = problem_desc(2, nel, sub_nel=sub, overlap=overlap, Emin=Emin,
                        precision=precision, eig_kmax=KMAX_FRAGMENTED)
    fixed = clamp_face_mask(desc, axis=0, side=0)
    f = point_load(desc, load, 1, -1.0)
    f[fixed == 1] = 0.0
    return Problem(name, desc, _to_element_order(rho), fixed, f)


def _cantilever_3d(name, nel, seed, *, ell, vf, nrods, widths, sub, overlap,
                   Emin, precision=1):
    rng = np.random.default_rng(seed)
    nx, ny, nz = nel
    rho = threshold(grf((nx, ny, nz), ell, rng), vf)
    rho = stamp_bars(rho, nrods, widths, rng)
    rho = fill_hinges(rho)
    # patch of 4x4 face nodes centred on the x = nx face
    lo = ny // 2 - 1
    hi = lo + 3
    rho[nx - 3:, lo:hi, lo:hi] = 1.0
    rho = connect_load_path(rho, (nx - 0.5, lo + 1.5, lo + 1.5))
    desc = problem_desc(3, nel, sub_nel=sub, overlap=overlap, Emin=Emin,
                        precision=precision, eig_kmax=KMAX_FRAGMENTED)
    fixed = clamp_face_mask(desc, axis=0, side=0)
    f = face_patch_load(desc, lo, hi, 1, -1.0)
    f[fixed == 1] = 0.0
    return Problem(name, desc, _to_element_order(rho), fixed, f)


CONFIG1_EMIN = (1e-3, 1e-6, 1e-9)

# Cap on heat modes per neighbourhood for the random-field workloads.  The
# paper caps at 6 for its own example; with 32-element coarse blocks and a
# two-scale field the threshold selects up to ~11 modes in a neighbourhood, so
# the cap is raised to leave the selection to the threshold.
KMAX_FRAGMENTED = 16


def config(k, Emin=None, precision=None):
    """Workload ``k`` (0, 1 or 2) with seed 1000 + k."""
    seed = 1000 + k
    if k == 0:
        return _cantilever_2d("cantilever2d_64x32", (64, 32), seed, ells=(8,),
                              vf=0.4, nbars=6, widths=(1, 2), sub=16,
                              overlap=2, Emin=1e-6 if Emin is None else Emin,
                              precision=0 if precision is None else precision)
    if k == 1:
        return _cantilever_2d("cantilever2d_512x256", (512, 256), seed,
                              ells=(32, 4), vf=0.4, nbars=40,
                              widths=(1, 2, 3), sub=32, overlap=2,
                              Emin=1e-6 if Emin is None else Emin,
                              precision=0 if precision is None else precision)
    if k == 2:
        return _cantilever_3d("cantilever3d_96x48x48", (96, 48, 48), seed,
                              ell=6, vf=0.3, nrods=100, widths=(1, 2), sub=6,
                              overlap=1, Emin=1e-6 if Emin is None else Emin,
                              precision=1 if precision is None else precision)
    raise ValueError(f"no workload {k}")


def scaled_cantilever_2d(nel, seed, *, sub=32, overlap=2, Emin=1e-6,
                         precision=0):
    """A config-1 style 2D cantilever of another size (used by batches)."""
    nx, ny = nel
    nb = max(1, int(round(40 * (nx * ny) / (512 * 256))))
    return _cantilever_2d(f"cantilever2d_{nx}x{ny}", nel, seed,
                          ells=(32, 4), vf=0.4, nbars=nb, widths=(1, 2, 3),
                          sub=sub, overlap=overlap, Emin=Emin,
                          precision=precision)


def scaled_cantilever_3d(nel, seed, *, sub=6, overlap=1, Emin=1e-6, precision=1):
    """A config-2 style 3D cantilever of another size (used by serving):
    rods scaled with the volume."""
    nx, ny, nz = nel
    nr = max(1, int(round(100 * (nx * ny * nz) / (96 * 48 * 48))))
    return _cantilever_3d(f"cantilever3d_{nx}x{ny}x{nz}", nel, seed, ell=6, vf=0.3,
                          nrods=nr, widths=(1, 2), sub=sub, overlap=overlap, Emin=Emin,
                          precision=precision)


def batch_configs(count=64, seed=3, sizes=((128, 64), (256, 128), (512, 256),
                                           (768, 384)), Emin=1e-6,
                  precision=1):
    """Batch of independent 2D cantilevers of uneven size."""
    rng = np.random.default_rng(seed)
    picks = rng.integers(0, len(sizes), count)
    return [scaled_cantilever_2d(sizes[p], 3000 + j, Emin=Emin,
                                 precision=precision)
            for j, p in enumerate(picks)]


def config_p(Emin=1.0, rho=None):
    """100 x 100 square, 10 x 10 coarse blocks of 10 x 10 elements, coarse
    vertex neighbourhoods as subdomains, zero displacement on every edge and
    two unit point forces (+x at (20, 20), -x at (80, 80)), PCG to 1e-6.
    With ``rho`` None the material is homogeneous (contrast 1)."""
    desc = problem_desc(2, (100, 100), sub_nel=10, overlap=0, sub_mode=1,
                        Emin=Emin)
    if rho is None:
        rho = np.ones(100 * 100)
    fixed = clamp_all_mask(desc)
    f = point_load(desc, (20, 20), 0, 1.0)
    f = point_load(desc, (80, 80), 0, -1.0, f)
    return Problem("square2d_100x100", desc, np.asarray(rho, np.float64),
                   fixed, f, tol=1e-6)


def output_dof_load(desc, rho, fixed, seed):
    """Adjoint load of a compliant-mechanism style output: a unit load on a
    seeded free DOF whose node touches solid material (rho >= 0.5)."""
    rng = np.random.default_rng(seed)
    dim = desc["dim"]
    nel = desc["nel"]
    shape = tuple(nel)
    solid = (np.asarray(rho).reshape(shape[::-1]).transpose() >= 0.5)
    node_solid = np.zeros(tuple(n + 1 for n in shape), dtype=bool)
    for corner in np.ndindex(*(2,) * dim):
        sl = tuple(slice(c, c + n) for c, n in zip(corner, shape))
        node_solid[sl] |= solid
    flat = np.ascontiguousarray(node_solid.transpose()).ravel()
    cand = [dim * p + c for p in np.nonzero(flat)[0] for c in range(dim)
            if fixed[dim * p + c] == 0]
    f = np.zeros(n_dofs(desc))
    f[cand[int(rng.integers(len(cand)))]] = 1.0
    return f


def probe_vector(fixed, seed):
    """Seeded residual for single-step parity probes: standard normal on the
    free DOFs, zero at clamped DOFs."""
    r = np.random.default_rng(seed).standard_normal(len(fixed))
    r[np.asarray(fixed) == 1] = 0.0
    return r


def perturb_seed(run, t):
    h = hashlib.sha256(f"{run}:{t}".encode()).digest()
    return int.from_bytes(h[:8], "little")


def perturb(rho_xyz_flat, nel, seed, amplitude=0.05, ell=8):
    """Smooth seeded density perturbation, clipped to [0, 1]."""
    rng = np.random.default_rng(seed)
    g = grf(tuple(nel), ell, rng)
    g = g / np.max(np.abs(g))
    d = _to_element_order(g)
    return np.clip(rho_xyz_flat + amplitude * d, 0.0, 1.0)
