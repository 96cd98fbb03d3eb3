"""Finite-element pieces of the oracle: SIMP, element matrices, assembly.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Element-local numbering: vertex ``a = ax + 2*ay (+ 4*az)`` with
``ax, ay, az`` in {0, 1}; local DOF ``dim*a + c``.  Global numbering is the
one of ``inputs``: node ``i + (nx+1)*(j + (ny+1)*k)``, DOF ``dim*node + c``,
element ``i + nx*(j + ny*k)``.
"""
from __future__ import annotations

import itertools
import math

import numpy as np
import scipy.sparse as sp


def simp_modulus(rho, E0, Emin, penal):
    """SIMP law of Section 1: E_e = Emin + rho_e^p (E0 - Emin)."""
    rho = np.asarray(rho, dtype=np.float64)
    return Emin + rho ** penal * (E0 - Emin)


# --------------------------------------------------------------------------
# element matrices by Gauss quadrature (2 points per axis: exact on bricks,
# the integrands being polynomials of degree <= 2 in each variable)
# --------------------------------------------------------------------------

_GP = (0.5 - 0.5 / math.sqrt(3.0), 0.5 + 0.5 / math.sqrt(3.0))


def _shape(dim, xi):
    """Values and reference gradients of the 2^dim multilinear functions."""
    nv = 2 ** dim
    N = np.empty(nv)
    dN = np.empty((nv, dim))
    for a in range(nv):
        bits = [(a >> d) & 1 for d in range(dim)]
        f = [xi[d] if bits[d] else 1.0 - xi[d] for d in range(dim)]
        g = [1.0 if bits[d] else -1.0 for d in range(dim)]
        N[a] = np.prod(f)
        for d in range(dim):
            dN[a, d] = g[d] * np.prod([f[e] for e in range(dim) if e != d])
    return N, dN


def constitutive(dim, nu):
    """C0: the material tensor at unit Young's modulus (Section 1.1).

    2D is plane stress; 3D uses the Lame constants of E = 1.  Voigt order
    2D: (xx, yy, xy); 3D: (xx, yy, zz, xy, yz, zx), engineering shears.
    """
    if dim == 2:
        return (1.0 / (1.0 - nu * nu)) * np.array(
            [[1.0, nu, 0.0], [nu, 1.0, 0.0], [0.0, 0.0, 0.5 * (1.0 - nu)]])
    lam = nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = 1.0 / (2.0 * (1.0 + nu))
    C = np.zeros((6, 6))
    C[:3, :3] = lam
    C[np.arange(3), np.arange(3)] += 2.0 * mu
    C[3, 3] = C[4, 4] = C[5, 5] = mu
    return C


def _strain_matrix(dim, dNdx):
    nv = dNdx.shape[0]
    if dim == 2:
        B = np.zeros((3, 2 * nv))
        for a in range(nv):
            B[0, 2 * a] = dNdx[a, 0]
            B[1, 2 * a + 1] = dNdx[a, 1]
            B[2, 2 * a] = dNdx[a, 1]
            B[2, 2 * a + 1] = dNdx[a, 0]
        return B
    B = np.zeros((6, 3 * nv))
    for a in range(nv):
        gx, gy, gz = dNdx[a]
        B[0, 3 * a] = gx
        B[1, 3 * a + 1] = gy
        B[2, 3 * a + 2] = gz
        B[3, 3 * a] = gy
        B[3, 3 * a + 1] = gx
        B[4, 3 * a + 1] = gz
        B[4, 3 * a + 2] = gy
        B[5, 3 * a] = gz
        B[5, 3 * a + 2] = gx
    return B


def elasticity_element(dim, nu, h=1.0):
    """Unit-modulus element stiffness K^_e = int B^T C0 B over an h-brick."""
    C = constitutive(dim, nu)
    nd = dim * 2 ** dim
    K = np.zeros((nd, nd))
    for xi in itertools.product(_GP, repeat=dim):
        _, dN = _shape(dim, xi)
        B = _strain_matrix(dim, dN / h)
        K += (0.5 ** dim) * (h ** dim) * (B.T @ C @ B)
    return K


def heat_element(dim, h=1.0):
    """Unit-coefficient scalar stiffness int grad N . grad N and consistent
    mass int N N^T on an h-brick (heat eigenproblem of Section 4.1)."""
    nv = 2 ** dim
    A = np.zeros((nv, nv))
    M = np.zeros((nv, nv))
    for xi in itertools.product(_GP, repeat=dim):
        N, dN = _shape(dim, xi)
        w = (0.5 ** dim) * (h ** dim)
        g = dN / h
        A += w * (g @ g.T)
        M += w * np.outer(N, N)
    return A, M


# --------------------------------------------------------------------------
# mesh helpers and assembly
# --------------------------------------------------------------------------

def node_coords(desc):
    """(n_nodes, dim) physical node coordinates, node order of ``inputs``."""
    nel = desc["nel"]
    axes = [np.arange(n + 1) * desc["h"] for n in nel]
    g = np.meshgrid(*axes, indexing="ij")
    return np.stack([np.ascontiguousarray(a.transpose()).ravel() for a in g],
                    axis=1)


def element_node_ids(desc):
    """(n_elems, 2^dim) global node ids of each element's vertices."""
    dim = desc["dim"]
    nel = desc["nel"]
    strides = [1]
    for d in range(dim - 1):
        strides.append(strides[-1] * (nel[d] + 1))
    axes = [np.arange(n) for n in nel]
    g = np.meshgrid(*axes, indexing="ij")
    base = sum(np.ascontiguousarray(a.transpose()).ravel() * s
               for a, s in zip(g, strides))
    out = np.empty((base.size, 2 ** dim), dtype=np.int64)
    for a in range(2 ** dim):
        off = sum(((a >> d) & 1) * strides[d] for d in range(dim))
        out[:, a] = base + off
    return out


def element_dof_ids(desc):
    dim = desc["dim"]
    nodes = element_node_ids(desc)
    dofs = np.empty((nodes.shape[0], dim * nodes.shape[1]), dtype=np.int64)
    for a in range(nodes.shape[1]):
        for c in range(dim):
            dofs[:, dim * a + c] = dim * nodes[:, a] + c
    return dofs


def assemble_stiffness(desc, E):
    """Global K = sum_e E_e P_e^T K^_e P_e (no boundary conditions)."""
    dim = desc["dim"]
    Ke = elasticity_element(dim, desc["nu"], desc["h"])
    dofs = element_dof_ids(desc)
    nd = Ke.shape[0]
    rows = np.repeat(dofs, nd, axis=1).ravel()
    cols = np.tile(dofs, (1, nd)).ravel()
    vals = (np.asarray(E)[:, None] * Ke.ravel()[None, :]).ravel()
    n = dim * int(np.prod([v + 1 for v in desc["nel"]]))
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, n))


def assemble_scalar(node_ids, coeff, Ae, n):
    """sum_e coeff_e P_e^T Ae P_e for scalar (one DOF per node) problems.

    ``node_ids`` (m, 2^dim) uses a local node numbering 0..n-1."""
    nv = Ae.shape[0]
    rows = np.repeat(node_ids, nv, axis=1).ravel()
    cols = np.tile(node_ids, (1, nv)).ravel()
    vals = (np.asarray(coeff)[:, None] * Ae.ravel()[None, :]).ravel()
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, n))


def rigid_body_modes(desc):
    """Columns spanning RBM(Omega): translations and infinitesimal rotations
    (Section 2.1; 3 modes in 2D, 6 in 3D), interleaved DOF order."""
    dim = desc["dim"]
    X = node_coords(desc)
    nn = X.shape[0]
    cols = []
    for c in range(dim):
        v = np.zeros((nn, dim))
        v[:, c] = 1.0
        cols.append(v.ravel())
    if dim == 2:
        v = np.stack([-X[:, 1], X[:, 0]], axis=1)
        cols.append(v.ravel())
    else:
        x, y, z = X[:, 0], X[:, 1], X[:, 2]
        zero = np.zeros(nn)
        cols.append(np.stack([zero, -z, y], axis=1).ravel())
        cols.append(np.stack([z, zero, -x], axis=1).ravel())
        cols.append(np.stack([-y, x, zero], axis=1).ravel())
    return np.stack(cols, axis=1)
