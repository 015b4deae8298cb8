"""P1 finite elements on structured meshes of the unit interval, square and cube.

Input generation only: these matrices build the SPDE priors of Sec. 2.2-2.4 and
App. A that the posterior path consumes; nothing here is on the timed path.

Conventions (fixed readings, see the design notes):
  * nodes sit on a uniform grid, node id = i0 + n0*(i1 + n1*i2) (first axis fastest);
  * 2D cells are split along the (i,j)-(i+1,j+1) diagonal into two triangles;
  * 3D cells use the Kuhn/Freudenthal split into 6 tetrahedra (one per axis
    permutation), whose edges are the 7 non-zero 0/1 vectors;
  * the mass matrix is lumped: M~_ii = sum over elements T containing i of |T|/(d+1);
  * matrix patterns are mesh-structural: every pair of nodes sharing an element
    is a stored entry even when its value is exactly zero (the P1 Laplacian
    vanishes on right-angle hypotenuses).
"""
from __future__ import annotations

import itertools
import math
from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp


@dataclass
class Mesh:
    dim: int
    shape: tuple          # nodes per axis
    h: tuple              # spacing per axis
    origin: tuple
    coords: np.ndarray    # (N, dim) float64
    elems: np.ndarray     # (E, dim+1) int64 vertex ids
    vol: float            # volume of every element (uniform mesh)

    @property
    def n(self) -> int:
        return int(self.coords.shape[0])


def structured_mesh(shape, lo=None, hi=None) -> Mesh:
    shape = tuple(int(s) for s in shape)
    d = len(shape)
    lo = (0.0,) * d if lo is None else tuple(lo)
    hi = (1.0,) * d if hi is None else tuple(hi)
    h = tuple((hi[a] - lo[a]) / (shape[a] - 1) for a in range(d))
    axes = [lo[a] + h[a] * np.arange(shape[a]) for a in range(d)]
    grid = np.meshgrid(*axes, indexing="ij")
    # node id with the first axis fastest -> flatten in Fortran order
    coords = np.stack([g.ravel(order="F") for g in grid], axis=1)

    def nid(idx):
        out = np.zeros_like(idx[0])
        stride = 1
        for a in range(d):
            out = out + idx[a] * stride
            stride *= shape[a]
        return out

    cells = np.meshgrid(*[np.arange(s - 1) for s in shape], indexing="ij")
    cells = [c.ravel(order="F") for c in cells]
    elems = []
    if d == 1:
        elems.append(np.stack([nid([cells[0]]), nid([cells[0] + 1])], axis=1))
    elif d == 2:
        i, j = cells
        a = nid([i, j]); b = nid([i + 1, j]); c = nid([i + 1, j + 1]); e = nid([i, j + 1])
        elems.append(np.stack([a, b, c], axis=1))
        elems.append(np.stack([a, c, e], axis=1))
    elif d == 3:
        for perm in itertools.permutations(range(3)):
            cur = [c.copy() for c in cells]
            verts = [nid(cur)]
            for ax in perm:
                cur[ax] = cur[ax] + 1
                verts.append(nid(cur))
            elems.append(np.stack(verts, axis=1))
    else:
        raise ValueError("dim must be 1, 2 or 3")
    elems = np.concatenate(elems, axis=0).astype(np.int64)
    vol = float(np.prod(h)) / math.factorial(d)
    return Mesh(d, shape, h, lo, coords, elems, vol)


def _p1_gradients(mesh: Mesh) -> np.ndarray:
    """Gradients of the d+1 barycentric basis functions on every element, (E, d+1, d)."""
    X = mesh.coords[mesh.elems]                      # (E, d+1, d)
    B = X[:, 1:, :] - X[:, :1, :]                    # (E, d, d) rows = edge vectors
    Binv = np.linalg.inv(B)                          # grad(phi_k) for k>=1 are columns of B^-T
    g = np.empty((X.shape[0], mesh.dim + 1, mesh.dim))
    g[:, 1:, :] = np.transpose(Binv, (0, 2, 1))
    g[:, 0, :] = -g[:, 1:, :].sum(axis=1)
    return g


def _assemble(mesh: Mesh, local: np.ndarray) -> sp.csr_matrix:
    E, k = mesh.elems.shape
    rows = np.repeat(mesh.elems, k, axis=1).ravel()
    cols = np.tile(mesh.elems, (1, k)).ravel()
    A = sp.coo_matrix((local.ravel(), (rows, cols)), shape=(mesh.n, mesh.n)).tocsr()
    A.sum_duplicates()   # keeps explicit zeros: the pattern stays mesh-structural
    A.sort_indices()
    return A


def stiffness(mesh: Mesh) -> sp.csr_matrix:
    """S_ij = integral grad(phi_i) . grad(phi_j) (P1 Laplacian, natural boundary)."""
    g = _p1_gradients(mesh)
    local = mesh.vol * np.einsum("eid,ejd->eij", g, g)
    return _assemble(mesh, local)


def convection(mesh: Mesh, axis: int = 0) -> sp.csr_matrix:
    """C_ij = integral phi_i d(phi_j)/dx_axis (non-symmetric)."""
    g = _p1_gradients(mesh)
    k = mesh.dim + 1
    local = (mesh.vol / k) * np.broadcast_to(g[:, None, :, axis], (g.shape[0], k, k))
    return _assemble(mesh, np.ascontiguousarray(local))


def lumped_mass(mesh: Mesh) -> np.ndarray:
    """Diagonal of the lumped mass matrix: sum over elements of |T|/(d+1)."""
    m = np.zeros(mesh.n)
    np.add.at(m, mesh.elems.ravel(), mesh.vol / (mesh.dim + 1))
    return m


def element_adjacency(mesh: Mesh) -> sp.csr_matrix:
    """Boolean node graph: i~j iff i and j share an element (diagonal included)."""
    k = mesh.dim + 1
    E = mesh.elems.shape[0]
    A = _assemble(mesh, np.ones((E, k, k)))
    A.data[:] = 1.0
    return A


def ring_pattern(mesh: Mesh, r: int) -> sp.csr_matrix:
    """Structural r-ring pattern (graph power r of the element adjacency), values 1."""
    A = element_adjacency(mesh)
    P = A.copy()
    for _ in range(r - 1):
        P = (P @ A).tocsr()
        P.data[:] = 1.0
    P.sort_indices()
    return P


def on_pattern(M: sp.spmatrix, P: sp.csr_matrix) -> sp.csr_matrix:
    """Return M's values placed on the (super)pattern P; entries of P absent in M are 0.

    Raises if M has an entry outside P."""
    M = M.tocsr(); M.sum_duplicates(); M.sort_indices()
    P = P.tocsr(); P.sort_indices()
    n = P.shape[1]
    pr = np.repeat(np.arange(P.shape[0], dtype=np.int64), np.diff(P.indptr))
    pk = pr * n + P.indices
    mr = np.repeat(np.arange(M.shape[0], dtype=np.int64), np.diff(M.indptr))
    mk = mr * n + M.indices
    pos = np.searchsorted(pk, mk)
    if np.any(pos >= pk.size) or np.any(pk[np.minimum(pos, pk.size - 1)] != mk):
        raise ValueError("matrix has entries outside the structural pattern")
    vals = np.zeros(pk.size)
    vals[pos] = M.data
    out = sp.csr_matrix((vals, P.indices.copy(), P.indptr.copy()), shape=P.shape)
    return out
