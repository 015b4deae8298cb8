"""Quadratic (P2) Lagrange elements on the structured triangulation of the unit square and the
linear-constraint boundaries of App. B (input generation, not the timed path).

Mesh: v x v vertices (h = 1/(v-1)), each cell split along its (i,j)-(i+1,j+1) diagonal; the
P2 nodes (vertices and edge midpoints) form the (2v-1) x (2v-1) grid of spacing h/2, node
id = I + (2v-1) J for grid indices (I, J).  Element matrices are computed once for the lower
and once for the upper triangle (all others are translates) with a degree-4 quadrature.

Lumped mass: the row-sum lumping of P2 triangles gives zero vertex weights, so the diagonal
of the consistent element mass is rescaled to the element area (HRZ lumping), which keeps
every weight positive.

Constraints (App. B): u_k = sum_l c_l u_h(l).  In every linear system the column of k is
added, scaled by c_l, to the columns h(l) and then zeroed.  The FEM matrices are eliminated
as in classic FEM (Sec. 2.2): the same operation on the rows too, then row k = e_k; for
homogeneous Dirichlet nodes the row operation is empty, for periodic pairs it gives the
torus operator and keeps K symmetric.  The lumped mass entry at k is set so that the
constrained unknown has a chosen small variance.  That unknown is the deviation from the constraint, decoupled from
all others; the field value at node k is u_k + sum_l c_l u_h(l) (homogeneous Dirichlet: no
h, value u_k; periodic: one h, the mirrored node, c = 1).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

# degree-4 quadrature on the reference triangle (Dunavant, 6 points), weights sum to 1/2
_QA, _QB = 0.445948490915965, 0.091576213509771
_WA, _WB = 0.223381589678011 / 2, 0.109951743655322 / 2
_QP = np.array([[_QA, _QA], [1 - 2 * _QA, _QA], [_QA, 1 - 2 * _QA],
                [_QB, _QB], [1 - 2 * _QB, _QB], [_QB, 1 - 2 * _QB]])
_QW = np.array([_WA, _WA, _WA, _WB, _WB, _WB])


def _basis(xi, eta):
    """P2 basis on the reference triangle (vertices 0: (0,0), 1: (1,0), 2: (0,1); midpoints
    3: edge 01, 4: edge 12, 5: edge 20) and its gradients w.r.t. (xi, eta)."""
    l0, l1, l2 = 1.0 - xi - eta, xi, eta
    phi = np.array([l0 * (2 * l0 - 1), l1 * (2 * l1 - 1), l2 * (2 * l2 - 1), 4 * l0 * l1, 4 * l1 * l2, 4 * l2 * l0])
    dl = np.array([[-1.0, -1.0], [1.0, 0.0], [0.0, 1.0]])
    g = np.zeros((6, 2))
    for i, li in enumerate((l0, l1, l2)):
        g[i] = (4 * li - 1) * dl[i]
    g[3] = 4 * (l0 * dl[1] + l1 * dl[0])
    g[4] = 4 * (l1 * dl[2] + l2 * dl[1])
    g[5] = 4 * (l2 * dl[0] + l0 * dl[2])
    return phi, g


def element_matrices(verts):
    """Consistent mass and stiffness of one P2 triangle with vertex coordinates verts (3, 2)."""
    B = np.array([verts[1] - verts[0], verts[2] - verts[0]]).T       # x = v0 + B (xi, eta)
    det = abs(np.linalg.det(B))
    Binv = np.linalg.inv(B)
    M = np.zeros((6, 6))
    S = np.zeros((6, 6))
    for (xi, eta), w in zip(_QP, _QW):
        phi, g = _basis(xi, eta)
        gx = g @ Binv                                                 # gradients in x
        M += w * det * np.outer(phi, phi)
        S += w * det * gx @ gx.T
    return M, S


class P2Mesh:
    def __init__(self, v: int):
        self.v = v
        self.g = 2 * v - 1                       # P2 grid points per side
        self.n = self.g * self.g
        self.h = 1.0 / (v - 1)
        I, J = np.meshgrid(np.arange(self.g), np.arange(self.g), indexing="ij")
        self.coords = np.stack([I.ravel(order="F") * self.h / 2, J.ravel(order="F") * self.h / 2], axis=1)
        ci, cj = np.meshgrid(np.arange(v - 1), np.arange(v - 1), indexing="ij")
        ci, cj = 2 * ci.ravel(order="F"), 2 * cj.ravel(order="F")
        nid = lambda a, b: a + self.g * b                              # noqa: E731
        # lower triangle (i,j),(i+1,j),(i+1,j+1); upper (i,j),(i+1,j+1),(i,j+1); local order
        # = 3 vertices then midpoints of edges 01, 12, 20
        self.lower = np.stack([nid(ci, cj), nid(ci + 2, cj), nid(ci + 2, cj + 2),
                               nid(ci + 1, cj), nid(ci + 2, cj + 1), nid(ci + 1, cj + 1)], axis=1)
        self.upper = np.stack([nid(ci, cj), nid(ci + 2, cj + 2), nid(ci, cj + 2),
                               nid(ci + 1, cj + 1), nid(ci + 1, cj + 2), nid(ci, cj + 1)], axis=1)
        h = self.h
        self.Ml, self.Sl = element_matrices(np.array([[0, 0], [h, 0], [h, h]], dtype=float))
        self.Mu, self.Su = element_matrices(np.array([[0, 0], [h, h], [0, h]], dtype=float))

    def _assemble(self, El, Eu, coef_lower=None, coef_upper=None):
        rows, cols, vals = [], [], []
        for T, E, c in ((self.lower, El, coef_lower), (self.upper, Eu, coef_upper)):
            rows.append(np.repeat(T, 6, axis=1).ravel())
            cols.append(np.tile(T, (1, 6)).ravel())
            v = np.tile(E.ravel(), (T.shape[0], 1))
            if c is not None:
                v = v * np.asarray(c, dtype=np.float64)[:, None]
            vals.append(v.ravel())
        A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                          shape=(self.n, self.n)).tocsr()
        A.sum_duplicates(); A.sort_indices()
        return A

    def stiffness(self, coef_lower=None, coef_upper=None):
        """Stiffness; with per-triangle coefficients (one per cell for each of the lower and
        upper triangles, cell id i + (v-1) j) that of -div(a grad u) for piecewise-constant a."""
        return self._assemble(self.Sl, self.Su, coef_lower, coef_upper)

    def mass(self):
        return self._assemble(self.Ml, self.Mu)

    def centroids(self):
        """Centroids of the lower and upper triangles of every cell, each (cells, 2)."""
        h = self.h
        ci, cj = np.meshgrid(np.arange(self.v - 1), np.arange(self.v - 1), indexing="ij")
        base = np.stack([ci.ravel(order="F") * h, cj.ravel(order="F") * h], axis=1)
        return base + np.array([2 * h / 3, h / 3]), base + np.array([h / 3, 2 * h / 3])

    def lumped_mass(self):
        """HRZ lumping: each element's consistent-mass diagonal scaled to the element area."""
        out = np.zeros(self.n)
        area = self.h * self.h / 2
        for T, E in ((self.lower, self.Ml), (self.upper, self.Mu)):
            d = np.diag(E) * (area / np.trace(E))
            np.add.at(out, T.ravel(), np.tile(d, T.shape[0]))
        return out

    def boundary_nodes(self):
        x = self.coords
        return np.flatnonzero(np.isclose(x[:, 0], 0) | np.isclose(x[:, 0], 1) |
                              np.isclose(x[:, 1], 0) | np.isclose(x[:, 1], 1))

    def periodic_pairs(self):
        """(k, mirror(k)) for the nodes on x = 1 or y = 1, mirrored to x = 0 / y = 0 (a torus)."""
        g = self.g
        I, J = np.arange(self.n) % g, np.arange(self.n) // g
        k = np.flatnonzero((I == g - 1) | (J == g - 1))
        mi = np.where(I[k] == g - 1, 0, I[k])
        mj = np.where(J[k] == g - 1, 0, J[k])
        return k, mi + g * mj

    def point_rows(self, pts):
        """P2 basis values at points (P, 2): CSR rows with the 6 nodes of the containing
        triangle (a point on the diagonal goes to the lower triangle)."""
        h = self.h
        t = pts / h
        i = np.clip(np.floor(t[:, 0]).astype(np.int64), 0, self.v - 2)
        j = np.clip(np.floor(t[:, 1]).astype(np.int64), 0, self.v - 2)
        a, b = t[:, 0] - i, t[:, 1] - j
        lower = b <= a
        cell = i + (self.v - 1) * j
        rows, cols, vals = [], [], []
        for r in range(pts.shape[0]):
            if lower[r]:
                xi, eta = a[r] - b[r], b[r]            # (h,0) -> xi, (h,h) -> eta... affine to reference
                phi, _ = _basis(xi, eta)
                nodes = self.lower[cell[r]]
            else:
                xi, eta = a[r], b[r] - a[r]
                phi, _ = _basis(xi, eta)
                nodes = self.upper[cell[r]]
            rows.append(np.full(6, r)); cols.append(nodes); vals.append(phi)
        A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                          shape=(pts.shape[0], self.n)).tocsr()
        A.sum_duplicates(); A.sort_indices()
        return A


def constraint_matrix(n, constrained, targets, coefs):
    """T with A T = A after the column operation of App. B: column k of A is added, scaled
    by c, to column h and then zeroed (targets < 0: no h, homogeneous Dirichlet)."""
    constrained = np.asarray(constrained, dtype=np.int64)
    targets = np.asarray(targets, dtype=np.int64)
    coefs = np.asarray(coefs, dtype=np.float64)
    keep = np.ones(n)
    keep[constrained] = 0.0
    free = np.flatnonzero(keep)
    has = targets >= 0
    rows = np.concatenate([free, constrained[has]])
    cols = np.concatenate([free, targets[has]])
    vals = np.concatenate([np.ones(free.size), coefs[has]])
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, n))


def constrain_columns(A, constrained, targets, coefs):
    """The column operation of App. B applied to any linear system matrix A."""
    A = sp.csr_matrix(A)
    out = (A @ constraint_matrix(A.shape[1], constrained, targets, coefs)).tocsr()
    out.sum_duplicates(); out.sort_indices()
    return out


def constrain_fem(K, m, constrained, targets, coefs, m_constrained):
    """Constrained FEM matrix and lumped mass, each constraint with at most one h.

    K' = T^T K T + sum_k e_k e_k^T with T of constraint_matrix: the column operation of App. B,
    the same operation on the rows (the elimination of classic FEM, which keeps K symmetric and,
    for periodic pairs, gives each mirrored node the test function of both sides), and row
    k = e_k.  The lumped mass transforms the same way and stays diagonal (m_h += c^2 m_k), with
    the entry m_constrained at k."""
    n = K.shape[0]
    T = constraint_matrix(n, constrained, targets, coefs)
    ek = np.zeros(n)
    ek[constrained] = 1.0
    Kc = (T.T @ sp.csr_matrix(K) @ T + sp.diags(ek)).tocsr()
    Kc.sum_duplicates(); Kc.eliminate_zeros(); Kc.sort_indices()
    mc = np.asarray((T.T @ sp.diags(np.asarray(m, dtype=np.float64)) @ T).diagonal()).ravel().copy()
    mc[constrained] = m_constrained
    return Kc, mc
