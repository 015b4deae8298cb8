"""Observation operators (Sec. 3.1): regression rows A_ij = phi_j(x_i) for point data
and FEM (Galerkin) rows of an implicit-Euler PDE residual.  Input generation only."""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import fem


def _locate(mesh: fem.Mesh, pts: np.ndarray):
    """Cell index (clamped to n-2 per axis) and local coordinates in [0,1]^d."""
    d = mesh.dim
    idx = np.empty((pts.shape[0], d), dtype=np.int64)
    loc = np.empty((pts.shape[0], d))
    for a in range(d):
        t = (pts[:, a] - mesh.origin[a]) / mesh.h[a]
        i = np.clip(np.floor(t).astype(np.int64), 0, mesh.shape[a] - 2)
        idx[:, a] = i
        loc[:, a] = t - i
    return idx, loc


def _nid(mesh, idx):
    out = np.zeros(idx.shape[0], dtype=np.int64)
    stride = 1
    for a in range(mesh.dim):
        out += idx[:, a] * stride
        stride *= mesh.shape[a]
    return out


def point_weights(mesh: fem.Mesh, pts: np.ndarray):
    """P1 basis values at the points: (cols (P, d+1) int64, weights (P, d+1)).

    2D: a point with local (xi, eta), eta <= xi lies in the lower triangle
    (i,j),(i+1,j),(i+1,j+1) (the diagonal goes to the lower triangle).
    3D: Freudenthal: sort the local coordinates descending, walk the cube corner
    along the sorted axes; weights are the successive differences."""
    d = mesh.dim
    idx, loc = _locate(mesh, pts)
    P = pts.shape[0]
    cols = np.empty((P, d + 1), dtype=np.int64)
    w = np.empty((P, d + 1))
    order = np.argsort(-loc, axis=1, kind="stable")
    srt = np.take_along_axis(loc, order, axis=1)
    cur = idx.copy()
    cols[:, 0] = _nid(mesh, cur)
    w[:, 0] = 1.0 - srt[:, 0]
    for s in range(d):
        ax = order[:, s]
        cur[np.arange(P), ax] += 1
        cols[:, s + 1] = _nid(mesh, cur)
        w[:, s + 1] = (srt[:, s] - srt[:, s + 1]) if s + 1 < d else srt[:, s]
    return cols, w


def point_rows(mesh: fem.Mesh, pts: np.ndarray, n_total: int, offset=None) -> sp.csr_matrix:
    """Regression operator rows (one row per point); offset shifts the columns of each
    row (space-time: slice_index * Ns)."""
    cols, w = point_weights(mesh, pts)
    if offset is not None:
        cols = cols + np.asarray(offset, dtype=np.int64)[:, None]
    P, k = cols.shape
    rows = np.repeat(np.arange(P), k)
    A = sp.coo_matrix((w.ravel(), (rows, cols.ravel())), shape=(P, n_total)).tocsr()
    A.sum_duplicates(); A.sort_indices()
    return A


def galerkin_euler_rows(G: sp.csr_matrix, m: np.ndarray, nt: int, dt: float,
                        first_slice: int = 1) -> sp.csr_matrix:
    """FEM observation rows of the implicit-Euler PDE residual
        (G u^(k) - M~ u^(k-1)) / dt = 0   for slices k = first_slice .. nt-1 (0-based),
    keeping G's structural pattern (explicit zeros stay stored)."""
    G = G.tocsr(); G.sort_indices()
    ns = G.shape[0]
    ks = np.arange(first_slice, nt)
    nrow = ks.size * ns
    gr = np.repeat(np.arange(ns), np.diff(G.indptr))
    rows, cols, vals = [], [], []
    for r, k in enumerate(ks):
        base_r = r * ns
        rows.append(base_r + gr); cols.append(k * ns + G.indices); vals.append(G.data / dt)
        rows.append(base_r + np.arange(ns)); cols.append((k - 1) * ns + np.arange(ns))
        vals.append(-m / dt)
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(nrow, nt * ns)).tocsr()
    A.sum_duplicates(); A.sort_indices()
    return A
