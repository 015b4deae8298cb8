"""SPDE priors as sparse precision matrices (input generation, not the timed path).

* Whittle-Matern (Sec. 2.2, eq. whittle-matern-spde and eq. sparse-prec-matrix):
  alpha = 2, (kappa^2 - Laplace) u = tau W  =>  K = kappa^2 M~ + S,
  Q = tau^-2 K M~^-1 K  (lumped mass M~, 2-ring pattern).
* Space-time prior from implicit Euler in time + FEM in space (Sec. 2.4 eq. st-ssm,
  App. A eq. block-tridiag-prec). With uniform step dt, G = M~ + dt*L_s (L_s the
  FEM matrix of the spatial operator), A = G^-1 M~, F = tau^2 dt G^-1 M~ Sigma M~ G^-T
  (the conditional covariance of u^(k+1) given u^(k)); then, with no inverse formed,
      F^-1      = tau^-2 dt^-1 G^T M~^-1 Sigma^-1 M~^-1 G
      A^T F^-1 A = tau^-2 dt^-1 Sigma^-1
      F^-1 A    = tau^-2 dt^-1 G^T M~^-1 Sigma^-1
  and the blocks are (1,1) = Q1 + A^T F^-1 A, (k,k) = F^-1 + A^T F^-1 A for
  1<k<Nt, (Nt,Nt) = F^-1, (k+1,k) = -F^-1 A, (k,k+1) = its transpose.
  Q1 is read as a precision (the (1,1) block adds Q1 itself).
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp

from . import fem


def _pattern(X) -> sp.csr_matrix:
    """Unit-valued copy of X's stored pattern (explicit zeros included)."""
    X = sp.csr_matrix(X)
    X.sum_duplicates()
    P = sp.csr_matrix((np.ones(X.indices.size), X.indices.copy(), X.indptr.copy()),
                      shape=X.shape)
    P.sort_indices()
    return P


def matern_range_to_kappa(rho: float, nu: float) -> float:
    """Effective range rho = sqrt(8 nu)/kappa (Lindgren et al. 2011)."""
    return math.sqrt(8.0 * nu) / rho


def matern_precision(mesh: fem.Mesh, kappa: float, tau: float, S=None, m=None):
    """Q = tau^-2 (kappa^2 M~ + S) M~^-1 (kappa^2 M~ + S) on the 2-ring pattern.

    Returns (Q csr, K csr, m lumped-mass vector)."""
    S = fem.stiffness(mesh) if S is None else S
    m = fem.lumped_mass(mesh) if m is None else m
    K = (S + sp.diags(kappa * kappa * m)).tocsr()
    K = fem.on_pattern(K, fem.ring_pattern(mesh, 1))
    Q = (K.T @ sp.diags(1.0 / m) @ K) / (tau * tau)
    Q = fem.on_pattern(Q, fem.ring_pattern(mesh, 2))
    return Q, K, m


def spacetime_precision(mesh: fem.Mesh, nt: int, dt: float, Ls: sp.spmatrix,
                        tau: float, Q1: sp.spmatrix, m: np.ndarray,
                        sigma_inv: sp.spmatrix | None = None):
    """Block-tridiagonal Q_ST over nt slices (slice-major ordering, slice k holds
    dofs k*Ns .. (k+1)*Ns-1).

    Ls:        FEM matrix of the spatial operator L_s (G = M~ + dt Ls).
    sigma_inv: Sigma^-1 of the spatial noise; None means white noise in space,
               for which the load covariance is M~, i.e. Sigma^-1 = M~.
    Returns (Q_ST csr with slice-structural pattern, G csr)."""
    ns = mesh.n
    Mt = sp.diags(m).tocsr()
    Minv = sp.diags(1.0 / m)
    G = (Mt + dt * Ls).tocsr()
    G = fem.on_pattern(G, _pattern(fem.ring_pattern(mesh, 1) + sp.eye(ns)))
    Sinv = Mt if sigma_inv is None else sigma_inv.tocsr()
    c = 1.0 / (tau * tau * dt)
    Finv = c * (G.T @ Minv @ Sinv @ Minv @ G)
    AtFA = c * Sinv
    FA = c * (G.T @ Minv @ Sinv)
    first = np.zeros(nt); first[0] = 1.0
    mid_a = np.ones(nt); mid_a[-1] = 0.0       # A^T F^-1 A on slices 1..nt-1
    mid_f = np.ones(nt); mid_f[0] = 0.0        # F^-1 on slices 2..nt
    sub = sp.diags([np.ones(nt - 1)], [-1], shape=(nt, nt))
    Q = (sp.kron(sp.diags(first), Q1) + sp.kron(sp.diags(mid_a), AtFA)
         + sp.kron(sp.diags(mid_f), Finv) - sp.kron(sub, FA) - sp.kron(sub.T, FA.T))
    Q = Q.tocsr()
    # Structural pattern from products of unit-valued patterns (all terms positive, so
    # no cancellation): diagonal blocks = pat(G)^T pat(Sigma^-1) pat(G) + pat(Q1) +
    # pat(Sigma^-1); off-diagonal blocks = pat(G)^T pat(Sigma^-1).
    PG = _pattern(G)
    PS = _pattern(Sinv)
    Pd = _pattern(PG.T @ PS @ PG + _pattern(Q1) + PS)
    Po = _pattern(PG.T @ PS)
    P = _pattern(sp.kron(sp.eye(nt), Pd) + sp.kron(sub, Po) + sp.kron(sub.T, Po.T))
    return fem.on_pattern(Q, P), G


def spacetime_precision_derivative(mesh: fem.Mesh, nt: int, dt: float, Ls: sp.spmatrix,
                                   dLs: sp.spmatrix, tau: float, m: np.ndarray,
                                   sigma_inv: sp.spmatrix | None = None) -> sp.csr_matrix:
    """dQ_ST for a change dLs of the spatial operator (Q1 and Sigma^-1 held fixed):
    with G = M~ + dt Ls, dG = dt dLs and W = M~^-1 Sigma^-1 M~^-1,
        d(F^-1)   = tau^-2 dt^-1 (dG^T W G + G^T W dG)
        d(F^-1 A) = tau^-2 dt^-1 dG^T M~^-1 Sigma^-1
        d(A^T F^-1 A) = 0,
    placed in the blocks of Q_ST like spacetime_precision (unstructured pattern; callers
    put it on Q's pattern)."""
    ns = mesh.n
    Mt = sp.diags(m).tocsr()
    Minv = sp.diags(1.0 / m)
    P1 = _pattern(fem.ring_pattern(mesh, 1) + sp.eye(ns))
    G = fem.on_pattern((Mt + dt * Ls).tocsr(), P1)
    dG = fem.on_pattern((dt * dLs).tocsr(), P1)
    Sinv = Mt if sigma_inv is None else sigma_inv.tocsr()
    c = 1.0 / (tau * tau * dt)
    W = Minv @ Sinv @ Minv
    dFinv = c * (dG.T @ W @ G + G.T @ W @ dG)
    dFA = c * (dG.T @ Minv @ Sinv)
    mid_f = np.ones(nt); mid_f[0] = 0.0
    sub = sp.diags([np.ones(nt - 1)], [-1], shape=(nt, nt))
    dQ = sp.kron(sp.diags(mid_f), dFinv) - sp.kron(sub, dFA) - sp.kron(sub.T, dFA.T)
    return dQ.tocsr()


def matern_precision_alpha3(mesh: fem.Mesh, kappa: float, tau: float, S=None, m=None):
    """(kappa^2 - Laplace)^(3/2) u = tau W (alpha = 3, i.e. nu = 2 in 2D):
    Q = tau^-2 K M~^-1 K M~^-1 K on the 3-ring pattern, K = kappa^2 M~ + S."""
    S = fem.stiffness(mesh) if S is None else S
    m = fem.lumped_mass(mesh) if m is None else m
    K = fem.on_pattern((S + sp.diags(kappa * kappa * m)).tocsr(), fem.ring_pattern(mesh, 1))
    Mi = sp.diags(1.0 / m)
    Q = (K.T @ Mi @ K @ Mi @ K) / (tau * tau)
    Q = fem.on_pattern(Q.tocsr(), fem.ring_pattern(mesh, 3))
    return Q, K, m
