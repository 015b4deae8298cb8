"""ORACLE -- test infrastructure only.  Log marginal likelihood of the observations and
its gradient with respect to hyper-parameters, in FP64 on the CPU.

lml_dense: the plain definition for tiny problems -- with mu = 0,
    y ~ N(b, A Q^-1 A^T + Q_eps^-1)   (the covariance form of the conditioning of Sec. 3.1),
    log p(y) = -1/2 r^T S^-1 r - 1/2 log det S - M/2 log 2 pi, r = y - b.
lml_sparse: the same value through the GMRF identity
    log p(y) = log p(y|u) + log p(u) - log p(u|y) at u = mu_post,
with log-dets from the oracle's sparse Cholesky factors (Sec. 3.2) of Q and Q_post, and the
gradient for given derivative matrices (dQ on Q's pattern, dq_eps diagonal):
    dLML = 1/2 tr(Q^-1 dQ) + 1/2 sum(dq_eps / q_eps) - 1/2 tr(Q_post^-1 (dQ + A^T diag(dq_eps) A))
           - 1/2 mu^T dQ mu - 1/2 sum(dq_eps r^2),
the traces read from the Takahashi selected inverses on the pattern (Sec. 3.2).  When the
observation operator depends on the parameter too (Galerkin PDE rows built from the
space-time operator G, Sec. 2.4 and 3.1), a derivative dA of A adds
    + r^T Q_eps dA mu      and   dQ_post += dA^T Q_eps A + A^T Q_eps dA
(the identity holds for every u, so at u = mu_post only the explicit dependence remains).
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp

from . import core


def lml_dense(Q, A, q_eps, y, b=None):
    Qd = sp.csr_matrix(Q).toarray()
    Ad = sp.csr_matrix(A).toarray()
    M = Ad.shape[0]
    Sy = Ad @ np.linalg.solve(Qd, Ad.T) + np.diag(1.0 / np.asarray(q_eps))
    r = np.asarray(y, dtype=np.float64) - (0.0 if b is None else b)
    sign, ld = np.linalg.slogdet(Sy)
    assert sign > 0
    return float(-0.5 * r @ np.linalg.solve(Sy, r) - 0.5 * ld - 0.5 * M * math.log(2.0 * math.pi))


def lml_sparse(Q, A, q_eps, y, b=None, coords=None, derivs=()):
    """Returns (LML, [dLML for each (dQ, dq_eps) in derivs], parts dict)."""
    Q = sp.csr_matrix(Q)
    A = sp.csr_matrix(A)
    q_eps = np.asarray(q_eps, dtype=np.float64)
    M = A.shape[0]
    perm = core.nd_order(coords, Q) if coords is not None else core.rcm_order(Q)
    F0 = core.cholesky(Q, perm)
    Qp, h = core.assemble(Q, A, q_eps, y, b)
    F1 = core.cholesky(Qp, perm)
    mu = core.solve(F1, h)
    r = np.asarray(y, dtype=np.float64) - (0.0 if b is None else b) - A @ mu
    quad = float(mu @ (Q @ mu))
    misfit = float(np.sum(q_eps * r * r))
    ld0, ld1 = core.logdet(F0), core.logdet(F1)
    lml = (-0.5 * M * math.log(2.0 * math.pi) + 0.5 * ld0 + 0.5 * math.fsum(np.log(q_eps).tolist())
           - 0.5 * ld1 - 0.5 * quad - 0.5 * misfit)
    grads = []
    if derivs:
        S0 = core.selinv(F0)
        S1 = core.selinv(F1)
        for dv in derivs:
            dQ, dqe = dv[0], dv[1]
            dA = sp.csr_matrix(dv[2]) if len(dv) > 2 and dv[2] is not None else None
            dQ = sp.csr_matrix(dQ)
            dqe = np.zeros(M) if dqe is None else np.asarray(dqe, dtype=np.float64)
            tr0 = float(np.dot(core.sigma_on_pattern(F0, S0, dQ), dQ.data)) if dQ.nnz else 0.0
            D1 = dQ + A.T @ sp.diags(dqe) @ A
            if dA is not None:
                D1 = D1 + dA.T @ sp.diags(q_eps) @ A + A.T @ sp.diags(q_eps) @ dA
            D1 = sp.csr_matrix(D1)
            D1.sum_duplicates()
            tr1 = float(np.dot(core.sigma_on_pattern(F1, S1, D1), D1.data)) if D1.nnz else 0.0
            g = (0.5 * tr0 + 0.5 * float(np.sum(dqe / q_eps)) - 0.5 * tr1
                 - 0.5 * float(mu @ (dQ @ mu)) - 0.5 * float(np.sum(dqe * r * r)))
            if dA is not None:
                g += float((q_eps * r) @ (dA @ mu))
            grads.append(g)
    return lml, grads, dict(mu=mu, r=r, quad=quad, misfit=misfit, logdet_prior=ld0, logdet_post=ld1)
