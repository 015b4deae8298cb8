"""ORACLE -- test infrastructure only (tests, the smoke check and the bench's CPU-baseline
leg may use it; the GPU library never does).  Plain FP64 CPU reference of the GMRF
posterior path of Sec. 3.1-3.2, sharing no code with the GPU library.

Permutation convention: perm[k] is the original index of the k-th pivot, so the
factored matrix is B = Q[perm][:, perm] = P Q P^T = L L^T.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle_chol.c")
_LIB = os.path.join(_HERE, "liboracle_chol.so")
_lib = None


def build() -> str:
    """Compile the plain-C part of the oracle with gcc."""
    subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-o", _LIB, _SRC, "-lm"])
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build()
    lib = ctypes.CDLL(_LIB)
    P = ctypes.c_void_p
    i64 = ctypes.c_int64
    lib.oc_symbolic.argtypes = [i64, P, P, P, P, ctypes.POINTER(P)]
    lib.oc_symbolic.restype = i64
    lib.oc_numeric.argtypes = [i64, P, P, P, P, P, P]
    lib.oc_numeric.restype = i64
    lib.oc_lsolve.argtypes = [i64, P, P, P, P, i64]
    lib.oc_ltsolve.argtypes = [i64, P, P, P, P, i64]
    lib.oc_takahashi.argtypes = [i64, P, P, P, P]
    lib.oc_free.argtypes = [P]
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


# ---------------------------------------------------------------- conditioning (Sec. 3.1)
def assemble(Q, A, q_eps, y, b=None, mu=None):
    """Q_post = Q + A^T diag(q_eps) A and h = A^T diag(q_eps) (y - A mu - b), so that the
    posterior mean is mu + Q_post^-1 h (Sec. 3.1, eq. posterior-mean)."""
    Q = sp.csr_matrix(Q)
    A = sp.csr_matrix(A)
    r = np.asarray(y, dtype=np.float64).copy()
    if b is not None:
        r -= b
    if mu is not None:
        r -= A @ mu
    D = (A.T @ sp.diags(np.asarray(q_eps, dtype=np.float64)) @ A).tocoo()
    Qc = Q.tocoo()
    # COO sum keeps every stored entry of Q (explicit zeros included) in the pattern
    Qp = sp.coo_matrix((np.concatenate([Qc.data, D.data]),
                        (np.concatenate([Qc.row, D.row]), np.concatenate([Qc.col, D.col]))),
                       shape=Q.shape).tocsr()
    Qp.sum_duplicates()
    Qp.sort_indices()
    h = A.T @ (q_eps * r)
    return Qp, h


# ---------------------------------------------------------------- orderings
def rcm_order(Q) -> np.ndarray:
    from scipy.sparse.csgraph import reverse_cuthill_mckee
    return np.asarray(reverse_cuthill_mckee(sp.csr_matrix(Q), symmetric_mode=True),
                      dtype=np.int64)


def nd_order(coords: np.ndarray, Q, leaf: int = 64) -> np.ndarray:
    """Geometric nested dissection: split the node set at the median of the coordinate
    axis with the largest extent; the separator is the set of low-side nodes with a
    neighbour on the high side; order = [low part, high part, separator]."""
    Q = sp.csr_matrix(Q)
    n = Q.shape[0]
    indptr, indices = Q.indptr, Q.indices
    side = np.zeros(n, dtype=np.int8)
    out = []

    def rec(nodes):
        if nodes.size <= leaf:
            out.append(nodes)
            return
        X = coords[nodes]
        ext = X.max(axis=0) - X.min(axis=0)
        ax = int(np.argmax(ext))
        if ext[ax] <= 0:
            out.append(nodes)
            return
        med = np.median(X[:, ax])
        lo_mask = X[:, ax] <= med
        if lo_mask.all() or not lo_mask.any():
            lo_mask = X[:, ax] < med
            if lo_mask.all() or not lo_mask.any():
                out.append(nodes)
                return
        lo, hi = nodes[lo_mask], nodes[~lo_mask]
        side[hi] = 1
        cnt = np.diff(indptr)[lo]
        rows = np.repeat(np.arange(lo.size), cnt)
        starts = indptr[lo]
        offs = np.arange(cnt.sum()) - np.repeat(np.cumsum(cnt) - cnt, cnt)
        nb = indices[np.repeat(starts, cnt) + offs]
        touch = np.zeros(lo.size, dtype=bool)
        np.logical_or.at(touch, rows, side[nb] == 1)
        side[hi] = 0
        sep = lo[touch]
        rec(lo[~touch])
        rec(hi)
        out.append(sep)

    rec(np.arange(n, dtype=np.int64))
    perm = np.concatenate(out) if out else np.zeros(0, dtype=np.int64)
    assert perm.size == n and np.unique(perm).size == n
    return perm.astype(np.int64)


# ---------------------------------------------------------------- Cholesky (Sec. 3.2)
@dataclass
class Factor:
    n: int
    perm: np.ndarray
    parent: np.ndarray
    Lp: np.ndarray
    Li: np.ndarray
    Lx: np.ndarray

    @property
    def nnz(self) -> int:
        return int(self.Lp[-1])

    def colcounts(self) -> np.ndarray:
        return np.diff(self.Lp)

    def flops_factor(self) -> int:
        c = self.colcounts().astype(np.int64)
        return int((c * c).sum())

    def L(self) -> sp.csc_matrix:
        return sp.csc_matrix((self.Lx, self.Li, self.Lp), shape=(self.n, self.n))


class NotSPDError(ValueError):
    def __init__(self, col):
        super().__init__(f"matrix is not positive definite (pivot at original index {col})")
        self.col = col


def cholesky(Qp, perm) -> Factor:
    """P Q_post P^T = L L^T with the given pivot order."""
    lib = _load()
    Qp = sp.csr_matrix(Qp)
    n = Qp.shape[0]
    perm = np.asarray(perm, dtype=np.int64)
    B = Qp[perm][:, perm]
    Bl = sp.tril(B, format="csc")
    Bl.sort_indices()
    Bp = np.ascontiguousarray(Bl.indptr, dtype=np.int64)
    Bi = np.ascontiguousarray(Bl.indices, dtype=np.int32)
    Bx = np.ascontiguousarray(Bl.data, dtype=np.float64)
    parent = np.empty(n, dtype=np.int32)
    Lp = np.empty(n + 1, dtype=np.int64)
    li_ptr = ctypes.c_void_p()
    nnz = lib.oc_symbolic(n, _ptr(Bp), _ptr(Bi), _ptr(parent), _ptr(Lp), ctypes.byref(li_ptr))
    Li = np.ctypeslib.as_array(ctypes.cast(li_ptr, ctypes.POINTER(ctypes.c_int32)),
                               shape=(max(nnz, 1),))[:nnz].copy()
    lib.oc_free(li_ptr)
    Lx = np.zeros(nnz)
    st = lib.oc_numeric(n, _ptr(Bp), _ptr(Bi), _ptr(Bx), _ptr(Lp), _ptr(Li), _ptr(Lx))
    if st != 0:
        raise NotSPDError(int(perm[-st - 1]))
    return Factor(n, perm, parent, Lp, Li, Lx)


def logdet(F: Factor) -> float:
    """log det = 2 sum_j log L_jj, summed exactly rounded with math.fsum."""
    d = F.Lx[F.Lp[:-1]]
    return 2.0 * math.fsum(np.log(d).tolist())


def solve(F: Factor, h) -> np.ndarray:
    """x = Q^-1 h = P^T L^-T L^-1 P h (one forward, one backward solve)."""
    lib = _load()
    h = np.asarray(h, dtype=np.float64)
    k = 1 if h.ndim == 1 else h.shape[1]
    v = np.asfortranarray(h[F.perm].reshape(F.n, k), dtype=np.float64).copy(order="F")
    lib.oc_lsolve(F.n, _ptr(F.Lp), _ptr(F.Li), _ptr(F.Lx), _ptr(v), k)
    lib.oc_ltsolve(F.n, _ptr(F.Lp), _ptr(F.Li), _ptr(F.Lx), _ptr(v), k)
    x = np.empty_like(v)
    x[F.perm] = v
    return x.reshape(h.shape)


def sample(F: Factor, mu, z) -> np.ndarray:
    """x = mu + P^T L^-T z (Sec. 3.2, sampling); z is indexed in pivot order, given as
    float32 and promoted exactly."""
    lib = _load()
    z = np.asarray(z)
    k = 1 if z.ndim == 1 else z.shape[1]
    v = np.asfortranarray(z.reshape(F.n, k).astype(np.float64)).copy(order="F")
    lib.oc_ltsolve(F.n, _ptr(F.Lp), _ptr(F.Li), _ptr(F.Lx), _ptr(v), k)
    x = np.empty_like(v)
    x[F.perm] = v
    x += np.asarray(mu, dtype=np.float64).reshape(F.n, 1)
    return x.reshape(z.shape)


def selinv(F: Factor) -> np.ndarray:
    """Sigma = Q^-1 on pattern(L) by the Takahashi recursion (layout of L)."""
    lib = _load()
    S = np.zeros_like(F.Lx)
    lib.oc_takahashi(F.n, _ptr(F.Lp), _ptr(F.Li), _ptr(F.Lx), _ptr(S))
    return S


def marginal_variances(F: Factor, S=None) -> np.ndarray:
    S = selinv(F) if S is None else S
    var = np.empty(F.n)
    var[F.perm] = S[F.Lp[:-1]]
    return var


def sigma_on_pattern(F: Factor, S, Q) -> np.ndarray:
    """Values of Sigma = Q^-1 at every stored entry of Q (CSR order, both triangles).
    Needs pattern(P Q P^T) within pattern(L + L^T), which holds for any ordering."""
    Q = sp.csr_matrix(Q)
    n = F.n
    ipos = np.empty(n, dtype=np.int64)
    ipos[F.perm] = np.arange(n)
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(Q.indptr))
    pi, pj = ipos[rows], ipos[Q.indices.astype(np.int64)]
    r, c = np.maximum(pi, pj), np.minimum(pi, pj)
    keys_L = np.repeat(np.arange(n, dtype=np.int64), np.diff(F.Lp)) * n + F.Li
    keys_q = c * n + r
    pos = np.searchsorted(keys_L, keys_q)
    if np.any(keys_L[np.minimum(pos, keys_L.size - 1)] != keys_q):
        raise ValueError("pattern of Q not contained in pattern of L + L^T")
    return S[pos]


def posterior(problem, perm=None, variances=True):
    """Posterior mean, marginal variances and log det Q_post of a Problem."""
    Qp, h = assemble(problem.Q, problem.A, problem.q_eps, problem.y, problem.b,
                     problem.mu)
    if perm is None:
        perm = nd_order(problem.coords, Qp) if problem.coords is not None else rcm_order(Qp)
    F = cholesky(Qp, perm)
    x = solve(F, h)
    if problem.mu is not None:
        x = x + problem.mu
    out = dict(Qpost=Qp, h=h, factor=F, mean=x, logdet=logdet(F))
    if variances:
        S = selinv(F)
        out["sigma_L"] = S
        out["var"] = marginal_variances(F, S)
    return out


def block_logdets(F: Factor, block_ptr) -> np.ndarray:
    """Per-block log det of a block-diagonal Q (blocks given in original numbering)."""
    d = np.log(F.Lx[F.Lp[:-1]])
    owner = np.searchsorted(np.asarray(block_ptr), F.perm, side="right") - 1
    nb = len(block_ptr) - 1
    return np.array([2.0 * math.fsum(d[owner == b].tolist()) for b in range(nb)])


# ---------------------------------------------------------------- dense references
def dense_posterior(problem):
    """Tiny problems only: mean by a dense solve, variances from the dense inverse,
    log det from the eigenvalues."""
    Qp, h = assemble(problem.Q, problem.A, problem.q_eps, problem.y, problem.b,
                     problem.mu)
    D = Qp.toarray()
    x = np.linalg.solve(D, h)
    if problem.mu is not None:
        x = x + problem.mu
    Sig = np.linalg.inv(D)
    ev = np.linalg.eigvalsh(D)
    return dict(mean=x, var=np.diag(Sig).copy(), logdet=float(np.sum(np.log(ev))),
                cov=Sig, Qpost=Qp, h=h)


# ------------------------------------------- conditioning of the scaled posterior precision
U32 = 2.0 ** -24    # unit roundoff of FP32 (round to nearest)
U64 = 2.0 ** -53    # unit roundoff of FP64


def jacobi_scaled(Q):
    """D^-1/2 Q D^-1/2 with D = diag(Q): the symmetric diagonal scaling a factorisation
    in reduced precision works on (unit diagonal)."""
    Q = sp.csr_matrix(Q)
    s = 1.0 / np.sqrt(Q.diagonal())
    return sp.csr_matrix(sp.diags(s) @ Q @ sp.diags(s))


def condition_number(Q, dense_max=2000):
    """2-norm condition number lambda_max / lambda_min of the Jacobi-scaled Q (Sec. 3.2
    concerns the cost of factoring Q; the accuracy of a reduced-precision factor is
    governed by this number: a backward error E with ||E|| ~ u ||Q^|| moves the inverse
    by about kappa u relative).  Dense eigenvalues up to dense_max unknowns, else
    Lanczos for the largest and shift-invert Lanczos (sigma = 0) for the smallest.
    Returns (kappa, lambda_min, lambda_max)."""
    Qh = jacobi_scaled(Q)
    n = Qh.shape[0]
    if n <= dense_max:
        w = np.linalg.eigvalsh(Qh.toarray())
        lo, hi = float(w[0]), float(w[-1])
    else:
        import scipy.sparse.linalg as spla
        hi = float(spla.eigsh(Qh, k=1, which="LA", tol=1e-6, return_eigenvectors=False)[0])
        lo = float(spla.eigsh(sp.csc_matrix(Qh), k=1, sigma=0.0, which="LM", tol=1e-6,
                              return_eigenvectors=False)[0])
    return hi / lo, lo, hi


# ------------------------------------------------- CG sampling and Rao-Blackwellised variances
def cg_sample_rhs(R, A, q_eps, w1, w2):
    """Right-hand side of CG sampling (Sec. 3.2): with Q = R R^T and Q_post = Q + A^T Q_eps A =
    [R, A^T Q_eps^1/2] [R, A^T Q_eps^1/2]^T, the vector R w1 + A^T Q_eps^1/2 w2 for standard
    normal w1, w2 has covariance Q_post, so Q_post^-1 of it is a N(0, Q_post^-1) draw.
    w1: (r, k), w2: (m, k); returns (n, k)."""
    R = sp.csr_matrix(R)
    A = sp.csr_matrix(A)
    return R @ np.asarray(w1, dtype=np.float64) + A.T @ (np.sqrt(np.asarray(q_eps))[:, None] * np.asarray(w2))


def rbmc_variances(Q, xs):
    """Rao-Blackwellised Monte Carlo estimate of diag(Q^-1) from draws x_s ~ N(0, Q^-1)
    (the estimator the paper cites as the alternative to the Takahashi recursion, Sec. 3.2):
    x_i | x_-i ~ N(-(1/Q_ii) sum_{j != i} Q_ij x_j, 1/Q_ii), so
      Var(x_i) = 1/Q_ii + E[((1/Q_ii) sum_{j != i} Q_ij x_j)^2]
    with the expectation replaced by the sample mean over the columns of xs (n, k)."""
    Q = sp.csr_matrix(Q)
    xs = np.asarray(xs, dtype=np.float64)
    d = Q.diagonal()
    off = (Q - sp.diags(d)).tocsr()
    t = (off @ xs) / d[:, None]
    return 1.0 / d + np.mean(t * t, axis=1)
