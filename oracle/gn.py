"""ORACLE -- test infrastructure only.  Gauss-Newton for the Galerkin implicit-Euler
Burgers residual and for residuals with a pointwise power nonlinearity (the lumped
Galerkin rows of -Laplace u + u^3 = f) (Sec. 3.3), one step at a time from a given
iterate, in FP64 on the CPU.

The step from u: linearise f(v) ~ f(u) + J (v - u); the minimiser of the linearised
objective 1/2 v^T Q v + 1/2 (f(u) + J (v - u) - y)^T Q_eps (...) is the affine posterior
mean with A = J, b = f(u) - J u (Sec. 3.1); d = x - u; backtracking line search on
phi(v) = 1/2 v^T Q v + 1/2 (f(v) - y)^T Q_eps (f(v) - y) with Armijo constant 1e-4 over
alpha = 1, 1/2, ..., 1/128, the first that passes; when none passes the step is not taken
(alpha = 0: the direction carries no decrease the arithmetic can resolve, so the iterate
is kept and the objective never increases).  Newton decrement lambda^2 = -grad phi(u)^T d.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import core


def burgers_residual_and_jacobian(u, nx, nt, dt, nu, mass, S, nonlinear=True):
    """f(u) with rows [initial condition (nx); PDE residual for slices 1..nt-1] and its
    Jacobian (CSR, same rows)."""
    U = np.asarray(u, dtype=np.float64).reshape(nt, nx)
    S = sp.csr_matrix(S)
    uk, ukm = U[1:], U[:-1]
    um = np.zeros_like(uk); um[:, 1:] = uk[:, :-1]
    up = np.zeros_like(uk); up[:, :-1] = uk[:, 1:]
    c = 1.0 if nonlinear else 0.0
    B = c * (up * up + uk * up - um * uk - um * um) / 6.0
    f_pde = mass[None, :] * (uk - ukm) / dt + nu * (S @ uk.T).T + B
    f = np.concatenate([U[0], f_pde.ravel()])
    blocks = []
    Nrow = nx * nt
    J = sp.lil_matrix((Nrow, nx * nt))
    # build J from sparse blocks: identity on slice 0, then per slice k
    I0 = sp.hstack([sp.eye(nx), sp.csr_matrix((nx, nx * (nt - 1)))])
    blocks.append(I0)
    for k in range(1, nt):
        u_k = U[k]
        u_m = np.concatenate([[0.0], u_k[:-1]])
        u_p = np.concatenate([u_k[1:], [0.0]])
        left = c * (-u_k - 2.0 * u_m) / 6.0
        diag = c * (u_p - u_m) / 6.0
        right = c * (2.0 * u_p + u_k) / 6.0
        dB = sp.diags([left[1:], diag, right[:-1]], [-1, 0, 1], shape=(nx, nx))
        Jk = sp.diags(mass / dt) + nu * S + dB
        Jkm = -sp.diags(mass / dt)
        row = [sp.csr_matrix((nx, nx)) for _ in range(nt)]
        row[k - 1] = Jkm
        row[k] = Jk
        blocks.append(sp.hstack(row))
    J = sp.vstack(blocks, format="csr")
    return f, J


def objective(Q, u, f, y, q_eps):
    r = f - y
    return 0.5 * float(u @ (Q @ u)) + 0.5 * float(np.sum(q_eps * r * r))


def gn_step(Q, u, y, q_eps, nx, nt, dt, nu, mass, S, perm=None, nonlinear=True):
    """One Gauss-Newton step with line search; returns (new iterate, record dict)."""
    Q = sp.csr_matrix(Q)
    f, J = burgers_residual_and_jacobian(u, nx, nt, dt, nu, mass, S, nonlinear)
    b = f - J @ u
    Qp, h = core.assemble(Q, J, q_eps, y, b)
    if perm is None:
        perm = core.rcm_order(Qp)
    F = core.cholesky(Qp, perm)
    x = core.solve(F, h)
    d = x - u
    phi0 = objective(Q, u, f, y, q_eps)
    slope = float((Q @ u) @ d) + float(np.sum(q_eps * (f - y) * (J @ d)))
    alpha = 0.0
    for j in range(8):
        a = 2.0 ** -j
        fa, _ = burgers_residual_and_jacobian(u + a * d, nx, nt, dt, nu, mass, S, nonlinear)
        if objective(Q, u + a * d, fa, y, q_eps) <= phi0 + 1e-4 * a * slope:
            alpha = a
            break
    return u + alpha * d, dict(phi0=phi0, alpha=alpha, decrement=-slope, slope=slope, x=x)


def pointwise_residual_and_jacobian(u, A_lin, nl_col, nl_coef, power):
    """f(u) = A_lin u + c * u[j]^p per row (c = nl_coef, j = nl_col; rows with j < 0 are
    linear) and its Jacobian A_lin + diag-placed p c u[j]^(p-1) (CSR, A_lin's rows)."""
    u = np.asarray(u, dtype=np.float64)
    A = sp.csr_matrix(A_lin)
    nl = np.flatnonzero(np.asarray(nl_col) >= 0)
    j = np.asarray(nl_col)[nl]
    c = np.asarray(nl_coef, dtype=np.float64)[nl]
    f = A @ u
    f[nl] += c * u[j] ** power
    D = sp.csr_matrix((power * c * u[j] ** (power - 1), (nl, j)), shape=A.shape)
    return f, (A + D).tocsr()


def gn_step_pointwise(Q, u, y, q_eps, A_lin, nl_col, nl_coef, power, perm=None):
    """One Gauss-Newton step with the same line search as gn_step, for the residual of
    pointwise_residual_and_jacobian; returns (new iterate, record dict)."""
    Q = sp.csr_matrix(Q)
    fun = lambda v: pointwise_residual_and_jacobian(v, A_lin, nl_col, nl_coef, power)  # noqa: E731
    f, J = fun(u)
    b = f - J @ u
    Qp, h = core.assemble(Q, J, q_eps, y, b)
    if perm is None:
        perm = core.rcm_order(Qp)
    F = core.cholesky(Qp, perm)
    x = core.solve(F, h)
    d = x - u
    phi0 = objective(Q, u, f, y, q_eps)
    slope = float((Q @ u) @ d) + float(np.sum(q_eps * (f - y) * (J @ d)))
    alpha = 0.0
    for k in range(8):
        a = 2.0 ** -k
        fa, _ = fun(u + a * d)
        if objective(Q, u + a * d, fa, y, q_eps) <= phi0 + 1e-4 * a * slope:
            alpha = a
            break
    return u + alpha * d, dict(phi0=phi0, alpha=alpha, decrement=-slope, slope=slope, x=x)
