"""Seeded synthetic workloads.  Every random number is drawn here with NumPy PCG64 from
a fixed seed, so the GPU path and the oracle see identical inputs.

Workloads (sizes are parameters so tests can shrink them with the same structure):
  matern2d      2D Matern prior (Sec. 2.2), P1 on an s x s grid, uniform point data
                on a seeded smooth target.                        (default 32x32)
  advdiff_st    space-time advection-diffusion prior (Sec. 2.3-2.4, App. A) on an
                ns x ns grid x nt implicit-Euler slices, white noise in space,
                Galerkin PDE rows on slices 2..nt plus 1% point data.  (128x128x64)
  matern_batch  many independent 2D Matern GMRFs of uneven size stacked block-
                diagonally.                                      (256 problems)
  matern3d      3D Matern prior on a Kuhn-split cube grid with point data. (64^3)
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import fem, obs, priors


@dataclass
class Problem:
    """Prior N(mu, Q^-1) and likelihood y | u ~ N(A u + b, Q_eps^-1) with diagonal Q_eps.

    CSR arrays: int64 row pointers, int32 column indices, float64 values; Q stores both
    triangles with a symmetric pattern."""
    n: int
    Q: sp.csr_matrix
    A: sp.csr_matrix
    q_eps: np.ndarray
    y: np.ndarray
    b: np.ndarray
    coords: np.ndarray
    block_ptr: np.ndarray | None = None
    mu: np.ndarray | None = None
    meta: dict = field(default_factory=dict)

    def csr(self, which: str):
        M = self.Q if which == "Q" else self.A
        return (np.ascontiguousarray(M.indptr, dtype=np.int64),
                np.ascontiguousarray(M.indices, dtype=np.int32),
                np.ascontiguousarray(M.data, dtype=np.float64))


def rng_for(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def smooth_target(rng: np.random.Generator, dim: int, terms: int = 8):
    """u*(x) = sum_k a_k cos(2 pi w_k . x + phi_k), a_k ~ N(0,1)/k, w_k in {1..4}^d,
    phi_k ~ U[0, 2 pi)."""
    a = rng.standard_normal(terms) / np.arange(1, terms + 1)
    w = rng.integers(1, 5, size=(terms, dim))
    phi = rng.uniform(0.0, 2.0 * math.pi, size=terms)

    def f(x):
        x = np.atleast_2d(x)
        return (a[None, :] * np.cos(2.0 * math.pi * (x @ w.T) + phi[None, :])).sum(axis=1)
    return f


def _sym_clean(Q: sp.csr_matrix) -> sp.csr_matrix:
    """Exact symmetrisation of values (the products above are symmetric only up to
    rounding); pattern must already be symmetric."""
    Qt = Q.T.tocsr(); Qt.sort_indices()
    if not (np.array_equal(Q.indptr, Qt.indptr) and np.array_equal(Q.indices, Qt.indices)):
        raise ValueError("pattern is not symmetric")
    return sp.csr_matrix((0.5 * (Q.data + Qt.data), Q.indices.copy(), Q.indptr.copy()),
                         shape=Q.shape)


def matern2d(side: int = 32, kappa: float = 5.0, tau: float = 1.0, n_obs: int = 100,
             sigma: float = 0.01, seed: int = 1) -> Problem:
    rng = rng_for(seed)
    mesh = fem.structured_mesh((side, side))
    Q, K, m = priors.matern_precision(mesh, kappa, tau)
    Q = _sym_clean(Q)
    target = smooth_target(rng, 2)
    pts = rng.uniform(0.0, 1.0, size=(n_obs, 2))
    A = obs.point_rows(mesh, pts, mesh.n)
    y = target(pts) + sigma * rng.standard_normal(n_obs)
    return Problem(mesh.n, Q, A, np.full(n_obs, 1.0 / sigma**2), y, np.zeros(n_obs),
                   mesh.coords.copy(),
                   meta=dict(workload="matern2d", side=side, kappa=kappa, tau=tau,
                             n_obs=n_obs, sigma=sigma, seed=seed, K=K, m=m, mesh=mesh))


def advdiff_spacetime(ns: int = 128, nt: int = 64, c: float = 0.5, nu: float = 0.01,
                      tau: float = 1.0, kappa1: float = 10.0, sigma_pde: float = 1e-3,
                      sigma: float = 1e-3, obs_frac: float = 0.01, seed: int = 2,
                      pde_rows: bool = True, noise: str = "white",
                      noise_range: float = 0.1) -> Problem:
    """du/dt + c du/dx - nu Laplace u = tau W on [0,1]^2 x [0,1]: Nt slices, dt=1/(Nt-1).
    Q1 = 2D Matern (alpha=2) with kappa1 and unit marginal variance
    tau1 = 1/(sqrt(4 pi) kappa1).  Observations: Galerkin implicit-Euler residual rows
    (G u^k - M~ u^(k-1))/dt = 0 on slices 2..Nt with noise sigma_pde, plus
    ceil(obs_frac N) points at uniform locations and uniform slice indices with noise
    sigma; the data come from the noiseless implicit-Euler FEM solution started from
    the seeded smooth target.

    noise = "white": white noise in space, Sigma^-1 = M~.  noise = "matern": spatial
    Matern noise (App. A), Sigma^-1 = Q_s = tau_s^-2 K_s M~^-1 K_s with K_s = kappa_s^2 M~ + S
    (alpha = 2, i.e. nu_s = 1 in 2D), kappa_s = sqrt(8 nu_s) / noise_range and
    tau_s = sqrt(4 pi) kappa_s (unit marginal variance tau_s^2 / (4 pi kappa_s^2)); the
    prior's blocks then reach the 4-ring (diagonal) and 3-ring (off-diagonal)."""
    rng = rng_for(seed)
    mesh = fem.structured_mesh((ns, ns))
    dt = 1.0 / (nt - 1)
    S = fem.stiffness(mesh)
    C = fem.convection(mesh, axis=0)
    m = fem.lumped_mass(mesh)
    tau1 = 1.0 / (math.sqrt(4.0 * math.pi) * kappa1)
    Q1, _, _ = priors.matern_precision(mesh, kappa1, tau1, S=S, m=m)
    Ls = nu * S + c * C
    if noise == "white":
        Sinv, kappa_s, tau_s = None, None, None
    elif noise == "matern":
        kappa_s = priors.matern_range_to_kappa(noise_range, 1.0)
        tau_s = math.sqrt(4.0 * math.pi) * kappa_s
        Sinv, _, _ = priors.matern_precision(mesh, kappa_s, tau_s, S=S, m=m)
    else:
        raise ValueError(f"unknown noise {noise!r}")
    Q, G = priors.spacetime_precision(mesh, nt, dt, Ls, tau, Q1, m, sigma_inv=Sinv)
    Q = _sym_clean(Q)
    N = ns * ns * nt
    # deterministic implicit-Euler trajectory from the smooth initial condition
    target = smooth_target(rng, 2)
    u = np.empty((nt, mesh.n))
    u[0] = target(mesh.coords)
    lu = spla.splu(G.tocsc())
    for k in range(1, nt):
        u[k] = lu.solve(m * u[k - 1])
    n_pts = int(math.ceil(obs_frac * N))
    pts = rng.uniform(0.0, 1.0, size=(n_pts, 2))
    kk = rng.integers(0, nt, size=n_pts)
    A_pt = obs.point_rows(mesh, pts, N, offset=kk * mesh.n)
    y_pt = A_pt @ u.ravel() + sigma * rng.standard_normal(n_pts)
    blocks, ys, qs = [], [], []
    if pde_rows:
        A_pde = obs.galerkin_euler_rows(G, m, nt, dt, first_slice=1)
        blocks.append(A_pde); ys.append(np.zeros(A_pde.shape[0]))
        qs.append(np.full(A_pde.shape[0], 1.0 / sigma_pde**2))
    blocks.append(A_pt); ys.append(y_pt); qs.append(np.full(n_pts, 1.0 / sigma**2))
    A = sp.vstack(blocks, format="csr")
    A.sort_indices()
    y = np.concatenate(ys)
    coords = np.concatenate([np.tile(mesh.coords, (nt, 1)),
                             np.repeat(np.arange(nt) * dt, mesh.n)[:, None]], axis=1)
    return Problem(N, Q, A, np.concatenate(qs), y, np.zeros(y.size), coords,
                   meta=dict(workload="advdiff_spacetime", ns=ns, nt=nt, dt=dt, c=c, nu=nu,
                             tau=tau, kappa1=kappa1, tau1=tau1, sigma_pde=sigma_pde,
                             sigma=sigma, n_pts=n_pts, seed=seed, G=G, m=m, Q1=Q1,
                             mesh=mesh, u_true=u, pde_rows=pde_rows, noise=noise,
                             Sigma_inv=Sinv, kappa_s=kappa_s, tau_s=tau_s))


def manufactured_cubic(x1: np.ndarray, x2: np.ndarray, terms: int = 600):
    """u*(x) = sum_{k=1}^{terms} k^-6 sin(k pi x1) sin(k pi x2) and f = -Laplace u* + u*^3 on the
    grid x1 (nx1) x x2 (nx2), as (nx1, nx2) arrays: u* vanishes on the boundary of the unit
    square and -Laplace u* = sum 2 k^2 pi^2 k^-6 sin sin."""
    k = np.arange(1, terms + 1, dtype=np.float64)
    s1 = np.sin(np.pi * k[:, None] * x1[None, :])
    s2 = np.sin(np.pi * k[:, None] * x2[None, :])
    u = s1.T @ (k[:, None] ** -6 * s2)
    lap = s1.T @ ((2.0 * np.pi**2 * k[:, None] ** -4) * s2)
    return u, lap + u**3


def elliptic_cubic(side: int = 1024, prior_range: float = 0.1, sigma_pde: float = 1e-3,
                   sigma_bdry: float | None = None, bdry_spacing: float = 1e-3) -> Problem:
    """Nonlinear elliptic -Laplace u + u^3 = f on [0, 1]^2, u = 0 on the boundary, with the
    manufactured solution of manufactured_cubic.  P1 on a side x side grid.

    Prior: Matern with effective range prior_range and nu = 2 (alpha = 3): kappa =
    sqrt(8 nu) / range, tau = sqrt(8 pi) kappa^2 (unit marginal variance
    tau^2 / (8 pi kappa^4)).  Observations (the linear part in A, the pointwise cubic in
    meta): Galerkin rows at the interior nodes i,
        f_i(u) = (S u)_i + m_i u_i^3 = m_i f(x_i)   (lumped quadrature of the cubic and the load),
    with noise sigma_pde * m_i (a pointwise residual noise sigma_pde), and the boundary
    condition as point data u(x_b) = 0 at points spaced bdry_spacing along the boundary
    with noise sigma_bdry, by default sigma_pde h^2: a Galerkin row (S u)_i has O(1)
    coefficients, so its noise sigma_pde m_i ~ sigma_pde h^2 is that size in units of u, and
    the boundary values are held as firmly as the equations.  (With a fixed sigma_bdry the
    harmonic extensions of boundary values, which the Galerkin rows do not see, are held only
    by the boundary data, and the condition number grows like h^-6 instead of h^-4.)  A holds the linear part; meta: nl_col (per row, the unknown of
    the cubic term or -1), nl_coef (m_i or 0), power 3, u_true (u* at the nodes)."""
    mesh = fem.structured_mesh((side, side))
    S = fem.stiffness(mesh)
    m = fem.lumped_mass(mesh)
    if sigma_bdry is None:
        sigma_bdry = sigma_pde / (side - 1) ** 2
    nu_m = 2.0
    kappa = math.sqrt(8.0 * nu_m) / prior_range
    tau = math.sqrt(8.0 * math.pi) * kappa * kappa
    Q, _, _ = priors.matern_precision_alpha3(mesh, kappa, tau, S=S, m=m)
    Q = _sym_clean(Q)
    x = mesh.coords
    g = np.linspace(0.0, 1.0, side)
    U, F = manufactured_cubic(g, g)
    u_true = U.ravel(order="F")          # node id = i + side * j, x1 fastest
    f_nodes = F.ravel(order="F")
    on_b = (np.isclose(x[:, 0], 0.0) | np.isclose(x[:, 0], 1.0) | np.isclose(x[:, 1], 0.0) |
            np.isclose(x[:, 1], 1.0))
    interior = np.flatnonzero(~on_b)
    A_pde = S[interior].tocsr()
    nb = int(round(1.0 / bdry_spacing))
    t = np.arange(nb) * bdry_spacing
    pts = np.concatenate([np.stack([t, np.zeros(nb)], 1), np.stack([np.ones(nb), t], 1),
                          np.stack([1.0 - t, np.ones(nb)], 1), np.stack([np.zeros(nb), 1.0 - t], 1)])
    A_bd = obs.point_rows(mesh, pts, mesh.n)
    A = sp.vstack([A_pde, A_bd], format="csr")
    A.sum_duplicates(); A.sort_indices()
    npde = interior.size
    y = np.concatenate([m[interior] * f_nodes[interior], np.zeros(A_bd.shape[0])])
    q_eps = np.concatenate([1.0 / (sigma_pde * m[interior]) ** 2, np.full(A_bd.shape[0], 1.0 / sigma_bdry**2)])
    nl_col = np.concatenate([interior, -np.ones(A_bd.shape[0], dtype=np.int64)]).astype(np.int32)
    nl_coef = np.concatenate([m[interior], np.zeros(A_bd.shape[0])])
    return Problem(mesh.n, Q, A, q_eps, y, np.zeros(y.size), mesh.coords.copy(),
                   meta=dict(workload="elliptic_cubic", side=side, kappa=kappa, tau=tau, mesh=mesh, m=m,
                             S=S, nl_col=nl_col, nl_coef=nl_coef, power=3, u_true=u_true, f=f_nodes,
                             n_pde=npde, sigma_pde=sigma_pde, sigma_bdry=sigma_bdry))


def prior_sqrt(problem: Problem) -> sp.csr_matrix:
    """A left square root R of the workload's prior precision, Q = R R^T, sparse (Sec. 3.2, CG
    sampling; App. A, square root of the space-time prior):
      Matern (alpha = 2): R = tau^-1 K M~^-1/2;
      space-time: block-bidiagonal with the slice-1 block Q1^1/2 = tau1^-1 K1 M~^-1/2 and, per
        transition k, the column block [A^T F^-1/2 on slice k; -F^-1/2 on slice k+1] with
        F^-1/2 = sqrt(c) G^T M~^-1 B, A^T F^-1/2 = sqrt(c) B, c = tau^-2 dt^-1 and Sigma^-1 = B B^T
        (white noise B = M~^1/2; Matern noise B = tau_s^-1 K_s M~^-1/2)."""
    meta = problem.meta
    if meta["workload"] == "matern2d":
        m = meta["m"]
        return sp.csr_matrix(meta["K"] @ sp.diags(1.0 / np.sqrt(m)) / meta["tau"])
    if meta["workload"] != "advdiff_spacetime":
        raise ValueError("no square root for this workload")
    mesh, nt, dt, m, G = meta["mesh"], meta["nt"], meta["dt"], meta["m"], meta["G"].tocsr()
    ns = mesh.n
    S = fem.stiffness(mesh)
    K1 = (S + sp.diags(meta["kappa1"] ** 2 * m)).tocsr()
    R1 = K1 @ sp.diags(1.0 / np.sqrt(m)) / meta["tau1"]
    if meta.get("noise", "white") == "white":
        B = sp.diags(np.sqrt(m))
    else:
        Ks = (S + sp.diags(meta["kappa_s"] ** 2 * m)).tocsr()
        B = Ks @ sp.diags(1.0 / np.sqrt(m)) / meta["tau_s"]
    c = 1.0 / (meta["tau"] ** 2 * dt)
    Fm = math.sqrt(c) * (G.T @ sp.diags(1.0 / m) @ B)
    AF = math.sqrt(c) * B
    blocks = [[None] * nt for _ in range(nt)]
    blocks[0][0] = R1
    for k in range(nt - 1):
        blocks[k][k + 1] = AF
        blocks[k + 1][k + 1] = -Fm
    for r in range(nt):
        for cc in range(nt):
            if blocks[r][cc] is None:
                blocks[r][cc] = sp.csr_matrix((ns, ns))
    R = sp.bmat(blocks, format="csr")
    R.sum_duplicates(); R.sort_indices()
    return R


def advdiff_values(problem: Problem, c: float, nu: float):
    """Values of the advection-diffusion workload's prior precision and observation
    operator at advection speed c and viscosity nu, on the workload's stored patterns
    (the data y, the noise and the point rows stay those of the workload).  Returns
    (q_data aligned with problem.Q.data, a_data aligned with problem.A.data)."""
    meta = problem.meta
    mesh, nt, dt, m = meta["mesh"], meta["nt"], meta["dt"], meta["m"]
    Ls = nu * fem.stiffness(mesh) + c * fem.convection(mesh, axis=0)
    Q, G = priors.spacetime_precision(mesh, nt, dt, Ls, meta["tau"], meta["Q1"], m,
                                      sigma_inv=meta.get("Sigma_inv"))
    q = fem.on_pattern(_sym_clean(Q), problem.Q).data
    blocks = []
    if meta.get("pde_rows", True):
        blocks.append(obs.galerkin_euler_rows(G, m, nt, dt, first_slice=1))
    npde = blocks[0].shape[0] if blocks else 0
    blocks.append(problem.A[npde:])
    a = fem.on_pattern(sp.vstack(blocks, format="csr"), problem.A).data
    return q, a


def advdiff_derivatives(problem: Problem, c: float | None = None, nu: float | None = None) -> dict:
    """Derivatives of the advection-diffusion workload's prior precision and of its
    Galerkin PDE observation rows with respect to the advection speed c and the
    viscosity nu (L_s = nu S + c C: dL_s/dc = C, dL_s/dnu = S); Q1, the noise and the
    point rows do not depend on them.  Returns {"c": (dq, da), "nu": (dq, da)} with dq
    aligned with problem.Q.data and da with problem.A.data (same stored patterns)."""
    meta = problem.meta
    mesh, nt, dt, m = meta["mesh"], meta["nt"], meta["dt"], meta["m"]
    S = fem.stiffness(mesh)
    C = fem.convection(mesh, axis=0)
    Ls = (meta["nu"] if nu is None else nu) * S + (meta["c"] if c is None else c) * C
    out = {}
    for name, dLs in (("c", C), ("nu", S)):
        dQ = priors.spacetime_precision_derivative(mesh, nt, dt, Ls, dLs, meta["tau"], m,
                                                   sigma_inv=meta.get("Sigma_inv"))
        dq = fem.on_pattern(dQ, problem.Q).data
        dQt = fem.on_pattern(dQ.T.tocsr(), problem.Q).data
        dq = 0.5 * (dq + dQt)
        blocks = []
        if meta.get("pde_rows", True):
            P1 = priors._pattern(fem.ring_pattern(mesh, 1) + sp.eye(mesh.n))
            dG = fem.on_pattern((dt * dLs).tocsr(), P1)
            blocks.append(obs.galerkin_euler_rows(dG, np.zeros(mesh.n), nt, dt, first_slice=1))
        n_pts = problem.A.shape[0] - (blocks[0].shape[0] if blocks else 0)
        blocks.append(sp.csr_matrix((n_pts, problem.n)))
        dA = sp.vstack(blocks, format="csr")
        da = fem.on_pattern(dA, problem.A).data
        out[name] = (dq, da)
    return out


def matern_batch(n_prob: int = 256, side_lo: int = 64, side_hi: int = 256,
                 kappa_lo: float = 1.0, kappa_hi: float = 20.0, tau: float = 1.0,
                 sigma: float = 0.01, seed: int = 4) -> Problem:
    """Block-diagonal stack of independent 2D Matern problems with sides ~ U{lo..hi},
    kappa ~ U[kappa_lo, kappa_hi], ceil(0.01 N_i) points each.

    Per side the FEM pieces are built once and Q is combined on the 2-ring pattern as
    Q = tau^-2 (kappa^4 M~ + 2 kappa^2 S + S M~^-1 S), i.e. K M~^-1 K with K = kappa^2 M~ + S."""
    rng = rng_for(seed)
    sides = rng.integers(side_lo, side_hi + 1, size=n_prob)
    kappas = rng.uniform(kappa_lo, kappa_hi, size=n_prob)
    cache = {}
    Qs, As, ys, qs, cs = [], [], [], [], []
    ptr = [0]
    for s_, kap in zip(sides, kappas):
        s_ = int(s_)
        if s_ not in cache:
            mesh = fem.structured_mesh((s_, s_))
            S = fem.stiffness(mesh)
            m = fem.lumped_mass(mesh)
            P2 = fem.ring_pattern(mesh, 2)
            cache[s_] = (mesh, m, P2,
                         fem.on_pattern(sp.diags(m), P2).data,
                         fem.on_pattern(S, P2).data,
                         fem.on_pattern(S @ sp.diags(1.0 / m) @ S, P2).data)
        mesh, m, P2, Md, Sd, SMSd = cache[s_]
        k2 = float(kap) ** 2
        data = (k2 * k2 * Md + 2.0 * k2 * Sd + SMSd) / (tau * tau)
        Q = sp.csr_matrix((data, P2.indices.copy(), P2.indptr.copy()), shape=P2.shape)
        target = smooth_target(rng, 2)
        npts = int(math.ceil(0.01 * mesh.n))
        pts = rng.uniform(0.0, 1.0, size=(npts, 2))
        As.append(obs.point_rows(mesh, pts, mesh.n))
        ys.append(target(pts) + sigma * rng.standard_normal(npts))
        qs.append(np.full(npts, 1.0 / sigma**2))
        Qs.append(_sym_clean(Q))
        cs.append(mesh.coords + 2.0 * len(cs))   # disjoint boxes per problem
        ptr.append(ptr[-1] + mesh.n)
    Q = sp.block_diag(Qs, format="csr"); Q.sort_indices()
    A = sp.block_diag(As, format="csr"); A.sort_indices()
    y = np.concatenate(ys)
    return Problem(ptr[-1], Q, A, np.concatenate(qs), y, np.zeros(y.size),
                   np.concatenate(cs), block_ptr=np.asarray(ptr, dtype=np.int64),
                   meta=dict(workload="matern_batch", n_prob=n_prob, sides=sides,
                             kappas=kappas, tau=tau, sigma=sigma, seed=seed))


def batch_block(problem: Problem, b: int) -> Problem:
    """The b-th independent problem of a block-diagonal batch as a Problem of its own."""
    lo, hi = int(problem.block_ptr[b]), int(problem.block_ptr[b + 1])
    Qb = problem.Q[lo:hi, lo:hi].tocsr()
    Ab_all = problem.A[:, lo:hi].tocsr()
    rows = np.flatnonzero(np.diff(Ab_all.indptr))
    Ab = Ab_all[rows].tocsr()
    return Problem(hi - lo, Qb, Ab, problem.q_eps[rows], problem.y[rows], problem.b[rows],
                   problem.coords[lo:hi], meta=dict(workload="matern_batch_block", block=b))


def matern3d(side: int = 64, kappa: float = 10.0, tau: float = 1.0, n_obs: int = 5000,
             sigma: float = 0.05, seed: int = 5) -> Problem:
    rng = rng_for(seed)
    mesh = fem.structured_mesh((side, side, side))
    Q, K, m = priors.matern_precision(mesh, kappa, tau)
    Q = _sym_clean(Q)
    target = smooth_target(rng, 3)
    pts = rng.uniform(0.0, 1.0, size=(n_obs, 3))
    A = obs.point_rows(mesh, pts, mesh.n)
    y = target(pts) + sigma * rng.standard_normal(n_obs)
    return Problem(mesh.n, Q, A, np.full(n_obs, 1.0 / sigma**2), y, np.zeros(n_obs),
                   mesh.coords.copy(),
                   meta=dict(workload="matern3d", side=side, kappa=kappa, tau=tau,
                             n_obs=n_obs, sigma=sigma, seed=seed, K=K, m=m, mesh=mesh))


def standard_normal_f32(n: int, k: int, seed: int) -> np.ndarray:
    """z ~ N(0, I) as float32, shape (n, k) column-major (Fortran order)."""
    rng = rng_for(seed)
    return np.asfortranarray(rng.standard_normal((n, k)).astype(np.float32))


def matern_pieces(problem: Problem):
    """Lumped mass, stiffness and S M~^-1 S placed on the stored pattern of a Matern
    problem's Q (arrays aligned with Q.data), from which the Matern precision of any
    (kappa, tau) is tau^-2 (kappa^4 M~ + 2 kappa^2 S + S M~^-1 S)."""
    meta = problem.meta
    K, m = meta["K"], meta["m"]
    S = (K - sp.diags(meta["kappa"] ** 2 * m)).tocsr()
    P = sp.csr_matrix((np.ones(problem.Q.nnz), problem.Q.indices, problem.Q.indptr),
                      shape=problem.Q.shape)
    Mq = fem.on_pattern(sp.diags(m), P).data
    Sq = fem.on_pattern(S, P).data
    SMSq = fem.on_pattern(S @ sp.diags(1.0 / m) @ S, P).data
    return Mq, Sq, SMSq


def matern_from_pieces(problem: Problem, pieces, kappa: float, tau: float):
    """(Q, dQ/dlog kappa) as CSR matrices on Q's pattern for the given hyper-parameters."""
    Mq, Sq, SMSq = pieces
    k2 = kappa * kappa
    q = (k2 * k2 * Mq + 2.0 * k2 * Sq + SMSq) / (tau * tau)
    dq = 4.0 * k2 * (k2 * Mq + Sq) / (tau * tau)
    mk = lambda v: sp.csr_matrix((v, problem.Q.indices.copy(), problem.Q.indptr.copy()),  # noqa: E731
                                 shape=problem.Q.shape)
    return mk(q), mk(dq)


def burgers_spacetime(nx: int = 1024, nt: int = 1024, nu: float = 0.01 / math.pi,
                      sigma_pde: float = 1e-3, sigma_ic: float = 1e-3, range_s: float = 0.02,
                      tau: float = 1.0, seed: int = 3) -> Problem:
    """Viscous Burgers u_t + u u_x = nu u_xx on [-1, 1] x [0, 1] (Sec. 2.3, 3.3).

    Prior: the linear stochastic proxy u_t - nu u_xx = tau W (the advection speed c is the
    mean of the initial condition, here 0), implicit Euler in time, P1 in space on nx
    interior nodes (homogeneous Dirichlet nodes at +-1 eliminated), spatial noise a 1D
    Matern field (alpha = 2, nu_s = 3/2) with range range_s, scaled to unit mean marginal
    variance of the discrete field, which is also the initial-slice precision.  Observations: nx initial-condition rows
    u^0_i = u0(x_i) (noise sigma_ic) and the Galerkin implicit-Euler Burgers residual rows
    on slices 2..nt (noise sigma_pde, data 0).  A holds the linearisation at u = 0; the
    library rewrites A and b at every Gauss-Newton iterate.  Initial condition
    u0 = -sin(pi x) + 0.1 sum_{k=2}^{4} a_k sin(k pi x), a_k ~ N(0, 1)."""
    rng = rng_for(seed)
    full = fem.structured_mesh((nx + 2,), lo=(-1.0,), hi=(1.0,))
    inner = np.arange(1, nx + 1)
    S = fem.stiffness(full)[inner][:, inner].tocsr()
    m = fem.lumped_mass(full)[inner]
    mesh = fem.structured_mesh((nx,), lo=(float(full.coords[1, 0]),), hi=(float(full.coords[nx, 0]),))
    dt = 1.0 / (nt - 1)
    kappa_s = priors.matern_range_to_kappa(range_s, 1.5)
    Ks = (S + sp.diags(kappa_s * kappa_s * m)).tocsr()
    Q0 = (Ks.T @ sp.diags(1.0 / m) @ Ks).tocsr()
    # tau_s gives the discrete noise field unit mean marginal variance
    tau_s = math.sqrt(1.0 / float(np.mean(np.diag(np.linalg.inv(Q0.toarray())))))
    Qs = fem.on_pattern(Q0 / (tau_s * tau_s), fem.ring_pattern(mesh, 2))
    Qs = _sym_clean(Qs)
    Q, G = priors.spacetime_precision(mesh, nt, dt, nu * S, tau, Qs, m, sigma_inv=Qs)
    Q = _sym_clean(Q)
    a = rng.standard_normal(3)
    x = full.coords[inner, 0]
    u0 = -np.sin(np.pi * x) + 0.1 * sum(a[k - 2] * np.sin(k * np.pi * x) for k in (2, 3, 4))
    # S rows as (left, diagonal, right) triplets
    s3 = np.zeros((nx, 3))
    Sd = S.toarray() if nx <= 4096 else None
    for i in range(nx):
        row = S.getrow(i)
        for j, v in zip(row.indices, row.data):
            s3[i, 1 + (j - i)] = v
    del Sd
    # A pattern and its linearisation at u = 0 (B vanishes there)
    rows, cols, vals = [], [], []
    rows.append(np.arange(nx)); cols.append(np.arange(nx)); vals.append(np.ones(nx))
    r = nx
    k = np.repeat(np.arange(1, nt), nx)
    i = np.tile(np.arange(nx), nt - 1)
    rr = nx + (k - 1) * nx + i
    rows.append(rr); cols.append((k - 1) * nx + i); vals.append(-m[i] / dt)
    sel = i > 0
    rows.append(rr[sel]); cols.append(k[sel] * nx + i[sel] - 1); vals.append(nu * s3[i[sel], 0])
    rows.append(rr); cols.append(k * nx + i); vals.append(m[i] / dt + nu * s3[i, 1])
    sel = i < nx - 1
    rows.append(rr[sel]); cols.append(k[sel] * nx + i[sel] + 1); vals.append(nu * s3[i[sel], 2])
    N = nx * nt
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(N, N)).tocsr()
    A.sum_duplicates(); A.sort_indices()
    y = np.concatenate([u0, np.zeros((nt - 1) * nx)])
    q_eps = np.concatenate([np.full(nx, 1.0 / sigma_ic**2), np.full((nt - 1) * nx, 1.0 / sigma_pde**2)])
    coords = np.stack([np.tile(x, nt), np.repeat(np.arange(nt) * dt, nx)], axis=1)
    return Problem(N, Q, A, q_eps, y, np.zeros(N), coords,
                   meta=dict(workload="burgers_spacetime", nx=nx, nt=nt, dt=dt, nu=nu, mass=m, s3=s3,
                             u0=u0, x=x, sigma_pde=sigma_pde, sigma_ic=sigma_ic, kappa_s=kappa_s,
                             tau_s=tau_s, seed=seed))


def darcy_p2(n_el: int = 300, boundary: str = "dirichlet", alpha: int = 3, eps2: float = 1e-8,
             sigma_pde: float = 1e-3, observations: str = "fem", n_obs: int = 2000,
             sigma: float = 1e-2, a_hi: float = 12.0, a_lo: float = 3.0, seed: int = 7) -> Problem:
    """GMRF-FEM for Darcy flow -div(a grad u) = 1 on the unit square (Sec. 5.1, App. C.1)
    with quadratic Lagrange triangles: n_el elements per side, (2 n_el + 1)^2 unknowns.

    Prior: Matern with nu = alpha - 1 (2D), effective range n_el^-1/2 and unit marginal
    variance: Q = tau^-2 K M~^-1 K (alpha = 2) or tau^-2 K M~^-1 K M~^-1 K (alpha = 3),
    K = kappa^2 M~ + S, M~ the HRZ-lumped P2 mass.  Boundary (App. B): "dirichlet"
    constrains every boundary node to 0, "periodic" ties the nodes on x = 1 / y = 1 to their
    mirrors on x = 0 / y = 0 (a torus), "natural" constrains nothing.  K and M~ are
    eliminated as in classic FEM (rows and columns, so K stays symmetric); the mass entry at
    a constrained node is (eps/tau)^(2/(alpha-1)), so that the constrained unknown is
    N(0, eps2) in the final precision.

    Observations: "fem" -- the Galerkin rows of -div(a grad u) = 1 at the unconstrained
    nodes (the constraint's column operation applied), data the consistent load, noise
    sigma_pde * m~_i (a pointwise residual noise sigma_pde); "points" -- n_obs uniform
    point values of a seeded smooth target with noise sigma; "none" -- the prior alone.  The permeability a is a
    seeded smooth random field thresholded to a_hi / a_lo per triangle (piecewise constant,
    like the two-valued coefficients of the Darcy benchmark)."""
    from . import p2
    if boundary not in ("dirichlet", "periodic", "natural"):
        raise ValueError(f"unknown boundary {boundary!r}")
    if alpha not in (2, 3):
        raise ValueError("alpha must be 2 or 3")
    rng = rng_for(seed)
    mesh = p2.P2Mesh(n_el + 1)
    S = mesh.stiffness()
    m = mesh.lumped_mass()
    nu_m = float(alpha - 1)
    kappa = priors.matern_range_to_kappa(n_el ** -0.5, nu_m)
    # unit marginal variance: tau^2 Gamma(nu) / (Gamma(alpha) 4 pi kappa^(2 nu)) = 1
    tau = math.sqrt(math.gamma(alpha) * 4.0 * math.pi * kappa ** (2.0 * nu_m) / math.gamma(nu_m))
    if boundary == "dirichlet":
        con = mesh.boundary_nodes()
        tgt = -np.ones(con.size, dtype=np.int64)
    elif boundary == "periodic":
        con, tgt = mesh.periodic_pairs()
    else:
        con = np.zeros(0, dtype=np.int64)
        tgt = np.zeros(0, dtype=np.int64)
    coef = np.ones(con.size)
    K = (S + sp.diags(kappa * kappa * m)).tocsr()
    m_con = (math.sqrt(eps2) / tau) ** (2.0 / (alpha - 1))
    Kc, mc = p2.constrain_fem(K, m, con, tgt, coef, m_con)
    Mi = sp.diags(1.0 / mc)
    Q = (Kc.T @ Mi @ Kc) if alpha == 2 else (Kc @ Mi @ Kc @ Mi @ Kc)
    Q = sp.csr_matrix(Q / (tau * tau))
    # the triple product is symmetric only up to rounding, and a cancelled entry can be stored
    # on one side only: take the symmetric part on the union pattern
    Q = sp.csr_matrix(0.5 * (Q + Q.T))
    Q.sum_duplicates(); Q.sort_indices()
    field_fn = smooth_target(rng, 2)
    cl, cu = mesh.centroids()
    a_l = np.where(field_fn(cl) > 0.0, a_hi, a_lo)
    a_u = np.where(field_fn(cu) > 0.0, a_hi, a_lo)
    free = np.setdiff1d(np.arange(mesh.n), con)
    if observations == "fem":
        Sa = mesh.stiffness(a_l, a_u)
        load = np.asarray(mesh.mass() @ np.ones(mesh.n)).ravel()
        A = p2.constrain_columns(Sa, con, tgt, coef)[free].tocsr()
        A.eliminate_zeros(); A.sort_indices()
        y = load[free].copy()
        q_eps = 1.0 / (sigma_pde * m[free]) ** 2
    elif observations == "points":
        pts = rng.uniform(0.0, 1.0, size=(n_obs, 2))
        A = p2.constrain_columns(mesh.point_rows(pts), con, tgt, coef)
        A.eliminate_zeros(); A.sort_indices()
        y = field_fn(pts) + sigma * rng.standard_normal(n_obs)
        q_eps = np.full(n_obs, 1.0 / sigma**2)
        Sa = load = None
    elif observations == "none":
        A = sp.csr_matrix((0, mesh.n))
        y = np.zeros(0)
        q_eps = np.zeros(0)
        Sa = load = None
    else:
        raise ValueError(f"unknown observations {observations!r}")
    return Problem(mesh.n, Q, A, q_eps, y, np.zeros(y.size), mesh.coords.copy(),
                   meta=dict(workload="darcy_p2", n_el=n_el, boundary=boundary, alpha=alpha, eps2=eps2,
                             kappa=kappa, tau=tau, mesh=mesh, constrained=con, targets=tgt, free=free,
                             a_lower=a_l, a_upper=a_u, S_a=Sa, load=load, observations=observations,
                             sigma_pde=sigma_pde, seed=seed))
