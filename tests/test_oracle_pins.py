"""Pins of the oracle against facts fixed by the paper and by the mathematics, not by
the oracle itself: dense inverse / eigenvalue log-det on tiny grids, closed forms of
the 1-node space-time prior (random walk and AR(1)), the state-space log-det identity
of the block-tridiagonal prior (App. A), Kalman filtering + RTS smoothing of the same
state-space model, the Matern log-det through a factorisation of
K, trace identities, the covariance (Woodbury) form of conditioning, sample
identities, ordering invariance and structural invariants."""
import math

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import gmrf_inputs as gi
import oracle as O
from gmrf_inputs import fem, priors

pytestmark = pytest.mark.filterwarnings("ignore::scipy.sparse.SparseEfficiencyWarning")


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _problems_tiny():
    return [gi.matern2d(side=7, n_obs=12, seed=11),
            gi.matern2d(side=10, kappa=2.0, n_obs=30, seed=12),
            gi.advdiff_spacetime(ns=5, nt=4, seed=13),
            gi.advdiff_spacetime(ns=6, nt=5, c=1.5, nu=0.05, seed=14),
            gi.matern3d(side=5, n_obs=20, seed=15)]


@pytest.mark.parametrize("k", range(5))
def test_P1_dense_inverse_and_eigen_logdet(k):
    p = _problems_tiny()[k]
    r = O.posterior(p)
    d = O.dense_posterior(p)
    assert _rel(r["mean"], d["mean"]) <= 1e-10
    assert np.max(np.abs(r["var"] - d["var"]) / d["var"]) <= 1e-10
    assert abs(r["logdet"] - d["logdet"]) <= 1e-10 * max(1.0, abs(d["logdet"]))
    # full Sigma on pattern(L) against the dense inverse, entry by entry
    F = r["factor"]
    Sig = d["cov"][np.ix_(F.perm, F.perm)]
    cols = np.repeat(np.arange(F.n), np.diff(F.Lp))
    ref = Sig[F.Li, cols]
    assert np.max(np.abs(r["sigma_L"] - ref)) <= 1e-10 * np.max(np.abs(ref))


def _one_node_chain(nt, dt, tau, q1, decay):
    mesh = fem.Mesh(1, (1,), (1.0,), (0.0,), np.zeros((1, 1)), np.zeros((0, 2), np.int64), 1.0)
    m = np.ones(1)
    Ls = sp.csr_matrix(np.array([[decay]]))
    Q1 = sp.csr_matrix(np.array([[q1]]))
    Q, G = priors.spacetime_precision(mesh, nt, dt, Ls, tau, Q1, m)
    return Q


def test_P2_random_walk_closed_form():
    nt, dt, tau, s0 = 40, 0.05, 1.7, 0.8
    s2 = tau * tau * dt
    Q = _one_node_chain(nt, dt, tau, 1.0 / s0**2, 0.0)
    i = np.arange(1, nt + 1)
    Sig = s0**2 + (np.minimum.outer(i, i) - 1) * s2
    # tridiagonal pattern and inverse of the closed-form covariance
    assert Q.nnz == 3 * nt - 2
    assert np.allclose(Q.toarray(), np.linalg.inv(Sig), rtol=1e-9, atol=1e-9 * abs(Q).max())
    for perm in (np.arange(nt), np.arange(nt)[::-1].copy(), O.rcm_order(Q)):
        F = O.cholesky(Q, perm)
        S = O.selinv(F)
        var = O.marginal_variances(F, S)
        assert np.max(np.abs(var - np.diag(Sig)) / np.diag(Sig)) <= 1e-12
        ld = -math.log(s0**2) - (nt - 1) * math.log(s2)
        assert abs(O.logdet(F) - ld) <= 1e-12 * abs(ld)
        cols = np.repeat(np.arange(nt), np.diff(F.Lp))
        ref = Sig[np.ix_(perm, perm)][F.Li, cols]
        assert np.max(np.abs(S - ref) / np.abs(ref)) <= 1e-12


def test_P3_ar1_closed_form():
    nt, dt, tau, decay = 30, 0.1, 0.9, 2.5
    G = 1.0 + dt * decay
    phi = 1.0 / G
    s2 = tau * tau * dt / G**2
    q1 = (1.0 - phi * phi) / s2                    # stationary start
    Q = _one_node_chain(nt, dt, tau, q1, decay)
    i = np.arange(nt)
    Sig = s2 * phi ** np.abs(np.subtract.outer(i, i)) / (1.0 - phi * phi)
    F = O.cholesky(Q, np.arange(nt))
    var = O.marginal_variances(F)
    assert np.max(np.abs(var - np.diag(Sig)) / np.diag(Sig)) <= 1e-12
    ld = -nt * math.log(s2) + math.log(1.0 - phi * phi)
    assert abs(O.logdet(F) - ld) <= 1e-12 * abs(ld)
    # the mean of a fully observed chain against a dense solve
    z = gi.rng_for(3).standard_normal(nt)
    x = O.solve(F, z)
    assert _rel(x, np.linalg.solve(np.linalg.inv(Sig), z)) <= 1e-10


def _splu_logabsdet(M):
    lu = spla.splu(sp.csc_matrix(M), permc_spec="COLAMD")
    return float(np.sum(np.log(np.abs(lu.U.diagonal()))) + np.sum(np.log(np.abs(lu.L.diagonal()))))


@pytest.mark.parametrize("ns,nt", [(6, 5), (12, 9)])
def test_P4_spacetime_prior_logdet_identity(ns, nt):
    """log|Q_ST| = log|Q1| + (Nt-1) log|F^-1| with
    log|F^-1| = -Ns log(tau^2 dt) + 2 log|det G| - 2 log|M~| + log|Sigma^-1|
    (unit-Jacobian change of variables in the state-space model, App. A)."""
    p = gi.advdiff_spacetime(ns=ns, nt=nt, seed=21)
    meta = p.meta
    m, G, Q1 = meta["m"], meta["G"], meta["Q1"]
    Ns = ns * ns
    logM = float(np.sum(np.log(m)))
    logFinv = (-Ns * math.log(meta["tau"] ** 2 * meta["dt"]) + 2 * _splu_logabsdet(G)
               - 2 * logM + logM)       # white noise: Sigma^-1 = M~
    logQ1 = (-2 * Ns * math.log(meta["tau1"])
             + 2 * _splu_logabsdet(Q1 * 0 + (sp.diags(meta["kappa1"] ** 2 * m)
                                             + fem.stiffness(meta["mesh"])))
             - logM)
    ref = logQ1 + (nt - 1) * logFinv
    F = O.cholesky(p.Q, O.nd_order(p.coords, p.Q))
    assert abs(O.logdet(F) - ref) <= 1e-9 * abs(ref)


def test_P4_spacetime_prior_logdet_identity_matern_noise():
    """The state-space log-det identity with spatial Matern noise (App. A):
    log|F^-1| = -Ns log(tau^2 dt) + 2 log|det G| - 2 log|M~| + log|Sigma^-1|, where
    log|Sigma^-1| = -2 Ns log tau_s + 2 log|det K_s| - log|M~| through K_s (a 1-ring matrix)."""
    ns, nt = 7, 6
    p = gi.advdiff_spacetime(ns=ns, nt=nt, seed=24, noise="matern", noise_range=0.3)
    meta = p.meta
    m, G, Q1 = meta["m"], meta["G"], meta["Q1"]
    Ns = ns * ns
    logM = float(np.sum(np.log(m)))
    Ks = sp.diags(meta["kappa_s"] ** 2 * m) + fem.stiffness(meta["mesh"])
    logSinv = -2 * Ns * math.log(meta["tau_s"]) + 2 * _splu_logabsdet(Ks) - logM
    logFinv = -Ns * math.log(meta["tau"] ** 2 * meta["dt"]) + 2 * _splu_logabsdet(G) - 2 * logM + logSinv
    logQ1 = (-2 * Ns * math.log(meta["tau1"])
             + 2 * _splu_logabsdet(sp.diags(meta["kappa1"] ** 2 * m) + fem.stiffness(meta["mesh"])) - logM)
    ref = logQ1 + (nt - 1) * logFinv
    F = O.cholesky(p.Q, O.nd_order(p.coords, p.Q))
    assert abs(O.logdet(F) - ref) <= 1e-9 * abs(ref)


@pytest.mark.parametrize("side,bound", [(33, 0.12), (65, 0.05)])
def test_P16_matern_interior_variance(side, bound):
    """Matern sanity check (Sec. 2.2): with (kappa^2 - Laplace) u = tau W in 2D (alpha = 2),
    the marginal variance away from the boundary tends to tau^2 / (4 pi kappa^2); the
    FEM prior's centre variance is within the discretisation error, which shrinks with h."""
    mesh = fem.structured_mesh((side, side))
    kappa, tau = 20.0, 2.0
    Q, _, _ = priors.matern_precision(mesh, kappa, tau)
    r = O.posterior(gi.Problem(mesh.n, Q, sp.csr_matrix((0, mesh.n)), np.zeros(0), np.zeros(0), np.zeros(0),
                               mesh.coords))
    centre = (side // 2) * side + side // 2
    rel = r["var"][centre] / (tau * tau / (4.0 * math.pi * kappa * kappa)) - 1.0
    assert 0.0 < rel <= bound


def test_P5_matern_logdet_via_K():
    p = gi.matern2d(side=20, kappa=3.0, tau=0.7, seed=22)
    K, m = p.meta["K"], p.meta["m"]
    ref = -2 * p.n * math.log(0.7) + 2 * _splu_logabsdet(K) - float(np.sum(np.log(m)))
    F = O.cholesky(p.Q, O.nd_order(p.coords, p.Q))
    assert abs(O.logdet(F) - ref) <= 1e-10 * abs(ref)
    p3 = gi.matern3d(side=8, kappa=4.0, seed=23)
    ref3 = (2 * _splu_logabsdet(p3.meta["K"]) - float(np.sum(np.log(p3.meta["m"]))))
    F3 = O.cholesky(p3.Q, O.nd_order(p3.coords, p3.Q))
    assert abs(O.logdet(F3) - ref3) <= 1e-10 * abs(ref3)


def test_P6_trace_identities():
    p = gi.matern2d(side=14, n_obs=40, seed=24)
    Qp, h = O.assemble(p.Q, p.A, p.q_eps, p.y)
    F = O.cholesky(Qp, O.nd_order(p.coords, Qp))
    S = O.selinv(F)
    Sq = O.sigma_on_pattern(F, S, Qp)
    assert abs(np.dot(Sq, Qp.data) - p.n) <= 1e-9 * p.n
    # tr(Q_post^-1 Q) + tr(Q_post^-1 A^T Q_eps A) = N, both read on pattern(Q_post)
    Qs = O.core.sp.csr_matrix(p.Q)
    Qon = gi.fem.on_pattern(Qs, Qp)
    D = (p.A.T @ sp.diags(p.q_eps) @ p.A).tocsr()
    Don = gi.fem.on_pattern(D, Qp)
    assert abs(np.dot(Sq, Qon.data) + np.dot(Sq, Don.data) - p.n) <= 1e-9 * p.n


def test_P7_sample_identities():
    p = gi.advdiff_spacetime(ns=6, nt=4, seed=25)
    Qp, h = O.assemble(p.Q, p.A, p.q_eps, p.y)
    F = O.cholesky(Qp, O.nd_order(p.coords, Qp))
    mu = O.solve(F, h)
    z = gi.standard_normal_f32(p.n, 3, seed=26)
    x = O.sample(F, mu, z)
    for c in range(3):
        d = x[:, c] - mu
        zc = z[:, c].astype(np.float64)
        assert abs(d @ (Qp @ d) - zc @ zc) <= 1e-9 * (zc @ zc)
        Ld = F.L().T @ d[F.perm]
        assert np.max(np.abs(Ld - zc)) <= 1e-9 * np.max(np.abs(zc))


def test_P7_sample_covariance_monte_carlo():
    p = gi.matern2d(side=5, kappa=3.0, n_obs=5, seed=27)
    Qp, h = O.assemble(p.Q, p.A, p.q_eps, p.y)
    F = O.cholesky(Qp, O.rcm_order(Qp))
    n_draw = 100000
    z = gi.standard_normal_f32(p.n, n_draw, seed=28)
    x = O.sample(F, np.zeros(p.n), z)
    C = x @ x.T / n_draw
    ref = np.linalg.inv(Qp.toarray())
    se = np.sqrt((np.outer(np.diag(ref), np.diag(ref)) + ref**2) / n_draw)
    assert np.max(np.abs(C - ref) / se) < 6.0


@pytest.mark.parametrize("seed,noise", [(81, "white"), (82, "white"), (83, "matern"), (84, "matern")])
def test_P8_kalman_rts_smoother(seed, noise):
    """The space-time GMRF is the precision form of a linear-Gaussian state-space model
    (Sec. 2.4, App. A): u_1 ~ N(0, Q1^-1), u_(k+1) = A u_k + e_k, e_k ~ N(0, F) with
    A = G^-1 M~ and F = tau^2 dt G^-1 M~ Sigma M~ G^-T (white noise in space: Sigma = M~^-1;
    Matern noise in space: Sigma = Q_s^-1, the covariance of the discretised spatial noise).
    With point data on single slices, a Kalman filter followed by the Rauch-Tung-Striebel
    smoother, run densely slice by slice, gives the posterior mean and marginal variances
    without the block-tridiagonal precision, its factorisation or the Takahashi recursion."""
    p = gi.advdiff_spacetime(ns=5, nt=6, obs_frac=0.3, pde_rows=False, seed=seed, noise=noise,
                             noise_range=0.5)
    meta = p.meta
    ns, nt, dt, tau = meta["mesh"].n, meta["nt"], meta["dt"], meta["tau"]
    G = meta["G"].toarray()
    M = np.diag(meta["m"])
    At = np.linalg.solve(G, M)
    Gi = np.linalg.inv(G)
    Sig = np.linalg.inv(M) if noise == "white" else np.linalg.inv(meta["Sigma_inv"].toarray())
    F = tau * tau * dt * Gi @ M @ Sig @ M @ Gi.T
    A = p.A.tocsr()
    slice_of_row = np.array([A.indices[A.indptr[i]] // ns for i in range(A.shape[0])])
    for i in range(A.shape[0]):
        assert np.all(A.indices[A.indptr[i]:A.indptr[i + 1]] // ns == slice_of_row[i])
    # filter
    mf, Pf, mp, Pp = [], [], [], []
    m_pred, P_pred = np.zeros(ns), np.linalg.inv(meta["Q1"].toarray())
    for k in range(nt):
        rows = np.flatnonzero(slice_of_row == k)
        m_k, P_k = m_pred, P_pred
        if rows.size:
            H = A[rows][:, k * ns:(k + 1) * ns].toarray()
            R = np.diag(1.0 / p.q_eps[rows])
            Sk = H @ P_k @ H.T + R
            K = np.linalg.solve(Sk, H @ P_k).T
            m_k = m_k + K @ (p.y[rows] - p.b[rows] - H @ m_k)
            IKH = np.eye(ns) - K @ H
            P_k = IKH @ P_k @ IKH.T + K @ R @ K.T     # Joseph form (data noise 1e-3)
        mp.append(m_pred); Pp.append(P_pred); mf.append(m_k); Pf.append(P_k)
        m_pred, P_pred = At @ m_k, At @ P_k @ At.T + F
    # smoother
    ms, Ps = [None] * nt, [None] * nt
    ms[-1], Ps[-1] = mf[-1], Pf[-1]
    for k in range(nt - 2, -1, -1):
        C = np.linalg.solve(Pp[k + 1], At @ Pf[k]).T
        ms[k] = mf[k] + C @ (ms[k + 1] - mp[k + 1])
        Ps[k] = Pf[k] + C @ (Ps[k + 1] - Pp[k + 1]) @ C.T
    mean = np.concatenate(ms)
    var = np.concatenate([np.diag(P) for P in Ps])
    r = O.posterior(p)
    # a wrong noise covariance (M~ dropped, or dt^2 for dt) moves these by 1e-5 .. 1
    assert _rel(r["mean"], mean) <= 1e-8
    assert np.max(np.abs(r["var"] - var) / var) <= 1e-8


def test_P9_woodbury_covariance_form():
    p = gi.matern2d(side=9, n_obs=25, seed=29)
    r = O.posterior(p)
    Sig0 = np.linalg.inv(p.Q.toarray())
    A = p.A.toarray()
    Sy = A @ Sig0 @ A.T + np.diag(1.0 / p.q_eps)
    mu = Sig0 @ A.T @ np.linalg.solve(Sy, p.y - p.b)
    cov = Sig0 - Sig0 @ A.T @ np.linalg.solve(Sy, A @ Sig0)
    assert _rel(r["mean"], mu) <= 1e-9
    assert np.max(np.abs(r["var"] - np.diag(cov)) / np.diag(cov)) <= 1e-9


def test_P10_invariants():
    p = gi.advdiff_spacetime(ns=8, nt=6, seed=30)
    Qp, h = O.assemble(p.Q, p.A, p.q_eps, p.y)
    assert (abs(Qp - Qp.T)).max() <= 1e-12 * abs(Qp).max()
    F = O.cholesky(Qp, O.nd_order(p.coords, Qp))
    assert np.all(F.Lx[F.Lp[:-1]] > 0)
    var = O.marginal_variances(F)
    F0 = O.cholesky(p.Q, O.nd_order(p.coords, p.Q))
    var0 = O.marginal_variances(F0)
    d = Qp.diagonal()
    assert np.all(var > 0)
    assert np.all(var >= (1.0 / d) * (1 - 1e-12))
    assert np.all(var <= var0 * (1 + 1e-10))


def test_P12_ordering_invariance():
    p = gi.advdiff_spacetime(ns=7, nt=5, seed=31)
    Qp, h = O.assemble(p.Q, p.A, p.q_eps, p.y)
    rng = gi.rng_for(32)
    outs = []
    for perm in (O.nd_order(p.coords, Qp), O.rcm_order(Qp), rng.permutation(p.n)):
        F = O.cholesky(Qp, perm)
        outs.append((O.solve(F, h), O.marginal_variances(F), O.logdet(F)))
    for o in outs[1:]:
        assert _rel(o[0], outs[0][0]) <= 1e-9
        assert np.max(np.abs(o[1] - outs[0][1]) / outs[0][1]) <= 1e-9
        assert abs(o[2] - outs[0][2]) <= 1e-11 * abs(outs[0][2])


def test_not_spd_reports_column():
    p = gi.matern2d(side=6, seed=33)
    Q = p.Q.tolil()
    Q[17, 17] = -1.0
    with pytest.raises(O.NotSPDError):
        O.cholesky(Q.tocsr(), np.arange(p.n))


def test_block_diagonal_batch_equals_separate_problems():
    p = gi.matern_batch(n_prob=4, side_lo=5, side_hi=9, seed=34)
    r = O.posterior(p)
    lds = O.block_logdets(r["factor"], p.block_ptr)
    for b in range(4):
        lo, hi = p.block_ptr[b], p.block_ptr[b + 1]
        Qb = p.Q[lo:hi, lo:hi]
        rows = np.unique(p.A[:, lo:hi].nonzero()[0])
        Ab = p.A[rows][:, lo:hi]
        sub = gi.Problem(hi - lo, Qb, Ab, p.q_eps[rows], p.y[rows], p.b[rows], p.coords[lo:hi])
        d = O.dense_posterior(sub)
        assert _rel(r["mean"][lo:hi], d["mean"]) <= 1e-10
        assert np.max(np.abs(r["var"][lo:hi] - d["var"]) / d["var"]) <= 1e-10
        assert abs(lds[b] - d["logdet"]) <= 1e-10 * abs(d["logdet"])


def test_condition_number_estimate_pins():
    """The condition estimate: the Lanczos branch against dense eigenvalues on a grid
    just above the dense limit; the 1-node RW1 precision (tridiagonal Toeplitz in the
    interior) against its closed-form eigenvalues 2 - 2 cos(k pi / (n+1)) for the
    Dirichlet second-difference matrix."""
    p = gi.matern2d(side=24, n_obs=40, seed=31)
    Qp, _ = O.assemble(p.Q, p.A, p.q_eps, p.y)
    k_l, lo_l, hi_l = O.condition_number(Qp, dense_max=100)
    w = np.linalg.eigvalsh(O.jacobi_scaled(Qp).toarray())
    assert abs(lo_l - w[0]) <= 1e-6 * w[0] and abs(hi_l - w[-1]) <= 1e-6 * w[-1]
    assert abs(k_l - w[-1] / w[0]) <= 1e-5 * w[-1] / w[0]
    n = 50
    T = sp.diags([-np.ones(n - 1), 2.0 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1], format="csr")
    k, lo, hi = O.condition_number(T)
    lam = 2.0 - 2.0 * np.cos(np.arange(1, n + 1) * np.pi / (n + 1))
    assert abs(lo - lam[0] / 2.0) <= 1e-12 and abs(hi - lam[-1] / 2.0) <= 1e-12


@pytest.mark.parametrize("maker", [lambda: gi.matern2d(side=12, seed=121),
                                   lambda: gi.advdiff_spacetime(ns=6, nt=5, seed=122),
                                   lambda: gi.advdiff_spacetime(ns=6, nt=5, seed=123, noise="matern")])
def test_prior_square_root_reproduces_precision(maker):
    """The left square roots used by CG sampling (Sec. 3.2; App. A's block-bidiagonal
    square root of the space-time prior, here with Q1 a precision): R R^T = Q."""
    p = maker()
    R = gi.prior_sqrt(p)
    assert abs(R @ R.T - p.Q).max() <= 1e-13 * abs(p.Q).max()


def test_cg_sampling_covariance_monte_carlo():
    """Q_post^-1 (R w1 + A^T Q_eps^1/2 w2) has covariance Q_post^-1: the sample covariance of
    40,000 draws on a tiny space-time grid against the dense inverse (MC error ~ 1/sqrt(N))."""
    p = gi.advdiff_spacetime(ns=4, nt=3, obs_frac=0.3, seed=124)
    Qp, _ = O.assemble(p.Q, p.A, p.q_eps, p.y)
    R = gi.prior_sqrt(p)
    rng = gi.rng_for(125)
    N = 40000
    rhs = O.cg_sample_rhs(R, p.A, p.q_eps, rng.standard_normal((R.shape[1], N)),
                          rng.standard_normal((p.A.shape[0], N)))
    X = np.linalg.solve(Qp.toarray(), rhs)
    C = X @ X.T / N
    Sig = np.linalg.inv(Qp.toarray())
    sd = np.sqrt(np.outer(np.diag(Sig), np.diag(Sig)))
    assert np.max(np.abs(C - Sig) / sd) <= 6.0 / np.sqrt(N) * 3


def test_rbmc_variance_estimator_unbiased_and_consistent():
    """Rao-Blackwellised MC variances: averaged over many independent draws the estimate
    equals diag(Q^-1) (it is unbiased) within the MC error, and it is far less noisy than
    the plain sample variance of the same draws."""
    p = gi.matern2d(side=10, n_obs=20, seed=126)
    Qp, _ = O.assemble(p.Q, p.A, p.q_eps, p.y)
    Sig = np.diag(np.linalg.inv(Qp.toarray()))
    F = O.cholesky(Qp, O.rcm_order(Qp))
    rng = gi.rng_for(127)
    z = rng.standard_normal((p.n, 4000))
    xs = O.sample(F, np.zeros(p.n), z)
    v = O.rbmc_variances(Qp, xs)
    plain = np.mean(xs * xs, axis=1)
    e_rb = np.max(np.abs(v - Sig) / Sig)
    e_pl = np.max(np.abs(plain - Sig) / Sig)
    assert e_rb <= 0.05 and e_rb < 0.5 * e_pl
