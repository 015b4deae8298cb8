"""Pins of the oracle's log marginal likelihood and gradient: the GMRF identity value
against the plain covariance-form definition on tiny grids, the trace-based gradient
against central finite differences of that plain definition, and the exact scaling
identity g_logtau + g_logsigma = -M + mu^T Q mu + r^T Q_eps r (scaling tau and sigma by
the same factor scales Cov(y) by its square)."""
import math

import numpy as np
import pytest
import scipy.sparse as sp

import gmrf_inputs as gi
import oracle as O


def _setup(maker, kappa, tau, sigma):
    p = maker()
    pieces = gi.matern_pieces(p)
    Q, dQk = gi.matern_from_pieces(p, pieces, kappa, tau)
    q_eps = np.full(p.A.shape[0], 1.0 / sigma**2)
    return p, pieces, Q, dQk, q_eps


def _lml_dense_theta(p, pieces, th):
    k, t, s = np.exp(th)
    Q, _ = gi.matern_from_pieces(p, pieces, k, t)
    return O.lml_dense(Q, p.A, np.full(p.A.shape[0], 1.0 / s**2), p.y, p.b)


@pytest.mark.parametrize("maker", [lambda: gi.matern2d(side=10, n_obs=30, seed=71),
                                   lambda: gi.matern3d(side=5, n_obs=25, seed=72)])
def test_lml_identity_matches_covariance_definition(maker):
    p, pieces, Q, dQk, q_eps = _setup(maker, 4.0, 0.8, 0.1)
    lml, _, _ = O.lml_sparse(Q, p.A, q_eps, p.y, p.b, p.coords)
    ref = O.lml_dense(Q, p.A, q_eps, p.y, p.b)
    assert abs(lml - ref) <= 1e-9 * max(1.0, abs(ref))


@pytest.mark.parametrize("maker", [lambda: gi.matern2d(side=9, n_obs=20, seed=73),
                                   lambda: gi.matern3d(side=5, n_obs=15, seed=74)])
def test_lml_gradient_matches_finite_differences(maker):
    kappa, tau, sigma = 3.0, 1.3, 0.2
    p, pieces, Q, dQk, q_eps = _setup(maker, kappa, tau, sigma)
    derivs = [(dQk, None), (-2.0 * Q, None), (0.0 * Q, -2.0 * q_eps)]
    _, g, _ = O.lml_sparse(Q, p.A, q_eps, p.y, p.b, p.coords, derivs)
    th = np.log([kappa, tau, sigma])
    h = 1e-5
    for i in range(3):
        e = np.zeros(3)
        e[i] = h
        fd = (_lml_dense_theta(p, pieces, th + e) - _lml_dense_theta(p, pieces, th - e)) / (2 * h)
        assert abs(g[i] - fd) <= 1e-5 * max(1.0, abs(fd)), (i, g[i], fd)


def test_scaling_identity_of_tau_and_sigma_gradients():
    kappa, tau, sigma = 5.0, 0.9, 0.05
    p, pieces, Q, dQk, q_eps = _setup(lambda: gi.matern2d(side=16, n_obs=60, seed=75), kappa, tau, sigma)
    derivs = [(-2.0 * Q, None), (0.0 * Q, -2.0 * q_eps)]
    _, g, parts = O.lml_sparse(Q, p.A, q_eps, p.y, p.b, p.coords, derivs)
    M = p.A.shape[0]
    assert abs(g[0] + g[1] - (-M + parts["quad"] + parts["misfit"])) <= 1e-8 * max(1.0, abs(g[0]))


@pytest.mark.parametrize("name", ["c", "nu"])
def test_spacetime_gradient_matches_fd_of_plain_definition(name):
    """Advection speed c and viscosity nu change both the space-time prior (through
    G = M~ + dt (nu S + c C)) and the Galerkin PDE observation rows: the oracle's
    gradient, with its observation-operator term, against central differences of the
    covariance-form LML at fixed data.  Leaving out either the r^T Q_eps dA mu term or
    the dA part of dQ_post moves the gradient far outside the tolerance."""
    kw = dict(ns=5, nt=4, seed=11, obs_frac=0.2)
    base = dict(c=0.5, nu=0.01)
    p = gi.advdiff_spacetime(**kw, **base)
    d = gi.advdiff_derivatives(p)
    dq, da = d[name]
    dQ = sp.csr_matrix((dq, p.Q.indices, p.Q.indptr), shape=p.Q.shape)
    dA = sp.csr_matrix((da, p.A.indices, p.A.indptr), shape=p.A.shape)
    _, g, _ = O.lml_sparse(p.Q, p.A, p.q_eps, p.y, p.b, p.coords, derivs=[(dQ, None, dA)])
    # the dense definition carries ~1e-7 absolute rounding on an LML of 3e5, so its
    # differences use h = 1e-4 (c) / 1e-5 (nu); the sparse identity's value (pinned to
    # the dense one elsewhere) allows h = 1e-5 / 1e-6 and a tighter comparison
    h = 1e-4 if name == "c" else 1e-5
    vals, svals = [], []
    for sgn in (1, -1):
        q = gi.advdiff_spacetime(**kw, **{**base, name: base[name] + sgn * h})
        vals.append(O.lml_dense(q.Q, q.A, p.q_eps, p.y, p.b))
        q = gi.advdiff_spacetime(**kw, **{**base, name: base[name] + sgn * h / 10})
        svals.append(O.lml_sparse(q.Q, q.A, p.q_eps, p.y, p.b, p.coords)[0])
    fd = (vals[0] - vals[1]) / (2 * h)
    fds = (svals[0] - svals[1]) / (2 * h / 10)
    print(f"[lml st] d/d{name}: oracle {g[0]:.10e} fd(dense) {fd:.10e} fd(sparse) {fds:.10e}")
    assert abs(g[0] - fd) <= 1e-6 * max(1.0, abs(fd))
    assert abs(g[0] - fds) <= 1e-8 * max(1.0, abs(fds))
    # without the observation-operator terms the gradient is wrong
    _, g0, _ = O.lml_sparse(p.Q, p.A, p.q_eps, p.y, p.b, p.coords, derivs=[(dQ, None)])
    assert abs(g0[0] - fd) > 1e-3 * max(1.0, abs(fd))
