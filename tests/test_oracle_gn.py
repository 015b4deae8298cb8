"""Pins of the oracle's Gauss-Newton step for the Burgers residual: its Jacobian against
central finite differences of the residual; for a linear residual (the nonlinear term
switched off) one step from any iterate equals the affine posterior mean exactly and the
full step passes the line search; the objective decreases along the nonlinear iteration."""
import numpy as np
import pytest
import scipy.sparse as sp

import gmrf_inputs as gi
import oracle as O
from gmrf_inputs import fem


def _prob(nx=12, nt=8, seed=91):
    p = gi.burgers_spacetime(nx=nx, nt=nt, seed=seed, range_s=0.5)
    m = p.meta
    full = fem.structured_mesh((nx + 2,), lo=(-1.0,), hi=(1.0,))
    inner = np.arange(1, nx + 1)
    S = fem.stiffness(full)[inner][:, inner].tocsr()
    return p, m, S


def test_jacobian_matches_finite_differences():
    p, m, S = _prob()
    u = gi.rng_for(92).standard_normal(p.n)
    f, J = O.burgers_residual_and_jacobian(u, m["nx"], m["nt"], m["dt"], m["nu"], m["mass"], S)
    h = 1e-6
    Jd = J.toarray()
    for j in gi.rng_for(93).choice(p.n, size=20, replace=False):
        e = np.zeros(p.n); e[j] = h
        fp, _ = O.burgers_residual_and_jacobian(u + e, m["nx"], m["nt"], m["dt"], m["nu"], m["mass"], S)
        fm, _ = O.burgers_residual_and_jacobian(u - e, m["nx"], m["nt"], m["dt"], m["nu"], m["mass"], S)
        fd = (fp - fm) / (2 * h)
        assert np.max(np.abs(fd - Jd[:, j])) <= 1e-6 * max(1.0, np.max(np.abs(Jd[:, j])))


def test_linear_residual_step_is_affine_posterior_mean():
    p, m, S = _prob(seed=94)
    u = gi.rng_for(95).standard_normal(p.n)
    unew, rec = O.gn_step(p.Q, u, p.y, p.q_eps, m["nx"], m["nt"], m["dt"], m["nu"], m["mass"], S,
                          nonlinear=False)
    _, J = O.burgers_residual_and_jacobian(u, m["nx"], m["nt"], m["dt"], m["nu"], m["mass"], S,
                                           nonlinear=False)
    lin = gi.Problem(p.n, p.Q, J, p.q_eps, p.y, np.zeros(p.n), p.coords)
    d = O.dense_posterior(lin)
    assert rec["alpha"] == 1.0
    assert np.linalg.norm(unew - d["mean"]) <= 1e-9 * np.linalg.norm(d["mean"])


def test_objective_decreases_along_iteration():
    p, m, S = _prob(nx=16, nt=10, seed=96)
    u = np.zeros(p.n)
    phis = []
    for _ in range(5):
        u, rec = O.gn_step(p.Q, u, p.y, p.q_eps, m["nx"], m["nt"], m["dt"], m["nu"], m["mass"], S)
        phis.append(rec["phi0"])
        assert rec["decrement"] >= -1e-12 * abs(rec["phi0"])
    assert all(b <= a for a, b in zip(phis, phis[1:]))
