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


def _quadrature_residual(u, nx, nt, dt, nu):
    """The Galerkin implicit-Euler Burgers residual rebuilt element by element from the
    P1 hat functions on [-1, 1] (nx interior nodes, zero Dirichlet values at +-1) with
    3-point Gauss-Legendre quadrature, exact for the cubic integrands here (Sec. 2.3 weak
    form of u_t + u u_x = nu u_xx; lumped mass = integral of each hat function).  Rows:
    u^0_i, then slices 1..nt-1."""
    h = 2.0 / (nx + 1)
    xg, wg = np.polynomial.legendre.leggauss(3)
    U = np.asarray(u, dtype=np.float64).reshape(nt, nx)
    out = [U[0].copy()]
    for k in range(1, nt):
        full = np.concatenate([[0.0], U[k], [0.0]])          # node values incl. boundary
        prev = np.concatenate([[0.0], U[k - 1], [0.0]])
        r = np.zeros(nx + 2)
        lump = np.zeros(nx + 2)
        for e in range(nx + 1):                                # element [x_e, x_{e+1}]
            xa = -1.0 + e * h
            for xi, w in zip(xg, wg):
                x = xa + 0.5 * h * (xi + 1.0)
                phi = np.array([(xa + h - x) / h, (x - xa) / h])
                dphi = np.array([-1.0 / h, 1.0 / h])
                uq = full[e] * phi[0] + full[e + 1] * phi[1]
                ux = full[e] * dphi[0] + full[e + 1] * dphi[1]
                for loc in range(2):
                    node = e + loc
                    jac = 0.5 * h * w
                    lump[node] += jac * phi[loc]
                    r[node] += jac * (nu * dphi[loc] * ux + phi[loc] * uq * ux)
        r += lump * (full - prev) / dt
        out.append(r[1:nx + 1])
    return np.concatenate(out)


def test_residual_matches_elementwise_quadrature():
    """The oracle's residual (mass, viscous and nonlinear terms) equals an independent
    element-by-element quadrature of the weak form on random iterates."""
    p, m, S = _prob(nx=11, nt=5, seed=97)
    for seed in (98, 99):
        u = gi.rng_for(seed).standard_normal(p.n)
        f, _ = O.burgers_residual_and_jacobian(u, m["nx"], m["nt"], m["dt"], m["nu"], m["mass"], S)
        g = _quadrature_residual(u, m["nx"], m["nt"], m["dt"], m["nu"])
        assert np.max(np.abs(f - g)) <= 1e-12 * max(1.0, np.max(np.abs(g)))


def test_nonlinear_term_closed_form_for_linear_u():
    """u = a + b x on a slice equal to its predecessor: the time term vanishes, the
    discrete Laplacian of a linear function is zero at nodes with two interior
    neighbours, and the weak nonlinear term is exactly b (a + b x_i) h there."""
    p, m, S = _prob(nx=15, nt=3, seed=90)
    nx, nt = m["nx"], m["nt"]
    h = 2.0 / (nx + 1)
    x = -1.0 + h * np.arange(1, nx + 1)
    a, b = 0.7, -1.3
    u = np.tile(a + b * x, nt)
    f, _ = O.burgers_residual_and_jacobian(u, nx, nt, m["dt"], m["nu"], m["mass"], S)
    f_pde = f[nx:].reshape(nt - 1, nx)
    want = b * (a + b * x) * h
    for k in range(nt - 1):
        assert np.max(np.abs(f_pde[k, 1:-1] - want[1:-1])) <= 1e-13


def _cubic(side, seed=None):
    p = gi.elliptic_cubic(side=side)
    m = p.meta
    return p, m


def test_pointwise_jacobian_matches_finite_differences():
    p, m = _cubic(12)
    u = gi.rng_for(111).standard_normal(p.n)
    f, J = O.pointwise_residual_and_jacobian(u, p.A, m["nl_col"], m["nl_coef"], m["power"])
    Jd = J.toarray()
    h = 1e-6
    for j in gi.rng_for(112).choice(p.n, size=15, replace=False):
        e = np.zeros(p.n); e[j] = h
        fp, _ = O.pointwise_residual_and_jacobian(u + e, p.A, m["nl_col"], m["nl_coef"], m["power"])
        fm, _ = O.pointwise_residual_and_jacobian(u - e, p.A, m["nl_col"], m["nl_coef"], m["power"])
        assert np.max(np.abs((fp - fm) / (2 * h) - Jd[:, j])) <= 1e-6 * max(1.0, np.max(np.abs(Jd[:, j])))


def test_pointwise_linear_step_is_affine_posterior_mean():
    p, m = _cubic(10)
    u = gi.rng_for(113).standard_normal(p.n)
    zero = np.zeros_like(m["nl_coef"])
    unew, rec = O.gn_step_pointwise(p.Q, u, p.y, p.q_eps, p.A, m["nl_col"], zero, 3)
    d = O.dense_posterior(gi.Problem(p.n, p.Q, p.A, p.q_eps, p.y, np.zeros(p.A.shape[0]), p.coords))
    assert rec["alpha"] == 1.0
    assert np.linalg.norm(unew - d["mean"]) <= 1e-9 * np.linalg.norm(d["mean"])


def test_cubic_rows_vanish_on_the_manufactured_solution_at_second_order():
    """The lumped Galerkin rows of -Laplace u + u^3 = f evaluated at the nodal values of
    the manufactured solution: the pointwise residual (f_i(u*) - m_i f(x_i)) / m_i is a
    consistency error that falls by about 4 per halving of h (second order); a wrong sign
    of the cubic or of the Laplacian leaves an O(1) residual."""
    errs = []
    for side in (33, 65, 129):
        p, m = _cubic(side)
        f, _ = O.pointwise_residual_and_jacobian(m["u_true"], p.A, m["nl_col"], m["nl_coef"], m["power"])
        npde = m["n_pde"]
        r = (f[:npde] - p.y[:npde]) / m["nl_coef"][:npde]
        errs.append(float(np.max(np.abs(r))))
    print(f"[cubic] max pointwise residual of u*: {errs}")
    assert errs[0] / errs[1] > 3.0 and errs[1] / errs[2] > 3.0
    assert errs[2] < 2e-3


def test_step_not_taken_when_no_trial_decreases(monkeypatch):
    """When the solve returns an ascent direction (here: the reflected minimiser, planted
    on the CPU), no trial step passes the Armijo test; the iterate is kept (alpha = 0) and
    the objective does not increase."""
    p, m = _cubic(10)
    u = gi.rng_for(114).standard_normal(p.n)
    good = O.core.solve

    def reflected(F, h):
        x = good(F, h)
        return 2.0 * u - x
    monkeypatch.setattr(O.core, "solve", reflected)
    unew, rec = O.gn_step_pointwise(p.Q, u, p.y, p.q_eps, p.A, m["nl_col"], m["nl_coef"], 3)
    assert rec["slope"] > 0
    assert rec["alpha"] == 0.0
    assert np.array_equal(unew, u)
