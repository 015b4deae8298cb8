"""The conjugate-gradient path (Sec. 3.2): preconditioned CG for the posterior mean with the
diagonal or the FP32 factor as preconditioner, warm starts, CG sampling from a left square
root of the prior, and Rao-Blackwellised Monte Carlo variances -- each against the oracle
on the same inputs."""
import numpy as np
import pytest
import scipy.sparse as sp

import gmrf_inputs as gi
import oracle as O

pytestmark = pytest.mark.gpu

CASES = {
    "matern2d_40": lambda: gi.matern2d(side=40, n_obs=150, seed=131),
    "spacetime_14x14x8": lambda: gi.advdiff_spacetime(ns=14, nt=8, seed=132),
}


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("precond", [0, 1])
def test_pcg_mean_matches_oracle(gpu_lib, name, precond):
    p = CASES[name]()
    r = O.posterior(p)
    ctx = gpu_lib.posterior_context(p, precision=gpu_lib.GMRF_FP32_REFINE)
    x, its, res = ctx.pcg(precond=precond, maxit=20000, tol=1e-13)
    e = _rel(x.cpu().numpy(), r["mean"])
    print(f"[pcg] {name} precond {precond}: {its[0]} iterations, residual {res[0]:.2e}, mean error {e:.2e}",
          flush=True)
    assert res[0] <= 1e-13 and e <= 1e-8
    if precond == 1:
        assert its[0] <= 10          # the FP32 factor leaves only a rounding-level error to remove
    # warm start from the converged iterate: nothing left to do
    x2, its2, _ = ctx.pcg(x0=x, precond=precond, maxit=100, tol=1e-13)
    assert its2[0] == 0
    ctx.close()


@pytest.mark.parametrize("name", sorted(CASES))
def test_sample_cg_matches_oracle(gpu_lib, name):
    import torch
    p = CASES[name]()
    ctx = gpu_lib.posterior_context(p, precision=gpu_lib.GMRF_FP64)
    mu, _, _ = ctx.solve()
    R = gi.prior_sqrt(p).tocsr()
    k = 3
    rng = gi.rng_for(133)
    w1 = rng.standard_normal((k, R.shape[1]))
    w2 = rng.standard_normal((k, p.A.shape[0]))
    t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a)).cuda().to(dt)  # noqa: E731
    x, its = ctx.sample_cg(t(R.indptr, torch.int64), t(R.indices, torch.int32), t(R.data, torch.float64),
                           t(w1, torch.float64), t(w2, torch.float64), precond=1, maxit=100, tol=1e-14)
    r = O.posterior(p)
    b = O.cg_sample_rhs(R, p.A, p.q_eps, w1.T, w2.T)
    xo = r["mean"][:, None] + np.linalg.solve(r["Qpost"].toarray(), b) if p.n <= 2000 else \
        r["mean"][:, None] + np.column_stack([O.solve(r["factor"], b[:, c]) for c in range(k)])
    e = max(_rel(x[c].cpu().numpy() - r["mean"], xo[:, c] - r["mean"]) for c in range(k))
    print(f"[sample cg] {name}: iterations {its}, error {e:.2e}", flush=True)
    assert e <= 1e-8
    ctx.close()


def test_rbmc_variances_match_oracle_and_exact(gpu_lib):
    import torch
    p = gi.matern2d(side=30, n_obs=60, seed=134)
    ctx = gpu_lib.posterior_context(p, precision=gpu_lib.GMRF_FP64)
    mu, _, _ = ctx.solve()
    k = 16
    z = torch.from_numpy(gi.rng_for(135).standard_normal((k, p.n)).astype(np.float32)).cuda()
    xs = ctx.sample(z) - mu[None, :]
    v = ctx.rbmc_variances(xs).cpu().numpy()
    r = O.posterior(p)
    vo = O.rbmc_variances(r["Qpost"], xs.cpu().numpy().T)
    e = float(np.max(np.abs(v - vo) / vo))
    # x_i | x_-i is N(-t_i, 1/Q_ii) with t_i ~ N(0, s_i), s_i = Sigma_ii - 1/Q_ii, so
    # k (v_i - 1/Q_ii) / s_i is chi-square with k degrees of freedom: standardised errors
    # (v_i - Sigma_ii) / (s_i sqrt(2/k)) have mean 0 and variance 1, and the chi-square tail
    # P(chi2_16 > 16 + 8 sqrt(32)) is below 1e-6 per node
    qd = r["Qpost"].diagonal()
    s = r["var"] - 1.0 / qd
    zstd = (v - r["var"]) / (s * np.sqrt(2.0 / k))
    # Rao-Blackwellisation: smaller error than the plain Monte Carlo estimate from the same draws
    xn = xs.cpu().numpy()
    v_mc = np.mean(xn * xn, axis=0)
    e_rb = float(np.mean(np.abs(v - r["var"]) / r["var"]))
    e_mc = float(np.mean(np.abs(v_mc - r["var"]) / r["var"]))
    print(f"[rbmc] k={k}: vs oracle estimator {e:.2e}; standardised error vs exact: max {np.max(np.abs(zstd)):.2f}, "
          f"mean {np.mean(zstd):.3f}; mean relative error RB {e_rb:.3f} vs plain MC {e_mc:.3f}", flush=True)
    assert e <= 1e-12
    assert np.max(np.abs(zstd)) <= 8.0
    assert e_rb < e_mc
    ctx.close()
