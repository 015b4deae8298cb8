"""Degenerate and edge cases of the GPU path, against closed forms and the dense oracle:
a diagonal posterior (every front one column, no fill, a forest of single-node trees), a
single unknown, a short chain with a few observations (one small front per column of the
elimination path), and the sampler's argument limits."""
import math

import numpy as np
import pytest
import scipy.sparse as sp

import gmrf_inputs as gi
import oracle as O

pytestmark = pytest.mark.gpu


def _diag_problem(n, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    d = rng.uniform(0.5, 4.0, n)
    q_eps = rng.uniform(1.0, 100.0, n)
    y = rng.standard_normal(n)
    p = gi.Problem(n, sp.diags(d).tocsr(), sp.identity(n, format="csr"), q_eps, y, np.zeros(n),
                   rng.uniform(0.0, 1.0, (n, 2)))
    return p, d, q_eps, y


@pytest.mark.parametrize("precision,use_coords", [(0, True), (0, False), (1, True)])
def test_diagonal_posterior_closed_form(gpu_lib, precision, use_coords):
    """Q = diag(d), A = I: Q_post = diag(d + q_eps), mean = q_eps y / (d + q_eps),
    variances 1 / (d + q_eps), log det = sum log(d + q_eps)."""
    p, d, q_eps, y = _diag_problem(1000, seed=91)
    ctx = gpu_lib.posterior_context(p, precision=precision, use_coords=use_coords)
    ld = ctx.logdet()[0]
    mu = ctx.solve(max_refine=20 if precision else 0, tol=1e-14, raise_not_converged=False)[0].cpu().numpy()
    var = ctx.selinv().cpu().numpy()
    ctx.close()
    qp = d + q_eps
    e_mu = np.max(np.abs(mu - q_eps * y / qp) / np.abs(q_eps * y / qp))
    e_var = np.max(np.abs(var - 1.0 / qp) * qp)
    ref = math.fsum(np.log(qp).tolist())
    e_ld = abs(ld - ref) / abs(ref)
    print(f"[diagonal] p={precision} coords={use_coords}: mean {e_mu:.1e} var {e_var:.1e} logdet {e_ld:.1e}",
          flush=True)
    assert e_mu <= 1e-13
    if precision == 0:
        assert e_var <= 1e-13 and e_ld <= 1e-13
    else:
        # the Jacobi-scaled Q_post is the identity (kappa = 1): first-order FP32 bounds
        # c kappa u32 (variances) and c n kappa u32 absolute (log-det), c = 10
        assert e_var <= 10 * O.U32 and e_ld <= 10 * p.n * O.U32 / abs(ref)


def test_single_unknown(gpu_lib):
    p = gi.Problem(1, sp.csr_matrix(np.array([[2.0]])), sp.csr_matrix(np.array([[1.0]])), np.array([4.0]),
                   np.array([0.5]), np.zeros(1), np.zeros((1, 2)))
    ctx = gpu_lib.posterior_context(p, precision=0)
    ld = ctx.logdet()[0]
    mu = ctx.solve()[0].cpu().numpy()
    var = ctx.selinv().cpu().numpy()
    ctx.close()
    assert abs(mu[0] - 1.0 / 3.0) <= 1e-15 and abs(var[0] - 1.0 / 6.0) <= 1e-16
    assert abs(ld - math.log(6.0)) <= 1e-15


@pytest.mark.parametrize("precision", [0, 1])
def test_short_chain_matches_dense_oracle(gpu_lib, precision):
    """A first-order random walk on 9 nodes plus a small diagonal (tridiagonal Q), three
    point observations: the dense oracle's mean, variances and log det."""
    n = 9
    Q = sp.diags([-np.ones(n - 1), np.r_[1.0, 2.0 * np.ones(n - 2), 1.0] + 0.1, -np.ones(n - 1)],
                 [-1, 0, 1]).tocsr()
    A = sp.csr_matrix((np.ones(3), (np.arange(3), np.array([1, 4, 7]))), shape=(3, n))
    p = gi.Problem(n, Q, A, np.full(3, 25.0), np.array([0.3, -1.0, 0.7]), np.zeros(3), None)
    ctx = gpu_lib.posterior_context(p, precision=precision, use_coords=False)
    ld = ctx.logdet()[0]
    mu = ctx.solve(max_refine=20 if precision else 0, tol=1e-14, raise_not_converged=False)[0].cpu().numpy()
    var = ctx.selinv().cpu().numpy()
    ctx.close()
    r = O.dense_posterior(p)
    e_var = np.max(np.abs(var - r["var"]) / r["var"])
    e_ld = abs(ld - r["logdet"]) / abs(r["logdet"])
    print(f"[chain] p={precision}: var {e_var:.1e} logdet {e_ld:.1e}", flush=True)
    assert np.max(np.abs(mu - r["mean"])) <= 1e-12 * np.max(np.abs(r["mean"]))
    if precision == 0:
        assert e_var <= 1e-12 and e_ld <= 1e-12
    else:
        Qp, _ = O.assemble(p.Q, p.A, p.q_eps, p.y)
        kappa = O.condition_number(Qp)[0]
        assert e_var <= 10 * kappa * O.U32 and e_ld <= 10 * n * kappa * O.U32 / abs(r["logdet"])


def test_sample_count_limits(gpu_lib):
    import torch
    p = gi.matern2d(side=12, n_obs=20, seed=92)
    ctx = gpu_lib.posterior_context(p, precision=0)
    ctx.solve()
    z = torch.zeros((17, p.n), dtype=torch.float32, device="cuda")
    x16 = ctx.sample(z[:16].contiguous())
    assert x16.shape == (16, p.n)
    with pytest.raises(gpu_lib.GmrfError) as e:
        ctx.sample(z)
    assert e.value.code == gpu_lib.GMRF_ERR_ARG
    ctx.close()
