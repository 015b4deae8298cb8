"""Full-size checks on the 128x128x64 advection-diffusion space-time posterior (1,048,576
unknowns) in the launch configuration the benchmark times (Sec. 3.1-3.2).  The oracle
cannot factor this size, so the checks are identities the exact posterior satisfies at any
size, evaluated with the oracle's own assembly of Q_post and h:
  * mean: Q_post mu = h (relative residual);
  * selected inverse on Q's pattern: (Q_post Sigma)_ii = 1 for every row i, where the row
    sum only involves Sigma on Q's pattern; the error bound scales with the row's absolute
    sum R_i = sum_j |Q_ij Sigma_ji|;
  * samples: (x - mu)^T Q_post (x - mu) = z^T z for x = mu + P^T L^-T z;
  * FP32+refine against FP64: log-det and marginal variances."""
import numpy as np
import pytest

import gmrf_inputs as gi
import oracle as O

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def full():
    p = gi.advdiff_spacetime()
    print(f"[full] n={p.n} nnz(Q)={p.Q.nnz}", flush=True)
    Qp, h = O.assemble(p.Q, p.A, p.q_eps, p.y, p.b)
    q_on = np.asarray(gi.fem.on_pattern(Qp, p.Q).data)
    return p, Qp, h, q_on, {}


# Bound on |(Q_post Sigma)_ii - 1| / R_i.  Sigma computed from a factor with
# L L^T = P (Q_post + E) P^T is the inverse of Q_post + E, so the row residual is -(E Sigma)_ii,
# of order c u R_i with u the unit roundoff of the factor (c: accumulation lengths, taken
# as 1e3): 1e-13 -> 1e-11 for the FP64 factor, 6e-8 -> 1e-4 for the FP32 one.
SIGMA_REL = {0: 1e-11, 1: 1e-4}


@pytest.mark.parametrize("precision", [0, 1])
def test_full_size_identities(gpu_lib, full, precision):
    import torch
    p, Qp, h, q_on, store = full
    ctx = gpu_lib.posterior_context(p, precision=precision)
    ld = ctx.logdet()
    mu, it, res = ctx.solve(max_refine=30 if precision == 1 else 0, tol=1e-12, raise_not_converged=False)
    mu = mu.cpu().numpy()
    r = Qp @ mu - h
    rel = float(np.linalg.norm(r) / np.linalg.norm(h))
    print(f"[full p={precision}] mean residual {rel:.3e} (refine iters {it})", flush=True)
    assert rel <= 1e-10
    z = gi.standard_normal_f32(p.n, 2, seed=71)
    x = ctx.sample(torch.from_numpy(np.ascontiguousarray(z.T)).cuda()).cpu().numpy().T
    for c in range(2):
        d = x[:, c] - mu
        zz = float(z[:, c].astype(np.float64) @ z[:, c].astype(np.float64))
        qf = float(d @ (Qp @ d))
        print(f"[full p={precision}] sample {c}: quadratic form / z'z - 1 = {qf / zz - 1:.3e}", flush=True)
        assert abs(qf - zz) <= (1e-9 if precision == 0 else 2e-2) * zz
    var, sq = ctx.selinv(with_pattern=True, nnzq=p.Q.nnz)
    var = var.cpu().numpy()
    sq = sq.cpu().numpy()
    starts = p.Q.indptr[:-1]
    rows = np.add.reduceat(q_on * sq, starts)
    absrow = np.add.reduceat(np.abs(q_on * sq), starts)
    dev = np.abs(rows - 1.0) / absrow
    print(f"[full p={precision}] max |(Q Sigma)_ii - 1| = {np.max(np.abs(rows - 1.0)):.3e}, "
          f"relative to R_i: {np.max(dev):.3e}", flush=True)
    assert np.all(var > 0)
    assert np.max(dev) <= SIGMA_REL[precision]
    store[precision] = (ld[0], var)
    ctx.close()
    if len(store) == 2:
        ld64, v64 = store[0]
        ld32, v32 = store[1]
        ldrel = abs(ld32 - ld64) / abs(ld64)
        vrel = float(np.max(np.abs(v32 - v64) / v64))
        print(f"[full] FP32 vs FP64: log-det {ldrel:.3e}, variances {vrel:.3e}", flush=True)
        assert ldrel <= 1e-6
        assert vrel <= 5e-3
