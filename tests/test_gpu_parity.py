"""GPU parity: the HIP path through the C ABI against the oracle, element by element, on
seeded inputs at sizes the oracle finishes in seconds that still span several tiles,
multi-block fronts and ragged tails.  FP64 results must match the oracle within 1e-10
(relative); the FP32-factor path must give the mean within 1e-8 after FP64 refinement,
and variances / log-det within the first-order bound of its rounding (c kappa u32, with
kappa the condition number of the Jacobi-scaled posterior precision) and within 10x of
the errors measured on the device."""
import math

import numpy as np
import pytest

import gmrf_inputs as gi
import oracle as O

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


# FP32 bounds (first order in the factor's backward error E, ||E|| <= c u32 ||Q^||, on the
# Jacobi-scaled posterior precision Q^ with condition number kappa): relative variance
# error and sample quadratic-form error <= c kappa u32 (|dSigma_ii| <= ||E|| ||Sigma|| Sigma_ii,
# z^T L^-1 E L^-T z <= ||E|| / lambda_min z^T z); absolute log-det error <= c n kappa u32
# (|tr(Sigma E)| <= n ||E|| / lambda_min).  c = 10 covers the accumulation constants.
C_BOUND = 10.0


def _fp32_bound(Qp):
    kappa, lo, hi = O.condition_number(Qp)
    return kappa, C_BOUND * kappa * O.U32


def _run(gpu_lib, p, precision, refine=0, tol=0.0, opts=None):
    ctx = gpu_lib.posterior_context(p, precision=precision, opts=opts)
    ld = ctx.logdet()
    mu, it, res = ctx.solve(max_refine=refine, tol=tol)
    var = ctx.selinv()
    return ctx, ld, mu.cpu().numpy(), var.cpu().numpy(), it, res


CASES_FP64 = {
    "matern2d_32": lambda: gi.matern2d(),
    "matern2d_45_ragged": lambda: gi.matern2d(side=45, kappa=3.0, n_obs=300, seed=41),
    "spacetime_16x16x8": lambda: gi.advdiff_spacetime(ns=16, nt=8, seed=42),
    "spacetime_20x20x12": lambda: gi.advdiff_spacetime(ns=20, nt=12, seed=43),
    "matern3d_12": lambda: gi.matern3d(side=12, n_obs=200, seed=44),
    "spacetime_24x24x16_multiblock": lambda: gi.advdiff_spacetime(ns=24, nt=16, seed=53),
}


_ORACLE = {}


def _oracle(name):
    """oracle posterior of a named case, computed once per test session"""
    if name not in _ORACLE:
        p = CASES_FP64[name]()
        _ORACLE[name] = (p, O.posterior(p))
    return _ORACLE[name]


@pytest.mark.parametrize("name", sorted(CASES_FP64))
def test_fp64_mean_var_logdet_match_oracle(gpu_lib, name):
    p, r = _oracle(name)
    print(f"[case] {name} n={p.n}", flush=True)
    ctx, ld, mu, var, _, res = _run(gpu_lib, p, gpu_lib.GMRF_FP64)
    assert _rel(mu, r["mean"]) <= 1e-10, _rel(mu, r["mean"])
    vrel = np.max(np.abs(var - r["var"]) / r["var"])
    assert vrel <= 1e-10, vrel
    bound = 1e-10 * np.sum(np.abs(np.log(r["factor"].Lx[r["factor"].Lp[:-1]]))) * 2
    assert abs(ld[0] - r["logdet"]) <= bound, (ld[0], r["logdet"])
    st = ctx.stats()
    assert st["failed_index"] == -1
    assert res < 1e-12
    ctx.close()


# FP32 factor / selected inversion (long products as six bf16 term products on the matrix
# cores) on the cases with multi-block fronts and ragged tails: mean within 1e-8 after FP64
# refinement; variances and log-det within the first-order bound c kappa u32 of FP32
# rounding, and within about 10x of the error measured on MI355X (a regression guard:
# FP32_MEASURED holds the errors measured with the current kernels).
FP32_MEASURED = {
    # name: (max relative variance error, relative log-det error)
    "matern2d_45_ragged": (1.420e-05, 1.520e-08),
    "matern3d_12": (1.000e-06, 2.250e-09),
    "spacetime_24x24x16_multiblock": (2.975e-05, 7.611e-09),
    "spacetime_20x20x10": (1.491e-05, 1.081e-08),
}


@pytest.mark.parametrize("name", ["matern2d_45_ragged", "matern3d_12", "spacetime_24x24x16_multiblock"])
def test_fp32_refine_matches_oracle(gpu_lib, name):
    p, r = _oracle(name)
    print(f"[case fp32] {name} n={p.n}", flush=True)
    ctx, ld, mu, var, it, res = _run(gpu_lib, p, gpu_lib.GMRF_FP32_REFINE, refine=30, tol=1e-14)
    vrel = float(np.max(np.abs(var - r["var"]) / r["var"]))
    ldabs = abs(ld[0] - r["logdet"])
    kappa, bound = _fp32_bound(r["Qpost"])
    print(f"[case fp32] {name}: kappa={kappa:.3e} bound c*kappa*u32={bound:.3e} iters={it} resid={res:.3e} "
          f"mean {_rel(mu, r['mean']):.3e} var {vrel:.3e} logdet abs {ldabs:.3e} "
          f"rel {ldabs / abs(r['logdet']):.3e} (bound n*c*kappa*u32 = {p.n * bound:.3e})", flush=True)
    assert _rel(mu, r["mean"]) <= 1e-8
    assert vrel <= bound
    assert ldabs <= p.n * bound
    if name in FP32_MEASURED:
        v_m, ld_m = FP32_MEASURED[name]
        assert vrel <= 10.0 * v_m
        assert ldabs / abs(r["logdet"]) <= 10.0 * ld_m
    assert ctx.stats()["failed_index"] == -1
    ctx.close()


def test_fp64_dense_pin_tiny(gpu_lib):
    p = gi.matern2d(side=9, n_obs=20, seed=45)
    ctx, ld, mu, var, _, _ = _run(gpu_lib, p, gpu_lib.GMRF_FP64)
    d = O.dense_posterior(p)
    assert _rel(mu, d["mean"]) <= 1e-10
    assert np.max(np.abs(var - d["var"]) / d["var"]) <= 1e-10
    assert abs(ld[0] - d["logdet"]) <= 1e-10 * abs(d["logdet"])


@pytest.mark.parametrize("precision", [0, 1])
def test_samples_match_oracle_with_library_pivot_order(gpu_lib, precision):
    import torch
    p = gi.advdiff_spacetime(ns=14, nt=6, seed=46)
    ctx = gpu_lib.posterior_context(p, precision=precision)
    mu, _, _ = ctx.solve(max_refine=20, tol=1e-13, raise_not_converged=False)
    perm = ctx.pivot_order().astype(np.int64)
    k = 5
    z = gi.standard_normal_f32(p.n, k, seed=47)          # (n, k) pivot order
    zt = torch.from_numpy(np.ascontiguousarray(z.T)).cuda()
    x = ctx.sample(zt).cpu().numpy().T                     # (n, k)
    Qp, h = O.assemble(p.Q, p.A, p.q_eps, p.y)
    F = O.cholesky(Qp, perm)
    mu_o = O.solve(F, h)
    xo = O.sample(F, mu_o, z)
    if precision == 0:
        assert np.max(np.abs(x - xo)) <= 1e-10 * np.max(np.abs(xo - mu_o[:, None]))
    # ordering-free identity (x - mu)^T Q_post (x - mu) = z^T z; FP32 factor: within
    # c kappa u32 and within 10x of the error measured on MI355X (SAMPLE_FP32_MEASURED)
    if precision == 0:
        tolr = 1e-9
    else:
        kappa, tolr = _fp32_bound(Qp)
        if SAMPLE_FP32_MEASURED is not None:
            tolr = min(tolr, 10.0 * SAMPLE_FP32_MEASURED)
    errs = []
    for c in range(k):
        d = x[:, c] - mu.cpu().numpy()
        zz = float(z[:, c].astype(np.float64) @ z[:, c].astype(np.float64))
        errs.append(abs(d @ (Qp @ d) - zz) / zz)
    print(f"[samples p={precision}] quadratic-form errors {max(errs):.3e} (tolerance {tolr:.3e})", flush=True)
    assert max(errs) <= tolr


SAMPLE_FP32_MEASURED = 1.197e-07   # max relative quadratic-form error of the FP32 samples


@pytest.mark.parametrize("precision", [0, 1])
def test_multi_rhs_sample_equals_single_rhs_samples(gpu_lib, precision):
    """Several right-hand sides in one backward pass (pairs sharing each load of L, a
    partial last pair) give bitwise the samples of one right-hand side per call: every
    column sum adds its terms in the same order either way."""
    import torch
    p = gi.matern_batch(n_prob=10, side_lo=8, side_hi=30, seed=49)
    ctx = gpu_lib.posterior_context(p, precision=precision)
    ctx.solve(max_refine=20 if precision else 0, tol=1e-12, raise_not_converged=False)
    z = torch.from_numpy(gi.rng_for(50).standard_normal((5, p.n)).astype(np.float32)).cuda()
    x = ctx.sample(z).clone()
    for r in range(5):
        assert torch.equal(ctx.sample(z[r:r + 1].contiguous())[0], x[r]), r
    ctx.close()


def test_fp32_refine_mean_and_bounds(gpu_lib):
    p = gi.advdiff_spacetime(ns=20, nt=10, seed=48)
    ctx, ld, mu, var, it, res = _run(gpu_lib, p, gpu_lib.GMRF_FP32_REFINE, refine=30, tol=1e-14)
    r = O.posterior(p)
    print(f"[fp32] iters={it} resid={res:.3e}", flush=True)
    assert _rel(mu, r["mean"]) <= 1e-8
    vrel = np.max(np.abs(var - r["var"]) / r["var"])
    ldrel = abs(ld[0] - r["logdet"]) / abs(r["logdet"])
    kappa, bound = _fp32_bound(r["Qpost"])
    print(f"[fp32] kappa={kappa:.3e} bound={bound:.3e} var max rel err {vrel:.3e}  logdet rel err {ldrel:.3e}",
          flush=True)
    assert vrel <= bound
    assert abs(ld[0] - r["logdet"]) <= p.n * bound
    if "spacetime_20x20x10" in FP32_MEASURED:
        v_m, ld_m = FP32_MEASURED["spacetime_20x20x10"]
        assert vrel <= 10.0 * v_m and ldrel <= 10.0 * ld_m


def test_batched_block_logdets_and_outputs(gpu_lib):
    p = gi.matern_batch(n_prob=7, side_lo=8, side_hi=30, seed=49)
    ctx, ld, mu, var, _, _ = _run(gpu_lib, p, gpu_lib.GMRF_FP64)
    r = O.posterior(p)
    lds = O.block_logdets(r["factor"], p.block_ptr)
    assert ld.shape == (7,)
    assert np.max(np.abs(ld - lds) / np.abs(lds)) <= 1e-10
    assert _rel(mu, r["mean"]) <= 1e-10
    assert np.max(np.abs(var - r["var"]) / r["var"]) <= 1e-10


def test_sigma_on_pattern_and_trace(gpu_lib):
    import torch
    p = gi.matern2d(side=30, n_obs=50, seed=50)
    ctx = gpu_lib.posterior_context(p, precision=gpu_lib.GMRF_FP64)
    var, sq = ctx.selinv(with_pattern=True, nnzq=p.Q.nnz)
    r = O.posterior(p)
    Qp = r["Qpost"]
    ref = O.sigma_on_pattern(r["factor"], r["sigma_L"], p.Q)
    sqn = sq.cpu().numpy()
    assert np.max(np.abs(sqn - ref)) <= 1e-10 * np.max(np.abs(ref))
    # tr(Q_post^-1 Q_post) = N through the library's deterministic dot
    qpost_on_q = torch.from_numpy(np.asarray(gi.fem.on_pattern(Qp, p.Q).data)).cuda()
    tr = ctx.dot(sq, qpost_on_q)
    assert abs(tr - p.n) <= 1e-9 * p.n


def test_update_values_refactor_matches_fresh(gpu_lib):
    import torch
    p = gi.matern2d(side=20, n_obs=40, seed=51)
    ctx = gpu_lib.posterior_context(p, precision=gpu_lib.GMRF_FP64)
    ctx.solve()
    p2 = gi.matern2d(side=20, kappa=7.0, n_obs=40, seed=51)    # same pattern, new values
    ctx.update_values(q_data=torch.from_numpy(p2.Q.data.copy()).cuda())
    ctx.factor(gpu_lib.GMRF_FP64)
    mu, _, _ = ctx.solve()
    ld = ctx.logdet()
    r = O.posterior(p2)
    assert _rel(mu.cpu().numpy(), r["mean"]) <= 1e-10
    assert abs(ld[0] - r["logdet"]) <= 1e-10 * abs(r["logdet"])


def test_not_spd_reports_original_index(gpu_lib):
    p = gi.matern2d(side=12, n_obs=5, seed=52)
    Q = p.Q.tolil()
    Q[37, 37] = -5.0
    p.Q = Q.tocsr()
    p.Q.sort_indices()
    ctx = gpu_lib.posterior_context(p, precision=gpu_lib.GMRF_FP64)
    with pytest.raises(gpu_lib.NotSPDError):
        ctx.logdet()
    st_fail = None
    try:
        ctx.stats()
    except gpu_lib.NotSPDError:
        st_fail = True
    assert st_fail


def test_call_order_errors(gpu_lib):
    ctx = gpu_lib.Context(0)
    with pytest.raises(gpu_lib.GmrfError) as e:
        ctx.factor(0)
    assert e.value.code == gpu_lib.GMRF_ERR_STATE


@pytest.mark.parametrize("precision", [0, 1])
def test_async_selinv_overlapping_solves_matches_sequential(gpu_lib, precision):
    """The selected inversion started on the second stream while the mean, a sample and
    the log-determinant are computed on the context's stream gives bitwise the results of
    the sequential calls (every reduction has a fixed order), also when repeated after a
    refactorisation."""
    import torch
    p = gi.advdiff_spacetime(ns=24, nt=16, seed=61)
    ctx = gpu_lib.posterior_context(p, precision=precision)
    refine = 20 if precision == 1 else 0
    z = torch.from_numpy(gi.rng_for(62).standard_normal((2, p.n)).astype(np.float32)).cuda()
    var_s, sq_s = ctx.selinv(with_pattern=True, nnzq=p.Q.nnz)
    mu_s = ctx.solve(max_refine=refine, tol=1e-12)[0].clone()
    x_s = ctx.sample(z).clone()
    ld_s = ctx.logdet()
    for _ in range(2):
        ctx.factor(precision)
        var_a, sq_a = ctx.selinv_submit(with_pattern=True, nnzq=p.Q.nnz)
        mu_a = ctx.solve(max_refine=refine, tol=1e-12)[0].clone()
        x_a = ctx.sample(z).clone()
        ld_a = ctx.logdet()
        ctx.selinv_wait()
        assert torch.equal(var_a, var_s) and torch.equal(sq_a, sq_s)
        assert torch.equal(mu_a, mu_s) and torch.equal(x_a, x_s)
        assert np.array_equal(ld_a, ld_s)
    ctx.close()
