"""Full-size checks on the 128x128x64 advection-diffusion space-time posterior (1,048,576
unknowns) in the launch configuration the benchmark times (Sec. 3.1-3.2).  The oracle
cannot factor this size, so the checks are identities the exact posterior satisfies at any
size, evaluated with the oracle's own assembly of Q_post and h:
  * mean: Q_post mu = h (relative residual);
  * selected inverse on Q's pattern: (Q_post Sigma)_ii = 1 for every row i, where the row
    sum only involves Sigma on Q's pattern; the error bound scales with the row's absolute
    sum R_i = sum_j |Q_ij Sigma_ji|;
  * samples: (x - mu)^T Q_post (x - mu) = z^T z for x = mu + P^T L^-T z;
  * FP32+refine against FP64: log-det and marginal variances, within the first-order
    bounds c kappa u32 (variances, sample identity) and c n kappa u32 (log-det), with
    kappa the condition number of the Jacobi-scaled posterior precision estimated by
    Lanczos (host products for lambda_max, the library's FP64 solves for lambda_min);
  * the prior alone (A empty): log-det against the state-space identity
    log|Q_ST| = log|Q1| + (Nt-1) log|F^-1| (App. A), which needs only factorisations of
    the 16,384-node spatial matrices G and K."""
import numpy as np
import pytest

import gmrf_inputs as gi
import oracle as O
from gpu_helpers import kappa_with_solves

pytestmark = pytest.mark.gpu


C_BOUND = 10.0


@pytest.fixture(scope="module")
def full():
    p = gi.advdiff_spacetime()
    print(f"[full] n={p.n} nnz(Q)={p.Q.nnz}", flush=True)
    Qp, h = O.assemble(p.Q, p.A, p.q_eps, p.y, p.b)
    q_on = np.asarray(gi.fem.on_pattern(Qp, p.Q).data)
    return p, Qp, h, q_on, {}


# Bound on |(Q_post Sigma)_ii - 1| / R_i.  Sigma computed from a factor with
# L L^T = P (Q_post + E) P^T is the inverse of Q_post + E, so the row residual is -(E Sigma)_ii,
# of order c u R_i with u the unit roundoff of the factor, independent of kappa; measured on
# MI355X 7.7e-15 (FP64) and 1.08e-6 (FP32), guarded at about 10x.
SIGMA_REL = {0: 1e-13, 1: 1e-5}


@pytest.mark.parametrize("precision", [0, 1])
def test_full_size_identities(gpu_lib, full, precision):
    import torch
    p, Qp, h, q_on, store = full
    if "kappa" not in store:
        c64 = gpu_lib.posterior_context(p, precision=gpu_lib.GMRF_FP64)
        store["kappa"] = kappa_with_solves(c64, Qp)
        c64.close()
        print(f"[full] kappa(Q_post^) = {store['kappa'][0]:.4e} (lambda {store['kappa'][1]:.4e} .. "
              f"{store['kappa'][2]:.4e}); c kappa u32 = {C_BOUND * store['kappa'][0] * O.U32:.3e}", flush=True)
    bound32 = C_BOUND * store["kappa"][0] * O.U32
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
        assert abs(qf - zz) <= (1e-9 if precision == 0 else min(bound32, 10.0 * FULL_FP32_MEASURED["sample"])) * zz
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
    if 0 in store and 1 in store:
        ld64, v64 = store[0]
        ld32, v32 = store[1]
        ldrel = abs(ld32 - ld64) / abs(ld64)
        verr = np.abs(v32 - v64) / v64
        vrel = float(np.max(verr))
        print(f"[full] FP32 vs FP64: log-det {ldrel:.3e} (abs {abs(ld32 - ld64):.3e}, bound "
              f"{p.n * bound32:.3e}), variances max {vrel:.3e} median {np.median(verr):.3e} "
              f"99.9% {np.quantile(verr, 0.999):.3e} (bound {bound32:.3e})", flush=True)
        assert abs(ld32 - ld64) <= p.n * bound32
        assert vrel <= bound32
        assert ldrel <= 10.0 * FULL_FP32_MEASURED["logdet"]
        assert vrel <= 10.0 * FULL_FP32_MEASURED["var"]


# FP32 errors measured on MI355X with the current kernels (regression guards at 10x):
# sample quadratic form 1.62e-7, log-det 1.93e-8 relative, variances 1.91e-3 relative
# (kappa(Q_post^) = 3.41e5, so 0.093 kappa u32: conditioning, see the scaling test)
FULL_FP32_MEASURED = {"sample": 1.62e-7, "logdet": 1.93e-8, "var": 1.91e-3}


@pytest.mark.parametrize("ns,nt", [(32, 16), (64, 32), (96, 48)])
def test_fp32_variance_error_tracks_conditioning(gpu_lib, ns, nt):
    """FP32 against FP64 variances of the same workload at growing sizes (the larger ones
    run the split-K Sigma[R', K] and panel-update branches of the full size): the error
    stays within c kappa u32 at every size, and its ratio to kappa u32 is reported."""
    p = gi.advdiff_spacetime(ns=ns, nt=nt, seed=2)
    Qp, _ = O.assemble(p.Q, p.A, p.q_eps, p.y, p.b)
    c64 = gpu_lib.posterior_context(p, precision=gpu_lib.GMRF_FP64)
    kappa = kappa_with_solves(c64, Qp)[0]
    v64 = c64.selinv().cpu().numpy()
    c64.close()
    c32 = gpu_lib.posterior_context(p, precision=gpu_lib.GMRF_FP32_REFINE)
    v32 = c32.selinv().cpu().numpy()
    c32.close()
    verr = np.abs(v32 - v64) / v64
    ratio = verr.max() / (kappa * O.U32)
    print(f"[scale {ns}x{ns}x{nt}] n={p.n} kappa={kappa:.3e} var err max {verr.max():.3e} "
          f"median {np.median(verr):.3e}; max / (kappa u32) = {ratio:.3e}", flush=True)
    # measured ratios 0.147, 0.160, 0.059 (and 0.093 at full size): the error is the
    # conditioning's, at every size; a ratio above 1 would point at accumulation
    assert ratio <= 1.0


def test_full_size_prior_logdet_state_space_identity(gpu_lib):
    """P4 at 1,048,576 unknowns: the GPU factor of the space-time prior alone (no
    observations) against log|Q1| + (Nt-1) log|F^-1|, log|F^-1| = -Ns log(tau^2 dt)
    + 2 log|det G| - 2 log|M~| + log|Sigma^-1| (white noise: Sigma^-1 = M~), from
    sparse LU factorisations of G and of K = kappa1^2 M~ + S (App. A)."""
    import math
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    import torch
    p = gi.advdiff_spacetime()
    meta = p.meta
    m, G = meta["m"], meta["G"]
    Ns = meta["ns"] ** 2

    def logabsdet(M):
        lu = spla.splu(sp.csc_matrix(M), permc_spec="COLAMD")
        return float(np.sum(np.log(np.abs(lu.U.diagonal()))) + np.sum(np.log(np.abs(lu.L.diagonal()))))

    logM = float(np.sum(np.log(m)))
    logFinv = -Ns * math.log(meta["tau"] ** 2 * meta["dt"]) + 2 * logabsdet(G) - 2 * logM + logM
    K = sp.diags(meta["kappa1"] ** 2 * m) + gi.fem.stiffness(meta["mesh"])
    logQ1 = -2 * Ns * math.log(meta["tau1"]) + 2 * logabsdet(K) - logM
    ref = logQ1 + (meta["nt"] - 1) * logFinv
    Q = p.Q.tocsr()
    qi = torch.from_numpy(Q.indptr.astype(np.int64)).cuda()
    qj = torch.from_numpy(Q.indices.astype(np.int32)).cuda()
    qv = torch.from_numpy(Q.data.astype(np.float64)).cuda()
    out = {}
    for prec in (0, 1):
        ctx = gpu_lib.Context(0)
        ctx.assemble(qi, qj, qv, None, None, None, None, None)
        ctx.analyze(p.coords)
        ctx.factor(prec)
        out[prec] = ctx.logdet()[0]
        if prec == 0:
            kappa = kappa_with_solves(ctx, Q)[0]
            st = ctx.stats()
        ctx.close()
    # FP64 within 1e-10 relative (measured 1.3e-15); FP32 within c n kappa u32 and within
    # 10x of the 1.1e-6 relative error measured on MI355X
    b64 = 1e-10 * abs(ref)
    b32 = min(p.n * C_BOUND * kappa * O.U32, 1.1e-5 * abs(ref))
    print(f"[P4 full] reference {ref:.12e}; FP64 {out[0]:.12e} (abs {abs(out[0] - ref):.3e}, bound {b64:.3e}); "
          f"FP32 {out[1]:.12e} (abs {abs(out[1] - ref):.3e}, bound {b32:.3e}); kappa(prior^) {kappa:.3e}; "
          f"nnz(L) {st['nnz_l']}", flush=True)
    assert abs(out[0] - ref) <= b64
    assert abs(out[1] - ref) <= b32
