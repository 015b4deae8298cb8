"""Log marginal likelihood of SPDE hyper-parameters and its adjoint gradient, on the GPU.

For a Whittle-Matern prior Q(kappa, tau) = tau^-2 K M~^-1 K, K = kappa^2 M~ + S (Sec. 2.2)
and point data y | u ~ N(A u + b, sigma^2 I) (Sec. 3.1), with mu_post the posterior mean
and r = y - b - A mu_post,

  LML = -M/2 log 2 pi + 1/2 log|Q| + 1/2 log|Q_eps| - 1/2 log|Q_post|
        - 1/2 mu_post^T Q mu_post - 1/2 r^T Q_eps r

(the Gaussian identity log p(y) = log p(y|u) + log p(u) - log p(u|y) at u = mu_post).
Differentiating at u = mu_post drops the terms through mu_post, leaving selected-inverse
traces on Q's pattern (the Takahashi entries of Sec. 3.2 are exactly what they need):

  dLML = 1/2 tr(Q^-1 dQ) + 1/2 tr(Q_eps^-1 dQ_eps) - 1/2 tr(Q_post^-1 (dQ + A^T dQ_eps A))
         - 1/2 mu^T dQ mu - 1/2 r^T dQ_eps r
  d/dlog kappa: dQ = 4 kappa^2 tau^-2 K;   d/dlog tau: dQ = -2 Q;   d/dlog sigma: dQ_eps = -2 Q_eps,
  with tr(Q_post^-1 A^T Q_eps A) = N - tr(Q_post^-1 Q).

Posterior-mean adjoint for a loss l(mu_post): lambda = Q_post^-1 dl/dmu (one extra solve),
dl/dtheta = lambda^T (dh - dQ_post mu_post); h does not depend on kappa, tau and gives
dh/dlog sigma = -2 h, which cancels against Q_post mu = h, so
  dl/dlog kappa = -lambda^T dQ mu,  dl/dlog tau = 2 lambda^T Q mu,  dl/dlog sigma = -2 lambda^T Q mu.

Every step runs in the library's kernels; this module marshals arguments and combines the
returned scalars.
"""
from __future__ import annotations

import math

import numpy as np

from . import binding


class MaternLML:
    """Prior and posterior contexts sharing one pattern, analysed once, refactored per
    hyper-parameter value (the reordering is reused, Sec. 3.3)."""

    def __init__(self, q_indptr, q_indices, m_on_q, s_on_q, sms_on_q, A, y, b=None, coords=None,
                 device=0, precision=binding.GMRF_FP64):
        import torch
        self.torch = torch
        self.dev = f"cuda:{device}"
        self.precision = precision
        t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a)).to(self.dev, dt)  # noqa: E731
        self.n = int(len(q_indptr) - 1)
        self.qi = t(q_indptr, torch.int64)
        self.qj = t(q_indices, torch.int32)
        self.mv = t(m_on_q, torch.float64)
        self.sv = t(s_on_q, torch.float64)
        self.smsv = t(sms_on_q, torch.float64)
        self.nnz = int(self.mv.numel())
        self.m = int(A.shape[0])
        self.ai = t(A.indptr, torch.int64)
        self.aj = t(A.indices, torch.int32)
        self.av = t(A.data, torch.float64)
        self.y = t(y, torch.float64)
        self.b = None if b is None else t(b, torch.float64)
        self.q = torch.empty(self.nnz, dtype=torch.float64, device=self.dev)
        self.dq = torch.empty_like(self.q)
        self.qeps = torch.ones(self.m, dtype=torch.float64, device=self.dev)
        self.prior = binding.Context(device)
        self.post = binding.Context(device)
        self.prior.matern_values(self.mv, self.sv, self.smsv, 1.0, 1.0, self.q, self.dq)
        self.prior.assemble(self.qi, self.qj, self.q, None, None, None, None, None)
        self.post.assemble(self.qi, self.qj, self.q, self.ai, self.aj, self.av, self.qeps, self.y, self.b)
        self.prior.analyze(coords)
        self.post.analyze(coords)
        self.tmp = torch.empty(self.n, dtype=torch.float64, device=self.dev)
        self.mu = None

    def close(self):
        self.prior.close()
        self.post.close()

    def _factor(self, log_kappa, log_tau, log_sigma):
        kappa, tau, sigma = math.exp(log_kappa), math.exp(log_tau), math.exp(log_sigma)
        self.post.matern_values(self.mv, self.sv, self.smsv, kappa, tau, self.q, self.dq)
        self.qeps.fill_(1.0 / (sigma * sigma))
        self.prior.update_values(q_data=self.q)
        self.post.update_values(q_data=self.q, q_eps=self.qeps)
        self.prior.factor(self.precision)
        self.post.factor(self.precision)
        return sigma

    def evaluate(self, log_kappa, log_tau, log_sigma, gradient=True):
        """Returns (LML, gradient w.r.t. (log kappa, log tau, log sigma) or None)."""
        sigma = self._factor(log_kappa, log_tau, log_sigma)
        N, M = self.n, self.m
        ld_prior = float(self.prior.logdet()[0])
        ld_post = float(self.post.logdet()[0])
        refine = 30 if self.precision == binding.GMRF_FP32_REFINE else 0
        mu, _, _ = self.post.solve(max_refine=refine, tol=1e-13, raise_not_converged=False)
        self.mu = mu
        self.post.spmv(self.q, mu, self.tmp)
        quad = self.post.dot(mu, self.tmp)                      # mu^T Q mu
        misfit = self.post.misfit(mu)                           # r^T Q_eps r
        logdet_qeps = -2.0 * M * math.log(sigma)
        lml = (-0.5 * M * math.log(2.0 * math.pi) + 0.5 * ld_prior + 0.5 * logdet_qeps
               - 0.5 * ld_post - 0.5 * quad - 0.5 * misfit)
        if not gradient:
            return lml, None
        _, sig_prior = self.prior.selinv(with_pattern=True, nnzq=self.nnz)
        _, sig_post = self.post.selinv(with_pattern=True, nnzq=self.nnz)
        tr_prior_dq = self.post.dot(sig_prior, self.dq)
        tr_post_dq = self.post.dot(sig_post, self.dq)
        tr_post_q = self.post.dot(sig_post, self.q)
        self.post.spmv(self.dq, mu, self.tmp)
        mu_dq_mu = self.post.dot(mu, self.tmp)
        g_kappa = 0.5 * tr_prior_dq - 0.5 * tr_post_dq - 0.5 * mu_dq_mu
        g_tau = -N + tr_post_q + quad
        g_sigma = -M + (N - tr_post_q) + misfit
        return lml, np.array([g_kappa, g_tau, g_sigma])

    def mean_adjoint(self, grad_mu):
        """dl/d(log kappa, log tau, log sigma) for a loss with gradient grad_mu w.r.t. the
        posterior mean of the last evaluate()."""
        lam = self.post.solve_rhs(grad_mu.contiguous())
        self.post.spmv(self.dq, self.mu, self.tmp)
        g_k = -self.post.dot(lam, self.tmp)
        self.post.spmv(self.q, self.mu, self.tmp)
        lqm = self.post.dot(lam, self.tmp)
        return np.array([g_k, 2.0 * lqm, -2.0 * lqm])


def _torch_function():
    import torch

    class GMRFLogML(torch.autograd.Function):
        """LML(theta) for theta = (log kappa, log tau, log sigma) with the hand-written
        adjoint gradient of MaternLML."""

        @staticmethod
        def forward(ctx, theta, engine):
            th = theta.detach().cpu().double().tolist()
            lml, g = engine.evaluate(*th)
            ctx.save_for_backward(torch.as_tensor(g, dtype=theta.dtype, device=theta.device))
            return torch.as_tensor(lml, dtype=theta.dtype, device=theta.device)

        @staticmethod
        def backward(ctx, grad_out):
            (g,) = ctx.saved_tensors
            return grad_out * g, None

    class GMRFPosteriorMean(torch.autograd.Function):
        """Posterior mean mu_post(theta) with the one-solve adjoint of MaternLML."""

        @staticmethod
        def forward(ctx, theta, engine):
            th = theta.detach().cpu().double().tolist()
            engine.evaluate(*th, gradient=False)
            ctx.engine = engine
            ctx.tdtype, ctx.tdev = theta.dtype, theta.device
            return engine.mu.clone()

        @staticmethod
        def backward(ctx, grad_mu):
            g = ctx.engine.mean_adjoint(grad_mu.double())
            return torch.as_tensor(g, dtype=ctx.tdtype, device=ctx.tdev), None

    return GMRFLogML, GMRFPosteriorMean


def log_ml(theta, engine):
    """Differentiable LML(theta) (torch); theta = (log kappa, log tau, log sigma)."""
    return _torch_function()[0].apply(theta, engine)


def posterior_mean(theta, engine):
    """Differentiable posterior mean (torch) with the hand-written adjoint."""
    return _torch_function()[1].apply(theta, engine)
