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

The same identity with derivatives of the observation operator gives the gradient with
respect to the advection speed c and viscosity nu of the space-time prior, whose Galerkin
PDE rows depend on them too (SpaceTimeLML).  Every step -- log-dets, refined mean,
selected inversions, traces, quadratic forms and their combination -- runs inside the
library call gmrf_lml_gradient; this module prepares derivative inputs and marshals.
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
        """Returns (LML, gradient w.r.t. (log kappa, log tau, log sigma) or None); the
        log-dets, refined mean, selected inversions, traces and reductions all run in
        gmrf_lml_gradient."""
        torch = self.torch
        self._factor(log_kappa, log_tau, log_sigma)
        refine = 30 if self.precision == binding.GMRF_FP32_REFINE else 0
        self.mu = torch.empty(self.n, dtype=torch.float64, device=self.dev)
        if gradient:
            # dQ/dlog kappa from the Matern kernel, dQ/dlog tau = -2 Q, dQ_eps/dlog sigma = -2 Q_eps
            dq = torch.stack([self.dq, -2.0 * self.q, torch.zeros_like(self.q)])
            dqeps = torch.stack([torch.zeros_like(self.qeps), torch.zeros_like(self.qeps), -2.0 * self.qeps])
            return self.post.lml_gradient(self.prior, dq=dq, dqeps=dqeps, max_refine=refine, tol=1e-13,
                                          mu_out=self.mu)
        lml, _ = self.post.lml_gradient(self.prior, max_refine=refine, tol=1e-13, mu_out=self.mu)
        return lml, None

    def mean_adjoint(self, grad_mu):
        """dl/d(log kappa, log tau, log sigma) for a loss with gradient grad_mu w.r.t. the
        posterior mean of the last evaluate()."""
        lam = self.post.solve_rhs(grad_mu.contiguous())
        self.post.spmv(self.dq, self.mu, self.tmp)
        g_k = -self.post.dot(lam, self.tmp)
        self.post.spmv(self.q, self.mu, self.tmp)
        lqm = self.post.dot(lam, self.tmp)
        return np.array([g_k, 2.0 * lqm, -2.0 * lqm])


class SpaceTimeLML:
    """LML of the advection-diffusion space-time workload (Sec. 2.4, App. A) as a function of
    the advection speed c and the viscosity nu, and its adjoint gradient.  Both enter the
    prior through G = M~ + dt (nu S + c C) and the Galerkin PDE observation rows through
    the same G (Sec. 3.1), so the gradient carries the observation-operator terms of
    gmrf_lml_gradient.  The prior and posterior contexts keep one pattern, analysed once
    and refactored per parameter value (Sec. 3.3); the values of Q, A and of their
    derivatives on those patterns come from the workload's generator."""

    def __init__(self, problem, device=0, precision=binding.GMRF_FP64):
        import gmrf_inputs as gi
        import torch
        self.torch = torch
        self.gi = gi
        self.p = problem
        self.dev = f"cuda:{device}"
        self.precision = precision
        d = binding.problem_to_device(problem, self.dev)
        self.prior = binding.Context(device)
        self.post = binding.Context(device)
        self.prior.assemble(d["q_indptr"], d["q_indices"], d["q_data"], None, None, None, None, None)
        self.post.assemble(**d)
        self.prior.analyze(problem.coords)
        self.post.analyze(problem.coords)
        self._keep = d

    def close(self):
        self.prior.close()
        self.post.close()

    def evaluate(self, c, nu, gradient=True):
        """Returns (LML, gradient w.r.t. (c, nu) or None)."""
        torch = self.torch
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(self.dev, torch.float64)  # noqa: E731
        q, a = self.gi.advdiff_values(self.p, float(c), float(nu))
        qd, ad = t(q), t(a)
        self.prior.update_values(q_data=qd)
        self.post.update_values(q_data=qd, a_data=ad)
        self.prior.factor(self.precision)
        self.post.factor(self.precision)
        refine = 30 if self.precision == binding.GMRF_FP32_REFINE else 0
        if not gradient:
            return self.post.lml_gradient(self.prior, max_refine=refine, tol=1e-13)[0], None
        der = self.gi.advdiff_derivatives(self.p, c=float(c), nu=float(nu))
        dq = t(np.stack([der["c"][0], der["nu"][0]]))
        da = t(np.stack([der["c"][1], der["nu"][1]]))
        return self.post.lml_gradient(self.prior, dq=dq, da=da, max_refine=refine, tol=1e-13)


def _torch_function():
    import torch

    class GMRFLogML(torch.autograd.Function):
        """LML(theta) with the hand-written adjoint gradient of an engine: MaternLML
        (theta = log kappa, log tau, log sigma) or SpaceTimeLML (theta = c, nu)."""

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
    """Differentiable LML(theta) (torch); theta as the engine takes it."""
    return _torch_function()[0].apply(theta, engine)


def posterior_mean(theta, engine):
    """Differentiable posterior mean (torch) with the hand-written adjoint."""
    return _torch_function()[1].apply(theta, engine)
