"""ORACLE -- test infrastructure only.

A plain, slow, FP64 CPU reference of the GMRF posterior path (Sec. 3.1-3.2 of the
paper): conditioning, sparse Cholesky, triangular solves, sampling, the Takahashi
recursion for marginal variances, log-determinant, and the log marginal likelihood
with its hyper-parameter gradient.  Only the test suite, the smoke check and the
bench's CPU-baseline leg may import it; the GPU library never does, and the two share
no code.
"""
from .core import (U32, U64, Factor, NotSPDError, assemble, block_logdets, build, cg_sample_rhs, cholesky,
                   condition_number, dense_posterior, jacobi_scaled, logdet,
                   marginal_variances, nd_order, posterior, rbmc_variances, rcm_order, sample, selinv,
                   sigma_on_pattern, solve)

from .lml import lml_dense, lml_sparse
from .gn import burgers_residual_and_jacobian, gn_step, gn_step_pointwise, pointwise_residual_and_jacobian

__all__ = ["lml_dense", "lml_sparse", "burgers_residual_and_jacobian", "gn_step", "gn_step_pointwise", "pointwise_residual_and_jacobian", "U32", "U64", "cg_sample_rhs", "rbmc_variances", "condition_number", "jacobi_scaled", "Factor", "NotSPDError", "assemble", "block_logdets", "build", "cholesky",
           "dense_posterior", "logdet", "marginal_variances", "nd_order", "posterior",
           "rcm_order", "sample", "selinv", "sigma_on_pattern", "solve"]
