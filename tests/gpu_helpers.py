"""Helpers shared by the GPU tests (no test functions here)."""
import numpy as np

import oracle as O


def kappa_with_solves(ctx, Q):
    """Condition number of D^-1/2 Q D^-1/2 (D = diag Q): Lanczos on the scaled matrix for
    lambda_max; Lanczos on its inverse D^1/2 Q^-1 D^1/2, applied through the context's
    FP64 factor of Q, for 1/lambda_min."""
    import scipy.sparse.linalg as spla
    import torch
    d = np.sqrt(Q.diagonal())
    hi = float(spla.eigsh(O.jacobi_scaled(Q), k=1, which="LA", tol=1e-4, return_eigenvectors=False)[0])

    def mv(v):
        t = torch.from_numpy(np.ascontiguousarray(d * np.ravel(v))).cuda()
        return d * ctx.solve_rhs(t).cpu().numpy()

    op = spla.LinearOperator(Q.shape, matvec=mv, dtype=np.float64)
    inv_lo = float(spla.eigsh(op, k=1, which="LA", tol=1e-4, return_eigenvectors=False)[0])
    return hi * inv_lo, 1.0 / inv_lo, hi
