"""Seeded synthetic inputs for the GMRF posterior path (FEM priors, observation
operators, data).  Shared by the GPU path's tests/bench and by the oracle; holds none
of the posterior computation itself."""
from .configs import (Problem, advdiff_derivatives, advdiff_spacetime, advdiff_values, batch_block, burgers_spacetime, darcy_p2, elliptic_cubic, manufactured_cubic, matern2d, matern3d, matern_batch,
                      matern_from_pieces, matern_pieces, prior_sqrt, rng_for, smooth_target,
                      standard_normal_f32)

__all__ = ["Problem", "advdiff_derivatives", "advdiff_spacetime", "advdiff_values", "batch_block", "burgers_spacetime", "darcy_p2", "elliptic_cubic", "manufactured_cubic", "matern2d", "matern3d", "matern_batch",
           "prior_sqrt", "rng_for", "smooth_target", "standard_normal_f32", "matern_pieces",
           "matern_from_pieces"]
