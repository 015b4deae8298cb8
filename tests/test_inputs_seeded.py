"""The synthetic workloads are seeded: the same seed gives byte-identical inputs (patterns,
values, observations, coordinates), another seed gives other random parts, and every
generated precision is symmetric with sorted CSR rows, the form the library's analysis
takes."""
import numpy as np
import pytest
import scipy.sparse as sp

import gmrf_inputs as gi

MAKERS = {
    "matern2d": lambda s: gi.matern2d(side=12, seed=s),
    "advdiff_spacetime": lambda s: gi.advdiff_spacetime(ns=8, nt=4, seed=s),
    "advdiff_matern_noise": lambda s: gi.advdiff_spacetime(ns=8, nt=4, seed=s, noise="matern"),
    "matern_batch": lambda s: gi.matern_batch(n_prob=4, side_lo=5, side_hi=9, seed=s),
    "matern3d": lambda s: gi.matern3d(side=6, n_obs=20, seed=s),
    "burgers_spacetime": lambda s: gi.burgers_spacetime(nx=16, nt=8, seed=s),
    "darcy_p2": lambda s: gi.darcy_p2(8, seed=s),
}


def _arrays(p):
    out = [p.Q.indptr, p.Q.indices, p.Q.data, p.A.indptr, p.A.indices, p.A.data, p.q_eps, p.y, p.b,
           p.coords]
    if p.block_ptr is not None:
        out.append(p.block_ptr)
    return [np.asarray(a) for a in out]


@pytest.mark.parametrize("name", sorted(MAKERS))
def test_same_seed_same_bytes_other_seed_other_data(name):
    a, b, c = MAKERS[name](11), MAKERS[name](11), MAKERS[name](12)
    for x, y in zip(_arrays(a), _arrays(b)):
        assert x.dtype == y.dtype and x.shape == y.shape and x.tobytes() == y.tobytes()
    assert any(x.shape != z.shape or x.tobytes() != z.tobytes() for x, z in zip(_arrays(a), _arrays(c)))
    Q = sp.csr_matrix(a.Q)
    assert abs(Q - Q.T).max() <= 1e-12 * abs(Q).max()
    assert Q.has_sorted_indices
    assert a.A.shape == (a.y.size, a.n) and a.q_eps.size == a.y.size and np.all(a.q_eps > 0)


def test_normal_draws_are_seeded():
    z1, z2, z3 = (gi.standard_normal_f32(50, 3, seed=s) for s in (1, 1, 2))
    assert z1.dtype == np.float32 and z1.tobytes() == z2.tobytes() and z1.tobytes() != z3.tobytes()
