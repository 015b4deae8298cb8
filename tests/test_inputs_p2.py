"""Pins of the quadratic-triangle (P2) workload and of the linear-constraint boundaries
(App. B), on the CPU.

  * element matrices against exact integration in barycentric coordinates
    (int lambda0^a lambda1^b lambda2^c = 2|T| a! b! c! / (a+b+c+2)!), and the consistent mass
    against the textbook P2 table; HRZ lumped weights |T|/19 (vertices) and 16|T|/57
    (midpoints);
  * the column operation of App. B: A' u equals A u for every u that satisfies the
    constraints;
  * FEM with the constraints converges to the PDE solution at the P2 rate (Dirichlet:
    -Laplace u = f; periodic: -Laplace u + u = f on the torus);
  * prior: a constrained unknown is N(0, eps^2) and independent of the rest; on the torus
    every vertex has the same marginal variance (the mesh is invariant under cell shifts);
  * posterior (oracle): with FEM observations of the Darcy problem and vanishing noise the
    posterior mean is the FEM solution of the constrained system."""
import math

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import gmrf_inputs as gi
import oracle as O
from gmrf_inputs import p2


# ----------------------------------------------------------- exact barycentric integration
def _pmul(a, b):
    out = {}
    for ka, va in a.items():
        for kb, vb in b.items():
            k = tuple(x + y for x, y in zip(ka, kb))
            out[k] = out.get(k, 0.0) + va * vb
    return out


def _pint(poly, area):
    s = 0.0
    for (a, b, c), v in poly.items():
        s += v * 2.0 * area * math.factorial(a) * math.factorial(b) * math.factorial(c) / math.factorial(a + b + c + 2)
    return s


def _pdiff(poly, j):
    out = {}
    for k, v in poly.items():
        if k[j] > 0:
            kk = list(k); kk[j] -= 1
            out[tuple(kk)] = out.get(tuple(kk), 0.0) + v * k[j]
    return out


def _e(i):
    return tuple(1 if j == i else 0 for j in range(3))


def _basis_bary():
    lam = [{_e(i): 1.0} for i in range(3)]
    one = {(0, 0, 0): 1.0}
    phis = [_pmul(lam[i], {**{k: 2.0 * v for k, v in lam[i].items()}, (0, 0, 0): -1.0}) for i in range(3)]
    for i, j in ((0, 1), (1, 2), (2, 0)):
        phis.append({k: 4.0 * v for k, v in _pmul(lam[i], lam[j]).items()})
    del one
    return phis


def _exact_element(verts):
    P = np.vstack([np.ones(3), verts.T])          # [1; x; y] = P lambda
    G = np.linalg.inv(P)[:, 1:]                   # grad lambda_j = G[j]
    area = abs(np.linalg.det(P)) / 2.0
    phis = _basis_bary()
    M = np.array([[_pint(_pmul(a, b), area) for b in phis] for a in phis])
    S = np.zeros((6, 6))
    for i, a in enumerate(phis):
        for k, b in enumerate(phis):
            S[i, k] = sum((G[j] @ G[l]) * _pint(_pmul(_pdiff(a, j), _pdiff(b, l)), area)
                          for j in range(3) for l in range(3))
    return M, S, area


@pytest.mark.parametrize("verts", [np.array([[0, 0], [0.25, 0], [0.25, 0.25]]),
                                   np.array([[0, 0], [0.25, 0.25], [0, 0.25]]),
                                   np.array([[0.1, 0.2], [0.7, 0.3], [0.3, 0.9]])])
def test_p2_element_matrices_exact(verts):
    M, S = p2.element_matrices(verts.astype(float))
    Me, Se, area = _exact_element(verts.astype(float))
    assert np.allclose(M, Me, rtol=0, atol=1e-14 * area * 10)
    assert np.allclose(S, Se, rtol=0, atol=1e-13)
    # textbook consistent P2 mass (vertices 0..2, midpoints of edges 01, 12, 20)
    tab = np.array([[6, -1, -1, 0, -4, 0], [-1, 6, -1, 0, 0, -4], [-1, -1, 6, -4, 0, 0],
                    [0, 0, -4, 32, 16, 16], [-4, 0, 0, 16, 32, 16], [0, -4, 0, 16, 16, 32]]) * area / 180.0
    assert np.allclose(M, tab, rtol=0, atol=1e-15)


def test_p2_global_matrices_and_hrz_weights():
    mesh = p2.P2Mesh(7)
    S, M, m = mesh.stiffness(), mesh.mass(), mesh.lumped_mass()
    x, y = mesh.coords[:, 0], mesh.coords[:, 1]
    assert np.max(np.abs(S @ np.ones(mesh.n))) < 1e-13
    # exact for global quadratics: grad(x^2 - y^2 + xy) . grad(x y + 3 y^2)
    u, v = x**2 - y**2 + x * y, x * y + 3 * y**2
    # integral over the unit square of (2x + y) y + (x - 2y)(x + 6y) = x^2 + 6xy - 11y^2
    exact = 1 / 3 + 6 / 4 - 11 / 3
    assert abs(u @ S @ v - exact) < 1e-12
    assert abs((x * x) @ M @ (y * y) - 1 / 9) < 1e-14          # u^T M v = int u v on P2
    # HRZ lumping: a vertex collects |T|/19 from each of its triangles, a midpoint 16|T|/57
    a = mesh.h**2 / 2
    g = mesh.g
    I, J = np.arange(mesh.n) % g, np.arange(mesh.n) // g
    vint = (I % 2 == 0) & (J % 2 == 0) & (I > 0) & (J > 0) & (I < g - 1) & (J < g - 1)
    mid = (I % 2 == 1) & (J % 2 == 0) & (J > 0) & (J < g - 1)
    assert np.allclose(m[vint], 6 * a / 19, rtol=1e-14)
    assert np.allclose(m[mid], 2 * 16 * a / 57, rtol=1e-14)
    assert abs(m.sum() - 1.0) < 1e-14


def test_column_operation_preserves_constrained_products():
    rng = np.random.default_rng(3)
    mesh = p2.P2Mesh(5)
    A = mesh.stiffness() + sp.diags(rng.uniform(1, 2, mesh.n))
    k, h = mesh.periodic_pairs()
    c = rng.uniform(-2, 2, k.size)
    Ac = p2.constrain_columns(A, k, h, c)
    u = rng.standard_normal(mesh.n)
    u_c = u.copy()
    u_c[k] = c * u[h]                      # satisfies the constraints
    assert np.allclose(A @ u_c, Ac @ u, rtol=0, atol=1e-13)
    assert np.all(np.abs(Ac[:, k]).sum(axis=0) == 0)
    # Dirichlet (no h): the columns simply vanish
    bd = mesh.boundary_nodes()
    Ad = p2.constrain_columns(A, bd, -np.ones(bd.size, dtype=np.int64), np.ones(bd.size))
    u_d = u.copy(); u_d[bd] = 0.0
    assert np.allclose(A @ u_d, Ad @ u, rtol=0, atol=1e-13)


def _fem_error(v, kind):
    mesh = p2.P2Mesh(v)
    x, y = mesh.coords[:, 0], mesh.coords[:, 1]
    S, M = mesh.stiffness(), mesh.mass()
    if kind == "dirichlet":
        u = np.sin(math.pi * x) * np.sin(math.pi * y)
        f = 2 * math.pi**2 * u
        K = S
        con = mesh.boundary_nodes(); tgt = -np.ones(con.size, dtype=np.int64)
    else:
        u = np.cos(2 * math.pi * x) * np.sin(2 * math.pi * y + 0.3)
        f = (8 * math.pi**2 + 1) * u
        K = S + M
        con, tgt = mesh.periodic_pairs()
    Kc, _ = p2.constrain_fem(K, np.ones(mesh.n), con, tgt, np.ones(con.size), 1.0)
    T = p2.constraint_matrix(mesh.n, con, tgt, np.ones(con.size))
    b = T.T @ (M @ f)                      # the load vector, eliminated the same way
    b[con] = 0.0
    uh = spla.spsolve(Kc.tocsc(), b)
    uh[con] = 0.0
    uh = T @ uh                            # field values at every node
    return float(np.max(np.abs(uh - u)))


@pytest.mark.parametrize("kind", ["dirichlet", "periodic"])
def test_constrained_fem_converges_at_p2_rate(kind):
    e = [_fem_error(v, kind) for v in (5, 9, 17)]
    rates = [math.log2(e[i] / e[i + 1]) for i in range(2)]
    assert e[-1] < (2e-4 if kind == "dirichlet" else 5e-4), e
    assert min(rates) > 2.7, (e, rates)


@pytest.mark.parametrize("boundary,alpha", [("dirichlet", 3), ("dirichlet", 2), ("periodic", 3), ("periodic", 2)])
def test_constrained_prior_variance_and_torus_invariance(boundary, alpha):
    p = gi.darcy_p2(6, boundary=boundary, alpha=alpha, observations="points", n_obs=20, eps2=1e-6)
    C = np.linalg.inv(p.Q.toarray())
    con = p.meta["constrained"]
    free = p.meta["free"]
    assert np.allclose(np.diag(C)[con], 1e-6, rtol=1e-9)
    assert np.max(np.abs(C[np.ix_(con, free)])) < 1e-12
    if boundary == "periodic":
        g = p.meta["mesh"].g
        I, J = np.arange(p.n) % g, np.arange(p.n) // g
        for sel in [(I % 2 == 0) & (J % 2 == 0), (I % 2 == 1) & (J % 2 == 0), (I % 2 == 1) & (J % 2 == 1)]:
            d = np.diag(C)[sel & (I < g - 1) & (J < g - 1)]
            assert np.max(d) - np.min(d) <= 1e-11 * np.max(d)


def test_darcy_posterior_mean_is_fem_solution_in_the_noise_limit():
    p = gi.darcy_p2(8, boundary="dirichlet", alpha=3, sigma_pde=1e-9)
    m = p.meta
    free = m["free"]
    Sa = m["S_a"].tocsr()
    u_fem = spla.spsolve(Sa[free][:, free].tocsc(), m["load"][free])
    r = O.posterior(p, variances=False)
    mu = r["mean"]
    assert np.max(np.abs(mu[m["constrained"]])) < 1e-12
    rel = np.linalg.norm(mu[free] - u_fem) / np.linalg.norm(u_fem)
    assert rel < 1e-7, rel
    # the permeability takes both values
    assert set(np.unique(np.concatenate([m["a_lower"], m["a_upper"]]))) == {3.0, 12.0}
