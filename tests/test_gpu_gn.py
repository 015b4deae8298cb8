"""GPU Gauss-Newton on the nonlinear Burgers space-time problem: each iteration against
the oracle's step from the same iterate (linearised posterior mean, line search,
decrement) in FP64 and in FP32 with FP64-residual refinement, hipGraph replays against
eager iterations (every iteration's record and the final iterate bitwise equal, also
across calls with new arguments and regrown buffers), and the full 1024 x 1024 problem
in FP32 with FP64 residuals against FP64, both run to convergence."""
import numpy as np
import pytest

import gmrf_inputs as gi
import oracle as O
from gmrf_inputs import fem

pytestmark = pytest.mark.gpu


def _dev(gpu_lib, p, precision=0):
    import torch
    ctx = gpu_lib.posterior_context(p, precision=precision)
    m = p.meta
    mass = torch.from_numpy(np.ascontiguousarray(m["mass"])).cuda()
    s3 = torch.from_numpy(np.ascontiguousarray(m["s3"].ravel())).cuda()
    return ctx, mass, s3


def _S(nx):
    full = fem.structured_mesh((nx + 2,), lo=(-1.0,), hi=(1.0,))
    inner = np.arange(1, nx + 1)
    return fem.stiffness(full)[inner][:, inner].tocsr()


@pytest.mark.parametrize("precision", [0, 1])
def test_gn_iterations_match_oracle_from_same_iterate(gpu_lib, precision):
    """Per-iteration parity (the oracle's step from the GPU's iterate).  FP32 factor:
    the linearised solve is refined with FP64 residuals to 1e-13, so the step matches
    the FP64 oracle to the refinement accuracy, not to FP32 rounding."""
    import torch
    p = gi.burgers_spacetime(nx=40, nt=32, seed=101, range_s=0.2)
    m = p.meta
    ctx, mass, s3 = _dev(gpu_lib, p, precision)
    S = _S(m["nx"])
    u = torch.zeros(p.n, dtype=torch.float64, device="cuda")
    refine, tol = (1, 0.0) if precision == 0 else (12, 1e-13)
    for it in range(3):
        u_in = u.cpu().numpy().copy()
        rec = ctx.gn_burgers(m["nx"], m["nt"], m["dt"], m["nu"], mass, s3, u, iters=1, precision=precision,
                             refine=refine, use_graph=False, refine_tol=tol)[0]
        uo, ro = O.gn_step(p.Q, u_in, p.y, p.q_eps, m["nx"], m["nt"], m["dt"], m["nu"], m["mass"], S)
        u_out = u.cpu().numpy()
        err = np.linalg.norm(u_out - uo) / np.linalg.norm(uo)
        print(f"[gn] precision {precision} it {it}: phi {rec[0]:.10e} / {ro['phi0']:.10e} alpha {rec[1]} / "
              f"{ro['alpha']} decrement {rec[2]:.4e} / {ro['decrement']:.4e} step err {err:.2e} "
              f"solve resid {rec[4]:.2e} after {rec[5]:.0f} corrections", flush=True)
        assert rec[1] == ro["alpha"]
        assert abs(rec[0] - ro["phi0"]) <= 1e-10 * abs(ro["phi0"])
        assert abs(rec[2] - ro["decrement"]) <= 1e-7 * max(1.0, abs(ro["decrement"]))
        if precision == 0:
            assert err <= 1e-10
        else:
            assert rec[4] <= tol and 1 <= rec[5] <= refine
            assert err <= 1e-8
    ctx.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_gn_graph_replays_match_eager(gpu_lib, precision):
    import torch
    p = gi.burgers_spacetime(nx=64, nt=48, seed=102, range_s=0.1)
    m = p.meta
    args = (m["nx"], m["nt"], m["dt"], m["nu"])
    ctx_e, mass, s3 = _dev(gpu_lib, p, precision)
    ctx_g, _, _ = _dev(gpu_lib, p, precision)
    ue = torch.zeros(p.n, dtype=torch.float64, device="cuda")
    ug = torch.zeros(p.n, dtype=torch.float64, device="cuda")
    re = ctx_e.gn_burgers(*args, mass, s3, ue, iters=6, precision=precision, refine=2, use_graph=False)
    rg = ctx_g.gn_burgers(*args, mass, s3, ug, iters=6, precision=precision, refine=2, use_graph=True)
    assert np.array_equal(re, rg)
    assert torch.equal(ue, ug)
    # eager work between the calls, then a second call that captures and replays its own graph
    torch.cuda.synchronize()
    _ = (ug * 2.0).sum().item()
    re2 = ctx_e.gn_burgers(*args, mass, s3, ue, iters=3, precision=precision, refine=2, use_graph=False)
    rg2 = ctx_g.gn_burgers(*args, mass, s3, ug, iters=3, precision=precision, refine=2, use_graph=True)
    assert np.array_equal(re2, rg2)
    assert torch.equal(ue, ug)
    phis = np.concatenate([re[:, 0], re2[:, 0]])
    assert np.all(np.diff(phis) <= 1e-12 * phis[:-1])
    ctx_e.close()
    ctx_g.close()


def test_gn_new_arguments_after_resize_match_eager(gpu_lib):
    """The captured graph lives for one call: a second call with another iterate tensor,
    another viscosity and refinement count, after gmrf_sample(k=16) has regrown the
    solve buffers, replays its own capture (bitwise equal to eager iterations)."""
    import torch
    p = gi.burgers_spacetime(nx=48, nt=40, seed=103, range_s=0.1)
    m = p.meta
    out = {}
    for use_graph in (False, True):
        ctx, mass, s3 = _dev(gpu_lib, p, 1)
        u1 = torch.zeros(p.n, dtype=torch.float64, device="cuda")
        r1 = ctx.gn_burgers(m["nx"], m["nt"], m["dt"], m["nu"], mass, s3, u1, iters=4, precision=1, refine=3,
                            use_graph=use_graph)
        z = torch.from_numpy(np.random.default_rng(5).standard_normal((16, p.n)).astype(np.float32)).cuda()
        xs = ctx.sample(z)
        u2 = torch.full((p.n,), 0.01, dtype=torch.float64, device="cuda")
        r2 = ctx.gn_burgers(m["nx"], m["nt"], m["dt"], 1.5 * m["nu"], mass, s3, u2, iters=4, precision=1,
                            refine=5, use_graph=use_graph, refine_tol=1e-12)
        out[use_graph] = (r1, u1.cpu().numpy(), xs.cpu().numpy(), r2, u2.cpu().numpy())
        del u1
        ctx.close()
    for a, b in zip(out[False], out[True]):
        assert np.array_equal(a, b)


def test_gn_full_size_fp32_vs_fp64(gpu_lib):
    """1024 x 1024 Burgers: FP32 supernodes with FP64-residual refinement and the FP64
    path, both iterated until the Newton decrement has stopped falling, reach the same
    mode to the refinement accuracy."""
    import time
    import torch
    p = gi.burgers_spacetime()       # 1024 x 1024 = 1,048,576 unknowns
    m = p.meta
    print(f"[gn] full size n={p.n}", flush=True)
    out = {}
    iters = 16
    for prec in (1, 0):
        ctx, mass, s3 = _dev(gpu_lib, p, prec)
        u = torch.zeros(p.n, dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rec = ctx.gn_burgers(m["nx"], m["nt"], m["dt"], m["nu"], mass, s3, u, iters=iters, precision=prec,
                             refine=30 if prec else 2, use_graph=True, refine_tol=1e-12)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        ld = ctx.logdet()[0]
        var = ctx.selinv().cpu().numpy()
        print(f"[gn] precision {prec}: {t:.3f} s for {iters} iterations; phi {rec[:, 0]}; alpha {rec[:, 1]}; "
              f"decrement {rec[:, 2]}; solve resid {rec[:, 4]}; corrections {rec[:, 5]}; logdet {ld:.6e}",
              flush=True)
        assert np.all(np.diff(rec[:, 0]) <= 1e-9 * rec[:-1, 0])
        assert np.all(rec[:, 4] <= 1e-12)
        assert np.isfinite(ld) and np.all(var > 0)
        out[prec] = (u.cpu().numpy(), rec, ld)
        ctx.close()
    u32, u64 = out[1][0], out[0][0]
    rel = np.linalg.norm(u32 - u64) / np.linalg.norm(u64)
    phi32, phi64 = out[1][1][-1, 0], out[0][1][-1, 0]
    dec32, dec64 = out[1][1][-1, 2], out[0][1][-1, 2]
    print(f"[gn] FP32 vs FP64: final iterate rel diff {rel:.3e}, final objective {phi32:.10e} / {phi64:.10e}, "
          f"final decrement {dec32:.3e} / {dec64:.3e}", flush=True)
    # measured: iterates 7.4e-10 apart, objectives 2.6e-12 apart (the rounding of the
    # objective's sums), final decrements 6e-15 and 2e-16 of an initial 5.7e8
    assert abs(phi32 - phi64) <= 1e-10 * phi64
    assert max(abs(dec32), abs(dec64)) <= 1e-10 * out[0][1][0, 2]
    assert rel <= 1e-8
