"""GPU Gauss-Newton on the nonlinear Burgers space-time problem: each iteration against
the oracle's step from the same iterate (linearised posterior mean, line search,
decrement), hipGraph replays against eager iterations (every iteration's record and the
final iterate bitwise equal, also across calls with eager work in between), and the full
1024 x 1024 problem in FP32 with FP64 residuals against FP64."""
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


def test_gn_iterations_match_oracle_from_same_iterate(gpu_lib):
    import torch
    p = gi.burgers_spacetime(nx=40, nt=32, seed=101, range_s=0.2)
    m = p.meta
    ctx, mass, s3 = _dev(gpu_lib, p)
    S = _S(m["nx"])
    u = torch.zeros(p.n, dtype=torch.float64, device="cuda")
    for it in range(3):
        u_in = u.cpu().numpy().copy()
        rec = ctx.gn_burgers(m["nx"], m["nt"], m["dt"], m["nu"], mass, s3, u, iters=1, precision=0,
                             refine=1, use_graph=False)[0]
        uo, ro = O.gn_step(p.Q, u_in, p.y, p.q_eps, m["nx"], m["nt"], m["dt"], m["nu"], m["mass"], S)
        u_out = u.cpu().numpy()
        print(f"[gn] it {it}: phi {rec[0]:.10e} / {ro['phi0']:.10e} alpha {rec[1]} / {ro['alpha']} "
              f"decrement {rec[2]:.4e} / {ro['decrement']:.4e}", flush=True)
        assert rec[1] == ro["alpha"]
        assert abs(rec[0] - ro["phi0"]) <= 1e-10 * abs(ro["phi0"])
        assert abs(rec[2] - ro["decrement"]) <= 1e-7 * max(1.0, abs(ro["decrement"]))
        assert np.linalg.norm(u_out - uo) <= 1e-10 * np.linalg.norm(uo)
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
    # eager work between replays, then more replays of the cached graph
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


def test_gn_full_size_fp32_vs_fp64(gpu_lib):
    import time
    import torch
    p = gi.burgers_spacetime()       # 1024 x 1024 = 1,048,576 unknowns
    m = p.meta
    print(f"[gn] full size n={p.n}", flush=True)
    out = {}
    for prec in (1, 0):
        ctx, mass, s3 = _dev(gpu_lib, p, prec)
        u = torch.zeros(p.n, dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rec = ctx.gn_burgers(m["nx"], m["nt"], m["dt"], m["nu"], mass, s3, u, iters=12, precision=prec,
                             refine=8 if prec else 1, use_graph=True)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        ld = ctx.logdet()[0]
        var = ctx.selinv().cpu().numpy()
        print(f"[gn] precision {prec}: {t:.3f} s for 12 iterations; phi {rec[:, 0]}; alpha {rec[:, 1]}; "
              f"decrement {rec[:, 2]}; logdet {ld:.6e}", flush=True)
        assert np.all(np.diff(rec[:, 0]) <= 1e-9 * rec[:-1, 0])
        assert rec[-1, 2] <= 1e-3 * rec[0, 2]
        assert np.isfinite(ld) and np.all(var > 0)
        out[prec] = (u.cpu().numpy(), rec, ld)
        ctx.close()
    # the trajectories differ at rounding level (inexact FP32 steps); both converge to the mode
    u32, u64 = out[1][0], out[0][0]
    rel = np.linalg.norm(u32 - u64) / np.linalg.norm(u64)
    phi32, phi64 = out[1][1][-1, 0], out[0][1][-1, 0]
    print(f"[gn] FP32 vs FP64: final iterate rel diff {rel:.3e}, final objective {phi32:.10e} / {phi64:.10e}",
          flush=True)
    assert abs(phi32 - phi64) <= 1e-7 * phi64
    assert rel <= 1e-4
