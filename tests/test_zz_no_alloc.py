"""The no-allocation log-determinant (gmrf_logdet_noalloc, the variant of gmrf_logdet for
callers that cannot allocate device memory) against gmrf_logdet through the C ABI: two
calls in a row on the device's shared workspace, the second on a smaller batch in the
other precision, each bitwise equal to gmrf_logdet's per-block values; the first batch
again afterwards (the workspace keeps no state between calls); and the size limit
rejected before anything is enqueued."""
import numpy as np
import pytest

import gmrf_inputs as gi

pytestmark = pytest.mark.gpu


def _noalloc(ctx, nblocks):
    import torch
    out = torch.full((nblocks,), float("nan"), dtype=torch.float64, device="cuda")
    ctx.logdet_noalloc(out)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def test_logdet_noalloc_matches_logdet(gpu_lib):
    big = gi.matern_batch(n_prob=24, side_lo=12, side_hi=40, seed=71)
    small = gi.matern_batch(n_prob=5, side_lo=8, side_hi=16, seed=72)
    c1 = gpu_lib.posterior_context(big, precision=gpu_lib.GMRF_FP64)
    ref1 = c1.logdet()
    got1 = _noalloc(c1, 24)
    print(f"[noalloc] 24 blocks: max |diff| {np.max(np.abs(got1 - ref1)):.3e}", flush=True)
    assert np.array_equal(got1, ref1)
    c2 = gpu_lib.posterior_context(small, precision=gpu_lib.GMRF_FP32_REFINE)
    ref2 = c2.logdet()
    got2 = _noalloc(c2, 5)
    print(f"[noalloc] 5 blocks: max |diff| {np.max(np.abs(got2 - ref2)):.3e}", flush=True)
    assert np.array_equal(got2, ref2)
    again = _noalloc(c1, 24)
    assert np.array_equal(again, ref1)
    c1.close()
    c2.close()


def test_logdet_noalloc_rejects_too_many_blocks(gpu_lib):
    import torch
    n = 8193                                  # one unknown per block, one block over the limit
    ctx = gpu_lib.Context(0)
    qi = torch.arange(n + 1, dtype=torch.int64, device="cuda")
    qj = torch.arange(n, dtype=torch.int32, device="cuda")
    qv = torch.full((n,), 2.0, dtype=torch.float64, device="cuda")
    ctx.assemble(qi, qj, qv, None, None, None, None, None, block_ptr=np.arange(n + 1))
    out = torch.zeros(n, dtype=torch.float64, device="cuda")
    with pytest.raises(gpu_lib.GmrfError) as e:
        ctx.logdet_noalloc(out)
    assert e.value.code == -1 and "8192" in str(e.value)
    ctx.close()
