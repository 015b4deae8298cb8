"""The supernode-shape autotuner: it times the library's factorisation + selected
inversion under candidate analysis options on the actual problem, keeps the fastest and
caches it per pattern; the tuned analysis still matches the oracle."""
import json

import numpy as np
import pytest

import gmrf_inputs as gi
import oracle as O

pytestmark = pytest.mark.gpu


def test_autotune_picks_fastest_and_caches(gpu_lib, tmp_path):
    from paper_2503_08343_amd import autotune as at
    p = gi.matern_batch(n_prob=12, side_lo=16, side_hi=40, seed=91)
    cache = str(tmp_path / "tune.json")
    cands = [(64, 8, 32, 128), (32, 4, 16, 64), (128, 16, 64, 256)]
    opts, rec = at.tune(p, precision=gpu_lib.GMRF_FP64, cache_path=cache, candidates=cands, reps=2)
    print(f"[autotune] {rec['trials']}", flush=True)
    best = min(rec["trials"], key=lambda r: r["ms"])
    assert rec["best"] == best["options"]
    assert opts == dict(leaf_size=best["options"][0], relax_small=best["options"][1],
                        relax_mid=best["options"][2], relax_big=best["options"][3])
    with open(cache) as f:
        assert len(json.load(f)) == 1
    # second call: read from the cache (no candidate is timed again)
    opts2, rec2 = at.tune(p, precision=gpu_lib.GMRF_FP64, cache_path=cache, candidates=[], reps=1)
    assert opts2 == opts and rec2["trials"] == rec["trials"]
    # the tuned analysis gives the same posterior (to the FP64 parity bar)
    ctx = gpu_lib.posterior_context(p, precision=gpu_lib.GMRF_FP64, opts=opts)
    mu, _, _ = ctx.solve()
    var = ctx.selinv().cpu().numpy()
    r = O.posterior(p)
    assert np.linalg.norm(mu.cpu().numpy() - r["mean"]) <= 1e-10 * np.linalg.norm(r["mean"])
    assert np.max(np.abs(var - r["var"]) / r["var"]) <= 1e-10
    ctx.close()
