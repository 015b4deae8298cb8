"""Supernode-shape autotuner.

The shapes of the dense fronts -- and so the tile shapes of every front kernel -- follow
from the nested-dissection leaf size and the relaxed-amalgamation thresholds of the
symbolic analysis (Sec. 3.2: the ordering and the supernodes fix the fill and the dense
work).  For one sparsity pattern this module times the library's own factorisation and
selected inversion (the two MFMA-bound phases) under a small set of candidate options
on the actual problem, keeps the fastest, and caches the choice in a JSON file keyed by
the device name, the precision and a hash of the pattern, so later runs on the same
pattern reuse it without measuring.  Only options are chosen here; all timed work runs
in the library.
"""
from __future__ import annotations

import hashlib
import json
import os
import time

import numpy as np

from . import binding

# (leaf_size, relax_small, relax_mid, relax_big): the library default first
CANDIDATES = [
    (64, 8, 32, 128),
    (64, 16, 64, 256),
    (32, 8, 32, 128),
    (128, 8, 32, 128),
    (64, 4, 16, 64),
    (128, 16, 64, 256),
]
DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "gmrf_autotune.json")


def pattern_key(problem, precision, device_name):
    h = hashlib.sha1()
    h.update(np.ascontiguousarray(problem.Q.indptr, dtype=np.int64).tobytes())
    h.update(np.ascontiguousarray(problem.Q.indices, dtype=np.int32).tobytes())
    if problem.A is not None and problem.A.shape[0]:
        h.update(np.ascontiguousarray(problem.A.indptr, dtype=np.int64).tobytes())
        h.update(np.ascontiguousarray(problem.A.indices, dtype=np.int32).tobytes())
    if problem.block_ptr is not None:
        h.update(np.ascontiguousarray(problem.block_ptr, dtype=np.int64).tobytes())
    return f"{device_name}|p{int(precision)}|n{problem.n}|{h.hexdigest()[:20]}"


def _options(c):
    return dict(leaf_size=c[0], relax_small=c[1], relax_mid=c[2], relax_big=c[3])


def _time_candidate(problem, precision, opts, reps):
    import torch
    ctx = binding.posterior_context(problem, precision=precision, opts=opts)
    try:
        ctx.selinv()                      # warm-up of factor-dependent allocations
        ts = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ctx.factor(precision)
            ctx.selinv()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        st = ctx.stats()
    finally:
        ctx.close()
    return float(np.median(ts)), st


def tune(problem, precision=binding.GMRF_FP32_REFINE, cache_path=DEFAULT_CACHE, reps=2,
         candidates=CANDIDATES, refresh=False, log=None):
    """Options (dict for binding.posterior_context(opts=...)) that gave the fastest
    factorisation + selected inversion of `problem`, measured on the current device or
    read from the cache.  Returns (opts, record)."""
    import torch
    dev = torch.cuda.get_device_name(0)
    key = pattern_key(problem, precision, dev)
    cache = {}
    if os.path.exists(cache_path):
        with open(cache_path) as f:
            cache = json.load(f)
    if key in cache and not refresh:
        rec = cache[key]
        return _options(rec["best"]), rec
    trials = []
    for c in candidates:
        t, st = _time_candidate(problem, precision, _options(c), reps)
        trials.append({"options": list(c), "ms": round(t * 1e3, 3), "n_super": st["n_super"],
                       "stored_l": st["stored_l"], "max_front": st["max_front"]})
        if log:
            log(f"[autotune] {c}: {t * 1e3:.2f} ms (supernodes {st['n_super']}, stored L {st['stored_l']:.4g})")
    best = min(trials, key=lambda r: r["ms"])
    rec = {"best": best["options"], "ms": best["ms"], "default_ms": trials[0]["ms"], "trials": trials}
    cache[key] = rec
    d = os.path.dirname(cache_path)
    if d:
        os.makedirs(d, exist_ok=True)
    tmp = cache_path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1)
    os.replace(tmp, cache_path)
    return _options(best["options"]), rec
