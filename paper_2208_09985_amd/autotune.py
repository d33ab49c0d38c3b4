"""Autotuner for the persistent alignment kernel's launch shape.

For a given batch and mode it times candidate configurations on the device
(kernel time from the HIP events the library records around each launch)
and keeps the fastest:

* kernel        -- error-row lanes or column blocks
* slots         -- windows in flight per wavefront (0: the library's automatic launch)
* waves_per_cu  -- persistent wavefronts per CU (capped by LDS occupancy)
* order         -- queue order of pairs (input order or longest first)
* tau           -- learned mode: confidence needed before a smaller row budget
* fixed_rows    -- fixed mode: constant row budget before falling back
* rows_lds      -- plain mode: the lowest stored rows of each window in LDS
* one_per_simd  -- plain mode: allow wavefronts to share a SIMD ("auto" reserves a
                   whole SIMD per wavefront when they fit one per SIMD)

Every candidate produces bit-identical output (the budget only changes how
many rows are tried first), which the tuner checks against the first
candidate; candidates that resolve to the same launch (the library reports
it) are timed once.  Results are cached as JSON keyed by the device (CU count), the
window parameters, the mode and a coarse signature of the batch (pair count
and length distribution), so a later call with a similar batch reuses them.
"""
from __future__ import annotations

import hashlib
import itertools
import json
import os
import time

import numpy as np

from . import api

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "scrooge_mi355x", "autotune.json")

SPACE = {
    "plain": {"kernel": ["columns"], "slots": [0, 4, 8, 10, 16], "waves_per_cu": [0], "order": ["input", "longest_first"],
              "rows_lds": [False, True], "one_per_simd": ["auto", False]},
    "fixed": {"kernel": ["rows"], "slots": [2, 4, 6, 8], "waves_per_cu": [0], "order": ["input"],
              "fixed_rows": [7, 11, 15, 23]},
    "learned": {"kernel": ["rows", "columns"], "slots": [4, 8], "waves_per_cu": [0], "order": ["input"],
                "tau": [0.7, 0.8, 0.9]},
}


def batch_signature(batch) -> dict:
    m = np.diff(batch.pat_off)
    n = np.diff(batch.txt_off)
    return {"pairs": int(len(m)), "m_mean": int(m.mean()) if len(m) else 0,
            "m_cv": round(float(m.std() / max(m.mean(), 1)), 1) if len(m) else 0.0,
            "n_over_m": round(float(n.sum() / max(m.sum(), 1)), 2)}


def cache_key(ctx, W, O, k, mode, sig) -> str:
    raw = json.dumps({"cus": ctx.cus, "W": W, "O": O, "k": k, "mode": mode, "sig": sig}, sort_keys=True)
    return hashlib.sha1(raw.encode()).hexdigest()[:16]


def _same(a, b) -> bool:
    if not (np.array_equal(a.edits, b.edits) and np.array_equal(a.n_runs, b.n_runs)
            and np.array_equal(a.text_end, b.text_end)):
        return False
    ra, rb = np.asarray(a.runs), np.asarray(b.runs)
    for i in range(0, len(a.n_runs), max(1, len(a.n_runs) // 64)):
        s, e = int(a.runs_off[i]), int(a.runs_off[i]) + int(a.n_runs[i])
        if not np.array_equal(ra[s:e], rb[s:e]):
            return False
    return True


def tune(ctx, batch, W=64, O=24, k=64, mode="plain", space=None, reps=2, cache_path=DEFAULT_CACHE,
         use_cache=True, log=None) -> tuple[dict, list]:
    """Return (best configuration as api.params keyword arguments, all timings)."""
    import torch
    sig = batch_signature(batch)
    key = cache_key(ctx, W, O, k, mode, sig)
    if use_cache and cache_path and os.path.exists(cache_path):
        try:
            cached = json.load(open(cache_path)).get(key)
            if cached:
                return cached["best"], cached["results"]
        except (OSError, ValueError):
            pass
    space = dict(space or SPACE[mode])
    names = list(space)
    results = []
    ref = None
    seen = {}
    for combo in itertools.product(*(space[n] for n in names)):
        cfg = dict(zip(names, combo))
        prm = api.params(W=W, O=O, k=k, mode=mode, **cfg)
        b = api.Batch(ctx, batch, prm)
        # the same launch under another name: reuse its timing
        launch = json.dumps([b.launch_shape(), {n: v for n, v in cfg.items() if n not in ("slots", "one_per_simd")}],
                            sort_keys=True)
        if launch in seen:
            results.append(dict(seen[launch], cfg=cfg))
            b.close()
            continue
        b.run()
        torch.cuda.synchronize()
        b.stats()
        for _ in range(reps):
            b.run()
        torch.cuda.synchronize()
        st = b.stats()
        res = b.result()
        if ref is None:
            ref = res
        elif not _same(ref, res):
            raise RuntimeError(f"autotune: configuration {cfg} changed the output")
        results.append({"cfg": cfg, "kernel_ms": st.kernel_ms_avg, "fallback_windows": int(st.fallback_windows),
                        "rounds": int(st.rounds)})
        seen[launch] = results[-1]
        if log:
            log(f"[autotune] {mode} {cfg}: {st.kernel_ms_avg:.3f} ms (fallback {st.fallback_windows}, "
                f"rounds {st.rounds})")
        b.close()
    best = min(results, key=lambda r: r["kernel_ms"])["cfg"]
    if cache_path:
        os.makedirs(os.path.dirname(cache_path), exist_ok=True)
        try:
            data = json.load(open(cache_path)) if os.path.exists(cache_path) else {}
        except (OSError, ValueError):
            data = {}
        data[key] = {"best": best, "results": results, "sig": sig, "mode": mode, "W": W, "O": O, "k": k,
                     "cus": ctx.cus, "time": time.time()}
        tmp = cache_path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(data, f, indent=1)
        os.replace(tmp, cache_path)
    return best, results
