"""Every workload at its full size, through the launch the benchmark times,
compared with the oracle pair by pair: status, edits, text_end and the whole
operation stream (bit-exact).

* short reads: 100,000 pairs of 250 bp, the default plain launch;
* long reads: 10,000 pairs of 10 kbp, the default plain launch (the
  benchmark's headline) and, with the committed predictor, learned mode;
* uneven lengths: 50,000 pairs of log-normal length, the default launch (the
  helpers holding the longest pairs; also with a bad byte in one of them) and the
  launch shape the autotuner picks, replayed from a captured hipGraph;
* mixed edit rates: 10,000 pairs of 10 kbp in learned mode with the
  committed predictor, in both kernels.
"""
import functools
import os

import numpy as np
import pytest

import oracle
from paper_2208_09985_amd import synth
from tests.gpu_helpers import compare, log

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]

WEIGHTS = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2208_09985_amd",
                       "weights", "budget_w64_o24.npz")


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2208_09985_amd import api
    c = api.Context(0)
    c.load_model(WEIGHTS)
    return c


@functools.lru_cache(maxsize=2)
def _workload(name):
    w = synth.WORKLOADS[name]
    log(f"[full] generating {name} ({w.npairs} pairs)")
    b = synth.make_batch(name)
    log(f"[full] oracle on {name}")
    ref = oracle.align_batch(b, w.W, w.O, w.k)
    return w, b, ref


def test_short_250bp_all_pairs():
    from paper_2208_09985_amd import api
    w, b, ref = _workload("short_250bp")
    c = api.Context(0)
    log("[full] short_250bp plain, default launch")
    res = api.align_batch(c, b, W=w.W, O=w.O, k=w.k)
    compare(b, res, ref, "short_250bp full")
    assert res.stats.windows == ref["stats"].windows
    assert res.stats.ops_alg == ref["stats"].ops_alg


def test_long_10kbp_all_pairs_plain_and_learned(ctx):
    import torch
    from paper_2208_09985_amd import api
    w, b, ref = _workload("long_10kbp")
    # the headline launch as the benchmark runs it: a prepared batch, warm-up run, timed runs
    bt = api.Batch(ctx, b, api.params(W=w.W, O=w.O, k=w.k, mode="plain"))
    shape = bt.launch_shape()
    log(f"[full] long_10kbp plain launch shape {shape}")
    if ctx.cus == 256:
        # 625 wavefronts of 16 windows, one per SIMD, and the off-track helper launch
        # of 4-window wavefronts on the other 399 SIMDs, their rows in LDS
        assert shape["kernel"] == "columns" and shape["slots"] == 16 and shape["one_per_simd"], shape
        assert shape["grid"] == 625 and shape["entry_bits"] == 48, shape
        assert shape["helper_grid"] == 399 and shape["helper_slots"] == 4 and shape["helper_lds_bytes"] > 0, shape
    for rep in range(2):
        log(f"[full] long_10kbp plain, benchmark launch, run {rep}")
        bt.edits.fill_(-7)
        bt.run()
        torch.cuda.synchronize()
        res = bt.result()
        compare(b, res, ref, f"long_10kbp full run {rep}")
    st = bt.stats()
    bt.close()
    assert st.windows == ref["stats"].windows and st.ops_alg == ref["stats"].ops_alg
    for slots, one, helpers in ((8, "auto", "auto"), (10, "auto", False), (10, False, False), (16, "auto", False)):
        log(f"[full] long_10kbp plain, {slots} windows per wavefront, one per SIMD: {one}, helpers: {helpers}")
        compare(b, api.align_batch(ctx, b, kernel="columns", slots=slots, one_per_simd=one, offtrack_helpers=helpers),
                ref, f"long_10kbp full slots={slots} one_per_simd={one} helpers={helpers}")
    for kw in (dict(rows_lds=True), dict(row_ring=True), dict(kernel="lanes")):
        log(f"[full] long_10kbp plain, {kw}")
        compare(b, api.align_batch(ctx, b, **{"kernel": "columns", **kw}), ref, f"long_10kbp full {kw}")
    log("[full] long_10kbp learned (committed predictor), default kernel")
    compare(b, api.align_batch(ctx, b, mode="learned"), ref, "long_10kbp full learned")


def test_uneven_lognormal_all_pairs_autotuned_graph(ctx):
    import torch
    from paper_2208_09985_amd import api, autotune
    w, b, ref = _workload("uneven_lognormal")
    # the default launch: lengths vary, so pairs go longest first; the batch needs more
    # chains in flight than one wavefront per SIMD holds, so the helper launch (one
    # wavefront per CU) holds the 768 longest pairs from the start and 16-window
    # wavefronts one per SIMD take the rest from the queue
    bt = api.Batch(ctx, b, api.params(W=w.W, O=w.O, k=w.k, mode="plain"))
    shape = bt.launch_shape()
    log(f"[full] uneven_lognormal default launch shape {shape}")
    if ctx.cus == 256:
        assert shape["kernel"] == "columns" and shape["slots"] == 16 and shape["one_per_simd"], shape
        assert shape["grid"] == 768 and shape["helper_grid"] == 256 and shape["helper_long_pairs"] == 768, shape
    bt.run()
    torch.cuda.synchronize()
    compare(b, bt.result(), ref, "uneven_lognormal full default launch")
    bt.close()
    # a pair with a non-ACGT byte among the longest ones (held by the helpers) is marked
    # as bad input, and every other pair keeps its result
    m = np.diff(b.pat_off)
    longest = int(np.argmax(m))
    bb = synth.PairBatch(b.pat.copy(), b.pat_off, b.txt, b.txt_off)
    bb.pat[int(b.pat_off[longest]) + 5] = ord("N")
    res = api.align_batch(ctx, bb, W=w.W, O=w.O, k=w.k)
    assert res.status[longest] == 2 and res.edits[longest] == -1
    keep = np.arange(b.npairs) != longest
    assert np.array_equal(res.edits[keep], ref["edits"][keep])
    assert np.array_equal(res.text_end[keep], ref["text_end"][keep])
    best, trials = autotune.tune(ctx, b, w.W, w.O, w.k, mode="plain", reps=1, cache_path=None, log=log)
    log(f"[full] uneven_lognormal autotuned {best}, graph launch")
    gb = api.Batch(ctx, b, api.params(W=w.W, O=w.O, k=w.k, mode="plain", graph=True, **best))
    for rep in range(2):
        gb.edits.fill_(-7)
        gb.n_runs.fill_(0)
        gb.run()
        torch.cuda.synchronize()
        compare(b, gb.result(), ref, f"uneven_lognormal full graph replay {rep} {best}")
        _ = torch.ones(1000, device=gb.dev).sum().item()   # eager work between replays
    gb.close()


def test_mixed_10kbp_all_pairs_one_lane_per_pair(ctx):
    from paper_2208_09985_amd import api
    w, b, ref = _workload("mixed_10kbp")
    log("[full] mixed_10kbp plain, one lane per pair")
    res = api.align_batch(ctx, b, W=w.W, O=w.O, k=w.k, kernel="lanes")
    compare(b, res, ref, "mixed_10kbp full lanes")
    assert res.stats.yields == 0


@pytest.mark.parametrize("kernel", ["auto", "columns"])
def test_mixed_10kbp_all_pairs_learned(ctx, kernel):
    from paper_2208_09985_amd import api
    w, b, ref = _workload("mixed_10kbp")
    log(f"[full] mixed_10kbp learned (committed predictor), kernel={kernel}")
    res = api.align_batch(ctx, b, W=w.W, O=w.O, k=w.k, mode="learned", kernel=kernel)
    compare(b, res, ref, f"mixed_10kbp full learned [{kernel}]")
    assert res.stats.windows == ref["stats"].windows
