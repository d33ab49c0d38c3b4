"""GPU path vs CPU oracle: bit-exact edits, text_end, status and full CIGAR
operation streams, through the C ABI, on seeded synthetic workloads."""
import numpy as np
import pytest

import oracle
from paper_2208_09985_amd import synth
from tests.gpu_helpers import compare, log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2208_09985_amd import api
    return api.Context(0)


def run_gpu(ctx, batch, **kw):
    from paper_2208_09985_amd import api
    return api.align_batch(ctx, batch, **kw)


KERNELS = ("rows", "columns")


def check(ctx, batch, W=64, O=24, k=64, what="", kernels=KERNELS, **kw):
    """Both fused kernels against the oracle; returns the last kernel's result."""
    ref = oracle.align_batch(batch, W, O, k)
    for kern in kernels:
        log(f"[parity] {what} pairs={batch.npairs} W={W} O={O} k={k} kernel={kern} {kw}")
        gpu = run_gpu(ctx, batch, W=W, O=O, k=k, kernel=kern, **kw)
        compare(batch, gpu, ref, f"{what} [{kern}]")
    return gpu, ref


def test_small_100bp_all_pairs_plain(ctx):
    b = synth.make_batch("small_100bp")
    ref = oracle.align_batch(b, 64, 24, 64)
    for kern in KERNELS + ("lanes",):
        gpu, _ = check(ctx, b, what="small_100bp plain", kernels=(kern,))
        assert gpu.stats.windows == ref["stats"].windows
        assert gpu.stats.ops_alg == ref["stats"].ops_alg


@pytest.mark.parametrize("mode,extra", [("fixed", dict(fixed_rows=1)), ("fixed", dict(fixed_rows=8)),
                                        ("fixed", dict(fixed_rows=16)), ("plain", dict(slots=4)),
                                        ("fixed", dict(fixed_rows=5, slots=16)), ("plain", dict(slots=8)),
                                        ("fixed", dict(fixed_rows=3, slots=8))])
def test_small_100bp_budgets_and_packing(ctx, mode, extra):
    b = synth.make_batch("small_100bp", 300)
    for kern in KERNELS:
        gpu, ref = check(ctx, b, mode=mode, what=f"small_100bp {mode} {extra}", kernels=(kern,), **extra)
        if mode == "fixed" and extra["fixed_rows"] == 1:
            assert gpu.stats.fallback_windows > 0


def test_short_250bp_subset(ctx):
    b = synth.make_batch("short_250bp", 20000)
    check(ctx, b, what="short_250bp")
    check(ctx, b, mode="fixed", fixed_rows=4, what="short_250bp fixed4")


def test_long_10kbp_sample(ctx):
    b = synth.make_batch("long_10kbp", 48)
    check(ctx, b, what="long_10kbp", kernels=KERNELS + ("lanes",))
    check(ctx, b, mode="fixed", fixed_rows=16, what="long_10kbp fixed16")


def test_uneven_and_mixed_samples(ctx):
    check(ctx, synth.make_batch("uneven_lognormal", 64), order="longest_first", what="uneven_lognormal")
    check(ctx, synth.make_batch("mixed_10kbp", 32), mode="fixed", fixed_rows=8, what="mixed_10kbp fixed8")


def test_uneven_chain_launch_one_per_simd(ctx):
    # 3,000 pairs of log-normal length: longest first, and the automatic launch keeps
    # about (all windows / longest chain) windows in flight, here one 4-window
    # wavefront per CU and per SIMD at most
    from paper_2208_09985_amd import api
    b = synth.make_batch("uneven_lognormal", 3000)
    ref = oracle.align_batch(b, 64, 24, 64)
    bt = api.Batch(ctx, b, api.params())
    shape = bt.launch_shape()
    bt.close()
    log(f"[parity] uneven 3,000 pairs, default launch shape {shape}")
    if ctx.cus == 256:
        assert shape["kernel"] == "columns" and shape["slots"] == 4 and shape["one_per_simd"], shape
        assert shape["grid"] == 256 and shape["helper_grid"] == 0, shape
    res = run_gpu(ctx, b)
    compare(b, res, ref, "uneven 3,000 pairs, chain launch")


@pytest.mark.parametrize("W,O,k", [(64, 33, 64), (32, 17, 32), (16, 9, 16), (8, 3, 8), (4, 3, 4), (64, 0, 64),
                                   (64, 63, 64), (1, 0, 1), (48, 20, 30), (64, 24, 6), (64, 17, 64), (64, 16, 64)])
def test_window_parameters(ctx, W, O, k):
    rng = np.random.default_rng(W * 100 + O)
    pats, txts = [], []
    for _ in range(150):
        p = synth.ALPHABET[rng.integers(0, 4, int(rng.integers(1, 400)))]
        t = p.copy()
        nedit = int(len(t) * rng.uniform(0, 0.3))
        for _ in range(nedit):
            pos = int(rng.integers(0, max(1, len(t))))
            r = rng.random()
            if r < 0.33 and len(t):
                t[pos] = synth.ALPHABET[rng.integers(0, 4)]
            elif r < 0.66:
                t = np.insert(t, pos, synth.ALPHABET[rng.integers(0, 4)])
            elif len(t):
                t = np.delete(t, pos)
        pats.append(p.tobytes())
        txts.append(t.tobytes())
    b = synth.from_lists(pats, txts)
    check(ctx, b, W=W, O=O, k=k, what=f"W{W}O{O}k{k}")
    check(ctx, b, W=W, O=O, k=k, mode="fixed", fixed_rows=3, what=f"W{W}O{O}k{k} fixed3")
    check(ctx, b, W=W, O=O, k=k, what=f"W{W}O{O}k{k} 10 windows per wavefront", kernels=("columns",), slots=10)
    check(ctx, b, W=W, O=O, k=k, what=f"W{W}O{O}k{k} edges stored", kernels=("columns",), store_edges=True)
    check(ctx, b, W=W, O=O, k=k, what=f"W{W}O{O}k{k} row ring", kernels=("columns",), row_ring=True)
    check(ctx, b, W=W, O=O, k=k, what=f"W{W}O{O}k{k} one lane per pair", kernels=("lanes",))


def test_edge_cases(ctx):
    pats = [b"", b"ACGT", b"ACGTACGT", b"A", b"acgtNacgt".replace(b"N", b"a"), b"G" * 300, b"ACGT" * 40,
            b"T" * 64, b"C" * 65, b"A" * 200]
    txts = [b"ACGT", b"", b"ACGTACGT" + b"T" * 500, b"C", b"ACGTAACGT", b"G" * 10, b"", b"A" * 64, b"C" * 64,
            b"T" * 200]
    b = synth.from_lists(pats, txts)
    check(ctx, b, what="edge cases")
    check(ctx, b, k=5, what="edge cases k=5 (not aligned)")
    check(ctx, b, what="edge cases, edges stored", kernels=("columns",), store_edges=True)
    check(ctx, b, what="edge cases, rows in LDS", kernels=("columns",), rows_lds=True)
    check(ctx, b, what="edge cases, row ring", kernels=("columns",), row_ring=True)
    check(ctx, b, what="edge cases, one lane per pair", kernels=("lanes",))
    check(ctx, b, k=5, what="edge cases k=5, one lane per pair", kernels=("lanes",))


def test_bad_device_input_marks_pair(ctx):
    from paper_2208_09985_amd import api
    b = synth.from_lists([b"ACGT", b"ACNT", b"ACGT"], [b"ACGT", b"ACGT", b"AXGT"])
    res = api.align_batch(ctx, b)
    assert list(res.status) == [0, 2, 2]
    assert list(res.edits) == [0, -1, -1]


def test_host_input_rejects_bad_alphabet(ctx):
    from paper_2208_09985_amd import api, _lib
    b = synth.from_lists([b"ACNT"], [b"ACGT"])
    with pytest.raises(_lib.ScgError) as e:
        api.Batch(ctx, b, device_input=False)
    assert e.value.code == _lib.EALPHABET


def test_single_pair_api(ctx):
    p, t = b"ACGTACGTTTGACCA" * 5, b"ACGTACGTTGACCAT" * 5
    e, te, cg = ctx.align(p, t)
    r = oracle.align_pair(p, t, 64, 24, 64)
    assert (e, te, cg) == (r["edits"], r["text_end"], oracle.cigar(r["ops"]))


def test_launch_shape_does_not_change_results(ctx):
    b = synth.make_batch("long_10kbp", indices=range(100, 132))
    ref = oracle.align_batch(b, 64, 24, 64)
    for kw in (dict(slots=1, waves_per_cu=1), dict(slots=3, order="longest_first"), dict(slots=16, waves_per_cu=2),
               dict(kernel="columns", slots=4, waves_per_cu=1), dict(kernel="columns", slots=8, order="longest_first"),
               dict(kernel="columns", slots=16, waves_per_cu=2), dict(kernel="columns", slots=32),
               dict(kernel="columns", slots=24, waves_per_cu=1), dict(kernel="columns", slots=10),
               dict(kernel="columns", slots=9, waves_per_cu=1)):
        log(f"[parity] launch shape {kw}")
        kw.setdefault("kernel", "rows")
        compare(b, run_gpu(ctx, b, mode="fixed", fixed_rows=12, **kw), ref, f"shape {kw}")


@pytest.mark.parametrize("W,O", [(64, 24), (64, 33), (64, 10), (32, 17)])
def test_one_wavefront_per_simd(ctx, W, O):
    # the form that reserves a SIMD per wavefront (48-, 32- and 64-bit stored
    # entries), 4, 8 and 10 windows per wavefront, with unrelated pairs mixed in
    mixed = synth.make_batch("mixed_10kbp", indices=range(300, 324))
    pats = [mixed.pat[mixed.pat_off[i]:mixed.pat_off[i + 1]].tobytes() for i in range(mixed.npairs)]
    txts = [mixed.txt[mixed.txt_off[i]:mixed.txt_off[i + 1]].tobytes() for i in range(mixed.npairs)]
    rng = np.random.default_rng(11)
    for _ in range(6):
        p, t = synth.random_pair(rng, 500, 520)
        pats.append(p)
        txts.append(t)
    b = synth.from_lists(pats, txts)
    ref = oracle.align_batch(b, W, O, W)
    for slots in (4, 8, 10):
        log(f"[parity] one wavefront per SIMD W={W} O={O} slots={slots}")
        gpu = run_gpu(ctx, b, W=W, O=O, k=W, kernel="columns", slots=slots, one_per_simd=True)
        compare(b, gpu, ref, f"one per SIMD W={W} O={O} slots={slots}")


def test_one_wavefront_per_simd_queue_cycles(ctx):
    # more wavefronts' worth of pairs than SIMDs: the capped grid takes pairs
    # from the queue until it is empty
    from paper_2208_09985_amd import api
    b = synth.make_batch("small_100bp", 4 * 4 * ctx.cus + 300)
    ref = oracle.align_batch(b, 64, 24, 64)
    bt = api.Batch(ctx, b, api.params(kernel="columns", slots=4, one_per_simd=True))
    shape = bt.launch_shape()
    bt.close()
    assert shape["one_per_simd"] and shape["grid"] == 4 * ctx.cus, shape
    compare(b, run_gpu(ctx, b, kernel="columns", slots=4, one_per_simd=True), ref, "one per SIMD, queue cycles")


def test_one_wavefront_per_simd_refused_forms(ctx):
    from paper_2208_09985_amd import _lib as L, api
    b = synth.make_batch("small_100bp", 16)
    for kw in (dict(mode="learned"), dict(rows_lds=True), dict(store_edges=True), dict(row_ring=True),
               dict(slots=32), dict(kernel="rows"), dict(kernel="lanes"), dict(W=96, O=24, k=96)):
        prm = dict(kernel="columns", one_per_simd=True)
        prm.update(kw)
        with pytest.raises(L.ScgError) as e:
            api.Batch(ctx, b, api.params(**prm))
        assert e.value.code == L.EINVAL, (kw, e.value)


def _offtrack_batch(n_mixed=40, n_unrelated=12, seed=5):
    # long pairs of which some lose the diagonal (unrelated sequences: every window deep)
    mixed = synth.make_batch("mixed_10kbp", indices=range(500, 500 + n_mixed))
    pats = [mixed.pat[mixed.pat_off[i]:mixed.pat_off[i + 1]].tobytes() for i in range(mixed.npairs)]
    txts = [mixed.txt[mixed.txt_off[i]:mixed.txt_off[i + 1]].tobytes() for i in range(mixed.npairs)]
    rng = np.random.default_rng(seed)
    for i in range(n_unrelated):
        p, t = synth.random_pair(rng, 1500 + 100 * i, 1500 + 100 * i)
        pats.append(p)
        txts.append(t)
    return synth.from_lists(pats, txts)


@pytest.mark.parametrize("W,O,rows_lds", [(64, 24, False), (64, 33, False), (32, 8, False), (64, 16, False),
                                           (64, 17, False), (64, 24, True), (64, 16, True)])
def test_offtrack_helpers_keep_results(ctx, W, O, rows_lds):
    # pairs handed to the 4-window helper launch after three deep windows come out
    # exactly as the oracle's; the helper launch leaves once every pair is finished.
    # The helpers keep their lowest rows in LDS (32-, 48- and 64-bit entries: W-O of
    # 31, 40 and 47, and 48); with rows_lds the main launch does too
    from paper_2208_09985_amd import api
    b = _offtrack_batch()
    ref = oracle.align_batch(b, W, O, W)
    bt = api.Batch(ctx, b, api.params(W=W, O=O, k=W, kernel="columns", offtrack_helpers=True, rows_lds=rows_lds))
    shape = bt.launch_shape()
    bt.close()
    log(f"[parity] off-track helpers W={W} O={O} rows_lds={rows_lds} shape {shape}")
    assert shape["helper_grid"] > 0 and shape["helper_slots"] == 4 and shape["slots"] == 16, shape
    assert (shape["lds_bytes"] > 0) == rows_lds and shape["helper_lds_bytes"] > 0, shape
    res = run_gpu(ctx, b, W=W, O=O, k=W, kernel="columns", offtrack_helpers=True, rows_lds=rows_lds)
    compare(b, res, ref, f"off-track helpers W={W} O={O} rows_lds={rows_lds}")
    assert res.stats.yields > 0, "no pair was handed over"


def test_offtrack_helpers_idle_and_repeated(ctx):
    # helpers that never receive a pair leave with the main launch; a prepared batch
    # with helpers runs several times with the same results
    import torch
    from paper_2208_09985_amd import api
    small = synth.make_batch("small_100bp", 600)
    ref = oracle.align_batch(small, 64, 24, 64)
    res = run_gpu(ctx, small, kernel="columns", offtrack_helpers=True)
    compare(small, res, ref, "helpers idle")
    assert res.stats.yields == 0
    b = _offtrack_batch(24, 8, seed=9)
    ref = oracle.align_batch(b, 64, 24, 64)
    bt = api.Batch(ctx, b, api.params(kernel="columns", offtrack_helpers=True, slots=10))
    for rep in range(3):
        bt.edits.fill_(-7)
        bt.run()
        torch.cuda.synchronize()
        compare(b, bt.result(), ref, f"helpers, run {rep}")
    bt.close()


def test_offtrack_helpers_stop_waiting(ctx, monkeypatch):
    # a helper that sees no beat of the main launch for idle_limit polls (forced small
    # from the host) closes the hand-over gate: pairs handed over before that are
    # still finished by the helpers, later ones stay in the main launch, and the
    # results are the oracle's either way
    from paper_2208_09985_amd import api
    b = _offtrack_batch(24, 8, seed=11)
    ref = oracle.align_batch(b, 64, 24, 64)
    for polls in ("0", "1", "3", "40"):
        monkeypatch.setenv("SCG_HELPER_IDLE_POLLS", polls)
        log(f"[parity] helpers stop waiting after {polls} idle polls")
        res = run_gpu(ctx, b, kernel="columns", offtrack_helpers=True)
        compare(b, res, ref, f"helpers stop waiting after {polls} polls")
        log(f"[parity]   pairs handed over: {res.stats.yields}")
    monkeypatch.delenv("SCG_HELPER_IDLE_POLLS")


def test_offtrack_helpers_graph_replays(ctx):
    # the graph flag on a batch with helpers: the launches are enqueued directly (the
    # helper launch must run beside the main one on the context's helper stream); every
    # run, with eager work between runs, gives the oracle's results
    import torch
    from paper_2208_09985_amd import api
    b = _offtrack_batch(24, 8, seed=13)
    ref = oracle.align_batch(b, 64, 24, 64)
    gb = api.Batch(ctx, b, api.params(kernel="columns", offtrack_helpers=True, graph=True))
    assert gb.launch_shape()["helper_grid"] > 0
    for rep in range(3):
        gb.edits.fill_(-7)
        gb.n_runs.fill_(0)
        gb.run()
        torch.cuda.synchronize()
        compare(b, gb.result(), ref, f"helpers with the graph flag, run {rep}")
        _ = torch.ones(1000, device=gb.dev).sum().item()
    gb.close()


def test_offtrack_helpers_two_batches_two_streams(ctx):
    # two batches of one context share the context's helper stream: run at once on two
    # streams (their helper launches take turns), both give the oracle's results, twice
    import torch
    from paper_2208_09985_amd import api
    b1 = _offtrack_batch(24, 8, seed=21)
    b2 = _offtrack_batch(16, 10, seed=22)
    ref1 = oracle.align_batch(b1, 64, 24, 64)
    ref2 = oracle.align_batch(b2, 64, 24, 64)
    g1 = api.Batch(ctx, b1, api.params(kernel="columns", offtrack_helpers=True))
    g2 = api.Batch(ctx, b2, api.params(kernel="columns", offtrack_helpers=True))
    assert g1.launch_shape()["helper_grid"] > 0 and g2.launch_shape()["helper_grid"] > 0
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    torch.cuda.synchronize()
    for rep in range(2):
        log(f"[parity] two helper batches on two streams, run {rep}")
        g1.run(s1)
        g2.run(s2)
        torch.cuda.synchronize()
        compare(b1, g1.result(), ref1, f"first of two batches on two streams, run {rep}")
        compare(b2, g2.result(), ref2, f"second of two batches on two streams, run {rep}")
    g1.close()
    g2.close()


def test_offtrack_helpers_refused_forms(ctx):
    from paper_2208_09985_amd import _lib as L, api
    b = synth.make_batch("small_100bp", 16)
    for kw in (dict(mode="fixed", fixed_rows=7), dict(rows_lds=True, slots=10), dict(store_edges=True),
               dict(slots=4), dict(yield_chars=64), dict(one_per_simd=False), dict(kernel="rows")):
        prm = dict(kernel="columns", offtrack_helpers=True)
        prm.update(kw)
        with pytest.raises(L.ScgError) as e:
            api.Batch(ctx, b, api.params(**prm))
        assert e.value.code == L.EINVAL, (kw, e.value)


@pytest.mark.parametrize("W,O", [(64, 24), (64, 40)])
def test_ablation_flags_keep_results(ctx, W, O):
    # no early termination / all columns stored: more work, same alignments
    b = synth.make_batch("long_10kbp", indices=range(200, 232))
    ref = oracle.align_batch(b, W, O, W)
    for kw in (dict(no_early_termination=True), dict(store_all_columns=True),
               dict(no_early_termination=True, store_all_columns=True, slots=4), dict(rows_lds=True),
               dict(rows_lds=True, store_all_columns=True, slots=16), dict(rows_lds=True, slots=4, waves_per_cu=1),
               dict(rows_lds=True, no_early_termination=True), dict(store_edges=True),
               dict(store_edges=True, no_early_termination=True, store_all_columns=True, slots=4),
               dict(store_edges=True, slots=16), dict(row_ring=True), dict(row_ring=True, slots=4),
               dict(row_ring=True, slots=16, store_edges=True, store_all_columns=True)):
        log(f"[parity] ablation W={W} O={O} {kw}")
        compare(b, run_gpu(ctx, b, W=W, O=O, k=W, kernel="columns", **kw), ref, f"ablation {kw}")


@pytest.mark.parametrize("kernel,mode", [("rows", "fixed"), ("columns", "plain")])
def test_graph_replays_match_eager(ctx, kernel, mode):
    import torch
    from paper_2208_09985_amd import api
    b = synth.make_batch("short_250bp", 3000)
    ref = oracle.align_batch(b, 64, 24, 64)
    gb = api.Batch(ctx, b, api.params(graph=True, mode=mode, fixed_rows=8, kernel=kernel))
    for rep in range(4):
        log(f"[parity] graph replay {kernel} {rep}")
        gb.edits.fill_(-7)
        gb.run()
        torch.cuda.synchronize()
        compare(b, gb.result(), ref, f"graph replay {kernel} {rep}")
        _ = torch.ones(1000, device=gb.dev).sum().item()   # eager work between replays
    gb.close()


@pytest.mark.parametrize("yield_chars,kw", [(40, dict(mode="fixed", fixed_rows=7, slots=4)), (40, dict()),
                                            (0, dict(mode="fixed", fixed_rows=15, slots=6)),
                                            (100, dict(mode="fixed", fixed_rows=11, slots=16, waves_per_cu=1))])
def test_yielding_queue_keeps_results(ctx, yield_chars, kw):
    """Pairs handed back to the queue every few windows (state saved and
    resumed on another wavefront) give the same alignments."""
    b = synth.make_batch("uneven_lognormal", indices=range(200, 260))
    ref = oracle.align_batch(b, 64, 24, 64)
    for kern in KERNELS:
        log(f"[parity] yield_chars={yield_chars} {kw} kernel={kern}")
        gpu = run_gpu(ctx, b, yield_chars=yield_chars, kernel=kern, **kw)
        compare(b, gpu, ref, f"yield {yield_chars} {kw} [{kern}]")
        if yield_chars:
            assert gpu.stats.yields > 0
        else:
            assert gpu.stats.yields == 0


def test_unrelated_pairs_long_tracebacks(ctx):
    """Unrelated sequences: windows with distances near the pattern length and
    tracebacks that run over several passes of the column kernel."""
    rng = np.random.default_rng(7)
    pats = [synth.ALPHABET[rng.integers(0, 4, int(rng.integers(50, 600)))].tobytes() for _ in range(300)]
    txts = [synth.ALPHABET[rng.integers(0, 4, int(rng.integers(50, 600)))].tobytes() for _ in range(300)]
    b = synth.from_lists(pats, txts)
    for slots in (4, 8, 10, 16):
        check(ctx, b, what=f"unrelated slots={slots}", kernels=("columns",), slots=slots)
    check(ctx, b, what="unrelated, edges stored", kernels=("columns",), store_edges=True)
    check(ctx, b, what="unrelated, rows in LDS", kernels=("columns",), rows_lds=True)
    # distances above W-O: the row ring wraps within a window
    for slots in (4, 8, 16):
        check(ctx, b, what=f"unrelated, row ring slots={slots}", kernels=("columns",), row_ring=True, slots=slots)
    check(ctx, b, W=64, O=40, k=64, what="unrelated, row ring W64 O40", kernels=("columns",), row_ring=True)
    check(ctx, b, what="unrelated, one lane per pair", kernels=("lanes",))
    check(ctx, b, W=64, O=40, k=64, what="unrelated, one lane per pair W64 O40", kernels=("lanes",))
    check(ctx, b, what="unrelated rows", kernels=("rows",))



def test_long_one_sided_indels(ctx):
    """Long insertions and deletions (16-30 bases): traceback paths far from
    the diagonal, in both kernels."""
    rng = np.random.default_rng(11)
    pats, txts = [], []
    for _ in range(200):
        p = synth.ALPHABET[rng.integers(0, 4, int(rng.integers(100, 500)))]
        t = p.copy()
        for _ in range(int(rng.integers(1, 4))):
            pos = int(rng.integers(0, len(t)))
            ln = int(rng.integers(16, 31))
            if rng.random() < 0.5:
                t = np.insert(t, pos, synth.ALPHABET[rng.integers(0, 4, ln)])
            else:
                t = np.delete(t, np.arange(pos, min(len(t), pos + ln)))
        pats.append(p.tobytes())
        txts.append(t.tobytes())
    b = synth.from_lists(pats, txts)
    check(ctx, b, what="long indels")
    for slots in (4, 10, 16):
        check(ctx, b, what=f"long indels slots={slots}", kernels=("columns",), slots=slots)
    check(ctx, b, what="long indels, one lane per pair", kernels=("lanes",))


def test_one_shot_batch_call(ctx):
    # scg_align_batch: host arrays in and out, and device arrays in and out, ASCII
    # or pre-packed 2-bit input; 2-bit operation streams out, rendered by
    # scg_ops_to_cigar
    from paper_2208_09985_amd import api
    b = synth.make_batch("uneven_lognormal", 24)
    pats = [b.pattern(i) for i in range(b.npairs)] + [b"", b"ACGT", b"acgtT", b"G" * 130]
    txts = [b.text(i) for i in range(b.npairs)] + [b"AC", b"", b"ACGTA", b"G" * 129 + b"T"]
    b = synth.from_lists(pats, txts)
    ref = oracle.align_batch(b, 64, 24, 64)
    for host in (True, False):
        for packed in (False, True):
            log(f"[parity] one-shot batch call host={host} packed={packed}")
            res = api.align_batch_once(ctx, b, host=host, packed=packed)
            compare(b, res, ref, f"one-shot host={host} packed={packed}")
            assert res.stats.windows == ref["stats"].windows and res.stats.kernel_ms > 0
            for i in range(b.npairs):
                assert res.cigar(i) == oracle.cigar(oracle.ops_of(ref, i)), i


@pytest.mark.parametrize("W,O,k,slots", [(128, 24, 128, 0), (128, 64, 128, 8), (96, 32, 96, 0), (65, 0, 65, 4),
                                         (128, 127, 128, 0), (100, 40, 30, 8), (128, 24, 5, 0), (128, 33, 128, 8),
                                         (128, 32, 128, 8), (128, 65, 128, 0), (128, 65, 128, 8)])
def test_wide_windows(ctx, W, O, k, slots):
    # windows of 65..128 characters (wide kernel), against the oracle's 128-bit instantiation
    rng = np.random.default_rng(W * 1000 + O * 10 + k)
    pats, txts = [], []
    for i in range(120):
        m = int(rng.integers(0, 700)) if i % 10 else int(rng.integers(0, 3))
        p = synth.ALPHABET[rng.integers(0, 4, m)]
        t = p.copy()
        for _ in range(int(m * rng.uniform(0, 0.3))):
            pos = int(rng.integers(0, max(1, len(t))))
            r = rng.random()
            if r < 0.33 and len(t):
                t[pos] = synth.ALPHABET[rng.integers(0, 4)]
            elif r < 0.66:
                t = np.insert(t, pos, synth.ALPHABET[rng.integers(0, 4, int(rng.integers(1, 6)))])
            elif len(t):
                t = np.delete(t, slice(pos, pos + int(rng.integers(1, 6))))
        if i % 17 == 0:
            t = synth.ALPHABET[rng.integers(0, 4, int(rng.integers(0, 300)))]   # unrelated text
        pats.append(p.tobytes())
        txts.append(t.tobytes())
    b = synth.from_lists(pats, txts)
    check(ctx, b, W=W, O=O, k=k, what=f"wide W{W}O{O}k{k} slots{slots}", kernels=("columns",), slots=slots)


def test_wide_windows_long_reads(ctx):
    b = synth.make_batch("long_10kbp", indices=range(300, 316))
    check(ctx, b, W=128, O=24, k=128, what="wide long_10kbp", kernels=("columns",))
