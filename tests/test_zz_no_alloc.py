"""The allocation-free entry point (scg_align_batch_noalloc) against the
allocating one (scg_batch_create + scg_batch_run with device input, which
returns the same run words), through the C ABI:
identical status, edits, text_end and run words for every pair, on calls in
a row whose second input is smaller than the first (the static workspace
keeps the previous call's contents).  Also its size limits and its handling
of inconsistent offsets."""
import ctypes

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


def same(a, b, what):
    n = len(a.edits)
    assert np.array_equal(a.status, b.status), f"{what}: status"
    assert np.array_equal(a.edits, b.edits), f"{what}: edits"
    assert np.array_equal(a.text_end, b.text_end), f"{what}: text_end"
    assert np.array_equal(a.n_runs, b.n_runs), f"{what}: n_runs"
    ra, rb = np.asarray(a.runs).view(np.uint32), np.asarray(b.runs).view(np.uint32)
    for i in range(n):
        s = int(a.runs_off[i])
        assert np.array_equal(ra[s:s + int(a.n_runs[i])], rb[s:s + int(b.n_runs[i])]), f"{what}: runs of pair {i}"


def test_noalloc_matches_align_batch_on_calls_in_a_row(ctx):
    from paper_2208_09985_amd import api
    big = synth.make_batch("long_10kbp", 600)
    pats = [big.pattern(i) for i in range(big.npairs)] + [b"", b"ACGT", b"A" * 70]
    txts = [big.text(i) for i in range(big.npairs)] + [b"ACG", b"", b"C" * 10]
    big = synth.from_lists(pats, txts)
    small = synth.make_batch("short_250bp", 37)
    for what, b, kw in (("first call, 603 pairs", big, {}), ("second call, 37 pairs", small, {}),
                        ("third call, 603 pairs, 4 windows per wavefront", big, dict(slots=4)),
                        ("fourth call, 37 pairs, W=32 O=17", small, dict(W=32, O=17, k=32))):
        log(f"[noalloc] {what}")
        got = api.align_batch_noalloc(ctx, b, **kw)
        want = api.align_batch(ctx, b, kernel="columns", **kw)
        same(got, want, what)
        W, O, k = kw.get("W", 64), kw.get("O", 24), kw.get("k", 64)
        compare(b, got, oracle.align_batch(b, W, O, k), what)


def test_noalloc_limits_and_bad_offsets(ctx):
    import torch
    from paper_2208_09985_amd import api, _lib as L
    lib = ctx._lib
    prm = api.params()
    z = ctypes.c_void_p(0)
    rc = lib.scg_align_batch_noalloc(ctx.handle, ctypes.byref(prm), L.NOALLOC_MAX_PAIRS + 1, z, z, 0, z, z, 0, z,
                                     z, z, z, z, z)
    assert rc == L.ELIMIT
    rc = lib.scg_align_batch_noalloc(ctx.handle, ctypes.byref(prm), 1, z, z, L.NOALLOC_MAX_BASES + 1, z, z, 0, z,
                                     z, z, z, z, z)
    assert rc == L.ELIMIT
    lprm = api.params(mode="fixed", fixed_rows=4)
    rc = lib.scg_align_batch_noalloc(ctx.handle, ctypes.byref(lprm), 1, z, z, 0, z, z, 0, z, z, z, z, z, z)
    assert rc == L.EINVAL
    # offsets out of order (checked on the device): every pair is bad input
    dev = torch.device("cuda:0")
    pat = torch.frombuffer(bytearray(b"ACGTACGTAC"), dtype=torch.uint8).to(dev)
    txt = torch.frombuffer(bytearray(b"ACGTACGTAC"), dtype=torch.uint8).to(dev)
    off = torch.tensor([0, 6, 4, 10], dtype=torch.int64, device=dev)
    outs = [torch.full((3,), -9, dtype=torch.int32, device=dev) for _ in range(4)]
    runs = torch.zeros(64, dtype=torch.int32, device=dev)
    torch.cuda.synchronize()
    P = lambda t: ctypes.c_void_p(t.data_ptr())
    rc = lib.scg_align_batch_noalloc(ctx.handle, ctypes.byref(prm), 3, P(pat), P(off), 10, P(txt), P(off), 10, z,
                                     P(outs[0]), P(outs[1]), P(outs[2]), P(runs), P(outs[3]))
    assert rc == L.OK
    torch.cuda.synchronize()
    assert outs[2].cpu().tolist() == [L.PAIR_BAD_INPUT] * 3
    assert outs[0].cpu().tolist() == [-1, -1, -1]
    # and the next call with good offsets is unaffected
    b = synth.make_batch("small_100bp", 50)
    compare(b, api.align_batch_noalloc(ctx, b), oracle.align_batch(b, 64, 24, 64), "after bad offsets")
