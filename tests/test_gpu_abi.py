"""The C ABI's calls and error paths on the GPU (through ctypes): predictor
file at context creation, pre-packed input in the batch API, the three-value
scg_last_stats, and the documented error codes: no predictor, window ranges,
too-small CIGAR and operation buffers."""
import ctypes
import os

import numpy as np
import pytest

import oracle
from paper_2208_09985_amd import synth
from tests.gpu_helpers import compare, log

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SCGW = os.path.join(ROOT, "paper_2208_09985_amd", "weights", "budget_w64_o24.scgw")


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2208_09985_amd import api
    return api.Context(0)


def test_predictor_file_at_creation(ctx, tmp_path):
    from paper_2208_09985_amd import api, _lib as L
    c = api.Context(0, weights_path=SCGW)
    b = synth.make_batch("mixed_10kbp", 16)
    ref = oracle.align_batch(b, 64, 24, 64)
    for kern in ("rows", "columns"):
        log(f"[abi] learned mode from the predictor file, kernel={kern}")
        compare(b, api.align_batch(c, b, mode="learned", kernel=kern), ref, f"scgw learned [{kern}]")
    c.close()
    with pytest.raises(L.ScgError) as e:
        api.Context(0, weights_path=str(tmp_path / "missing.scgw"))
    assert e.value.code == L.EINVAL
    bad = tmp_path / "bad.scgw"
    bad.write_bytes(open(SCGW, "rb").read()[:-2])   # truncated
    with pytest.raises(L.ScgError) as e:
        api.Context(0, weights_path=str(bad))
    assert e.value.code == L.EINVAL


def test_learned_mode_without_predictor(ctx):
    from paper_2208_09985_amd import api, _lib as L
    c = api.Context(0)
    b = synth.make_batch("small_100bp", 4)
    with pytest.raises(L.ScgError) as e:
        api.Batch(c, b, api.params(mode="learned"))
    assert e.value.code == L.ENOMODEL
    with pytest.raises(L.ScgError) as e:
        api.align_batch_once(c, b, mode="learned")
    assert e.value.code == L.ENOMODEL


@pytest.mark.parametrize("kw", [dict(W=0, O=0, k=0), dict(W=129, O=24, k=64), dict(W=64, O=64, k=64),
                                dict(W=64, O=-1, k=64), dict(W=64, O=24, k=65), dict(W=64, O=24, k=-1),
                                dict(W=96, O=24, k=96, mode="learned"), dict(W=96, O=24, k=96, mode="fixed"),
                                dict(W=64, O=24, k=64, mode="fixed", fixed_rows=0),
                                dict(W=64, O=24, k=64, slots=33), dict(W=64, O=24, k=64, yield_chars=10)])
def test_window_and_launch_ranges(kw):
    from paper_2208_09985_amd import api, _lib as L
    c = api.Context(0, weights_path=SCGW)
    b = synth.make_batch("small_100bp", 4)
    with pytest.raises(L.ScgError) as e:
        api.Batch(c, b, api.params(**kw))
    assert e.value.code == L.EINVAL, kw
    with pytest.raises(L.ScgError) as e:
        api.align_batch_once(c, b, **kw)
    assert e.value.code == L.EINVAL, kw


def test_single_pair_cigar_buffer_too_small(ctx):
    lib = ctx._lib
    from paper_2208_09985_amd import _lib as L
    p, t = b"ACGTACGTTTGACCA" * 5, b"ACGTACGTTGACCAT" * 5
    want = oracle.cigar(oracle.align_pair(p, t, 64, 24, 64)["ops"]).encode()
    e, te, ln = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    small = ctypes.create_string_buffer(4)
    rc = lib.scg_align(ctx.handle, p, len(p), t, len(t), 64, 24, 64, ctypes.byref(e), ctypes.byref(te), small, 4,
                       ctypes.byref(ln))
    assert rc == L.ERANGE and ln.value == len(want)
    buf = ctypes.create_string_buffer(len(want) + 1)
    rc = lib.scg_align(ctx.handle, p, len(p), t, len(t), 64, 24, 64, ctypes.byref(e), ctypes.byref(te), buf,
                       len(want) + 1, ctypes.byref(ln))
    assert rc == L.OK and buf.value == want
    rc = lib.scg_align(ctx.handle, p, len(p), t, len(t), 64, 24, 65, ctypes.byref(e), ctypes.byref(te), buf,
                       len(want) + 1, ctypes.byref(ln))
    assert rc == L.EINVAL


def test_operation_buffer_too_small_and_last_stats(ctx):
    from paper_2208_09985_amd import api, _lib as L
    lib = ctx._lib
    b = synth.make_batch("short_250bp", 8)
    n = b.npairs
    prm = api.params()
    off = api.ops_offsets(b)
    off[3:] -= 1                      # pair 2 one byte short
    outs = [np.zeros(n, np.int32) for _ in range(4)]
    ops = np.zeros(int(off[-1]) + 8, np.uint8)
    P = lambda a: ctypes.c_void_p(a.ctypes.data)
    rc = lib.scg_align_batch(ctx.handle, ctypes.byref(prm), n, P(b.pat), P(b.pat_off), P(b.txt), P(b.txt_off),
                             L.INPUT_ASCII, L.WHERE_HOST, None, P(outs[0]), P(outs[1]), P(outs[2]), P(ops), P(off),
                             P(outs[3]))
    assert rc == L.ERANGE
    res = api.align_batch_once(ctx, b)
    ref = oracle.align_batch(b, 64, 24, 64)
    compare(b, res, ref, "last stats run")
    km, oa, fb = ctypes.c_double(), ctypes.c_int64(), ctypes.c_int64()
    assert lib.scg_last_stats(ctx.handle, ctypes.byref(km), ctypes.byref(oa), ctypes.byref(fb)) == L.OK
    assert km.value > 0 and oa.value == ref["stats"].ops_alg and fb.value == 0
    assert lib.scg_last_stats(ctx.handle, None, ctypes.byref(oa), None) == L.OK


@pytest.mark.parametrize("host", [True, False])
def test_packed_input_prepared_batch(ctx, host):
    from paper_2208_09985_amd import api
    b = synth.make_batch("long_10kbp", 24)
    pats = [b.pattern(i) for i in range(b.npairs)] + [b"", b"A", b"C" * 64, b"G" * 65]
    txts = [b.text(i) for i in range(b.npairs)] + [b"T", b"", b"C" * 64, b"G" * 31]
    b = synth.from_lists(pats, txts)
    ref = oracle.align_batch(b, 64, 24, 64)
    for kern, mode in (("columns", "plain"), ("rows", "plain"), ("rows", "fixed")):
        log(f"[abi] packed input host={host} kernel={kern} mode={mode}")
        bt = api.Batch(ctx, b, api.params(kernel=kern, mode=mode, fixed_rows=9), device_input=not host, packed=True)
        bt.run()
        import torch
        torch.cuda.synchronize()
        compare(b, bt.result(), ref, f"packed host={host} [{kern} {mode}]")
        bt.close()
