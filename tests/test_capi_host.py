"""Host-only checks of the C ABI (no GPU needed): the library builds and loads,
exports every function include/scrooge.h declares, and its pure-host helpers
behave as documented."""
import ctypes
import os
import re

import numpy as np

from paper_2208_09985_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "scrooge.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(scg_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    lib = L.load()
    names = declared_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(L.EXPORTED)


def test_strerror_and_defaults():
    lib = L.load()
    assert lib.scg_strerror(0) == b"ok"
    assert lib.scg_strerror(L.EALPHABET) == b"character outside A/C/G/T"
    assert lib.scg_strerror(12345) == b"unknown status"
    p = L.Params()
    lib.scg_params_default(ctypes.byref(p))
    assert (p.W, p.O, p.k, p.mode) == (64, 24, 64, L.MODE_PLAIN)


def test_runs_to_cigar():
    lib = L.load()
    runs = np.array([(12 << 2) | 0, (1 << 2) | 1, (3 << 2) | 2, (2 << 2) | 3], dtype=np.uint32)
    buf = ctypes.create_string_buffer(64)
    n = ctypes.c_int32()
    assert lib.scg_runs_to_cigar(runs.ctypes.data, 4, buf, 64, ctypes.byref(n)) == 0
    assert buf.value == b"12=1X3I2D" and n.value == 9
    small = ctypes.create_string_buffer(4)
    assert lib.scg_runs_to_cigar(runs.ctypes.data, 4, small, 4, ctypes.byref(n)) == L.ERANGE
    assert n.value == 9
    assert lib.scg_runs_to_cigar(None, -1, buf, 64, ctypes.byref(n)) == L.EINVAL
    assert lib.scg_runs_to_cigar(None, 0, buf, 64, ctypes.byref(n)) == 0 and buf.value == b""


def test_null_arguments_are_rejected_without_a_device():
    lib = L.load()
    assert lib.scg_create(None, 0, None) == L.EINVAL
    assert lib.scg_last_stats(None, None, None, None) == L.EINVAL
    assert lib.scg_last_stats_all(None, None) == L.EINVAL
    assert lib.scg_align_batch(None, None, 0, *([None] * 4), 0, 0, *([None] * 7)) == L.EINVAL
    assert lib.scg_align_batch_noalloc(None, None, 0, None, None, 0, None, None, 0, *([None] * 6)) == L.EINVAL
    assert lib.scg_batch_runs_capacity(None) == -1
    assert lib.scg_batch_stats(None, None) == L.EINVAL
    assert lib.scg_batch_run(None, None, None, None, None, None, None) == L.EINVAL
    assert lib.scg_set_model(None, 16, 64, 4, None, None, None, None, None) == L.EINVAL
    assert lib.scg_mlp_forward(4, 15, 64, 4, *([None] * 11)) == L.EINVAL
    assert lib.scg_adam_step(4, None, None, None, None, None, 1e-3, 0.9, 0.999, 1e-8, 0, None) == L.EINVAL


def test_ops_to_cigar():
    """2-bit operation streams (op t in byte t // 4, bits 2 (t % 4)..) rendered
    with runs merged, against a run list written out by hand."""
    lib = L.load()
    ops = [0] * 12 + [1] + [2] * 3 + [3] * 2 + [0]
    packed = np.zeros((len(ops) + 3) // 4, np.uint8)
    for t, o in enumerate(ops):
        packed[t // 4] |= o << (2 * (t % 4))
    buf = ctypes.create_string_buffer(64)
    n = ctypes.c_int32()
    assert lib.scg_ops_to_cigar(packed.ctypes.data, len(ops), buf, 64, ctypes.byref(n)) == 0
    assert buf.value == b"12=1X3I2D1=" and n.value == 11
    small = ctypes.create_string_buffer(5)
    assert lib.scg_ops_to_cigar(packed.ctypes.data, len(ops), small, 5, ctypes.byref(n)) == L.ERANGE
    assert n.value == 11
    # only the first n_ops operations count, whatever the rest of the last byte holds
    packed[-1] |= 0xC0   # bits of a 20th operation
    assert lib.scg_ops_to_cigar(packed.ctypes.data, len(ops), buf, 64, ctypes.byref(n)) == 0
    assert buf.value == b"12=1X3I2D1="
    assert lib.scg_ops_to_cigar(None, 0, buf, 64, ctypes.byref(n)) == 0 and buf.value == b""
    assert lib.scg_ops_to_cigar(None, 3, buf, 64, ctypes.byref(n)) == L.EINVAL


def test_packed_input_helper():
    """The binding's 2-bit packer (input preparation for SCG_INPUT_PACKED2):
    base t of a sequence at bits 2t of its words, sequences word-aligned."""
    from paper_2208_09985_amd import api, synth
    b = synth.from_lists([b"ACGTTGCA" * 5, b"", b"t" * 33], [b"A", b"CC", b"G" * 64])
    w = api.pack2(b.pat, b.pat_off)
    assert w.dtype == np.uint64 and w.size == 2 + 0 + 2
    codes = {ord("A"): 0, ord("C"): 1, ord("G"): 2, ord("T"): 3}
    seq = b"ACGTTGCA" * 5
    for t, ch in enumerate(seq):
        assert (int(w[t // 32]) >> (2 * (t % 32))) & 3 == codes[ch]
    assert int(w[1]) >> 16 == 0                      # past the 40th base
    assert int(w[2]) == (1 << 64) - 1 and int(w[3]) == 3


def test_predictor_file_matches_npz():
    """The committed predictor file scg_create reads holds the same numbers as
    the npz the training run wrote."""
    z = np.load(os.path.join(ROOT, "paper_2208_09985_amd", "weights", "budget_w64_o24.npz"), allow_pickle=False)
    raw = open(os.path.join(ROOT, "paper_2208_09985_amd", "weights", "budget_w64_o24.scgw"), "rb").read()
    assert raw[:4] == b"SCGW"
    ver, F, H, C = np.frombuffer(raw[4:20], "<i4")
    assert (ver, F, H, C) == (1, 16, z["w1"].shape[1], z["w2"].shape[1])
    rows = np.frombuffer(raw[20:20 + 4 * C], "<i4")
    assert np.array_equal(rows, z["budget_rows"])
    h = np.frombuffer(raw[20 + 4 * C:], "<f2")
    parts = np.split(h, np.cumsum([F * H, H, H * C]))
    for got, key in zip(parts, ("w1", "b1", "w2", "b2")):
        assert np.array_equal(got, z[key].astype(np.float16).reshape(-1))
