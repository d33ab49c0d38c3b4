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
    assert lib.scg_create(None, 0) == L.EINVAL
    assert lib.scg_batch_runs_capacity(None) == -1
    assert lib.scg_batch_stats(None, None) == L.EINVAL
    assert lib.scg_batch_run(None, None, None, None, None, None, None) == L.EINVAL
    assert lib.scg_set_model(None, 16, 64, 4, None, None, None, None, None) == L.EINVAL
    assert lib.scg_mlp_forward(4, 15, 64, 4, *([None] * 11)) == L.EINVAL
    assert lib.scg_adam_step(4, None, None, None, None, None, 1e-3, 0.9, 0.999, 1e-8, 0, None) == L.EINVAL
