"""CPU oracle for windowed GenASM alignment (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product path never does, and it
shares no code with the GPU library: the C source here has its own encoder,
mask builder, table layout and traceback.

``build()`` compiles ``scrooge_oracle.c`` with gcc into ``_build/``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "scrooge_oracle.c")
INC = os.path.join(HERE, "oracle_width.inc")   # width-generic body, included twice by SRC
BUILD_DIR = os.path.join(HERE, "_build")
LIB_PATH = os.path.join(BUILD_DIR, "liboracle.so")

OK, NOT_ALIGNED = 0, 1
OP_M, OP_S, OP_I, OP_D = 0, 1, 2, 3
OP_CHARS = "=XID"


class Stats(ctypes.Structure):
    _fields_ = [
        ("windows", ctypes.c_int64),
        ("ops_alg", ctypes.c_int64),
        ("ops_genasm", ctypes.c_int64),
        ("tb_steps", ctypes.c_int64),
        ("max_col_read", ctypes.c_int32),
        ("max_bit_read", ctypes.c_int32),
        ("max_row_above_dw", ctypes.c_int32),
        ("max_rows_below_dw", ctypes.c_int32),
    ]


WINDOW_DTYPE = np.dtype([(n, np.int32) for n in
                         ("pair", "p0", "t0", "m_w", "n_w", "k_w", "d_w", "adv_p", "adv_t", "edits")])


def build(sanitize: bool = False) -> str:
    """Compile the oracle shared library (gcc, -O2, pthreads)."""
    os.makedirs(BUILD_DIR, exist_ok=True)
    out = LIB_PATH if not sanitize else os.path.join(BUILD_DIR, "liboracle_san.so")
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-fPIC", "-shared", "-pthread", SRC, "-o", out + ".tmp"]
    if sanitize:
        cmd[1:2] = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer"]
    subprocess.check_call(cmd)
    os.replace(out + ".tmp", out)
    return out


_lib = None


def lib():
    global _lib
    if _lib is None and os.environ.get("SCG_ORACLE_LIB"):
        # an explicitly chosen build (the sanitizer build in the tests)
        _lib = _declare(ctypes.CDLL(os.environ["SCG_ORACLE_LIB"]))
    if _lib is None:
        if not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < max(os.path.getmtime(SRC),
                                                                              os.path.getmtime(INC)):
            build()
        _lib = _declare(ctypes.CDLL(LIB_PATH))
    return _lib


def _declare(L):
    """ctypes signatures of the oracle's exported functions."""
    P = ctypes.c_void_p
    i32, i64 = ctypes.c_int32, ctypes.c_int64
    L.or_dc_table.argtypes = [P, i32, P, i32, i32, P, P]
    L.or_dc_table.restype = ctypes.c_int
    L.or_dc_table_wide.argtypes = [P, i32, P, i32, i32, P, P]
    L.or_dc_table_wide.restype = ctypes.c_int
    L.or_pattern_masks.argtypes = [P, i32, P]
    L.or_pattern_masks.restype = ctypes.c_int
    L.or_align_pair.argtypes = [P, i32, P, i32, i32, i32, i32, P, P, P, i64, P, P, P, i64, P, i32]
    L.or_align_pair.restype = ctypes.c_int
    L.or_align_batch.argtypes = [i32, P, P, P, P, i32, i32, i32, i32, P, P, P, P, P, P, P]
    L.or_align_batch.restype = ctypes.c_int
    return L


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def dc_table(pattern: bytes, text: bytes, k: int):
    """Algorithm 1 on one window.  Returns (R, d) with R[i, d] as uint64 in the
    paper's bit order (bit j of the pattern at machine bit m-1-j); d = -1 when
    no row 0..k has a 0 in the msb of R[0][d]."""
    m, n = len(pattern), len(text)
    R = np.zeros((n + 1, k + 1), dtype=np.uint64)
    dw = ctypes.c_int32(0)
    p = np.frombuffer(pattern, np.uint8).copy()
    t = np.frombuffer(text, np.uint8).copy() if n else np.zeros(1, np.uint8)
    rc = lib().or_dc_table(_ptr(p), m, _ptr(t), n, k, _ptr(R), ctypes.byref(dw))
    if rc != 0:
        raise ValueError(f"or_dc_table rc={rc}")
    return R, dw.value


def dc_table_wide(pattern: bytes, text: bytes, k: int):
    """Algorithm 1 on one window of up to 128 characters (the 128-bit
    instantiation).  Returns (R, d): R[i, d] as Python ints in the paper's bit
    order (bit j of the pattern at bit m-1-j), d as in dc_table."""
    m, n = len(pattern), len(text)
    R2 = np.zeros((n + 1) * (k + 1) * 2, dtype=np.uint64)
    dw = ctypes.c_int32(0)
    p = np.frombuffer(pattern, np.uint8).copy()
    t = np.frombuffer(text, np.uint8).copy() if n else np.zeros(1, np.uint8)
    rc = lib().or_dc_table_wide(_ptr(p), m, _ptr(t), n, k, _ptr(R2), ctypes.byref(dw))
    if rc != 0:
        raise ValueError(f"or_dc_table_wide rc={rc}")
    R = np.empty((n + 1, k + 1), dtype=object)
    for x in range((n + 1) * (k + 1)):
        R.flat[x] = int(R2[2 * x]) | (int(R2[2 * x + 1]) << 64)
    return R, dw.value


def pattern_masks(pattern: bytes) -> np.ndarray:
    """PM[A], PM[C], PM[G], PM[T] of a window pattern (paper bit order)."""
    PM = np.zeros(4, np.uint64)
    p = np.frombuffer(pattern, np.uint8).copy()
    rc = lib().or_pattern_masks(_ptr(p), len(pattern), _ptr(PM))
    if rc != 0:
        raise ValueError(f"or_pattern_masks rc={rc}")
    return PM


def align_pair(pattern: bytes, text: bytes, W: int, O: int, k: int, want_windows: bool = False):
    """Align one pair.  Returns dict(status, edits, text_end, ops (uint8 array),
    stats, windows (structured array, if requested))."""
    m, n = len(pattern), len(text)
    p = np.frombuffer(pattern, np.uint8).copy() if m else np.zeros(1, np.uint8)
    t = np.frombuffer(text, np.uint8).copy() if n else np.zeros(1, np.uint8)
    ops = np.zeros(m + n + 1, np.uint8)
    e, te = ctypes.c_int32(), ctypes.c_int32()
    nops, nwin = ctypes.c_int64(), ctypes.c_int64()
    st = Stats()
    st.max_col_read = st.max_bit_read = -1
    wcap = (m // max(1, W - O) + 4) * 4 + n + 4 if want_windows else 0
    wrec = np.zeros(max(wcap, 1), WINDOW_DTYPE)
    rc = lib().or_align_pair(_ptr(p), m, _ptr(t), n, W, O, k, ctypes.byref(e), ctypes.byref(te),
                             _ptr(ops), ops.size, ctypes.byref(nops), ctypes.byref(st),
                             _ptr(wrec) if want_windows else None, wcap, ctypes.byref(nwin), 0)
    if rc < 0:
        raise ValueError(f"or_align_pair rc={rc}")
    out = dict(status=rc, edits=e.value, text_end=te.value, ops=ops[:nops.value].copy(), stats=st)
    if want_windows:
        out["windows"] = wrec[:min(nwin.value, wcap)].copy()
    return out


def align_batch(batch, W: int, O: int, k: int, threads: int | None = None):
    """Align a CSR batch (``synth.PairBatch``-like: pat, pat_off, txt, txt_off)
    on ``threads`` host threads.  Returns dict of numpy arrays + stats."""
    npairs = len(batch.pat_off) - 1
    if threads is None:
        threads = len(os.sched_getaffinity(0))
    lens = np.diff(batch.pat_off) + np.diff(batch.txt_off)
    ops_off = np.zeros(npairs + 1, np.int64)
    ops_off[1:] = np.cumsum(lens)
    ops = np.zeros(max(1, int(ops_off[-1])), np.uint8)
    edits = np.zeros(npairs, np.int32)
    text_end = np.zeros(npairs, np.int32)
    status = np.zeros(npairs, np.int32)
    n_ops = np.zeros(npairs, np.int64)
    st = Stats()
    pat = batch.pat if batch.pat.size else np.zeros(1, np.uint8)
    txt = batch.txt if batch.txt.size else np.zeros(1, np.uint8)
    rc = lib().or_align_batch(npairs, _ptr(pat), _ptr(batch.pat_off), _ptr(txt), _ptr(batch.txt_off),
                              W, O, k, threads, _ptr(edits), _ptr(text_end), _ptr(status),
                              _ptr(ops), _ptr(ops_off), _ptr(n_ops), ctypes.byref(st))
    if rc < 0:
        raise ValueError(f"or_align_batch rc={rc}")
    return dict(edits=edits, text_end=text_end, status=status, ops=ops, ops_off=ops_off, n_ops=n_ops,
                stats=st, threads=threads)


def ops_of(res, i: int) -> np.ndarray:
    s = res["ops_off"][i]
    return res["ops"][s:s + res["n_ops"][i]]


def cigar(ops: np.ndarray) -> str:
    """Run-length encode an op list with '=', 'X', 'I', 'D'."""
    if len(ops) == 0:
        return ""
    ops = np.asarray(ops)
    change = np.flatnonzero(np.diff(ops)) + 1
    starts = np.concatenate([[0], change])
    ends = np.concatenate([change, [len(ops)]])
    return "".join(f"{e - s}{OP_CHARS[ops[s]]}" for s, e in zip(starts, ends))
