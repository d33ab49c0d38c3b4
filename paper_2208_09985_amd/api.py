"""Python interface over the C ABI: contexts, prepared batches, one-pair calls.

PyTorch provides device memory and the stream; every alignment step runs in
the library's HIP kernels.  Names follow include/scrooge.h.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os

import numpy as np

from . import _lib as L

OP_CHARS = "=XID"


def _ptr(x) -> ctypes.c_void_p:
    """Raw pointer of a numpy array or torch tensor (None -> NULL)."""
    if x is None:
        return ctypes.c_void_p(0)
    if isinstance(x, np.ndarray):
        return ctypes.c_void_p(x.ctypes.data)
    return ctypes.c_void_p(x.data_ptr())


def _stream_ptr(stream) -> ctypes.c_void_p:
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def params(W=64, O=24, k=64, mode="plain", slots=0, waves_per_cu=0, order="auto", fixed_rows=None, tau=None,
           graph=False, yield_chars=None, kernel="auto", no_early_termination=False,
           store_all_columns=False, rows_lds=False, store_edges=False, row_ring=False,
           one_per_simd="auto", offtrack_helpers="auto") -> L.Params:
    p = L.Params()
    L.load().scg_params_default(ctypes.byref(p))
    p.W, p.O, p.k = W, O, k
    p.mode = {"plain": L.MODE_PLAIN, "learned": L.MODE_LEARNED, "fixed": L.MODE_FIXED}[mode]
    p.slots, p.waves_per_cu = slots, waves_per_cu
    p.order = {"input": L.ORDER_INPUT, "longest_first": L.ORDER_LONGEST_FIRST, "auto": L.ORDER_AUTO}[order]
    if fixed_rows is not None:
        p.fixed_rows = fixed_rows
    if tau is not None:
        p.tau = tau
    p.flags = ((L.FLAG_GRAPH if graph else 0) | (L.FLAG_NO_EARLY_TERMINATION if no_early_termination else 0)
               | (L.FLAG_STORE_ALL_COLUMNS if store_all_columns else 0) | (L.FLAG_ROWS_LDS if rows_lds else 0)
               | (L.FLAG_STORE_EDGES if store_edges else 0) | (L.FLAG_ROW_RING if row_ring else 0))
    if yield_chars is not None:
        p.yield_chars = yield_chars
    p.kernel = {"auto": L.KERNEL_AUTO, "rows": L.KERNEL_ROWS, "columns": L.KERNEL_COLUMNS,
                "lanes": L.KERNEL_LANES}[kernel]
    p.one_per_simd = {"auto": 0, True: 1, False: -1}[one_per_simd]
    p.offtrack_helpers = {"auto": 0, True: 1, False: -1}[offtrack_helpers]
    return p


class Context:
    """A device context (scg_create).  Holds the learned predictor, if any."""

    def __init__(self, device: int = 0, weights_path: str | None = None):
        self._lib = L.load()
        h = ctypes.c_void_p()
        wp = None if weights_path is None else os.fsencode(weights_path)
        L.check(self._lib.scg_create(ctypes.byref(h), device, wp), "scg_create")
        self.handle = h
        self.device = device

    @property
    def cus(self) -> int:
        return self._lib.scg_device_cus(self.handle)

    def set_model(self, w1, b1, w2, b2, budget_rows) -> None:
        """fp16 arrays (numpy float16 or uint16 views) w1[F,H], b1[H], w2[H,C], b2[C]."""
        arrs = [np.ascontiguousarray(np.asarray(a, dtype=np.float16)).view(np.uint16) for a in (w1, b1, w2, b2)]
        F, H = arrs[0].shape
        C = arrs[2].shape[1]
        br = np.ascontiguousarray(budget_rows, dtype=np.int32)
        L.check(self._lib.scg_set_model(self.handle, F, H, C, *[_ptr(a) for a in arrs], _ptr(br)), "scg_set_model")
        self._model = (arrs, br)

    def load_model(self, path: str) -> None:
        z = np.load(path, allow_pickle=False)
        self.set_model(z["w1"], z["b1"], z["w2"], z["b2"], z["budget_rows"])

    def close(self) -> None:
        if getattr(self, "handle", None):
            self._lib.scg_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def align(self, pattern: bytes, text: bytes, W: int = 64, O: int = 24, k: int = 64):
        """One pair in host memory (scg_align).  Returns (edits, text_end, cigar)."""
        e, te, ln = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        cap = 2 * (len(pattern) + len(text)) * 11 + 16
        buf = ctypes.create_string_buffer(cap)
        rc = self._lib.scg_align(self.handle, pattern, len(pattern), text, len(text), W, O, k,
                                 ctypes.byref(e), ctypes.byref(te), buf, cap, ctypes.byref(ln))
        L.check(rc, "scg_align")
        return e.value, te.value, buf.value.decode()


@dataclasses.dataclass
class Result:
    edits: object
    text_end: object
    status: object
    runs: object
    n_runs: object
    runs_off: np.ndarray

    def to_host(self) -> "Result":
        def h(x):
            return x.cpu().numpy() if hasattr(x, "cpu") else x
        return Result(h(self.edits), h(self.text_end), h(self.status), h(self.runs), h(self.n_runs), self.runs_off)

    def run_words(self, i: int) -> np.ndarray:
        r = self.to_host() if hasattr(self.runs, "cpu") else self
        s = int(r.runs_off[i])
        return np.asarray(r.runs[s:s + int(r.n_runs[i])], dtype=np.uint32)

    def ops(self, i: int) -> np.ndarray:
        """Expanded op list (0..3) of pair i."""
        w = self.run_words(i)
        return np.repeat((w & 3).astype(np.uint8), (w >> 2).astype(np.int64))

    def cigar(self, i: int) -> str:
        return "".join(f"{int(x) >> 2}{OP_CHARS[int(x) & 3]}" for x in self.run_words(i))


class Batch:
    """A prepared batch (scg_batch_create) and its output buffers."""

    def __init__(self, ctx: Context, batch, prm: L.Params | None = None, device_input: bool = True, stream=None,
                 packed: bool = False):
        import torch
        self.ctx = ctx
        self._lib = ctx._lib
        self.prm = prm if prm is not None else params()
        self.npairs = int(len(batch.pat_off) - 1)
        self.dev = torch.device(f"cuda:{ctx.device}")
        pat_off = np.ascontiguousarray(batch.pat_off, dtype=np.int64)
        txt_off = np.ascontiguousarray(batch.txt_off, dtype=np.int64)
        self._keep = [pat_off, txt_off]
        pat_in, txt_in = batch.pat, batch.txt
        if packed:
            pat_in, txt_in = pack2(batch.pat, pat_off), pack2(batch.txt, txt_off)
        if device_input:
            pat = torch.from_numpy(np.ascontiguousarray(pat_in)).to(self.dev)
            txt = torch.from_numpy(np.ascontiguousarray(txt_in)).to(self.dev)
            torch.cuda.synchronize(self.dev)
            self._keep += [pat, txt]
            where = L.WHERE_DEVICE
        else:
            pat = np.ascontiguousarray(pat_in)
            txt = np.ascontiguousarray(txt_in)
            self._keep += [pat, txt]
            where = L.WHERE_HOST
        h = ctypes.c_void_p()
        kind = L.INPUT_PACKED2 if packed else L.INPUT_ASCII
        rc = self._lib.scg_batch_create(ctx.handle, ctypes.byref(self.prm), self.npairs, _ptr(pat), _ptr(pat_off),
                                        _ptr(txt), _ptr(txt_off), kind, where, _stream_ptr(stream), ctypes.byref(h))
        L.check(rc, "scg_batch_create")
        self.handle = h
        cap = int(self._lib.scg_batch_runs_capacity(h))
        self.runs_off = np.zeros(self.npairs + 1, np.int64)
        L.check(self._lib.scg_batch_runs_offsets(h, _ptr(self.runs_off)), "scg_batch_runs_offsets")
        n = max(self.npairs, 1)
        self.edits = torch.empty(n, dtype=torch.int32, device=self.dev)
        self.text_end = torch.empty(n, dtype=torch.int32, device=self.dev)
        self.status = torch.empty(n, dtype=torch.int32, device=self.dev)
        self.n_runs = torch.empty(n, dtype=torch.int32, device=self.dev)
        self.runs = torch.empty(max(cap, 1), dtype=torch.int32, device=self.dev)

    def run(self, stream=None) -> None:
        rc = self._lib.scg_batch_run(self.handle, _stream_ptr(stream), _ptr(self.edits), _ptr(self.text_end),
                                     _ptr(self.status), _ptr(self.runs), _ptr(self.n_runs))
        L.check(rc, "scg_batch_run")

    def launch_shape(self) -> dict:
        out = (ctypes.c_int32 * 10)()
        L.check(self._lib.scg_batch_launch_shape(self.handle, out), "scg_batch_launch_shape")
        kernel = {L.KERNEL_ROWS: "rows", L.KERNEL_COLUMNS: "columns", L.KERNEL_LANES: "lanes", 4: "wide"}[out[0]]
        return {"kernel": kernel, "slots": out[1], "grid": out[2], "lds_bytes": out[3], "one_per_simd": bool(out[4]),
                "entry_bits": out[5], "helper_grid": out[6], "helper_slots": out[7], "helper_lds_bytes": out[8],
                "helper_long_pairs": out[9]}

    def stats(self) -> L.Stats:
        st = L.Stats()
        L.check(self._lib.scg_batch_stats(self.handle, ctypes.byref(st)), "scg_batch_stats")
        return st

    def result(self) -> Result:
        n = self.npairs
        return Result(self.edits[:n], self.text_end[:n], self.status[:n], self.runs.view(-1), self.n_runs[:n],
                      self.runs_off).to_host()

    def features(self, windows: np.ndarray, stream=None):
        """Features (uint16 [nwin, 16]) of windows given as int32 [nwin, 3] (pair, p0, t0)."""
        import torch
        w = torch.from_numpy(np.ascontiguousarray(windows, dtype=np.int32)).to(self.dev)
        out = torch.empty((max(len(windows), 1), L.NFEATURES), dtype=torch.int16, device=self.dev)
        L.check(self._lib.scg_features(self.handle, len(windows), _ptr(w), _ptr(out), _stream_ptr(stream)),
                "scg_features")
        return out[:len(windows)]

    def close(self) -> None:
        if getattr(self, "handle", None):
            self._lib.scg_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def align_batch(ctx: Context, batch, W=64, O=24, k=64, mode="plain", **kw) -> Result:
    """Prepare, run once and return host results (convenience)."""
    import torch
    b = Batch(ctx, batch, params(W=W, O=O, k=k, mode=mode, **kw))
    b.run()
    torch.cuda.synchronize(b.dev)
    res = b.result()
    st = b.stats()
    b.close()
    res.stats = st
    return res


def pack2(seq: np.ndarray, off: np.ndarray) -> np.ndarray:
    """ASCII CSR sequences -> the library's pre-packed input form
    (SCG_INPUT_PACKED2): two bits per base, 32 bases per uint64 (base t in
    bits 2t, 2t+1), every sequence from a word boundary.  Codes A0 C1 G2 T3.
    Input preparation only: the library converts it to its own layout."""
    seq = np.asarray(seq, dtype=np.uint8)
    lens = np.diff(np.asarray(off, dtype=np.int64))
    words = (lens + 31) // 32
    wo = np.zeros(len(lens) + 1, np.int64)
    np.cumsum(words, out=wo[1:])
    lut = np.zeros(256, np.uint64)
    for ch, c in ((b"A", 0), (b"C", 1), (b"G", 2), (b"T", 3)):
        lut[ch[0]] = c
        lut[ch.lower()[0]] = c
    codes = lut[seq]
    # position of every base in the padded word stream
    first = np.repeat(wo[:-1] * 32 - np.asarray(off[:-1], np.int64), lens)
    pos = np.arange(seq.size, dtype=np.int64) + first
    out = np.zeros(max(int(wo[-1]), 1), np.uint64)
    np.bitwise_or.at(out, pos // 32, codes << (2 * (pos % 32)).astype(np.uint64))
    return out[:max(int(wo[-1]), 1)]


@dataclasses.dataclass
class OpsResult:
    """Output of scg_align_batch: per-pair 2-bit operation streams."""
    edits: np.ndarray
    text_end: np.ndarray
    status: np.ndarray
    ops: np.ndarray       # uint8, op t of pair p in byte ops_off[p] + t // 4, bits 2 (t % 4) ..
    ops_off: np.ndarray
    n_ops: np.ndarray

    def ops_of(self, i: int) -> np.ndarray:
        """Expanded op list (0..3) of pair i."""
        n = int(self.n_ops[i])
        b = self.ops[int(self.ops_off[i]):int(self.ops_off[i]) + (n + 3) // 4]
        x = np.stack([(b >> (2 * e)) & 3 for e in range(4)], axis=1).reshape(-1)
        return x[:n].astype(np.uint8)

    def cigar(self, i: int, lib=None) -> str:
        """scg_ops_to_cigar of pair i."""
        lib = lib or L.load()
        n = int(self.n_ops[i])
        b = np.ascontiguousarray(self.ops[int(self.ops_off[i]):int(self.ops_off[i]) + (n + 3) // 4 + 1])
        cap = 11 * n + 16
        buf = ctypes.create_string_buffer(cap)
        ln = ctypes.c_int32()
        L.check(lib.scg_ops_to_cigar(_ptr(b), n, buf, cap, ctypes.byref(ln)), "scg_ops_to_cigar")
        return buf.value.decode()


def ops_offsets(batch) -> np.ndarray:
    """Byte offsets of the per-pair op streams: ceil((m + n) / 4) bytes each."""
    lens = np.diff(np.asarray(batch.pat_off, np.int64)) + np.diff(np.asarray(batch.txt_off, np.int64))
    off = np.zeros(len(lens) + 1, np.int64)
    np.cumsum((lens + 3) // 4, out=off[1:])
    return off


def align_batch_once(ctx: Context, batch, W=64, O=24, k=64, mode="plain", host=True, packed=False,
                     **kw) -> OpsResult:
    """One scg_align_batch call: host arrays in and out (host=True), or device
    tensors in and out (host=False); ASCII or pre-packed input.  Returns host
    results with .stats (scg_last_stats_all)."""
    import torch
    prm = params(W=W, O=O, k=k, mode=mode, **kw)
    n = int(len(batch.pat_off) - 1)
    pat_off = np.ascontiguousarray(batch.pat_off, dtype=np.int64)
    txt_off = np.ascontiguousarray(batch.txt_off, dtype=np.int64)
    ops_off = ops_offsets(batch)
    nbytes = max(int(ops_off[-1]), 1)
    pat_in, txt_in = (pack2(batch.pat, pat_off), pack2(batch.txt, txt_off)) if packed else (batch.pat, batch.txt)
    lib = ctx._lib
    if host:
        pat, txt = np.ascontiguousarray(pat_in), np.ascontiguousarray(txt_in)
        outs = [np.zeros(max(n, 1), np.int32) for _ in range(4)]
        ops = np.zeros(nbytes, np.uint8)
        where = L.WHERE_HOST
    else:
        dev = torch.device(f"cuda:{ctx.device}")
        pat = torch.from_numpy(np.ascontiguousarray(pat_in)).to(dev)
        txt = torch.from_numpy(np.ascontiguousarray(txt_in)).to(dev)
        outs = [torch.zeros(max(n, 1), dtype=torch.int32, device=dev) for _ in range(4)]
        ops = torch.zeros(nbytes, dtype=torch.uint8, device=dev)
        torch.cuda.synchronize(dev)
        where = L.WHERE_DEVICE
    kind = L.INPUT_PACKED2 if packed else L.INPUT_ASCII
    rc = lib.scg_align_batch(ctx.handle, ctypes.byref(prm), n, _ptr(pat), _ptr(pat_off), _ptr(txt), _ptr(txt_off),
                             kind, where, _stream_ptr(None), _ptr(outs[0]), _ptr(outs[1]), _ptr(outs[2]), _ptr(ops),
                             _ptr(ops_off), _ptr(outs[3]))
    L.check(rc, "scg_align_batch")
    st = L.Stats()
    L.check(lib.scg_last_stats_all(ctx.handle, ctypes.byref(st)), "scg_last_stats_all")

    def h(x):
        return x.cpu().numpy() if hasattr(x, "cpu") else x
    res = OpsResult(h(outs[0])[:n], h(outs[1])[:n], h(outs[2])[:n], h(ops), ops_off, h(outs[3])[:n])
    res.stats = st
    return res


def align_batch_noalloc(ctx: Context, batch, W=64, O=24, k=64, stream=None, **kw) -> Result:
    """scg_align_batch_noalloc: device arrays in and out, the library's static
    workspace instead of allocations.  Returns host results."""
    import torch
    prm = params(W=W, O=O, k=k, mode="plain", **kw)
    n = int(len(batch.pat_off) - 1)
    dev = torch.device(f"cuda:{ctx.device}")
    pat_off = np.ascontiguousarray(batch.pat_off, dtype=np.int64)
    txt_off = np.ascontiguousarray(batch.txt_off, dtype=np.int64)
    lens = (pat_off[1:] - pat_off[:-1]) + (txt_off[1:] - txt_off[:-1]) + 1
    runs_off = np.zeros(n + 1, np.int64)
    np.cumsum(lens, out=runs_off[1:])
    pat = torch.from_numpy(np.ascontiguousarray(batch.pat)).to(dev)
    txt = torch.from_numpy(np.ascontiguousarray(batch.txt)).to(dev)
    po = torch.from_numpy(pat_off).to(dev)
    to = torch.from_numpy(txt_off).to(dev)
    outs = [torch.full((max(n, 1),), -9, dtype=torch.int32, device=dev) for _ in range(4)]
    runs = torch.zeros(max(int(runs_off[-1]), 1), dtype=torch.int32, device=dev)
    torch.cuda.synchronize(dev)
    rc = ctx._lib.scg_align_batch_noalloc(ctx.handle, ctypes.byref(prm), n, _ptr(pat), _ptr(po), int(pat_off[-1]),
                                          _ptr(txt), _ptr(to), int(txt_off[-1]), _stream_ptr(stream), _ptr(outs[0]),
                                          _ptr(outs[1]), _ptr(outs[2]), _ptr(runs), _ptr(outs[3]))
    L.check(rc, "scg_align_batch_noalloc")
    torch.cuda.synchronize(dev)
    res = Result(outs[0][:n], outs[1][:n], outs[2][:n], runs, outs[3][:n], runs_off).to_host()
    res.runs = np.asarray(res.runs).view(np.uint32)
    return res
