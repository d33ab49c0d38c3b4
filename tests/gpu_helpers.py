"""Helpers for GPU-vs-oracle parity tests."""
from __future__ import annotations

import sys

import numpy as np


def log(msg: str) -> None:
    print(msg, flush=True)
    sys.stdout.flush()


def _gather(data: np.ndarray, starts: np.ndarray, counts: np.ndarray) -> np.ndarray:
    """Concatenation of data[starts[i] : starts[i] + counts[i]] over i."""
    counts = np.asarray(counts, dtype=np.int64)
    total = int(counts.sum())
    if total == 0:
        return data[:0]
    first = np.zeros(len(counts), np.int64)
    np.cumsum(counts[:-1], out=first[1:])
    idx = np.arange(total, dtype=np.int64) - np.repeat(first - np.asarray(starts, np.int64), counts)
    return data[idx]


def expand_runs(res, npairs):
    """GPU run words -> (ops concatenated, per-pair op offsets, run words concatenated, per-pair run counts)."""
    runs = np.asarray(res.runs).view(np.uint32) if np.asarray(res.runs).dtype.itemsize == 4 else \
        np.asarray(res.runs).astype(np.uint32)
    n_runs = np.asarray(res.n_runs)[:npairs].astype(np.int64)
    words = _gather(runs, np.asarray(res.runs_off)[:npairs], n_runs)
    lens = (words >> 2).astype(np.int64)
    ops = np.repeat((words & 3).astype(np.uint8), lens)
    per_pair = np.zeros(npairs, np.int64)
    if npairs:
        nz = n_runs > 0
        first = np.zeros(npairs, np.int64)
        np.cumsum(n_runs[:-1], out=first[1:])
        sums = np.add.reduceat(lens, first[nz]) if lens.size else np.zeros(0, np.int64)
        per_pair[nz] = sums
    offs = np.zeros(npairs + 1, np.int64)
    np.cumsum(per_pair, out=offs[1:])
    return ops, offs, words, n_runs


def compare(batch, gpu, ref, what=""):
    """Bit-exact comparison of GPU results with oracle results: status,
    edits, text_end and the complete operation sequence of every pair
    (vectorised over the whole batch), and run words that are maximal."""
    n = batch.npairs
    st_ref = np.where(ref["status"] == 0, 0, 1)
    assert np.array_equal(np.asarray(gpu.status)[:n], st_ref), (
        f"{what}: status differs at {np.flatnonzero(np.asarray(gpu.status)[:n] != st_ref)[:10]}")
    assert np.array_equal(np.asarray(gpu.edits)[:n], ref["edits"]), (
        f"{what}: edits differ at {np.flatnonzero(np.asarray(gpu.edits)[:n] != ref['edits'])[:10]}")
    assert np.array_equal(np.asarray(gpu.text_end)[:n], ref["text_end"]), (
        f"{what}: text_end differs at {np.flatnonzero(np.asarray(gpu.text_end)[:n] != ref['text_end'])[:10]}")
    if hasattr(gpu, "n_ops"):   # a 2-bit operation stream (scg_align_batch)
        counts = np.asarray(gpu.n_ops)[:n].astype(np.int64)
        packed = np.asarray(gpu.ops, np.uint8)
        unpacked = np.stack([(packed >> (2 * e)) & 3 for e in range(4)], axis=1).reshape(-1).astype(np.uint8)
        ops = _gather(unpacked, 4 * np.asarray(gpu.ops_off)[:n], counts)
        offs = np.zeros(n + 1, np.int64)
        np.cumsum(counts, out=offs[1:])
        words = n_runs = None
    else:
        ops, offs, words, n_runs = expand_runs(gpu, n)
    ref_counts = np.asarray(ref["n_ops"])[:n].astype(np.int64)
    gpu_counts = np.diff(offs)
    bad = np.flatnonzero(gpu_counts != ref_counts)
    assert bad.size == 0, f"{what}: op count differs at pairs {bad[:10]} ({gpu_counts[bad[:3]]} vs {ref_counts[bad[:3]]})"
    ref_ops = _gather(ref["ops"], np.asarray(ref["ops_off"])[:n], ref_counts)
    if not np.array_equal(ops, ref_ops):
        at = int(np.argmax(ops != ref_ops))
        pair = int(np.searchsorted(offs, at, side="right") - 1)
        raise AssertionError(f"{what}: op stream of pair {pair} differs (first at op {at - int(offs[pair])})")
    if words is None:
        return
    # runs are maximal: no empty run and no two consecutive words of a pair with the same op
    assert np.all((words >> 2) > 0), f"{what}: empty run"
    if words.size > 1:
        same = np.diff((words & 3).astype(np.int8)) == 0
        first = np.zeros(n, np.int64)
        if n:
            np.cumsum(n_runs[:-1], out=first[1:])
        boundary = np.zeros(words.size, bool)
        boundary[first[(n_runs > 0) & (first > 0)]] = True
        assert not np.any(same & ~boundary[1:]), f"{what}: unmerged runs"
