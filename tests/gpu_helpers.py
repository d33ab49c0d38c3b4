"""Helpers for GPU-vs-oracle parity tests."""
from __future__ import annotations

import sys

import numpy as np

import oracle


def log(msg: str) -> None:
    print(msg, flush=True)
    sys.stdout.flush()


def expand_runs(res, npairs):
    """GPU run words -> (ops concatenated, per-pair op offsets)."""
    runs = np.asarray(res.runs).astype(np.uint32)
    lens, offs = [], [0]
    chunks = []
    for i in range(npairs):
        s = int(res.runs_off[i])
        w = runs[s:s + int(res.n_runs[i])]
        ops = np.repeat((w & 3).astype(np.uint8), (w >> 2).astype(np.int64))
        chunks.append(ops)
        offs.append(offs[-1] + ops.size)
    return (np.concatenate(chunks) if chunks else np.zeros(0, np.uint8)), np.asarray(offs)


def compare(batch, gpu, ref, what=""):
    """Bit-exact comparison of GPU results with oracle results: status,
    edits, text_end and the complete operation sequence of every pair."""
    n = batch.npairs
    st_ref = np.where(ref["status"] == 0, 0, 1)
    assert np.array_equal(np.asarray(gpu.status)[:n], st_ref), f"{what}: status differs"
    assert np.array_equal(np.asarray(gpu.edits)[:n], ref["edits"]), (
        f"{what}: edits differ at {np.flatnonzero(np.asarray(gpu.edits)[:n] != ref['edits'])[:10]}")
    assert np.array_equal(np.asarray(gpu.text_end)[:n], ref["text_end"]), f"{what}: text_end differs"
    ops, offs = expand_runs(gpu, n)
    for i in range(n):
        g = ops[offs[i]:offs[i + 1]]
        o = oracle.ops_of(ref, i)
        if not np.array_equal(g, o):
            k = int(np.argmax(g[:min(len(g), len(o))] != o[:min(len(g), len(o))])) if min(len(g), len(o)) else 0
            raise AssertionError(f"{what}: op stream of pair {i} differs (len {len(g)} vs {len(o)}, first at {k})")
    # runs are maximal: no two consecutive words with the same op
    runs = np.asarray(gpu.runs).astype(np.uint32)
    for i in range(n):
        s = int(gpu.runs_off[i])
        w = runs[s:s + int(gpu.n_runs[i])]
        assert np.all((w >> 2) > 0), f"{what}: empty run in pair {i}"
        assert np.all(np.diff((w & 3).astype(np.int8)) != 0), f"{what}: unmerged runs in pair {i}"
