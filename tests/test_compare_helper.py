"""The GPU-vs-oracle comparator itself, on the CPU: oracle results rewritten
as run words must compare equal, and any planted difference (an op, a run
split in two, an edit count, a status) must be caught."""
import types

import numpy as np
import pytest

import oracle
from paper_2208_09985_amd import synth
from tests.gpu_helpers import compare


def as_runs(ref, n):
    """Oracle op lists -> a GPU-like result of merged run words."""
    lens = np.diff(np.asarray(ref["ops_off"]))[:n] + 1
    runs_off = np.zeros(n + 1, np.int64)
    np.cumsum(lens, out=runs_off[1:])
    runs = np.zeros(int(runs_off[-1]) + 1, np.uint32)
    n_runs = np.zeros(n, np.int32)
    for i in range(n):
        ops = oracle.ops_of(ref, i)
        k = 0
        j = 0
        while j < len(ops):
            e = j
            while e < len(ops) and ops[e] == ops[j]:
                e += 1
            runs[runs_off[i] + k] = ((e - j) << 2) | int(ops[j])
            k += 1
            j = e
        n_runs[i] = k
    st = np.where(ref["status"] == 0, 0, 1).astype(np.int32)
    return types.SimpleNamespace(status=st, edits=ref["edits"].copy(), text_end=ref["text_end"].copy(),
                                 runs=runs, n_runs=n_runs, runs_off=runs_off)


@pytest.fixture(scope="module")
def case():
    b = synth.make_batch("small_100bp", 60)
    pats = [b.pattern(i) for i in range(b.npairs)] + [b"", b"ACGT"]
    txts = [b.text(i) for i in range(b.npairs)] + [b"ACG", b""]
    b = synth.from_lists(pats, txts)
    ref = oracle.align_batch(b, 64, 24, 64)
    return b, ref


def test_identical_results_compare_equal(case):
    b, ref = case
    compare(b, as_runs(ref, b.npairs), ref, "self")


def test_planted_differences_are_caught(case):
    b, ref = case
    g = as_runs(ref, b.npairs)
    w = g.runs[g.runs_off[5]]
    g.runs[g.runs_off[5]] = (w & ~np.uint32(3)) | ((w + 1) & 3)   # another op in one run
    with pytest.raises(AssertionError):
        compare(b, g, ref, "op")
    g = as_runs(ref, b.npairs)
    g.edits[7] += 1
    with pytest.raises(AssertionError):
        compare(b, g, ref, "edits")
    g = as_runs(ref, b.npairs)
    g.status[3] = 1
    with pytest.raises(AssertionError):
        compare(b, g, ref, "status")
    g = as_runs(ref, b.npairs)
    # split the first run of pair 9 in two (same ops, runs no longer maximal)
    i = 9
    s, k = int(g.runs_off[i]), int(g.n_runs[i])
    w = int(g.runs[s])
    assert (w >> 2) >= 2
    g.runs[s + 1:s + k + 1] = g.runs[s:s + k].copy()
    g.runs[s] = (1 << 2) | (w & 3)
    g.runs[s + 1] = (((w >> 2) - 1) << 2) | (w & 3)
    g.n_runs[i] = k + 1
    with pytest.raises(AssertionError):
        compare(b, g, ref, "split")
    g = as_runs(ref, b.npairs)
    g.n_runs[11] -= 1   # a run dropped
    with pytest.raises(AssertionError):
        compare(b, g, ref, "dropped")
