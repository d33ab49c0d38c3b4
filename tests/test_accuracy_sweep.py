"""Accuracy of the windowing heuristic (Section 2.2.3) against the exact
optimum, on pairs of the 10 kbp, 15%-edit workload (CPU only).

The windows align the whole pattern to a text prefix greedily, so a pair's
windowed edit count can never fall below min over L of edit(pattern,
text[0:L]); the test checks that bound for every pair and window geometry and
prints the mean ratio per geometry (``pytest -s`` shows the table;
SCG_ACCURACY_PAIRS sets how many pairs, 6 by default)."""
import os

import numpy as np
import pytest

import oracle
from paper_2208_09985_amd import synth
from tests import refs

GEOMETRIES = ((64, 24), (64, 33), (64, 16), (64, 40), (32, 8), (96, 32), (128, 24), (128, 64))
PAIRS = range(int(os.environ.get("SCG_ACCURACY_PAIRS", "6")))


def test_prefix_distance_matches_bruteforce():
    rng = np.random.default_rng(11)
    for _ in range(300):
        m, n = int(rng.integers(0, 9)), int(rng.integers(0, 10))
        p = bytes(rng.choice(list(b"ACGT"), m))
        t = bytes(rng.choice(list(b"ACGT"), n))
        assert refs.prefix_distance(p, t) == refs.shw_bruteforce(p, t), (p, t)


@pytest.fixture(scope="module")
def exact():
    b = synth.make_batch("long_10kbp", indices=list(PAIRS))
    return b, [refs.prefix_distance(b.pattern(i), b.text(i)) for i in range(b.npairs)]


def test_windowed_edits_against_exact_optimum(exact):
    b, opt = exact
    rows = []
    for W, O in GEOMETRIES:
        res = oracle.align_batch(b, W, O, W)
        assert np.all(res["status"] == 0)
        ed = res["edits"].astype(np.int64)
        assert np.all(ed >= np.asarray(opt)), (W, O)
        r = ed / np.asarray(opt)
        rows.append((W, O, float(ed.mean()), float(r.mean()), float(np.median(r)), float(r.max())))
    print(f"\nwindowed edits vs exact optimum, long_10kbp pairs 0..{len(PAIRS) - 1}: exact mean {np.mean(opt):.1f}")
    for W, O, mean_ed, ratio, med, worst in rows:
        print(f"  W={W:2d} O={O:2d}: windowed mean {mean_ed:7.1f}; ratio mean {ratio:.3f}, median {med:.3f}, max {worst:.3f}")
