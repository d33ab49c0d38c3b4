"""Pins for the CPU oracle, against what the paper and the mathematics fix.

Each test names the passage it follows.  None of them compares the oracle with
itself: the references are textbook dynamic programming on characters
(tests/refs.py), brute force over text prefixes, printed values, or
properties the paper states.
"""
import json
import os

import numpy as np
import pytest

import oracle
from paper_2208_09985_amd import synth
from tests import refs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
RNG = np.random.default_rng(12345)


def pbit(v, j, m):
    """paper bit j (j = 0 is the msb) of an m-bit vector; bit m reads 0."""
    return 0 if j >= m else (int(v) >> (m - 1 - j)) & 1


def rand_seq(rng, n):
    return synth.ALPHABET[rng.integers(0, 4, n)].tobytes()


def mutate(rng, s: bytes, rate: float) -> bytes:
    out = bytearray()
    for c in s:
        r = rng.random()
        if r < rate / 3:
            out.append(b"ACGT"[(b"ACGT".index(c) + rng.integers(1, 4)) % 4])
        elif r < 2 * rate / 3:
            out.append(c)
            out.append(b"ACGT"[rng.integers(0, 4)])
        elif r < rate:
            continue
        else:
            out.append(c)
    return bytes(out)


# --- Section 2.2.1, Fig. 1: the printed worked example -------------------------------------

def test_worked_example_fig1():
    g = json.load(open(os.path.join(GOLDEN, "fig1_worked_example.json")))
    text, pattern, k = g["text"].encode(), g["pattern"].encode(), g["k"]
    R, d = oracle.dc_table(pattern, text, k)
    z = g["zero_at"]
    assert pbit(R[z["i"], z["d"]], z["j"], len(pattern)) == 0
    # the same bit one row up (d = 0) must be 1: no exact match of "GT" vs "GA"
    assert pbit(R[z["i"], z["d"] - 1], z["j"], len(pattern)) == 1
    assert d == g["edit_distance"]
    PM = oracle.pattern_masks(pattern)
    for x, want in g["pattern_masks_j0_first"].items():
        got = "".join(str(pbit(PM["ACGT".index(x)], j, len(pattern))) for j in range(len(pattern)))
        assert got == want, (x, got, want)


# --- Theorem 1: every bit of every entry ---------------------------------------------------

def _check_theorem1(pattern, text, k, wide=False):
    m, n = len(pattern), len(text)
    R, d = (oracle.dc_table_wide if wide else oracle.dc_table)(pattern, text, k)
    D = refs.suffix_dp(pattern, text)
    for i in range(n + 1):
        for dd in range(k + 1):
            for j in range(m):
                want = 1 if D[i][j] > dd else 0
                assert pbit(R[i, dd], j, m) == want, (pattern, text, i, j, dd)
    expect = D[0][0] if D[0][0] <= k else -1
    assert d == expect


def test_suffix_dp_is_prefix_alignment_with_free_text_tail():
    # The distance of Theorem 1 under Algorithm 1's init and zero shift-in:
    # pattern suffix fully consumed, text tail free.  Pin the textbook
    # recurrence used below against brute force over every text prefix.
    rng = np.random.default_rng(7)
    for _ in range(150):
        m, n = int(rng.integers(0, 7)), int(rng.integers(0, 8))
        p, t = rand_seq(rng, m), rand_seq(rng, n)
        D = refs.suffix_dp(p, t)
        for i in range(n + 1):
            for j in range(m + 1):
                assert D[i][j] == refs.shw_bruteforce(p[j:], t[i:]), (p, t, i, j)


def test_theorem1_small_windows():
    rng = np.random.default_rng(1)
    for _ in range(300):
        m, n = int(rng.integers(1, 13)), int(rng.integers(0, 14))
        p = rand_seq(rng, m)
        t = mutate(rng, p, 0.3)[:n] if rng.random() < 0.5 else rand_seq(rng, n)
        _check_theorem1(p, t, int(rng.integers(0, m + 1)))


def test_theorem1_full_width_windows():
    # 64-bit vectors (m = 64): the widest window, every bit position used.
    rng = np.random.default_rng(2)
    for rate in (0.0, 0.05, 0.15, 0.5):
        p = rand_seq(rng, 64)
        t = mutate(rng, p + rand_seq(rng, 8), rate)[:64]
        _check_theorem1(p, t, 64)
    _check_theorem1(rand_seq(rng, 64), rand_seq(rng, 64), 64)


def test_theorem1_windows_wider_than_64():
    # the 128-bit instantiation: windows of 65..128 characters, every bit
    rng = np.random.default_rng(21)
    for m, n, rate in ((65, 70, 0.1), (96, 96, 0.15), (128, 128, 0.05), (128, 128, 0.3), (100, 0, 0.0)):
        p = rand_seq(rng, m)
        t = mutate(rng, p + rand_seq(rng, 16), rate)[:n]
        _check_theorem1(p, t, min(m, 40), wide=True)


def test_wide_instantiation_agrees_with_64_bit_one():
    # windows of up to 64 characters give the same table in both widths
    rng = np.random.default_rng(22)
    for _ in range(40):
        m, n = int(rng.integers(1, 65)), int(rng.integers(0, 65))
        p, t = rand_seq(rng, m), mutate(rng, rand_seq(rng, n), 0.2)[:n]
        k = int(rng.integers(0, m + 1))
        R64, d64 = oracle.dc_table(p, t, k)
        R128, d128 = oracle.dc_table_wide(p, t, k)
        assert d64 == d128
        assert all(int(R64.flat[x]) == R128.flat[x] for x in range(R64.size))


# --- Section 2.2.3: a single window with no overlap is the exact optimum ---------------------

def test_single_window_o0_equals_bruteforce_optimum():
    rng = np.random.default_rng(3)
    for W in (4, 8, 16):
        for _ in range(80):
            m, n = int(rng.integers(1, W + 1)), int(rng.integers(0, W + 1))
            p = rand_seq(rng, m)
            t = mutate(rng, p, 0.3)[:n] if rng.random() < 0.6 else rand_seq(rng, n)
            r = oracle.align_pair(p, t, W, 0, W)
            assert r["status"] == 0
            assert r["edits"] == refs.shw_bruteforce(p, t), (W, p, t)
            e, used = refs.replay(p, t, r["ops"])
            assert (e, used) == (r["edits"], r["text_end"])


def test_single_wide_window_o0_equals_optimum():
    rng = np.random.default_rng(23)
    for W in (65, 96, 128):
        for _ in range(12):
            m, n = int(rng.integers(1, W + 1)), int(rng.integers(0, W + 1))
            p = rand_seq(rng, m)
            t = mutate(rng, p, 0.2)[:n] if rng.random() < 0.7 else rand_seq(rng, n)
            r = oracle.align_pair(p, t, W, 0, W)
            assert r["status"] == 0
            assert r["edits"] == refs.suffix_dp(p, t)[0][0], (W, p, t)
            e, used = refs.replay(p, t, r["ops"])
            assert (e, used) == (r["edits"], r["text_end"])


# --- CIGAR replay and optimality bound on windowed pairs ----------------------------------

def _replay_all(batch, res):
    for i in range(batch.npairs):
        p, t = batch.pattern(i), batch.text(i)
        assert res["status"][i] == 0
        e, used = refs.replay(p, t, oracle.ops_of(res, i))
        assert e == res["edits"][i], i
        assert used == res["text_end"][i], i


def test_replay_small_workload():
    b = synth.make_batch("small_100bp")
    res = oracle.align_batch(b, 64, 24, 64)
    _replay_all(b, res)


def test_replay_long_sample():
    b = synth.make_batch("long_10kbp", indices=[0, 17, 999, 4242])
    res = oracle.align_batch(b, 64, 24, 64)
    _replay_all(b, res)


def test_windowed_edits_bounded_below_by_optimum():
    rng = np.random.default_rng(4)
    for W, O in ((64, 24), (16, 9), (8, 3), (128, 24), (96, 33)):
        for _ in range(25):
            p = rand_seq(rng, int(rng.integers(1, 90)))
            t = mutate(rng, p, 0.15)
            r = oracle.align_pair(p, t, W, O, W)
            D = refs.suffix_dp(p, t)
            assert r["edits"] >= D[0][0]
            refs.replay(p, t, r["ops"])


# --- Traceback is tight: each window spends exactly d_w - D(stop) ---------------------------

def test_traceback_is_tight_per_window():
    rng = np.random.default_rng(5)
    W, O = 16, 6
    for _ in range(60):
        p = rand_seq(rng, int(rng.integers(10, 60)))
        t = mutate(rng, p, 0.2)
        r = oracle.align_pair(p, t, W, O, W, want_windows=True)
        for w in r["windows"]:
            pw = p[w["p0"]:w["p0"] + w["m_w"]]
            tw = t[w["t0"]:w["t0"] + w["n_w"]]
            D = refs.suffix_dp(pw, tw)
            assert w["d_w"] == D[0][0]
            assert w["edits"] == w["d_w"] - D[w["adv_t"]][w["adv_p"]]


def test_match_edge_available_whenever_characters_agree():
    # Diagonal monotonicity: on a tight state (D(i,j) = d) with text[i] ==
    # pattern[j], the M term always has its 0 (bit j+1 of R[i+1][d] is 0).
    rng = np.random.default_rng(6)
    for _ in range(120):
        m, n = int(rng.integers(1, 12)), int(rng.integers(1, 13))
        p = rand_seq(rng, m)
        t = mutate(rng, p, 0.3)[:n] if rng.random() < 0.5 else rand_seq(rng, n)
        n = len(t)
        R, _ = oracle.dc_table(p, t, m)
        D = refs.suffix_dp(p, t)
        for i in range(n):
            for j in range(m):
                if t[i] == p[j] and D[i][j] <= m:
                    assert pbit(R[i + 1, D[i][j]], j + 1, m) == 0


# --- Supplementary 8.2: the work of one full W = 64 window -----------------------------------

def test_full_window_op_count_28865():
    p = rand_seq(np.random.default_rng(8), 64)
    r = oracle.align_pair(p, p, 64, 0, 64)   # one window, all matches
    st = r["stats"]
    assert st.windows == 1
    assert st.ops_genasm == 28865
    assert st.ops_alg == 1 + 2 * 64          # d_w = 0: right column + top row


# --- Sections 2.4.2 / 2.4.3 and supplementary S1: what traceback reads ---------------------

@pytest.mark.parametrize("W,O", [(4, 3), (64, 24), (64, 33), (32, 17), (128, 24), (96, 40)])
def test_traceback_reads_stay_in_dent_region(W, O):
    rng = np.random.default_rng(9)
    st_all = []
    for _ in range(40):
        p = rand_seq(rng, int(rng.integers(1, 4 * W)))
        t = mutate(rng, p, 0.25) if rng.random() < 0.7 else rand_seq(rng, int(rng.integers(0, 4 * W)))
        st_all.append(oracle.align_pair(p, t, W, O, W)["stats"])
    # DENT: only the first W-O+1 columns and bits are ever read
    assert max(s.max_col_read for s in st_all) <= W - O
    assert max(s.max_bit_read for s in st_all) <= W - O
    # ET: traceback never reads a row beyond d_w (it never goes south)
    assert max(s.max_row_above_dw for s in st_all) == 0
    # extended DENT (S1): at most W-O rows below d_w are read
    assert max(s.max_rows_below_dw for s in st_all) <= W - O


# --- Supplementary S10 (Lemma S1) and the ET claim of Section 2.4.3 --------------------------

def test_random_window_distance_bound_and_et_savings():
    rng = np.random.default_rng(10)
    ds = []
    for _ in range(300):
        p, t = rand_seq(rng, 64), rand_seq(rng, 64)
        _, d = oracle.dc_table(p, t, 64)
        ds.append(d)
    mean_d = float(np.mean(ds))
    assert mean_d <= 3 * 64 / 4                    # Lemma S1
    assert 1.0 - (mean_d + 1) / 65 >= 0.25         # rows skippable by ET


# --- edge cases -----------------------------------------------------------------------------

def test_edge_cases():
    r = oracle.align_pair(b"", b"ACGT", 64, 24, 64)
    assert (r["status"], r["edits"], r["text_end"], len(r["ops"])) == (0, 0, 0, 0)
    r = oracle.align_pair(b"ACGTACGT", b"", 64, 24, 64)
    assert (r["status"], r["edits"], r["text_end"]) == (0, 8, 0)
    assert set(r["ops"].tolist()) == {oracle.OP_I}
    r = oracle.align_pair(b"AAAAAAAA", b"CCCCCCCC", 64, 24, 2)
    assert r["status"] == oracle.NOT_ALIGNED and r["edits"] == -1
    r = oracle.align_pair(b"acgt", b"ACGT", 64, 24, 64)
    assert r["edits"] == 0
    with pytest.raises(ValueError):
        oracle.align_pair(b"ACNT", b"ACGT", 64, 24, 64)
    with pytest.raises(ValueError):
        oracle.align_pair(b"ACGT", b"ACGT", 64, 64, 64)
    # long text tail is free
    r = oracle.align_pair(b"ACGTACGTAC", b"ACGTACGTAC" + b"G" * 200, 64, 24, 64)
    assert (r["edits"], r["text_end"]) == (0, 10)


# --- Section 2.2.2: the traceback's edge order, restated on the integer table ---------------

@pytest.mark.parametrize("W,O,length", [(8, 3, 60), (16, 5, 120), (64, 24, 260), (128, 40, 300)])
def test_traceback_order_matches_integer_table_traceback(W, O, length):
    """Windowed alignment with an independent traceback over the textbook
    suffix-distance table (tests/refs.py) gives the oracle's exact op stream.
    The table traceback takes M, S, I, D in that order, so a swap of any two
    edges in the oracle changes the path at the first tie; the test checks
    that ties between I and D (the ones a tight path can meet) occur."""
    rng = np.random.default_rng(W * 7 + O)
    ties = 0
    for case in range(24):
        p = rand_seq(rng, int(rng.integers(length // 2, length)))
        t = mutate(rng, p, 0.2) if case % 6 else rand_seq(rng, int(rng.integers(length // 2, length)))
        st, e, te, ops, tie = refs.windowed_dp_align(p, t, W, O, W)
        ties += tie
        r = oracle.align_pair(p, t, W, O, W)
        assert r["status"] == st == 0
        assert (r["edits"], r["text_end"]) == (e, te), case
        assert r["ops"].tolist() == ops, case
    assert ties > 0
