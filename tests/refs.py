"""Textbook references used by the oracle's pins (pure Python, tiny inputs).

These are independent of both the oracle and the GPU path: plain dynamic
programming over characters, no bitvectors.
"""
from __future__ import annotations


def levenshtein(a: bytes, b: bytes) -> int:
    """Classic Wagner-Fischer edit distance (unit costs)."""
    prev = list(range(len(b) + 1))
    for i in range(1, len(a) + 1):
        cur = [i] + [0] * len(b)
        for j in range(1, len(b) + 1):
            cur[j] = min(prev[j] + 1, cur[j - 1] + 1, prev[j - 1] + (a[i - 1] != b[j - 1]))
        prev = cur
    return prev[-1]


def shw_bruteforce(pattern: bytes, text: bytes) -> int:
    """min over L of levenshtein(pattern, text[0:L]) -- prefix alignment with a
    free text tail, by trying every text prefix."""
    return min(levenshtein(pattern, text[:L]) for L in range(len(text) + 1))


def suffix_dp(pattern: bytes, text: bytes):
    """D[i][j] = min_L edit(text[i:i+L), pattern[j:m)) by the textbook
    recurrence over suffixes: D[i][m] = 0, D[n][j] = m - j."""
    m, n = len(pattern), len(text)
    D = [[0] * (m + 1) for _ in range(n + 1)]
    for j in range(m + 1):
        D[n][j] = m - j
    for i in range(n - 1, -1, -1):
        D[i][m] = 0
        for j in range(m - 1, -1, -1):
            D[i][j] = min(D[i][j + 1] + 1, D[i + 1][j] + 1,
                          D[i + 1][j + 1] + (text[i] != pattern[j]))
    return D


def prefix_distance(pattern: bytes, text: bytes) -> int:
    """min over L of levenshtein(pattern, text[0:L]) for long inputs: the
    Wagner-Fischer rows over the text, one pattern character at a time, with
    the in-row recurrence cur[i] = min(a[i], cur[i-1] + 1) solved as
    i + running-min(a[k] - k) (numpy, O(m n) work, O(n) memory)."""
    import numpy as np
    t = np.frombuffer(text, np.uint8)
    n = len(t)
    idx = np.arange(n + 1, dtype=np.int64)
    prev = idx.copy()                           # pattern prefix of length 0
    for j, c in enumerate(pattern, start=1):
        a = np.empty(n + 1, np.int64)
        a[0] = j
        a[1:] = np.minimum(prev[:-1] + (t != c), prev[1:] + 1)
        prev = idx + np.minimum.accumulate(a - idx)
    return int(prev.min())


def replay(pattern: bytes, text: bytes, ops) -> tuple[int, int]:
    """Walk an op list over the two strings.  Returns (edits, text consumed).
    Raises AssertionError if an op contradicts the strings or the pattern is
    not fully consumed."""
    i = j = edits = 0
    for op in ops:
        op = int(op)
        if op == 0:
            assert i < len(text) and j < len(pattern) and text[i] == pattern[j], ("M", i, j)
            i += 1; j += 1
        elif op == 1:
            assert i < len(text) and j < len(pattern) and text[i] != pattern[j], ("S", i, j)
            i += 1; j += 1; edits += 1
        elif op == 2:
            assert j < len(pattern), ("I", i, j)
            j += 1; edits += 1
        elif op == 3:
            assert i < len(text), ("D", i, j)
            i += 1; edits += 1
        else:
            raise AssertionError(("bad op", op))
    assert j == len(pattern), ("pattern not consumed", j, len(pattern))
    return edits, i


# Traceback priority used throughout: match, then substitution, then a pattern
# character missing from the text (I), then a text character missing from the
# pattern (D).
OP_M, OP_S, OP_I, OP_D = 0, 1, 2, 3


def dp_traceback(pattern: bytes, text: bytes, d: int, cap: int, D=None):
    """GenASM-TB restated on the integer table: from (0, 0) at distance d,
    take the first available of M, S, I, D, where an edge is available when it
    reaches a cell whose suffix distance is within the remaining budget
    (Theorem 1: a 0 at bit j of R[i][e] means D(i, j) <= e).  Stops once cap
    characters of either sequence are consumed or the pattern is used up.
    Returns (ops, text consumed, pattern consumed, I/D ties met)."""
    if D is None:
        D = suffix_dp(pattern, text)
    m, n = len(pattern), len(text)
    i = j = ties = 0
    ops = []
    while j < m and i < cap and j < cap:
        has_t = i < n
        if has_t and text[i] == pattern[j] and D[i + 1][j + 1] <= d:
            op = OP_M
        else:
            s_ok = has_t and d > 0 and D[i + 1][j + 1] <= d - 1
            i_ok = d > 0 and D[i][j + 1] <= d - 1
            d_ok = has_t and d > 0 and D[i + 1][j] <= d - 1
            ties += int(not s_ok and i_ok and d_ok)
            if s_ok:
                op = OP_S
            elif i_ok:
                op = OP_I
            elif d_ok:
                op = OP_D
            else:
                raise AssertionError(("no edge", i, j, d))
        ops.append(op)
        i += op != OP_I
        j += op != OP_D
        d -= op != OP_M
    return ops, i, j, ties


def windowed_dp_align(pattern: bytes, text: bytes, W: int, O: int, k: int):
    """The windowing of the method with the integer-table traceback above:
    window at (p0, t0) over at most W characters of each sequence, budget
    min(k, m_w), advance by what the traceback consumed.  Returns (status,
    edits, text_end, ops, I/D ties met); status 1 = some window's distance
    exceeds its budget."""
    m, n = len(pattern), len(text)
    p0 = t0 = ties = 0
    ops = []
    while p0 < m:
        pw, tw = pattern[p0:p0 + W], text[t0:t0 + W]
        D = suffix_dp(pw, tw)
        if D[0][0] > min(k, len(pw)):
            return 1, -1, -1, [], ties
        wops, di, dj, t = dp_traceback(pw, tw, D[0][0], W - O, D)
        ops += wops
        ties += t
        p0 += dj
        t0 += di
    return 0, sum(op != OP_M for op in ops), t0, ops, ties
