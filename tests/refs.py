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
