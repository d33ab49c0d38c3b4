"""Seeded synthetic read-pair generator.

This module produces inputs only: random patterns and the texts derived from
them by random substitutions, insertions and deletions.  It holds none of the
alignment arithmetic, so both the GPU path and the CPU oracle may use it.

Every pair is drawn from its own counter-based stream
``PCG64(SeedSequence([seed, pair_index]))``, so any subset of a workload (the
first N pairs, a random sample of pair indices) is reproduced exactly without
generating the rest.

Workloads (pattern = read, text = the same read with edits applied):

=====================  ========  =======================================  ==========  ==================
name                   pairs     pattern length                           edit rate   sub / ins / del
=====================  ========  =======================================  ==========  ==================
``small_100bp``        1,000     100                                      5 %         1/3 each, length 1
``short_250bp``        100,000   250                                      2 %         0.8 / 0.1 / 0.1
``long_10kbp``         10,000    10,000                                   15 %        0.2 / 0.4 / 0.4, geometric indels (mean 1.5)
``uneven_lognormal``   50,000    log-normal, median 5,000, sigma 1.0,     U(5,15) %   as ``long_10kbp``
                                 clipped to [1,000, 50,000]
``mixed_10kbp``        10,000    10,000                                   U(5,15) %   as ``long_10kbp``
``train_10kbp``        1,000     10,000                                   U(5,15) %   as ``long_10kbp`` (disjoint seed)
=====================  ========  =======================================  ==========  ==================

Edit model: the number of edited bases is E = round(rate * m).  Events are
drawn (type by the mix; substitutions have length 1, indels length 1 or
Geometric(2/3)) until their lengths sum to E, the last one truncated.  Event
positions are uniform in [0, m).  A substitution picks one of the three other
bases uniformly, an insertion adds uniform random bases before the position,
a deletion removes bases starting at the position.
"""
from __future__ import annotations

import dataclasses
import numpy as np

ALPHABET = np.frombuffer(b"ACGT", dtype=np.uint8)


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    npairs: int
    seed: int
    length: tuple          # ("fixed", m) | ("lognormal", median, sigma, lo, hi)
    rate: tuple            # ("fixed", r) | ("uniform", lo, hi)
    mix: tuple             # probabilities of (substitution, insertion, deletion)
    geometric_indels: bool
    W: int = 64
    O: int = 24
    k: int = 64


WORKLOADS = {
    w.name: w
    for w in [
        Workload("small_100bp", 1000, 1001, ("fixed", 100), ("fixed", 0.05), (1 / 3, 1 / 3, 1 / 3), False),
        Workload("short_250bp", 100000, 1002, ("fixed", 250), ("fixed", 0.02), (0.8, 0.1, 0.1), False),
        Workload("long_10kbp", 10000, 1003, ("fixed", 10000), ("fixed", 0.15), (0.2, 0.4, 0.4), True),
        Workload("uneven_lognormal", 50000, 1004, ("lognormal", 5000, 1.0, 1000, 50000), ("uniform", 0.05, 0.15),
                 (0.2, 0.4, 0.4), True),
        Workload("mixed_10kbp", 10000, 1005, ("fixed", 10000), ("uniform", 0.05, 0.15), (0.2, 0.4, 0.4), True),
        Workload("train_10kbp", 1000, 2005, ("fixed", 10000), ("uniform", 0.05, 0.15), (0.2, 0.4, 0.4), True),
    ]
}


@dataclasses.dataclass
class PairBatch:
    """Sequences in CSR form: ASCII bytes plus int64 offsets (npairs + 1)."""
    pat: np.ndarray
    pat_off: np.ndarray
    txt: np.ndarray
    txt_off: np.ndarray

    @property
    def npairs(self) -> int:
        return len(self.pat_off) - 1

    def pattern(self, i: int) -> bytes:
        return self.pat[self.pat_off[i]:self.pat_off[i + 1]].tobytes()

    def text(self, i: int) -> bytes:
        return self.txt[self.txt_off[i]:self.txt_off[i + 1]].tobytes()

    def subset(self, idx) -> "PairBatch":
        return from_lists([self.pattern(i) for i in idx], [self.text(i) for i in idx])


def _pair_rng(seed: int, index: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, index])))


def _draw_length(rng, spec) -> int:
    if spec[0] == "fixed":
        return int(spec[1])
    if spec[0] == "lognormal":
        _, median, sigma, lo, hi = spec
        v = rng.lognormal(np.log(median), sigma)
        return int(min(max(round(v), lo), hi))
    raise ValueError(spec)


def _draw_rate(rng, spec) -> float:
    if spec[0] == "fixed":
        return float(spec[1])
    if spec[0] == "uniform":
        return float(rng.uniform(spec[1], spec[2]))
    raise ValueError(spec)


def make_pair(w: Workload, index: int) -> tuple[np.ndarray, np.ndarray]:
    """Return (pattern, text) as uint8 codes 0..3 for pair ``index`` of ``w``."""
    rng = _pair_rng(w.seed, index)
    m = _draw_length(rng, w.length)
    rate = _draw_rate(rng, w.rate)
    pat = rng.integers(0, 4, m, dtype=np.uint8)
    budget = int(round(rate * m))
    if budget == 0:
        return pat, pat.copy()
    cmix = np.cumsum(np.asarray(w.mix, dtype=np.float64))
    cmix[-1] = 1.0
    n_draw = budget + 16
    types = np.searchsorted(cmix, rng.random(n_draw), side="right").astype(np.int8)
    lens = np.ones(n_draw, dtype=np.int64)
    if w.geometric_indels:
        g = rng.geometric(2.0 / 3.0, n_draw)
        lens = np.where(types > 0, g, 1)
    cum = np.cumsum(lens)
    while cum[-1] < budget:  # extremely unlikely; extend deterministically
        extra = np.ones(n_draw, dtype=np.int64)
        types = np.concatenate([types, np.zeros(n_draw, dtype=np.int8)])
        lens = np.concatenate([lens, extra])
        cum = np.cumsum(lens)
    nev = int(np.searchsorted(cum, budget, side="left")) + 1
    types = types[:nev]
    lens = lens[:nev].copy()
    lens[-1] -= cum[nev - 1] - budget
    pos = rng.integers(0, m, nev)

    txt = pat.copy()
    sub = types == 0
    if sub.any():
        sp = pos[sub]
        txt[sp] = (pat[sp] + rng.integers(1, 4, sp.size, dtype=np.uint8)) % 4
    deleted = np.zeros(m + 1, dtype=np.int64)
    dl = types == 2
    if dl.any():
        starts = pos[dl]
        ends = np.minimum(starts + lens[dl], m)
        np.add.at(deleted, starts, 1)
        np.add.at(deleted, ends, -1)
    keep = np.cumsum(deleted[:m]) == 0
    kept_idx = np.flatnonzero(keep)
    out = txt[keep]
    ins = types == 1
    if ins.any():
        ip = np.searchsorted(kept_idx, pos[ins], side="left")
        il = lens[ins]
        where = np.repeat(ip, il)
        vals = rng.integers(0, 4, int(il.sum()), dtype=np.uint8)
        out = np.insert(out, where, vals)
    return pat, out


def from_lists(patterns, texts) -> PairBatch:
    """Build a CSR batch from sequences given as bytes/str (ASCII)."""
    def csr(seqs):
        bs = [s.encode() if isinstance(s, str) else bytes(s) for s in seqs]
        off = np.zeros(len(bs) + 1, dtype=np.int64)
        off[1:] = np.cumsum([len(b) for b in bs])
        data = np.frombuffer(b"".join(bs), dtype=np.uint8).copy() if bs else np.zeros(0, np.uint8)
        return data, off
    p, po = csr(patterns)
    t, to = csr(texts)
    return PairBatch(p, po, t, to)


def make_batch(name: str, npairs: int | None = None, indices=None) -> PairBatch:
    """Generate workload ``name``; ``indices`` (or the first ``npairs``) picks pairs."""
    w = WORKLOADS[name]
    if indices is None:
        indices = range(w.npairs if npairs is None else npairs)
    pats, txts = [], []
    for i in indices:
        p, t = make_pair(w, int(i))
        pats.append(ALPHABET[p])
        txts.append(ALPHABET[t])

    def csr(arrs):
        off = np.zeros(len(arrs) + 1, dtype=np.int64)
        off[1:] = np.cumsum([a.size for a in arrs])
        data = np.concatenate(arrs) if arrs else np.zeros(0, np.uint8)
        return data, off
    p, po = csr(pats)
    t, to = csr(txts)
    return PairBatch(p, po, t, to)


def random_pair(rng: np.random.Generator, m: int, n: int) -> tuple[bytes, bytes]:
    """Two uncorrelated uniform ACGT strings (ASCII bytes) of lengths m and n."""
    return ALPHABET[rng.integers(0, 4, m)].tobytes(), ALPHABET[rng.integers(0, 4, n)].tobytes()
