"""Write the predictor's training windows from the oracle.

    python -m oracle.training_windows [--out PATH] [--windows 200000]

Runs the oracle on the ``train_10kbp`` workload (disjoint seed) and records,
for every window it aligns, (pair, p0, t0, m_w, n_w, k_w, d_w).  The label of
a window is the smallest row budget holding d_w (``mlp_ref.budget_class``).
Only the oracle computes these values; the trainer reads the file.
"""
from __future__ import annotations

import argparse
import os

import numpy as np

from oracle import align_pair
from paper_2208_09985_amd import synth

DEFAULT_OUT = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2208_09985_amd",
                           "weights", "train_windows_w64_o24.npz")


def collect(workload: str = "train_10kbp", max_windows: int = 200000, W=64, O=24, k=64):
    wl = synth.WORKLOADS[workload]
    recs = []
    total = 0
    npairs = 0
    for i in range(wl.npairs):
        batch = synth.make_batch(workload, indices=[i])
        r = align_pair(batch.pattern(0), batch.text(0), W, O, k, want_windows=True)
        w = r["windows"]
        w["pair"] = i
        recs.append(w)
        total += len(w)
        npairs = i + 1
        if total >= max_windows:
            break
    win = np.concatenate(recs)[:max_windows]
    return win, npairs


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=DEFAULT_OUT)
    ap.add_argument("--windows", type=int, default=200000)
    args = ap.parse_args()
    win, npairs = collect(max_windows=args.windows)
    os.makedirs(os.path.dirname(args.out), exist_ok=True)
    np.savez(args.out, pair=win["pair"], p0=win["p0"], t0=win["t0"], m_w=win["m_w"], n_w=win["n_w"],
             k_w=win["k_w"], d_w=win["d_w"], npairs=np.int64(npairs), workload="train_10kbp")
    print(f"{len(win)} windows from {npairs} pairs -> {args.out}")


if __name__ == "__main__":
    main()
