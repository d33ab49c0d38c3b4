"""Benchmark: windowed GenASM alignment throughput on one MI355X.

    python bench.py [--steps K] [--warmup W] [--workload long_10kbp]

A step aligns the whole workload once: encode + pack to 2-bit planes, then
the persistent fused DC+TB kernel (every window's DC, early termination,
traceback, CIGAR runs).  The ASCII input is resident in HBM before timing.
Prints ONE JSON line on stdout; progress goes to stderr.

Headline: the plain method (every window may use all rows 0..k_w) on 10,000
pairs of 10 kbp with 15% edits, W=64, O=24, k=64, in the library's default
kernel for it (column blocks, exact early termination per window).  Variants
on the same input run the error-row lane kernel, where a window's row budget
decides how many lanes it takes: plain, a constant budget and the learned
budget, each with full-row fallback and each checked bit-identical to the
headline's output.  Two more workloads are reported under "workloads":
10,000 x 10 kbp pairs with a per-pair edit rate of 5-15% (learned vs plain),
and 50,000 pairs of log-normal length (1-50 kbp) as one hipGraph-captured
launch with the launch shape picked by the autotuner.

Roofline: the kernel is bound by 32-bit bitwise VALU issue.  One 64-bit op of
the paper's accounting is two 32-bit lane operations, so the nominal peak is
256 CU x 64 lanes x 2.4 GHz / 2 = 19.66 T 64-bit op/s; `peak` is the figure
the bitwise-VALU microbenchmark measured on the device
(profiles/peak_microbench.txt, with the shader clock it ran at), the
nominal one when that summary is missing.  `achieved` is
ops_alg (sum over windows of (d_w+1) + 2 n_w + 7 n_w d_w) per launch divided
by the kernel's mean duration from HIP events recorded around each timed
launch on its stream.  `traffic` (HBM bytes per launch) comes from the
committed rocprofv3 counter summary when it was taken from the current kernel
sources (their hash is recorded beside the figures), else it is null.

    python bench.py --copy-probe 1024   # device copy of 1 GiB, for counter calibration
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_NOMINAL = 256 * 64 * 2.4e9 / 2 / 1e12    # 19.66 T 64-bit op/s
PEAK_FILE = os.path.join(ROOT, "profiles", "peak_microbench.txt")


def measured_peak():
    """(T 64-bit op/s, shader MHz) from the committed microbenchmark summary,
    or (nominal, None) when it is missing."""
    try:
        for line in open(PEAK_FILE):
            if line.startswith("{"):
                d = json.loads(line)
                return d["valu_t64_ops_per_s"] / 1e12, d.get("sclk_mhz")
    except (OSError, ValueError, KeyError):
        pass
    return PEAK_NOMINAL, None


PEAK_T64OPS, PEAK_SCLK = measured_peak()
METRIC = "alignments/s and Gbitops/s vs roofline, 10 kbp @15% err; learned-k vs plain"
WEIGHTS = os.path.join(ROOT, "paper_2208_09985_amd", "weights", "budget_w64_o24.npz")
TRAFFIC = os.path.join(ROOT, "profiles", "cols_kernel_long_10kbp_traffic.txt")
KERNEL_SOURCES = ("align_cols.hip", "colblock.h", "predictor.h", "internal.h")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def timed_steps(batch, steps: int, warmup: int):
    import torch
    for _ in range(warmup):
        batch.run()
    torch.cuda.synchronize()
    batch.stats()                      # clear the timing ring
    t0 = time.perf_counter()
    for _ in range(steps):
        batch.run()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    st = batch.stats()
    return wall / steps * 1e3, st


def same_output(a, b) -> bool:
    """Identical edits, text_end, status and CIGAR run words for every pair."""
    if not (np.array_equal(a.edits, b.edits) and np.array_equal(a.text_end, b.text_end)
            and np.array_equal(a.status, b.status) and np.array_equal(a.n_runs, b.n_runs)):
        return False
    ra, rb = np.asarray(a.runs), np.asarray(b.runs)
    for i in range(len(a.n_runs)):
        s, e = int(a.runs_off[i]), int(a.runs_off[i]) + int(a.n_runs[i])
        if not np.array_equal(ra[s:e], rb[s:e]):
            return False
    return True


def cpu_baseline(workload, W, O, k, budget_core_s=15.0):
    """The oracle (unchanged) on a bounded sample of the same workload, all host cores."""
    import oracle
    from paper_2208_09985_amd import synth
    cores = len(os.sched_getaffinity(0))
    probe = synth.make_batch(workload, 64)
    t = time.perf_counter()
    oracle.align_batch(probe, W, O, k, threads=1)
    per_pair_core_s = (time.perf_counter() - t) / probe.npairs
    n = int(min(synth.WORKLOADS[workload].npairs, max(64, budget_core_s / max(per_pair_core_s, 1e-9))))
    sample = synth.make_batch(workload, n)
    t = time.perf_counter()
    res = oracle.align_batch(sample, W, O, k, threads=cores)
    dt = time.perf_counter() - t
    return {"value": round(n / dt, 3), "unit": "alignments/s", "cores": int(res["threads"]), "kind": "oracle",
            "sample": f"first {n} of {synth.WORKLOADS[workload].npairs} pairs of {workload} "
                      f"({dt:.2f} s wall on {res['threads']} threads, plain full-table oracle)",
            "ops_alg_per_s": round(res["stats"].ops_alg / dt, 1)}


def spec(t):
    """("fixed", x) -> x; other distributions -> "kind(a, b, ...)"."""
    return t[1] if t[0] == "fixed" else f"{t[0]}{tuple(t[1:])}"


def stored_form(cap):
    """Template argument of the plain column-block kernel for W - O = cap: 1 keeps
    32-bit entries, 2 keeps 48-bit entries in two planes, 0 whole 64-bit ones."""
    return 1 if cap <= 31 else (2 if cap <= 47 else 0)


def kernel_source_hash() -> str:
    """Hash of the measured kernel's sources with comments and blank space
    removed, so that the counters stay valid across comment-only edits (the
    sources hold no comment markers inside string literals)."""
    import re
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2208_09985_amd", "csrc", f), encoding="utf-8") as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed counter summary,
    or None when the summary is missing or was taken from other sources."""
    if not os.path.exists(TRAFFIC):
        return None
    vals = {}
    for line in open(TRAFFIC):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("source_hash") != kernel_source_hash():
        return None
    try:
        return int(float(vals[f"{kernel}.hbm_bytes_per_launch"]))
    except (KeyError, ValueError):
        return None


def copy_probe(mib: int, reps: int = 5):
    """A plain device copy of known size (counter calibration)."""
    import torch
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_each_way": n * 4, "reps": reps}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="long_10kbp")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-variants", action="store_true", help="only the plain headline")
    ap.add_argument("--no-workloads", action="store_true", help="skip the extra workloads")
    ap.add_argument("--fixed-rows", type=int, default=15)
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: pairs are independent, so several GPUs would each run this "
              "kernel on their own share of the pairs; run with --gpus 1.", file=sys.stderr)
        sys.exit(2)
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return

    import torch
    from paper_2208_09985_amd import api, autotune, synth

    ctx = api.Context(0)
    have_model = os.path.exists(WEIGHTS)
    if have_model:
        ctx.load_model(WEIGHTS)

    shapes = {}

    def measure(batch, name, prm, steps, warmup):
        log(f"[bench] {name}: prepare")
        b = api.Batch(ctx, batch, prm)
        shapes[name] = b.launch_shape()
        ms, st = timed_steps(b, steps, warmup)
        res = b.result()
        ok = bool(np.all(res.status == 0))
        log(f"[bench] {name}: {ms:.3f} ms/step, kernel {st.kernel_ms_avg:.3f} ms, windows {st.windows}, "
            f"fallback {st.fallback_windows}, all pairs aligned: {ok}")
        b.close()
        return ms, st, res

    def summary(batch, ms, st, same=None, ref_ms=None):
        d = dict(alignments_per_s=round(batch.npairs / (ms / 1e3), 1), ms_per_step=round(ms, 4),
                 kernel_ms=round(st.kernel_ms_avg, 4), fallback_windows=int(st.fallback_windows),
                 rows_budgeted=int(st.rows_budgeted), lane_steps=int(st.lane_steps),
                 t64ops=round(st.ops_alg / (st.kernel_ms_avg / 1e3) / 1e12, 4))
        if same is not None:
            d["identical_to_plain"] = same
        if ref_ms is not None:
            d["speedup_vs_plain"] = round(ref_ms / ms, 3)
        return d

    w = synth.WORKLOADS[args.workload]
    log(f"[bench] generating {args.workload} ({w.npairs} pairs)")
    t = time.perf_counter()
    batch = synth.make_batch(args.workload)
    log(f"[bench] generated in {time.perf_counter() - t:.1f}s: {batch.pat.size} + {batch.txt.size} bases")

    ms, st, res = measure(batch, "plain", api.params(W=w.W, O=w.O, k=w.k, mode="plain"), args.steps, args.warmup)
    variants = {}
    if not args.no_variants:
        # the row budget acts in the error-row lane kernel: plain vs fixed vs learned there
        rms, rst, rres = measure(batch, "plain (row lanes)", api.params(W=w.W, O=w.O, k=w.k, mode="plain", kernel="rows"),
                                 args.steps, args.warmup)
        variants["plain_row_lanes"] = summary(batch, rms, rst, same_output(rres, res), ms)
        fms, fst, fres = measure(batch, "fixed (row lanes)", api.params(W=w.W, O=w.O, k=w.k, mode="fixed",
                                                                          fixed_rows=args.fixed_rows, kernel="rows"),
                                 args.steps, args.warmup)
        variants[f"fixed_{args.fixed_rows}_rows_row_lanes"] = summary(batch, fms, fst, same_output(fres, res), rms)
        if have_model:
            lms, lst, lres = measure(batch, "learned (row lanes)", api.params(W=w.W, O=w.O, k=w.k, mode="learned",
                                                                              kernel="rows"), args.steps, args.warmup)
            variants["learned_row_lanes"] = summary(batch, lms, lst, same_output(lres, res), rms)
            variants["learned_row_lanes"]["speedup_vs_headline"] = round(ms / lms, 3)

    workloads = {}
    if not args.no_workloads:
        # short reads (the paper's short-read results, Section 3.2): plain, default launch
        # short reads: the library's automatic launch, and the launch autotune.tune picks
        # (shallow windows favour fewer lanes per window: a shorter skew)
        for name in ("small_100bp", "short_250bp"):
            sb = synth.make_batch(name)
            sw = synth.WORKLOADS[name]
            sms, sst, sres = measure(sb, f"{name} plain", api.params(W=sw.W, O=sw.O, k=sw.k, mode="plain"), 10, 2)
            e = summary(sb, sms, sst)
            e.update(pairs=sb.npairs, windows=int(sst.windows), launch=shapes[f"{name} plain"],
                     frac=round(sst.ops_alg / (sst.kernel_ms_avg / 1e3) / 1e12 / PEAK_T64OPS, 5))
            best, _ = autotune.tune(ctx, sb, sw.W, sw.O, sw.k, mode="plain", reps=2, cache_path=None, log=log)
            tms, tst, tres = measure(sb, f"{name} plain tuned {best}",
                                     api.params(W=sw.W, O=sw.O, k=sw.k, mode="plain", **best), 10, 2)
            t = summary(sb, tms, tst, same_output(tres, sres))
            t.update(autotuned=best, launch=shapes[f"{name} plain tuned {best}"],
                     frac=round(tst.ops_alg / (tst.kernel_ms_avg / 1e3) / 1e12 / PEAK_T64OPS, 5))
            e["autotuned"] = t
            workloads[name] = e
            del sb
        # per-pair edit rate 5-15%: learned budget vs plain
        name = "mixed_10kbp"
        wb = synth.make_batch(name)
        ww = synth.WORKLOADS[name]
        pms, pst, pres = measure(wb, f"{name} plain", api.params(W=ww.W, O=ww.O, k=ww.k, mode="plain"), 5, 1)
        entry = {"pairs": wb.npairs, "plain": summary(wb, pms, pst)}
        rms, rst, rres = measure(wb, f"{name} plain (row lanes)",
                                 api.params(W=ww.W, O=ww.O, k=ww.k, mode="plain", kernel="rows"), 5, 1)
        entry["plain_row_lanes"] = summary(wb, rms, rst, same_output(rres, pres), pms)
        if have_model:
            lms, lst, lres = measure(wb, f"{name} learned (row lanes)",
                                     api.params(W=ww.W, O=ww.O, k=ww.k, mode="learned", kernel="rows"), 5, 1)
            entry["learned_row_lanes"] = summary(wb, lms, lst, same_output(lres, pres), rms)
            entry["learned_row_lanes"]["speedup_vs_headline_kernel"] = round(pms / lms, 3)
        workloads[name] = entry
        del wb
        # uneven lengths: autotuned launch shape, one hipGraph-captured launch per step (a batch
        # with off-track helpers is enqueued directly)
        name = "uneven_lognormal"
        log(f"[bench] generating {name}")
        wb = synth.make_batch(name)
        ww = synth.WORKLOADS[name]
        entry = {"pairs": wb.npairs, "bases": int(wb.pat.size)}
        ref = None
        for mode in (("plain", "learned") if have_model else ("plain",)):
            best, trials = autotune.tune(ctx, wb, ww.W, ww.O, ww.k, mode=mode, reps=1, cache_path=None, log=log)
            gms, gst, gres = measure(wb, f"{name} {mode} graph {best}",
                                     api.params(W=ww.W, O=ww.O, k=ww.k, mode=mode, graph=True, **best), 5, 1)
            e = summary(wb, gms, gst, None if ref is None else same_output(gres, ref[1]),
                        None if ref is None else ref[0])
            e["autotuned"] = best
            gshape = shapes[f"{name} {mode} graph {best}"]
            # the library enqueues a batch with off-track helpers directly, graph flag or not
            e["graph"] = gshape["helper_grid"] == 0
            e["launch"] = gshape
            e["candidates"] = len(trials)
            entry[mode] = e
            if ref is None:
                ref = (gms, gres)
        workloads[name] = entry
        del wb
        # window geometry on the headline batch: throughput and windowed edit counts per (W, O);
        # W - O <= 31 stores 32-bit entries, W > 64 runs 128-bit bitvectors
        sweep = {}
        for (W, O) in ((64, 24), (64, 33), (64, 16), (64, 40), (32, 8), (96, 32), (128, 24), (128, 64)):
            sms, sst, sres = measure(batch, f"window sweep W={W} O={O}", api.params(W=W, O=O, k=W, mode="plain"), 5, 1)
            e = summary(batch, sms, sst)
            ach = sst.ops_alg / (sst.kernel_ms_avg / 1e3) / 1e12
            e.update(windows=int(sst.windows), frac=round(ach / PEAK_T64OPS, 5),
                     stored_entry_bits=((96 if W - O <= 95 else 128) if W > 64 else {1: 32, 2: 48, 0: 64}[stored_form(W - O)]),
                     mean_edits=round(float(np.mean(sres.edits[sres.status == 0])), 2),
                     aligned=int(np.sum(sres.status == 0)))
            sweep[f"W{W}_O{O}"] = e
        workloads["window_sweep_long_10kbp"] = sweep
        # lanes per window in the column-block kernel: 16, 8, 4 or 2 lanes (4, 8, 16 or 32 windows per
        # wavefront); the error-row lane kernel's plain figure is in `variants`
        # (10: six lanes of 12 columns), each with the automatic SIMD placement, and 8 and 10 also
        # with wavefronts allowed to share a SIMD; none of them with the off-track helpers (the
        # headline's launch is 16 windows per wavefront plus the helpers)
        lanes = {}
        for ng, one in ((4, "auto"), (8, "auto"), (8, False), (10, "auto"), (10, False), (16, "auto"), (32, "auto")):
            tag = f"windows_per_wavefront_{ng}" + ("_shared_simds" if one is False else "")
            lms_, lst_, _ = measure(batch, f"columns, {ng} windows per wavefront, one per SIMD {one}",
                                    api.params(W=w.W, O=w.O, k=w.k, mode="plain", kernel="columns", slots=ng,
                                               one_per_simd=one, offtrack_helpers=False), 5, 1)
            e = summary(batch, lms_, lst_)
            e["lanes_per_window"] = 6 if ng == 10 else 64 // ng
            e["one_wavefront_per_simd"] = shapes[f"columns, {ng} windows per wavefront, one per SIMD {one}"]["one_per_simd"]
            e["frac"] = round(lst_.ops_alg / (lst_.kernel_ms_avg / 1e3) / 1e12 / PEAK_T64OPS, 5)
            lanes[tag] = e
        # the other end of the mapping: one lane per pair, rows in order (the paper's CPU mapping),
        # and the column-block kernel with its stored rows as a ring (DENT extended to rows) or with
        # the lowest rows in LDS
        for tag, kw in (("one_lane_per_pair_rowwise", dict(kernel="lanes")),
                        ("columns_row_ring", dict(kernel="columns", row_ring=True)),
                        ("columns_rows_in_lds", dict(kernel="columns", rows_lds=True))):
            xms, xst, xres = measure(batch, f"mapping {tag}", api.params(W=w.W, O=w.O, k=w.k, mode="plain", **kw), 3, 1)
            e = summary(batch, xms, xst, same_output(xres, res))
            e["frac"] = round(xst.ops_alg / (xst.kernel_ms_avg / 1e3) / 1e12 / PEAK_T64OPS, 5)
            lanes[tag] = e
        workloads["column_blocks_long_10kbp"] = lanes
        # the paper's three improvements (SENE: entries, not edges; DENT: only the columns traceback
        # reads; ET: rows stop at d_w) switched off in every combination, with the stored rows in global
        # memory (default) or the lowest rows in LDS, at W=64 with O=24 (the headline) and O=33
        # (32-bit entries); every combination gives the same alignments
        abl = {}
        for (W, O) in ((64, 24), (64, 33)):
            ref_res = None
            for sene in (True, False):
                for dent in (True, False):
                    for et in (True, False):
                        for lds in ((False, True) if sene else (False,)):
                            on = "+".join(x for x, f in (("SENE", sene), ("DENT", dent), ("ET", et)) if f) or "none"
                            tag = f"W{W}_O{O}_{on}" + ("_lds" if lds else "")
                            kw = dict(no_early_termination=not et, store_all_columns=not dent, store_edges=not sene,
                                      rows_lds=lds)
                            steps_ = 5 if (sene and et) else 2
                            ams, ast, ares = measure(batch, f"ablation {tag}",
                                                     api.params(W=W, O=O, k=W, mode="plain", kernel="columns", **kw),
                                                     steps_, 1)
                            if ref_res is None:
                                ref_res = ares
                            e = summary(batch, ams, ast, same_output(ares, ref_res))
                            e.update(rows_computed=int(ast.rows_budgeted), sene=sene, dent=dent, et=et,
                                     stored_rows="lds+global" if lds else "global")
                            abl[tag] = e
        workloads["ablation_long_10kbp"] = abl
        # more pairs of the headline shape: how far latency hiding goes once the GPU holds more wavefronts
        scale = {}
        for n in (20000, 40000):
            sb = synth.make_batch(args.workload, n)
            sms, sst, _ = measure(sb, f"{args.workload} x{n}", api.params(W=w.W, O=w.O, k=w.k, mode="plain"), 5, 1)
            e = summary(sb, sms, sst)
            e["frac"] = round(sst.ops_alg / (sst.kernel_ms_avg / 1e3) / 1e12 / PEAK_T64OPS, 5)
            scale[str(n)] = e
            del sb
        workloads["more_pairs_long_10kbp"] = scale

    achieved = st.ops_alg / (st.kernel_ms_avg / 1e3) / 1e12
    shape = shapes["plain"]
    kname = (f"cols_kernel<false, {shape['slots']}, {stored_form(w.W - w.O)}, 0"
             + (", true>" if shape["one_per_simd"] else ">"))
    if shape.get("helper_grid", 0) > 0:
        # the off-track helper launch runs beside the main one; the kernel time spans both
        kname += f" + cols_kernel<false, {shape['helper_slots']}, {stored_form(w.W - w.O)}, 0, true>"
    lanes_per_window = 64 // shape["slots"] if shape["slots"] != 10 else 6
    out = {
        "metric": METRIC,
        "value": round(batch.npairs / (ms / 1e3), 1),
        "unit": "alignments/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": args.workload, "pairs": batch.npairs, "pattern_length": spec(w.length),
                   "edit_rate": spec(w.rate), "W": w.W, "O": w.O, "k": w.k, "mode": "plain"},
        "gbitops_per_s": round(achieved * 1e3, 2),
        "roofline": {"bound": "alu", "achieved": round(achieved, 4), "peak": round(PEAK_T64OPS, 3),
                     "unit": "T 64-bit op/s", "frac": round(achieved / PEAK_T64OPS, 5),
                     "peak_source": "measured (profiles/peak_microbench.txt)" if PEAK_SCLK else "nominal",
                     "peak_sclk_mhz": round(PEAK_SCLK, 1) if PEAK_SCLK else None,
                     "peak_nominal": round(PEAK_NOMINAL, 3),
                     "traffic": measured_traffic("cols_kernel_plain"),
                     "kernel": kname, "kernel_ms": round(st.kernel_ms_avg, 4),
                     "launch": shape,
                     "ops_alg_per_launch": int(st.ops_alg), "windows_per_launch": int(st.windows),
                     # lockstep: a pass of a wavefront runs as many row steps as its deepest
                     # window needs; rows_needed is the mean of d_w + 1 (row steps of both
                     # launches when the off-track helpers run, each counted at its own width)
                     "lockstep": {"row_steps_per_window": round(st.lane_steps / 64 * shape["slots"] / max(st.windows, 1), 2)
                                  if not shape.get("helper_grid") else None,
                                  "rows_needed_per_window": round(st.rows_budgeted / max(st.windows, 1), 2),
                                  "skew_steps": lanes_per_window - 1},
                     "offtrack_pairs_handed_over": int(st.yields) if shape.get("helper_grid") else 0},
        "variants": variants,
        "workloads": workloads,
    }
    if not args.no_cpu:
        log("[bench] CPU oracle baseline")
        out["cpu_baseline"] = cpu_baseline(args.workload, w.W, w.O, w.k)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
