"""Train the learned row-budget predictor on the GPU.

    python -m paper_2208_09985_amd.train [--windows PATH] [--out PATH]

Input: windows labelled by their distance d_w (pair, p0, t0, m_w, n_w, k_w,
d_w) of a seeded workload, written by the oracle's training-window script.
Every numeric step runs in the library's kernels through the C ABI:
features (scg_features), the FP16 MLP forward with softmax cross-entropy
(scg_mlp_forward), the backward pass (scg_mlp_backward) and Adam
(scg_adam_step) on FP32 master weights with an FP16 copy.
Output: an .npz with the FP16 weights and the budget classes, loaded by
Context.load_model for SCG_MODE_LEARNED.
"""
from __future__ import annotations

import argparse
import ctypes
import os
import time

import numpy as np

from . import _lib as L
from . import api, synth

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_WINDOWS = os.path.join(HERE, "weights", "train_windows_w64_o24.npz")
DEFAULT_OUT = os.path.join(HERE, "weights", "budget_w64_o24.npz")
BUDGET_ROWS = (7, 15, 31, 64)
F = L.NFEATURES


def budget_class(d_w, m_w, k_w, budget_rows=BUDGET_ROWS):
    """Smallest budget class holding rows 0..d_w (row m_w is implicit)."""
    d_w, m_w, k_w = (np.asarray(a, np.int64) for a in (d_w, m_w, k_w))
    rows_full = np.where(k_w == m_w, m_w, k_w + 1)
    need = np.minimum(d_w + 1, rows_full)
    br = np.asarray(budget_rows, np.int64)
    return np.minimum(np.searchsorted(br, need, side="left"), len(br) - 1).astype(np.int32)


class Mlp:
    """FP32 master weights + FP16 copy + Adam moments, flat on the device."""

    def __init__(self, H=64, C=4, seed=0, device="cuda"):
        import torch
        self.H, self.C = H, C
        g = np.random.default_rng(seed)
        w1 = g.normal(0, np.sqrt(2.0 / F), (F, H))
        b1 = np.zeros(H)
        w2 = g.normal(0, np.sqrt(2.0 / H), (H, C))
        b2 = np.zeros(C)
        flat = np.concatenate([w1.ravel(), b1, w2.ravel(), b2]).astype(np.float32)
        self.n = flat.size
        self.p = torch.tensor(flat, device=device)
        self.p16 = self.p.to(torch.float16)
        self.g = torch.zeros_like(self.p)
        self.m = torch.zeros_like(self.p)
        self.v = torch.zeros_like(self.p)
        self.step = 0

    def views(self, t):
        H, C = self.H, self.C
        o1 = F * H
        o2 = o1 + H
        o3 = o2 + H * C
        return t[:o1], t[o1:o2], t[o2:o3], t[o3:o3 + C]

    def numpy_fp16(self):
        w1, b1, w2, b2 = (x.detach().cpu().numpy() for x in self.views(self.p16))
        return w1.reshape(F, self.H), b1, w2.reshape(self.H, self.C), b2


def forward(lib, mlp, x16, labels=None, stream=None):
    """Run scg_mlp_forward; returns (logits, hidden, loss, dlogits)."""
    import torch
    B = x16.shape[0]
    logits = torch.empty((B, mlp.C), dtype=torch.float32, device=x16.device)
    hidden = torch.empty((B, mlp.H), dtype=torch.float16, device=x16.device)
    loss = dl = None
    if labels is not None:
        loss = torch.empty(B, dtype=torch.float32, device=x16.device)
        dl = torch.empty((B, mlp.C), dtype=torch.float32, device=x16.device)
    w1, b1, w2, b2 = mlp.views(mlp.p16)
    P = api._ptr
    rc = lib.scg_mlp_forward(B, F, mlp.H, mlp.C, P(x16), P(w1), P(b1), P(w2), P(b2), P(logits), P(hidden),
                             P(labels), P(loss), P(dl), api._stream_ptr(stream))
    L.check(rc, "scg_mlp_forward")
    return logits, hidden, loss, dl


def backward(lib, mlp, x16, hidden, dlogits, stream=None):
    import torch
    gw1, gb1, gw2, gb2 = mlp.views(mlp.g)
    _, _, w2, _ = mlp.views(mlp.p16)
    P = api._ptr
    need = int(lib.scg_mlp_backward_workspace(x16.shape[0], mlp.H, mlp.C))
    ws = getattr(mlp, "workspace", None)
    if ws is None or ws.numel() < max(need, 1):
        ws = mlp.workspace = torch.empty(max(need, 1), dtype=torch.float32, device=x16.device)
    rc = lib.scg_mlp_backward(x16.shape[0], F, mlp.H, mlp.C, P(x16), P(hidden), P(w2), P(dlogits),
                              P(gw1), P(gb1), P(gw2), P(gb2), P(ws), ws.numel(), api._stream_ptr(stream))
    L.check(rc, "scg_mlp_backward")


def adam(lib, mlp, lr, stream=None):
    mlp.step += 1
    P = api._ptr
    rc = lib.scg_adam_step(mlp.n, P(mlp.p), P(mlp.g), P(mlp.m), P(mlp.v), P(mlp.p16), ctypes.c_float(lr),
                           ctypes.c_float(0.9), ctypes.c_float(0.999), ctypes.c_float(1e-8), mlp.step,
                           api._stream_ptr(stream))
    L.check(rc, "scg_adam_step")


def window_features(ctx, win, workload):
    """GPU features of the labelled windows (uint16 [N, 16] on the device)."""
    npairs = int(win["npairs"])
    batch = synth.make_batch(workload, npairs)
    b = api.Batch(ctx, batch, api.params())
    tri = np.stack([win["pair"], win["p0"], win["t0"]], axis=1).astype(np.int32)
    feats = b.features(tri)
    return feats, b


def train(windows_path=DEFAULT_WINDOWS, out=DEFAULT_OUT, epochs=12, batch_size=4096, lr=3e-3, seed=0, H=64,
          val_frac=0.1, log=print):
    import torch
    z = np.load(windows_path, allow_pickle=False)
    win = {k: z[k] for k in z.files}
    workload = str(win.get("workload", "train_10kbp"))
    ctx = api.Context(0)
    lib = ctx._lib
    t0 = time.time()
    feats, keep = window_features(ctx, win, workload)
    x16 = (feats.to(torch.int32).to(torch.float32) / 64.0).to(torch.float16).contiguous()
    y = torch.tensor(budget_class(win["d_w"], win["m_w"], win["k_w"]), device=x16.device)
    N = x16.shape[0]
    g = torch.Generator(device="cpu").manual_seed(seed)
    perm = torch.randperm(N, generator=g).to(x16.device)
    nval = int(N * val_frac)
    val_idx, tr_idx = perm[:nval], perm[nval:]
    mlp = Mlp(H=H, C=len(BUDGET_ROWS), seed=seed, device=x16.device)
    hist = []
    for ep in range(epochs):
        order = tr_idx[torch.randperm(tr_idx.numel(), generator=g).to(x16.device)]
        tot = 0.0
        nb = 0
        for s in range(0, order.numel(), batch_size):
            idx = order[s:s + batch_size]
            xb = x16[idx].contiguous()
            yb = y[idx].contiguous().to(torch.int32)
            _, hid, loss, dl = forward(lib, mlp, xb, yb)
            backward(lib, mlp, xb, hid, dl)
            adam(lib, mlp, lr * (0.5 ** (ep // 4)))
            tot += float(loss.mean())
            nb += 1
        acc, vloss = evaluate(lib, mlp, x16[val_idx].contiguous(), y[val_idx].contiguous())
        hist.append(dict(epoch=ep, train_loss=tot / nb, val_loss=vloss, val_acc=acc))
        log(f"[train] epoch {ep}: train loss {tot / nb:.4f}  val loss {vloss:.4f}  val acc {acc:.4f}")
    w1, b1, w2, b2 = mlp.numpy_fp16()
    os.makedirs(os.path.dirname(out), exist_ok=True)
    np.savez(out, w1=w1, b1=b1, w2=w2, b2=b2, budget_rows=np.asarray(BUDGET_ROWS, np.int32),
             feature_scale=np.float32(1 / 64), windows=np.int64(N), workload=workload,
             val_acc=np.float32(hist[-1]["val_acc"]), val_loss=np.float32(hist[-1]["val_loss"]))
    write_scgw(out, os.path.splitext(out)[0] + ".scgw")
    log(f"[train] {N} windows, {time.time() - t0:.1f}s -> {out}")
    keep.close()
    return hist


def write_scgw(npz_path: str, out: str) -> None:
    """The predictor file scg_create reads: "SCGW", uint32 version 1, int32 F,
    H, C, int32 budget_rows[C], then FP16 w1, b1, w2, b2 (little-endian)."""
    z = np.load(npz_path, allow_pickle=False)
    w1, b1, w2, b2 = (np.ascontiguousarray(z[k], dtype=np.float16) for k in ("w1", "b1", "w2", "b2"))
    F, H = w1.shape
    C = w2.shape[1]
    rows = np.ascontiguousarray(z["budget_rows"], dtype="<i4")
    with open(out + ".tmp", "wb") as f:
        f.write(b"SCGW")
        f.write(np.asarray([1, F, H, C], dtype="<i4").tobytes())
        f.write(rows.tobytes())
        for a in (w1, b1, w2, b2):
            f.write(a.astype("<f2").tobytes())
    os.replace(out + ".tmp", out)


def evaluate(lib, mlp, x16, y):
    import torch
    logits, _, loss, _ = forward(lib, mlp, x16, y.to(torch.int32))
    pred = logits.argmax(dim=1)
    return float((pred == y).float().mean()), float(loss.mean())


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--windows", default=DEFAULT_WINDOWS)
    ap.add_argument("--out", default=DEFAULT_OUT)
    ap.add_argument("--epochs", type=int, default=12)
    ap.add_argument("--lr", type=float, default=3e-3)
    args = ap.parse_args()
    train(args.windows, args.out, epochs=args.epochs, lr=args.lr)


if __name__ == "__main__":
    main()
