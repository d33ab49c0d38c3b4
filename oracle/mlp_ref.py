"""Float64 reference of the learned row budget (test infrastructure only).

The learned budget is not part of the paper: it predicts, per window, how
many error rows GenASM-DC (Algorithm 1) must compute before early
termination (Section 2.4.3) finds d_w, so that a window can start with fewer
rows and fall back to all rows when the prediction is too small.  This module
states its pieces in the plainest form, for checking the GPU kernels:

* ``window_features`` -- the 16 integer features of one window, by explicit
  loops over characters;
* ``forward`` / ``loss_and_grads`` -- a 2-layer MLP (ReLU hidden layer,
  softmax cross-entropy over budget classes) and its gradients in float64;
* ``budget_class`` -- the training label of a window.

Only tests/, the smoke check and the benchmark's CPU baseline import it.
"""
from __future__ import annotations

import numpy as np

NFEATURES = 16
BUDGET_ROWS = (7, 15, 31, 64)


def window_features(pattern_w: bytes, text_w: bytes) -> np.ndarray:
    """Features of the window (pattern_w = P[p0:p0+m_w], text_w = T[t0:t0+n_w]).

    f[0..6]   for delta = -3..3: number of t with pattern_w[t:t+4] ==
              text_w[t+delta:t+delta+4], all eight positions inside the window
    f[7..13]  for delta = -3..3: number of t with pattern_w[t] == text_w[t+delta]
    f[14]     m_w
    f[15]     n_w
    """
    m, n = len(pattern_w), len(text_w)
    f = np.zeros(NFEATURES, dtype=np.int64)
    for k, delta in enumerate(range(-3, 4)):
        ones = 0
        fours = 0
        for t in range(m):
            u = t + delta
            if 0 <= u < n and pattern_w[t] == text_w[u]:
                ones += 1
            if t + 3 < m and u >= 0 and u + 3 < n and pattern_w[t:t + 4] == text_w[u:u + 4]:
                fours += 1
        f[k] = fours
        f[7 + k] = ones
    f[14] = m
    f[15] = n
    return f


def features_to_input(f: np.ndarray) -> np.ndarray:
    """Network input: features / 64 (the GPU stores it as fp16)."""
    return np.asarray(f, dtype=np.float64) / 64.0


def budget_class(d_w: int, m_w: int, k_w: int, budget_rows=BUDGET_ROWS) -> int:
    """Smallest class whose row budget holds rows 0..d_w (row m_w is never
    computed: when k_w == m_w a window with no earlier hit has d_w = m_w)."""
    rows_full = m_w if k_w == m_w else k_w + 1
    need = min(d_w + 1, rows_full)
    for c, b in enumerate(budget_rows):
        if b >= need:
            return c
    return len(budget_rows) - 1


def forward(x, w1, b1, w2, b2):
    """h = relu(x @ w1 + b1); logits = h @ w2 + b2 (all float64)."""
    x, w1, b1, w2, b2 = (np.asarray(a, dtype=np.float64) for a in (x, w1, b1, w2, b2))
    pre = x @ w1 + b1
    h = np.maximum(pre, 0.0)
    return h, h @ w2 + b2


def softmax(z):
    z = z - z.max(axis=1, keepdims=True)
    e = np.exp(z)
    return e / e.sum(axis=1, keepdims=True)


def loss_and_grads(x, y, w1, b1, w2, b2, hidden=None):
    """Mean softmax cross-entropy and its gradients.  With ``hidden`` given
    (the forward pass's post-ReLU activations) the backward pass uses it in
    place of recomputing h, as the GPU kernels do."""
    x = np.asarray(x, dtype=np.float64)
    B = x.shape[0]
    h, logits = forward(x, w1, b1, w2, b2)
    if hidden is not None:
        h = np.asarray(hidden, dtype=np.float64)
        logits = h @ np.asarray(w2, np.float64) + np.asarray(b2, np.float64)
    p = softmax(logits)
    loss = -np.mean(np.log(p[np.arange(B), y]))
    dlog = p.copy()
    dlog[np.arange(B), y] -= 1.0
    dlog /= B
    gw2 = h.T @ dlog
    gb2 = dlog.sum(axis=0)
    dh = (dlog @ np.asarray(w2, np.float64).T) * (h > 0)
    gw1 = x.T @ dh
    gb1 = dh.sum(axis=0)
    return loss, dlog, (gw1, gb1, gw2, gb2)
