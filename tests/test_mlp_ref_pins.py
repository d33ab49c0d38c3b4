"""Pins for the float64 predictor reference (oracle/mlp_ref.py)."""
import numpy as np
import pytest

from oracle import mlp_ref


def rand_seq(rng, n):
    return bytes(b"ACGT"[i] for i in rng.integers(0, 4, n))


def test_features_identical_window():
    # pattern == text: every position matches on diagonal 0
    p = rand_seq(np.random.default_rng(1), 64)
    f = mlp_ref.window_features(p, p)
    assert f[3] == 64 - 3          # 4-mers on delta = 0
    assert f[10] == 64             # single characters on delta = 0
    assert (f[14], f[15]) == (64, 64)


def test_features_shifted_text_uses_positive_delta():
    # text = X + pattern: pattern[t] == text[t+1] -> diagonal delta = +1
    p = rand_seq(np.random.default_rng(2), 40)
    t = b"A" + p
    f = mlp_ref.window_features(p, t)
    assert f[11] == 40 and f[4] == 40 - 3
    # pattern = X + text: pattern[t] == text[t-1] -> delta = -1
    f2 = mlp_ref.window_features(b"C" + p, p)
    assert f2[9] == 40 and f2[2] == 40 - 3


def test_features_counting_ranges():
    # a homopolymer makes every in-range comparison a match: count the ranges
    for m, n in ((10, 13), (13, 10), (5, 5), (3, 9), (64, 0)):
        f = mlp_ref.window_features(b"A" * m, b"A" * n)
        for k, delta in enumerate(range(-3, 4)):
            ones = sum(1 for t in range(m) if 0 <= t + delta < n)
            fours = sum(1 for t in range(m - 3) if t + delta >= 0 and t + delta + 3 < n)
            assert f[7 + k] == ones and f[k] == fours, (m, n, delta)


def test_budget_class():
    assert mlp_ref.budget_class(0, 64, 64) == 0
    assert mlp_ref.budget_class(6, 64, 64) == 0      # 7 rows: 0..6
    assert mlp_ref.budget_class(7, 64, 64) == 1
    assert mlp_ref.budget_class(30, 64, 64) == 2
    assert mlp_ref.budget_class(31, 64, 64) == 3
    assert mlp_ref.budget_class(64, 64, 64) == 3     # implicit row m_w: 64 rows
    assert mlp_ref.budget_class(5, 5, 5) == 0        # short last window


def params(rng, F=16, H=64, C=4, scale=0.5):
    return (rng.normal(0, scale, (F, H)), rng.normal(0, 0.1, H), rng.normal(0, scale, (H, C)), rng.normal(0, 0.1, C))


def test_forward_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(3)
    w1, b1, w2, b2 = params(rng)
    x = rng.random((37, 16))
    y = rng.integers(0, 4, 37)
    h, logits = mlp_ref.forward(x, w1, b1, w2, b2)
    xt = torch.tensor(x)
    ht = torch.relu(xt @ torch.tensor(w1) + torch.tensor(b1))
    lt = ht @ torch.tensor(w2) + torch.tensor(b2)
    assert np.allclose(logits, lt.numpy(), rtol=1e-12, atol=1e-12)
    loss, _, _ = mlp_ref.loss_and_grads(x, y, w1, b1, w2, b2)
    lt_loss = torch.nn.functional.cross_entropy(lt, torch.tensor(y)).item()
    assert abs(loss - lt_loss) < 1e-12


def test_gradients_by_finite_differences():
    rng = np.random.default_rng(4)
    w1, b1, w2, b2 = params(rng, H=8, scale=1.0)
    x = rng.random((11, 16))
    y = rng.integers(0, 4, 11)
    _, _, grads = mlp_ref.loss_and_grads(x, y, w1, b1, w2, b2)
    ps = [w1, b1, w2, b2]
    eps = 1e-6
    for pi, g in enumerate(grads):
        flat = ps[pi].reshape(-1)
        for idx in rng.choice(flat.size, min(flat.size, 12), replace=False):
            old = flat[idx]
            flat[idx] = old + eps
            lp, _, _ = mlp_ref.loss_and_grads(x, y, *ps)
            flat[idx] = old - eps
            lm, _, _ = mlp_ref.loss_and_grads(x, y, *ps)
            flat[idx] = old
            fd = (lp - lm) / (2 * eps)
            assert abs(fd - g.reshape(-1)[idx]) < 1e-6 * max(1.0, abs(fd)), (pi, idx, fd, g.reshape(-1)[idx])
