"""Learned row budget on the GPU: features, FP16 MLP forward/backward and
training against the float64 reference; learned mode bit-exact with the
oracle; and what the trained network saves over the method without it."""
import os
import tempfile

import numpy as np
import pytest

import oracle
from oracle import mlp_ref, training_windows
from paper_2208_09985_amd import synth
from tests.gpu_helpers import compare, log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    from paper_2208_09985_amd import api
    return api.Context(0)


@pytest.fixture(scope="module")
def model_path(ctx):
    """A predictor trained here from oracle-labelled windows (GPU kernels)."""
    from paper_2208_09985_amd import train
    win, npairs = training_windows.collect(max_windows=60000)
    d = tempfile.mkdtemp()
    wpath = os.path.join(d, "win.npz")
    np.savez(wpath, pair=win["pair"], p0=win["p0"], t0=win["t0"], m_w=win["m_w"], n_w=win["n_w"], k_w=win["k_w"],
             d_w=win["d_w"], npairs=np.int64(npairs), workload="train_10kbp")
    out = os.path.join(d, "model.npz")
    hist = train.train(wpath, out, epochs=4, log=log)
    assert hist[-1]["val_loss"] < hist[0]["val_loss"] * 1.01
    return out


def test_features_match_reference(ctx):
    from paper_2208_09985_amd import api
    b = synth.make_batch("uneven_lognormal", 6)
    b = synth.from_lists([b.pattern(i) for i in range(6)] + [b"ACGTTGCA" * 3, b"A" * 70],
                         [b.text(i) for i in range(6)] + [b"ACG", b""])
    rng = np.random.default_rng(0)
    wins = []
    for i in range(b.npairs):
        m, n = len(b.pattern(i)), len(b.text(i))
        for _ in range(60 if m > 100 else 6):
            wins.append((i, int(rng.integers(0, m)), int(rng.integers(0, n + 1))))
        wins.append((i, max(0, m - 5), n))          # short pattern tail, empty text window
        wins.append((i, 0, max(0, n - 3)))
    wins = np.array(wins, np.int32)
    bt = api.Batch(ctx, b, api.params())
    got = bt.features(wins).cpu().numpy().astype(np.int64)
    bt.close()
    for (pi, p0, t0), g in zip(wins, got):
        pw = b.pattern(pi)[p0:p0 + 64]
        tw = b.text(pi)[t0:t0 + 64]
        want = mlp_ref.window_features(pw, tw)
        assert np.array_equal(g, want), (pi, p0, t0, g, want)


def _rand_model(rng, H=64, C=4):
    w1 = rng.normal(0, 0.6, (16, H)).astype(np.float16)
    b1 = rng.normal(0, 0.2, H).astype(np.float16)
    w2 = rng.normal(0, 0.5, (H, C)).astype(np.float16)
    b2 = rng.normal(0, 0.2, C).astype(np.float16)
    return w1, b1, w2, b2


@pytest.mark.parametrize("H,C,B", [(64, 4, 1000), (40, 3, 37), (64, 2, 16)])
def test_mlp_forward_backward_match_reference(ctx, H, C, B):
    import torch
    from paper_2208_09985_amd import train
    rng = np.random.default_rng(H * 10 + C)
    w1, b1, w2, b2 = _rand_model(rng, H, C)
    x = (rng.integers(0, 65, (B, 16)) / 64.0).astype(np.float16)
    y = rng.integers(0, C, B).astype(np.int32)
    mlp = train.Mlp(H=H, C=C)
    flat = np.concatenate([w1.ravel(), b1, w2.ravel(), b2]).astype(np.float32)
    mlp.p.copy_(torch.tensor(flat))
    mlp.p16.copy_(mlp.p.to(torch.float16))
    xd = torch.tensor(x, device="cuda")
    yd = torch.tensor(y, device="cuda")
    logits, hidden, loss, dl = train.forward(ctx._lib, mlp, xd, yd)
    train.backward(ctx._lib, mlp, xd, hidden, dl)
    torch.cuda.synchronize()
    h_ref, _ = mlp_ref.forward(x, w1, b1, w2, b2)
    h_gpu = hidden.cpu().numpy().astype(np.float64)
    # hidden: fp32 accumulation of fp16 products, rounded to fp16
    assert np.allclose(h_gpu, h_ref, rtol=2e-3, atol=2e-3)
    # logits and gradients from the GPU's own fp16 hidden activations
    lg_ref = h_gpu @ w2.astype(np.float64) + b2.astype(np.float64)
    assert np.allclose(logits.cpu().numpy(), lg_ref, rtol=1e-4, atol=1e-4)
    loss_ref, dl_ref, grads_ref = mlp_ref.loss_and_grads(x, y, w1, b1, w2, b2, hidden=h_gpu)
    assert abs(float(loss.mean()) - loss_ref) < 1e-4
    assert np.allclose(dl.cpu().numpy(), dl_ref, rtol=1e-4, atol=1e-7)
    for got, want in zip(mlp.views(mlp.g), grads_ref):
        got = got.cpu().numpy().astype(np.float64).reshape(want.shape)
        assert np.allclose(got, want, rtol=1e-3, atol=1e-6), np.abs(got - want).max()


def test_adam_step_matches_reference(ctx):
    import torch
    from paper_2208_09985_amd import train
    mlp = train.Mlp(H=8, C=2)
    rng = np.random.default_rng(5)
    g = rng.normal(0, 1, mlp.n).astype(np.float32)
    p0 = mlp.p.cpu().numpy().astype(np.float64)
    mlp.g.copy_(torch.tensor(g))
    m = np.zeros(mlp.n)
    v = np.zeros(mlp.n)
    p = p0.copy()
    for step in range(1, 4):
        train.adam(ctx._lib, mlp, 1e-2)
        m = 0.9 * m + 0.1 * g
        v = 0.999 * v + 0.001 * g.astype(np.float64) ** 2
        p = p - 1e-2 * (m / (1 - 0.9 ** step)) / (np.sqrt(v / (1 - 0.999 ** step)) + 1e-8)
    torch.cuda.synchronize()
    assert np.allclose(mlp.p.cpu().numpy(), p, rtol=1e-5, atol=1e-6)
    assert np.allclose(mlp.p16.cpu().numpy().astype(np.float64), p, rtol=1e-3, atol=1e-3)


def test_learned_mode_is_bit_exact(ctx, model_path):
    from paper_2208_09985_amd import api
    ctx.load_model(model_path)
    for name, n in (("small_100bp", 400), ("long_10kbp", 24), ("mixed_10kbp", 24), ("uneven_lognormal", 24)):
        b = synth.make_batch(name, n)
        ref = oracle.align_batch(b, 64, 24, 64)
        for tau in (0.5, 0.9, 0.99):
            for kern in ("rows", "columns"):
                log(f"[learned] {name} tau={tau} kernel={kern}")
                compare(b, api.align_batch(ctx, b, mode="learned", tau=tau, kernel=kern), ref,
                        f"{name} learned tau={tau} [{kern}]")


def test_learned_budget_saves_work_over_plain_and_constant_budgets(ctx, model_path):
    """What the trained network gains in the row-lane kernel (where rows above
    a window's budget are lanes not spent): identical output with fewer rows
    computed than the plain method and fewer fallback attempts than constant
    budgets."""
    from paper_2208_09985_amd import api
    ctx.load_model(model_path)
    b = synth.make_batch("mixed_10kbp", 300)
    runs = {}
    for name, kw in (("plain", dict(mode="plain")), ("fixed7", dict(mode="fixed", fixed_rows=7)),
                     ("fixed15", dict(mode="fixed", fixed_rows=15)), ("learned", dict(mode="learned", tau=0.9))):
        runs[name] = api.align_batch(ctx, b, kernel="rows", **kw)
        st = runs[name].stats
        log(f"[gain] {name}: lane_steps={st.lane_steps} rows={st.rows_budgeted} fallback={st.fallback_windows} "
            f"rounds={st.rounds} kernel_ms={st.kernel_ms:.3f}")
    for name in ("fixed7", "fixed15", "learned"):
        assert np.array_equal(runs[name].edits, runs["plain"].edits)
        for i in range(0, b.npairs, 7):
            assert np.array_equal(runs[name].ops(i), runs["plain"].ops(i))
    L, P = runs["learned"].stats, runs["plain"].stats
    assert L.rows_budgeted < 0.5 * P.rows_budgeted
    assert L.fallback_windows < runs["fixed7"].stats.fallback_windows
    assert L.rows_budgeted < runs["fixed15"].stats.rows_budgeted
