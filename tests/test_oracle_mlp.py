"""Pins of the FP64 MLP cost-model oracle."""
import numpy as np
import pytest

import synth
from oracle import mlp


def _data(n=50, k=4, seed=0):
    rng = np.random.default_rng(seed)
    shapes = [(int(rng.integers(16, 4097)), int(rng.integers(16, 4097)), int(rng.integers(16, 4097)),
               int(rng.integers(1, 65)), int(rng.integers(0, 2)), int(rng.integers(0, 2)))
              for _ in range(n)]
    X = mlp.features(shapes)
    Y = rng.uniform(0, 1, size=(n, k))
    return X, Y


def test_features_closed_form():
    X = mlp.features([(4096, 16, 1, 64, 1, 0)])
    assert X.tolist() == [[1.0, 4 / 12, 0.0, 1.0, 1.0, 0.0]]


def test_gradients_vs_central_differences():
    X, Y = _data()
    p = synth.mlp_init(4)
    rng = np.random.default_rng(1)
    for name in mlp.PARAM_ORDER:            # nonzero biases so every path is exercised
        if name.startswith("b"):
            p[name] = rng.uniform(-0.1, 0.1, size=p[name].shape)
    g, _ = mlp.grads(p, X, Y)
    h = 1e-6
    for name in mlp.PARAM_ORDER:
        flat = p[name].reshape(-1)
        for idx in rng.choice(flat.size, size=min(12, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + h
            lp = mlp.loss(p, X, Y)
            flat[idx] = old - h
            lm = mlp.loss(p, X, Y)
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            an = g[name].reshape(-1)[idx]
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)) + 1e-9, (name, idx, fd, an)


def test_zero_network_closed_form():
    X, Y = _data(n=20, k=3)
    p = {k: np.zeros_like(v) for k, v in synth.mlp_init(3).items()}
    p["b3"] = np.array([0.1, -0.2, 0.3])
    y, _ = mlp.forward(p, X)
    assert np.array_equal(y, np.broadcast_to(p["b3"], y.shape))
    g, _ = mlp.grads(p, X, Y)
    n, k = Y.shape
    assert np.allclose(g["b3"], 2 * (p["b3"][None, :] - Y).sum(axis=0) / (n * k), rtol=0, atol=1e-15)
    for name in ("W1", "b1", "W2", "b2", "W3"):
        assert not g[name].any()


def test_first_adam_step_closed_form():
    X, Y = _data(n=30, k=4)
    p0 = synth.mlp_init(4)
    g, _ = mlp.grads(p0, X, Y)
    p1, _ = mlp.train(p0, X, Y, 1, lr=1e-3)
    for name in mlp.PARAM_ORDER:
        want = p0[name] - 1e-3 * g[name] / (np.abs(g[name]) + 1e-8)
        assert np.allclose(p1[name], want, rtol=1e-12, atol=1e-15)


def test_against_torch_autograd():
    torch = pytest.importorskip("torch")
    X, Y = _data(n=40, k=5, seed=3)
    p = synth.mlp_init(5)
    g, l = mlp.grads(p, X, Y)
    tp = {k: torch.tensor(v, dtype=torch.float64, requires_grad=True) for k, v in p.items()}
    tX, tY = torch.tensor(X), torch.tensor(Y)
    h1 = torch.relu(tX @ tp["W1"].T + tp["b1"])
    h2 = torch.relu(h1 @ tp["W2"].T + tp["b2"])
    out = h2 @ tp["W3"].T + tp["b3"]
    loss = torch.mean((out - tY) ** 2)
    loss.backward()
    assert abs(loss.item() - l) < 1e-12
    for k in mlp.PARAM_ORDER:
        assert np.allclose(tp[k].grad.numpy(), g[k], rtol=1e-10, atol=1e-14)
    # Adam against torch.optim.Adam for a few steps
    tp2 = {k: torch.tensor(v, dtype=torch.float64, requires_grad=True) for k, v in p.items()}
    opt = torch.optim.Adam([tp2[k] for k in mlp.PARAM_ORDER], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    for _ in range(5):
        opt.zero_grad()
        h1 = torch.relu(tX @ tp2["W1"].T + tp2["b1"])
        h2 = torch.relu(h1 @ tp2["W2"].T + tp2["b2"])
        torch.mean((h2 @ tp2["W3"].T + tp2["b3"] - tY) ** 2).backward()
        opt.step()
    p5, _ = mlp.train(p, X, Y, 5)
    for k in mlp.PARAM_ORDER:
        assert np.allclose(tp2[k].detach().numpy(), p5[k], rtol=1e-9, atol=1e-12)


def test_training_reduces_loss_and_select_is_argmax():
    X, Y = _data(n=60, k=3, seed=4)
    p, losses = mlp.train(synth.mlp_init(3), X, Y, 200)
    assert losses[-1] < losses[0]
    y, _ = mlp.forward(p, X)
    assert np.array_equal(mlp.select(p, X), np.argmax(y, axis=1))
