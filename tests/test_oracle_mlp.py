"""Pins of the oracle MLP: gradients against central finite differences and
against torch autograd (float64, CPU), Adam against torch.optim.Adam."""
import numpy as np
import torch

import synth
from oracle import mlp


def _theta(seed=0):
    u = synth.uniform_f32(seed, synth.STREAM["mlp_init"], mlp.NPARAM, -0.3, 0.3)
    return u.astype(np.float64)


def _data(n=37):
    x = synth.uniform_f32(1, 5, n * 16, 0.0, 1.0).reshape(n, 16).astype(np.float64)
    t = synth.uniform_f32(1, 6, n, 0.5, 2.0).astype(np.float64)
    return x, t


def test_param_count():
    assert mlp.NPARAM == 5313


def test_gradient_finite_differences():
    th = _theta()
    x, t = _data()
    g = mlp.grad(th, x, t)
    rng = np.random.default_rng(0)
    for i in rng.choice(mlp.NPARAM, 60, replace=False):
        e = np.zeros_like(th)
        e[i] = 1e-6
        fd = (mlp.loss(th + e, x, t) - mlp.loss(th - e, x, t)) / 2e-6
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])) + 1e-8


def _torch_net(th):
    parts = [torch.tensor(p, dtype=torch.float64, requires_grad=True)
             for p in mlp.unpack(th)]
    return parts


def test_gradient_matches_torch_autograd():
    th = _theta(3)
    x, t = _data(50)
    W1, b1, W2, b2, W3, b3 = _torch_net(th)
    X = torch.tensor(x)
    y = (torch.relu(torch.relu(X @ W1 + b1) @ W2 + b2) @ W3 + b3)[:, 0]
    loss = torch.mean((y - torch.tensor(t)) ** 2)
    loss.backward()
    ref = np.concatenate([p.grad.numpy().ravel() for p in (W1, b1, W2, b2, W3, b3)])
    assert np.max(np.abs(mlp.grad(th, x, t) - ref)) < 1e-12
    assert abs(mlp.loss(th, x, t) - loss.item()) < 1e-12


def test_adam_matches_torch():
    th = _theta(4)
    x, t = _data(64)
    order = np.stack([np.arange(64), np.arange(64)[::-1]])
    got = mlp.train(th.copy(), x, t, epochs=2, batch=16, order=order, lr=1e-3)
    parts = _torch_net(th)
    opt = torch.optim.Adam(parts, lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    X, T = torch.tensor(x), torch.tensor(t)
    for e in range(2):
        for s in range(0, 64, 16):
            idx = torch.tensor(order[e][s:s + 16])
            W1, b1, W2, b2, W3, b3 = parts
            y = (torch.relu(torch.relu(X[idx] @ W1 + b1) @ W2 + b2) @ W3 + b3)[:, 0]
            opt.zero_grad()
            torch.mean((y - T[idx]) ** 2).backward()
            opt.step()
    ref = np.concatenate([p.detach().numpy().ravel() for p in parts])
    assert np.max(np.abs(got - ref)) < 1e-10
