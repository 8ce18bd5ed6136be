"""GPU parity of the surrogate network's kernels against the float64 oracle:
forward values, batch gradients (1e-4 normwise) and parameters after 20
Adam steps (1e-3 normwise), on seeded inputs through the C ABI."""
import numpy as np
import pytest
import torch

import synth
from oracle import mlp as O
from paper_1303_5164_amd import surrogate as S

pytestmark = pytest.mark.gpu


def _data(n=512, seed=3):
    x = synth.uniform_f32(seed, synth.STREAM["synthk"], n * 16, -1.0, 1.0).reshape(n, 16)
    t = (np.sin(3.0 * x[:, 0]) + x[:, 1] * x[:, 2] - 0.5 * x[:, 3] ** 2).astype(np.float32)
    order = np.argsort(synth.raw_u64(seed, synth.STREAM["mlp_shuffle"], n), kind="stable")
    return x, t, order.astype(np.int32)


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


def test_forward_matches_oracle():
    theta = S.init_params(0)
    x, _, _ = _data(300)
    net = S.Net(theta)
    y = net.forward(torch.from_numpy(x).cuda()).cpu().numpy()
    ref, _ = O.forward(theta.astype(np.float64), x.astype(np.float64))
    assert _rel(y, ref) < 1e-5


@pytest.mark.parametrize("batch", [1, 64, 300])
def test_gradient_matches_oracle(batch):
    theta = S.init_params(1)
    x, t, order = _data()
    idx = order[:batch]
    net = S.Net(theta)
    g = net.grad(torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda(),
                 torch.from_numpy(idx).cuda()).cpu().numpy()
    ref = O.grad(theta.astype(np.float64), x[idx].astype(np.float64), t[idx].astype(np.float64))
    assert _rel(g, ref) < 1e-4


def test_adam_steps_match_oracle():
    theta = S.init_params(2)
    x, t, order = _data()
    batch, steps = 64, 20
    net = S.Net(theta)
    xd, td = torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda()
    th = theta.astype(np.float64)
    m = np.zeros_like(th)
    v = np.zeros_like(th)
    for s in range(steps):
        idx = order[(s * batch) % 512:(s * batch) % 512 + batch]
        net.train_step(xd, td, torch.from_numpy(idx).cuda(), lr=1e-3)
        g = O.grad(th, x[idx].astype(np.float64), t[idx].astype(np.float64))
        th, m, v = O.adam_step(th, m, v, g, s + 1, lr=1e-3)
    torch.cuda.synchronize()
    assert _rel(net.params(), th) < 1e-3
    # and it learned: the loss fell
    assert O.loss(net.params().astype(np.float64), x, t) < O.loss(theta.astype(np.float64), x, t)
