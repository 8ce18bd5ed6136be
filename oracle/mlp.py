"""CPU ORACLE -- TEST INFRASTRUCTURE ONLY.

The surrogate network that ranks candidate co-schedules: a fully connected
16 -> 64 -> 64 -> 1 network with ReLU hidden layers, mean-squared-error
loss and the Adam optimiser (Kingma & Ba, 2015: m = b1 m + (1-b1) g,
v = b2 v + (1-b2) g^2, w -= lr * (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps)),
in float64.  Parameters are row-major: W1 [16,64], b1 [64], W2 [64,64],
b2 [64], W3 [64,1], b3 [1] (5313 numbers), packed in that order.
Initial values are inputs (drawn by the seeded generator), not drawn here.
"""
from __future__ import annotations

import numpy as np

SHAPES = [(16, 64), (64,), (64, 64), (64,), (64, 1), (1,)]
NPARAM = sum(int(np.prod(s)) for s in SHAPES)


def unpack(theta):
    out, o = [], 0
    for s in SHAPES:
        n = int(np.prod(s))
        out.append(np.asarray(theta[o:o + n], dtype=np.float64).reshape(s))
        o += n
    return out


def pack(parts):
    return np.concatenate([np.asarray(p, np.float64).reshape(-1) for p in parts])


def forward(theta, x):
    W1, b1, W2, b2, W3, b3 = unpack(theta)
    z1 = x @ W1 + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2 + b2
    h2 = np.maximum(z2, 0.0)
    y = (h2 @ W3 + b3)[:, 0]
    return y, (x, z1, h1, z2, h2)


def loss(theta, x, t):
    y, _ = forward(theta, x)
    return float(np.mean((y - t) ** 2))


def grad(theta, x, t):
    """Gradient of the mean-squared error with respect to theta."""
    W1, b1, W2, b2, W3, b3 = unpack(theta)
    y, (x, z1, h1, z2, h2) = forward(theta, x)
    n = x.shape[0]
    dy = 2.0 * (y - t) / n                 # [n]
    gW3 = h2.T @ dy[:, None]
    gb3 = np.array([dy.sum()])
    dh2 = dy[:, None] @ W3.T
    dz2 = dh2 * (z2 > 0)
    gW2 = h1.T @ dz2
    gb2 = dz2.sum(0)
    dh1 = dz2 @ W2.T
    dz1 = dh1 * (z1 > 0)
    gW1 = x.T @ dz1
    gb1 = dz1.sum(0)
    return pack([gW1, gb1, gW2, gb2, gW3, gb3])


def adam_step(theta, m, v, g, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (step counts from 1).  Returns new (theta, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def train(theta, x, t, epochs, batch, order, lr=1e-3):
    """Mini-batch Adam.  `order` [epochs, n] gives the sample order of each
    epoch (an input).  Returns the final theta."""
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    step = 0
    n = x.shape[0]
    for e in range(epochs):
        for s in range(0, n, batch):
            idx = order[e][s:s + batch]
            step += 1
            g = grad(theta, x[idx], t[idx])
            theta, m, v = adam_step(theta, m, v, g, step, lr)
    return theta
