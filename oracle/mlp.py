"""Float64 reference of the load predictor's network (test infrastructure).

A 6 -> 64 -> 64 -> 1 multilayer perceptron with ReLU hidden layers, mean
squared error, and the Adam update (Kingma and Ba, ICLR 2015).  Parameters
are one flat vector in this order:

    W1[64][6], b1[64], W2[64][64], b2[64], W3[64], b3       (4,673 values)

followed, in the full weight buffer, by the input normalisation
mean[6], std[6] (features are used as (x - mean) / std).

Written from the definitions with plain numpy: forward pass, chain rule by
hand for the backward pass.  Pinned by central finite differences and by
closed forms in tests/test_oracle_mlp.py.
"""
from __future__ import annotations

import numpy as np

D_IN, H1, H2 = 6, 64, 64
N_PARAMS = H1 * D_IN + H1 + H2 * H1 + H2 + H2 + 1          # 4673
N_WEIGHTS = N_PARAMS + 2 * D_IN                              # + mean, std


def unpack(p: np.ndarray):
    p = np.asarray(p, dtype=np.float64)
    o = 0
    W1 = p[o:o + H1 * D_IN].reshape(H1, D_IN); o += H1 * D_IN
    b1 = p[o:o + H1]; o += H1
    W2 = p[o:o + H2 * H1].reshape(H2, H1); o += H2 * H1
    b2 = p[o:o + H2]; o += H2
    W3 = p[o:o + H2]; o += H2
    b3 = p[o]; o += 1
    return W1, b1, W2, b2, W3, b3


def pack(W1, b1, W2, b2, W3, b3) -> np.ndarray:
    return np.concatenate([np.ravel(W1), b1, np.ravel(W2), b2, W3, [b3]]).astype(np.float64)


def normalise(x: np.ndarray, mean: np.ndarray, std: np.ndarray) -> np.ndarray:
    return (np.asarray(x, dtype=np.float64) - mean) / std


def forward(p: np.ndarray, x: np.ndarray):
    """Predictions and the intermediate values needed by backward (x already normalised)."""
    W1, b1, W2, b2, W3, b3 = unpack(p)
    x = np.asarray(x, dtype=np.float64)
    z1 = x @ W1.T + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2.T + b2
    h2 = np.maximum(z2, 0.0)
    out = h2 @ W3 + b3
    return out, (x, z1, h1, z2, h2)


def loss(p: np.ndarray, x: np.ndarray, y: np.ndarray) -> float:
    out, _ = forward(p, x)
    return float(np.mean((out - np.asarray(y, dtype=np.float64)) ** 2))


def grad(p: np.ndarray, x: np.ndarray, y: np.ndarray):
    """Loss (mean squared error over the batch) and its gradient, by the chain rule."""
    W1, b1, W2, b2, W3, b3 = unpack(p)
    out, (x, z1, h1, z2, h2) = forward(p, x)
    B = x.shape[0]
    r = out - np.asarray(y, dtype=np.float64)
    L = float(np.mean(r ** 2))
    d_out = 2.0 * r / B                      # dL/d out
    gW3 = h2.T @ d_out
    gb3 = d_out.sum()
    d_h2 = np.outer(d_out, W3)               # dL/d h2
    d_z2 = d_h2 * (z2 > 0)
    gW2 = d_z2.T @ h1
    gb2 = d_z2.sum(axis=0)
    d_h1 = d_z2 @ W2
    d_z1 = d_h1 * (z1 > 0)
    gW1 = d_z1.T @ x
    gb1 = d_z1.sum(axis=0)
    return L, pack(gW1, gb1, gW2, gb2, gW3, gb3)


def adam_step(p, g, m, v, step: int, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step counts from 1).  Returns new (p, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    return p - lr * mhat / (np.sqrt(vhat) + eps), m, v


def train(p, x, y, epochs: int, batch: int, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """Minibatch Adam over the samples in the given order, epoch after epoch.
    Returns parameters and per-step losses."""
    p = np.array(p, dtype=np.float64)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    S = x.shape[0]
    step = 0
    losses = []
    for _ in range(epochs):
        for s0 in range(0, S, batch):
            xb, yb = x[s0:s0 + batch], y[s0:s0 + batch]
            L, g = grad(p, xb, yb)
            step += 1
            p, m, v = adam_step(p, g, m, v, step, lr, beta1, beta2, eps)
            losses.append(L)
    return p, np.array(losses)
