"""FP64 reference MLP with a hand-written backward pass and Adam (oracle).

Network: x (n_in) -> tanh(W1 x + b1) (n_h) -> tanh(W2 h1 + b2) (n_h) ->
y = W3 h2 + b3 (n_out).  Parameters are one flat vector in the order
W1 (n_h x n_in, row-major), b1, W2 (n_h x n_h), b2, W3 (n_out x n_h), b3.
Loss: mean over all batch entries and outputs of (y - t)^2.  Adam
(Kingma & Ba) with bias correction.  The backward pass is pinned by central
finite differences in the tests.
"""
from __future__ import annotations

import numpy as np


def shapes(n_in=8, n_h=64, n_out=27):
    return [(n_h, n_in), (n_h,), (n_h, n_h), (n_h,), (n_out, n_h), (n_out,)]


def n_params(n_in=8, n_h=64, n_out=27):
    return sum(int(np.prod(s)) for s in shapes(n_in, n_h, n_out))


def unpack(params, n_in=8, n_h=64, n_out=27):
    out = []
    off = 0
    for s in shapes(n_in, n_h, n_out):
        n = int(np.prod(s))
        out.append(np.asarray(params[off:off + n], dtype=np.float64).reshape(s))
        off += n
    return out


def init_params(seed, n_in=8, n_h=64, n_out=27):
    """Xavier-uniform weights, zero biases."""
    rng = np.random.default_rng(seed)
    parts = []
    for s in shapes(n_in, n_h, n_out):
        if len(s) == 2:
            a = np.sqrt(6.0 / (s[0] + s[1]))
            parts.append(rng.uniform(-a, a, size=s).reshape(-1))
        else:
            parts.append(np.zeros(s))
    return np.concatenate(parts)


def forward(params, X, n_in=8, n_h=64, n_out=27):
    W1, b1, W2, b2, W3, b3 = unpack(params, n_in, n_h, n_out)
    X = np.asarray(X, dtype=np.float64)
    H1 = np.tanh(X @ W1.T + b1)
    H2 = np.tanh(H1 @ W2.T + b2)
    Y = H2 @ W3.T + b3
    return Y, (X, H1, H2)


def loss(Y, T):
    D = Y - T
    return float(np.mean(D * D))


def loss_grad(Y, T):
    return 2.0 * (Y - T) / Y.size


def backward(params, cache, dY, n_in=8, n_h=64, n_out=27):
    """Gradient of sum(dY * Y) w.r.t. the flat parameters."""
    W1, b1, W2, b2, W3, b3 = unpack(params, n_in, n_h, n_out)
    X, H1, H2 = cache
    gW3 = dY.T @ H2
    gb3 = dY.sum(axis=0)
    dH2 = dY @ W3
    dA2 = dH2 * (1.0 - H2 * H2)
    gW2 = dA2.T @ H1
    gb2 = dA2.sum(axis=0)
    dH1 = dA2 @ W2
    dA1 = dH1 * (1.0 - H1 * H1)
    gW1 = dA1.T @ X
    gb1 = dA1.sum(axis=0)
    return np.concatenate([g.reshape(-1) for g in (gW1, gb1, gW2, gb2, gW3, gb3)])


def adam_step(params, grads, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns new (params, m, v)."""
    m = b1 * m + (1.0 - b1) * grads
    v = b2 * v + (1.0 - b2) * grads * grads
    mhat = m / (1.0 - b1 ** step)
    vhat = v / (1.0 - b2 ** step)
    return params - lr * mhat / (np.sqrt(vhat) + eps), m, v
