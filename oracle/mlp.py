"""FP64 reference of the rank-predicting multilayer perceptron (test
infrastructure only; the paper has no learned component -- this network and
its loss are choices of this library, not of the paper).

Network: x (32) -> ReLU(W1 x + b1) (64) -> ReLU(W2 h1 + b2) (64) -> W3 h2 + b3 (1).
The forward pass uses the weights rounded to bfloat16 (round to nearest even),
as the device does; biases stay FP32.  Loss: asymmetric Huber on
e = prediction - label (label = log of the kept rank), weight 4 when e < 0
(an under-predicted rank forces a fallback), threshold 1, mean over the batch.
The gradient is taken w.r.t. the FP32 master weights through the rounding as
the identity (straight-through), matching the device.

Parameter vector order: W1 (64x32, row-major), b1, W2 (64x64), b2, W3 (1x64), b3.
"""

from __future__ import annotations

import numpy as np

SIZES = [(64, 32), (64,), (64, 64), (64,), (1, 64), (1,)]
N_PARAMS = sum(int(np.prod(s)) for s in SIZES)
UNDER_WEIGHT = 4.0
HUBER_DELTA = 1.0


def unpack(p):
    out, o = [], 0
    for s in SIZES:
        n = int(np.prod(s))
        out.append(np.asarray(p[o:o + n], dtype=np.float64).reshape(s))
        o += n
    return out


def bf16_round(x):
    """float32 -> bfloat16 -> float32, round to nearest even (finite inputs)."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)


def forward(params, X, quantize: bool = True):
    W1, b1, W2, b2, W3, b3 = unpack(params)
    q = (lambda W: bf16_round(W).astype(np.float64)) if quantize else (lambda W: W)
    W1q, W2q, W3q = q(W1), q(W2), q(W3)
    X = np.asarray(X, dtype=np.float64)
    z1 = X @ W1q.T + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2q.T + b2
    h2 = np.maximum(z2, 0.0)
    y = (h2 @ W3q.T)[:, 0] + b3[0]
    return y, (X, z1, h1, z2, h2, W2q, W3q)


def loss_and_grad(params, X, labels, quantize: bool = True):
    y, (X, z1, h1, z2, h2, W2q, W3q) = forward(params, X, quantize)
    e = y - np.asarray(labels, dtype=np.float64)
    w = np.where(e < 0, UNDER_WEIGHT, 1.0)
    a = np.abs(e)
    per = np.where(a <= HUBER_DELTA, 0.5 * e * e, HUBER_DELTA * (a - 0.5 * HUBER_DELTA))
    B = len(e)
    loss = float(np.sum(w * per) / B)
    g = w * np.clip(e, -HUBER_DELTA, HUBER_DELTA) / B          # dL/dy
    dW3 = g[None, :] @ h2                                        # (1, 64)
    db3 = np.array([g.sum()])
    dh2 = np.outer(g, W3q[0]) * (z2 > 0)
    dW2 = dh2.T @ h1
    db2 = dh2.sum(0)
    dh1 = (dh2 @ W2q) * (z1 > 0)
    dW1 = dh1.T @ X
    db1 = dh1.sum(0)
    grad = np.concatenate([dW1.ravel(), db1, dW2.ravel(), db2, dW3.ravel(), db3])
    return loss, grad


def features(spectrum, floor=1e-30):
    """32 leading log(s_j / s_0) of a descending spectrum, padded with log(floor)."""
    s = np.zeros(32)
    sp = np.asarray(spectrum, dtype=np.float64)[:32]
    s[:len(sp)] = sp
    out = np.full(32, np.log(floor))
    if s[0] > 0:
        r = s / s[0]
        ok = r > floor
        out[ok] = np.log(r[ok])
    return out


def adam_step(params, grad, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015, Algorithm 1) of the FP32 master
    parameters; step is the 1-based update count.  Returns (params, m, v)."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mhat = m / (1 - b1 ** step)
    vhat = v / (1 - b2 ** step)
    return params - lr * mhat / (np.sqrt(vhat) + eps), m, v
