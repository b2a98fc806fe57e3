"""FP64 reference of the step-size network (not in the paper).

A multilayer perceptron 16 -> 128 -> 128 -> 128 -> 6 with ReLU hidden layers.
Outputs 0..4 are acceptance logits for the step multipliers 2^-1, 2^0, 2^1,
2^2, 2^3; output 5 is the secant blend weight.  Loss over a batch of B rows
with targets Y and 0/1 mask M:

    loss = (1/B) sum_b [ sum_{k<5} M_bk BCE(o_bk, Y_bk) + M_b5 (o_b5 - Y_b5)^2 ]
    BCE(o, y) = max(o, 0) - o y + log(1 + exp(-|o|))

Gradients by the chain rule written out layer by layer; Adam with bias
correction.  The flat parameter layout is that of ``synth.policy``.

Parity: pinned in ``tests/test_oracle_mlp.py`` by central finite differences
in FP64, the value log 2 of the loss at zero logits, the first Adam step
(which moves every parameter with a nonzero gradient by lr * sign(g) up to eps)
and three Adam steps written out in exact rationals (bias correction).
"""

from __future__ import annotations

import numpy as np

LAYERS = [16, 128, 128, 128, 6]


def unpack(p, layers=LAYERS):
    out, off = [], 0
    for i, o in zip(layers[:-1], layers[1:]):
        W = p[off: off + o * i].reshape(o, i)
        off += o * i
        b = p[off: off + o]
        off += o
        out.append((W, b))
    return out


def forward(p, X, layers=LAYERS):
    """Returns (outputs, list of layer inputs H_0=X, H_1, ...)."""
    hs = [np.asarray(X, dtype=np.float64)]
    params = unpack(p, layers)
    for li, (W, b) in enumerate(params):
        z = hs[-1] @ W.T + b
        if li < len(params) - 1:
            z = np.maximum(z, 0.0)
        hs.append(z)
    return hs[-1], hs


def loss(p, X, Y, M, layers=LAYERS) -> float:
    o, _ = forward(p, X, layers)
    B = o.shape[0]
    lo = o[:, :-1]
    bce = np.maximum(lo, 0) - lo * Y[:, :-1] + np.log1p(np.exp(-np.abs(lo)))
    mse = (o[:, -1] - Y[:, -1]) ** 2
    return float(((M[:, :-1] * bce).sum() + (M[:, -1] * mse).sum()) / B)


def loss_and_grad(p, X, Y, M, layers=LAYERS):
    o, hs = forward(p, X, layers)
    B = o.shape[0]
    g = np.zeros_like(o)
    lo = o[:, :-1]
    g[:, :-1] = M[:, :-1] * (1.0 / (1.0 + np.exp(-lo)) - Y[:, :-1]) / B
    g[:, -1] = M[:, -1] * 2.0 * (o[:, -1] - Y[:, -1]) / B
    params = unpack(p, layers)
    grads = []
    dz = g
    for li in range(len(params) - 1, -1, -1):
        W, _ = params[li]
        h = hs[li]
        dW = dz.T @ h
        db = dz.sum(axis=0)
        grads.append((dW, db))
        if li > 0:
            dh = dz @ W
            dz = dh * (hs[li] > 0)
    grads.reverse()
    flat = np.concatenate([np.concatenate([dW.ravel(), db]) for dW, db in grads])
    return loss(p, X, Y, M, layers), flat


def adam_step(p, g, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns new (p, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
