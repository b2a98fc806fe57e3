"""Pins for the FP64 network reference: finite differences, loss value, Adam's first step."""

import numpy as np
import pytest

from oracle.mlp import adam_step, loss, loss_and_grad
from synth.policy import init_params, n_params, random_batch

SMALL = [4, 6, 5, 3]


def test_gradient_matches_central_differences():
    p = init_params(3, SMALL)
    X, Y, M = random_batch(4, 7, SMALL)
    _, g = loss_and_grad(p, X, Y, M, SMALL)
    h = 1e-6
    for idx in range(0, p.size, 3):
        e = np.zeros_like(p)
        e[idx] = h
        fd = (loss(p + e, X, Y, M, SMALL) - loss(p - e, X, Y, M, SMALL)) / (2 * h)
        assert abs(fd - g[idx]) <= 1e-6 * max(1.0, abs(fd)), idx


def test_loss_at_zero_logits_is_log2_per_target():
    p = np.zeros(n_params(SMALL))
    X, Y, M = random_batch(5, 9, SMALL)
    Y[:, -1] = 0.0
    expect = (M[:, :-1].sum() * np.log(2.0)) / X.shape[0]
    assert abs(loss(p, X, Y, M, SMALL) - expect) < 1e-14


def test_first_adam_step_moves_by_lr_sign():
    p = init_params(6, SMALL)
    g = np.linspace(-1, 1, p.size)
    g[g == 0] = 0.5
    p1, _, _ = adam_step(p, g, np.zeros_like(p), np.zeros_like(p), 1, lr=1e-3, eps=1e-12)
    assert np.allclose(p1 - p, -1e-3 * np.sign(g), rtol=0, atol=1e-12)


def test_default_layout_size():
    assert n_params() == 16 * 128 + 128 + 2 * (128 * 128 + 128) + 128 * 6 + 6


def test_three_adam_steps_by_hand():
    # Adam (Kingma & Ba) with bias correction, written out for one scalar parameter and the
    # gradients 1/2, -1/4, 1 in exact rationals: m_k = b1 m + (1-b1) g, v_k = b2 v + (1-b2) g^2,
    # p -= lr (m_k / (1 - b1^k)) / (sqrt(v_k / (1 - b2^k)) + eps).  Dropping the bias
    # correction, using k-1 for k, or putting eps under the root changes steps 2 and 3.
    from fractions import Fraction as F
    import math

    b1, b2, lr, eps = F(9, 10), F(999, 1000), 0.1, 1e-8
    grads = [F(1, 2), F(-1, 4), F(1)]
    m = v = F(0)
    p_ref = 1.0
    expect = []
    for k, g in enumerate(grads, start=1):
        m = b1 * m + (1 - b1) * g
        v = b2 * v + (1 - b2) * g * g
        mh = m / (1 - b1**k)
        vh = v / (1 - b2**k)
        p_ref = p_ref - lr * float(mh) / (math.sqrt(float(vh)) + eps)
        expect.append(p_ref)
    # the first two values, also by hand: step 1 moves by lr * (1/2)/(1/2 + eps);
    # step 2 has m = 1/50, v = 31225/10^8, mh = 2/19, vh = 31225/199900
    assert expect[0] == pytest.approx(1.0 - 0.1 * 0.5 / (0.5 + 1e-8), rel=1e-15)
    assert expect[1] == pytest.approx(expect[0] - 0.1 * (2 / 19) / (math.sqrt(31225 / 199900) + 1e-8), rel=1e-15)

    p = np.array([1.0])
    mm = np.zeros(1)
    vv = np.zeros(1)
    for k, g in enumerate(grads, start=1):
        p, mm, vv = adam_step(p, np.array([float(g)]), mm, vv, k, lr=lr, b1=0.9, b2=0.999, eps=eps)
        assert p[0] == pytest.approx(expect[k - 1], rel=1e-14, abs=1e-15), k
