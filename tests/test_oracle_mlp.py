"""Pins for the FP64 network reference: finite differences, loss value, Adam's first step."""

import numpy as np

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
