"""Seeded initial parameters of the step-size network (random draws only).

Layer sizes ``LAYERS`` = [16 features, 128, 128, 128, 6 outputs]; the flat
parameter vector lists, for each layer, its weight matrix [out][in]
(row-major) and then its bias [out].  Weights are uniform in
[-sqrt(6/in), sqrt(6/in)], biases zero, drawn with PCG64(seed).
"""

from __future__ import annotations

import numpy as np

LAYERS = [16, 128, 128, 128, 6]


def n_params(layers=LAYERS) -> int:
    return sum(o * i + o for i, o in zip(layers[:-1], layers[1:]))


def init_params(seed: int, layers=LAYERS) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for i, o in zip(layers[:-1], layers[1:]):
        lim = np.sqrt(6.0 / i)
        out.append(rng.uniform(-lim, lim, size=(o, i)).ravel())
        out.append(np.zeros(o))
    return np.concatenate(out)


def random_batch(seed: int, batch: int, layers=LAYERS):
    """Synthetic (features, targets, mask) for gradient checks: features N(0,1),
    five 0/1 targets, one real target, random mask."""
    rng = np.random.Generator(np.random.PCG64(seed))
    X = rng.standard_normal((batch, layers[0]))
    Y = np.concatenate([(rng.random((batch, layers[-1] - 1)) < 0.5).astype(float),
                        rng.uniform(0.0, 1.5, (batch, 1))], axis=1)
    M = (rng.random((batch, layers[-1])) < 0.8).astype(float)
    return X, Y, M
