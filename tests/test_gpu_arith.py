"""Multiword arithmetic kernels vs exact rational results."""

from fractions import Fraction

import numpy as np
import pytest

from oracle.arith import err_units, exact_complex, exact_real, scale_complex, scale_real
from synth.systems import random_limbs
from tests.gpu_helpers import say

pytestmark = pytest.mark.gpu

# bound in units of u_L = 2^(-53L) times the componentwise scale of the op
BOUND = {1: {"add": 1, "sub": 1, "mul": 1, "div": 1, "cadd": 1, "csub": 1, "cmul": 2, "cdiv": 8, "cfms": 4,
             "cinv": 8},
         2: {"add": 4, "sub": 4, "mul": 6, "div": 12, "cadd": 4, "csub": 4, "cmul": 8, "cdiv": 32, "cfms": 16,
             "cinv": 32},
         4: {"add": 16, "sub": 16, "mul": 32, "div": 64, "cadd": 16, "csub": 16, "cmul": 64, "cdiv": 256,
             "cfms": 128, "cinv": 256}}


def _dev(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _run(op, L, *arrs):
    import paper_1109_0545_amd as q

    say("arith", op, "L", L, "count", arrs[0].shape[0])
    d = [_dev(a) for a in arrs]
    while len(d) < 3:
        d.append(None)
    out = q.arith_batch(op, L, d[0], d[1], d[2])
    return out.cpu().numpy()


def _cases(L, count, seed, spread):
    return random_limbs((count,), L, seed, exp_spread=spread)


@pytest.mark.parametrize("L", [1, 2, 4])
@pytest.mark.parametrize("op", ["add", "sub", "mul", "div"])
def test_real_ops_random(L, op):
    a = _cases(L, 300, 11 + L, 6)
    b = _cases(L, 300, 23 + L, 6)
    out = _run(op, L, a, b)
    worst = 0.0
    for k in range(a.shape[0]):
        e = err_units(out[k], exact_real(op, a[k], b[k]), scale_real(op, a[k], b[k]), L)
        worst = max(worst, e)
    assert worst <= BOUND[L][op], worst


@pytest.mark.parametrize("L", [2, 4])
def test_add_cancellation_and_limb_gaps(L):
    # a + b with b = -a + tiny perturbation, and limbs with wide gaps
    a = _cases(L, 200, 5, 3)
    b = -a.copy()
    b[:, -1] += np.ldexp(a[:, 0], -53 * L - 3)
    out = _run("add", L, a, b)
    for k in range(a.shape[0]):
        ex = exact_real("add", a[k], b[k])
        e = err_units(out[k], ex, scale_real("add", a[k], b[k]), L)
        assert e <= BOUND[L]["add"], (k, e)
    gap = np.zeros((50, L))
    gap[:, 0] = 1.0
    gap[:, L - 1] = np.ldexp(1.0, -300)  # a huge gap between limbs
    out = _run("mul", L, gap, gap)
    for k in range(50):
        e = err_units(out[k], exact_real("mul", gap[k], gap[k]), scale_real("mul", gap[k], gap[k]), L)
        assert e <= BOUND[L]["mul"]


@pytest.mark.parametrize("L", [1, 2, 4])
@pytest.mark.parametrize("op", ["cadd", "csub", "cmul", "cdiv", "cfms", "cinv"])
def test_complex_ops_random(L, op):
    a = random_limbs((200, 2), L, 101 + L, 4)
    b = random_limbs((200, 2), L, 202 + L, 4)
    c = random_limbs((200, 2), L, 303 + L, 4)
    out = _run(op, L, a, b, c)
    worst = 0.0
    for k in range(a.shape[0]):
        ex = exact_complex(op, a[k], b[k], c[k])
        sre, sim = scale_complex(op, a[k], b[k], c[k])
        worst = max(worst, err_units(out[k][0], ex.re, sre, L), err_units(out[k][1], ex.im, sim, L))
    assert worst <= BOUND[L][op], worst


@pytest.mark.parametrize("L", [2, 4])
def test_zero_and_exact_cases(L):
    z = np.zeros((4, 2, L))
    one = np.zeros((4, 2, L))
    one[:, 0, 0] = 1.0
    out = _run("cmul", L, z, one)
    assert np.all(out == 0.0)
    out = _run("cmul", L, one, one)
    assert np.all(out == one)
    out = _run("cinv", L, one)
    assert np.all(out == one)
