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


@pytest.mark.parametrize("L", [1, 2, 4])
def test_pivot_search_matches_argmax(L):
    # the wavefront maximum the elimination uses to pick pivots: per group of
    # 64, the index of the largest |Re| + |Im| of the leading limbs, compared
    # on the high 32 bits of that FP64 value, ties to the lowest index
    import torch

    import paper_1109_0545_amd as q

    rng = np.random.Generator(np.random.PCG64(40 + L))
    groups = 60
    a = np.zeros((groups * 64, 2, L))
    a[:, :, 0] = rng.standard_normal((groups * 64, 2)) * np.exp(rng.uniform(-30, 30, (groups * 64, 1)))
    a[:64, :, 0] = 1.0                      # all equal: index 0
    a[64:128, :, 0] = 0.0                   # all zero: no pivot
    a[64 + 17, 0, 0] = -3e-300              # one tiny nonzero: index 17
    a[128:192, :, 0] = rng.uniform(0.5, 1.0, (64, 2))
    a[128 + 40] = a[128 + 5] = [[7.0] + [0.0] * (L - 1), [-2.0] + [0.0] * (L - 1)]  # tie: 5
    a[192 + 63, 1, 0] = 1e300                # the last lane
    say("pivot search L", L)
    out = q.arith_batch("pivot", L, torch.from_numpy(a).cuda()).cpu().numpy()[:, 0]
    key = np.abs(a[:, 0, 0]) + np.abs(a[:, 1, 0])
    hi = (key.view(np.uint64) >> np.uint64(32)).reshape(groups, 64)
    for g in range(groups):
        got = out[g * 64: (g + 1) * 64]
        assert np.all(got == got[0])  # every lane holds the group's answer
        if np.all(key[g * 64: (g + 1) * 64] == 0):
            assert got[0] == -1
        else:
            assert got[0] == int(np.flatnonzero(hi[g] == hi[g].max())[0]), g
    assert out[0] == 0 and out[64] == 17 and out[128] == 5 and out[192] == 63
