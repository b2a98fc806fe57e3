"""Shared pieces of the GPU parity tests (no oracle arithmetic here)."""

import json
import os
import sys

import mpmath
import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))


def say(*a):
    """Name the case before each GPU step (flushed, so a crash still shows it)."""
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def fixture(name):
    with open(os.path.join(HERE, "golden", f"path_{name}.json")) as fh:
        return json.load(fh)


def zss_mpc(fix):
    from oracle.numbers import mpc_of

    with mpmath.workprec(600):
        return [mpc_of(np.array(v)) for v in fix["zss_limbs"]]


def err_over_scale(got_limbs, ref_mpc, scale):
    """|got - ref| / scale as float (mpmath at 600 bits)."""
    from oracle.numbers import mpc_of

    with mpmath.workprec(600):
        d = abs(mpc_of(got_limbs) - ref_mpc)
        if scale == 0:
            return 0.0 if d == 0 else float("inf")
        return float(d / scale)


def start_power_bounds(L, t, gamma_limbs, x_limbs, d):
    """Rounding bounds of the start-system terms of the homotopy as the GPU
    forms them: x^d by binary powering in L limbs takes at most d - 1 roundings'
    worth of relative error (a rounding made at power k is carried into x^d
    with weight d/k; summed over the powering chain this is at most d - 1
    times the error of one complex product), each complex product rounds by
    at most 4u (u = 2^(-53 L)).  Returns (bound on |error| of (1-t) gamma x^d,
    bound on |error| of (1-t) gamma d x^(d-1))."""
    u = 2.0 ** (-53 * L)
    w = abs(1.0 - t) * abs(complex(float(np.sum(gamma_limbs[0])), float(np.sum(gamma_limbs[1]))))
    r = abs(complex(float(np.sum(x_limbs[0])), float(np.sum(x_limbs[1]))))
    return 4.0 * d * u * w * r ** d * 1.01, 4.0 * d * u * w * d * r ** max(d - 1, 0) * 1.01
