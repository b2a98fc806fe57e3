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
