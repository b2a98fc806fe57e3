"""Pins for the oracle's multiword value and exact-operation layer (hand-computed dyadic identities)."""

from fractions import Fraction

import numpy as np
import pytest

from oracle.arith import err_units, exact_complex, exact_real, scale_complex
from oracle.numbers import QC, cfrac, frac, to_limbs_real

E60 = 2.0**-60


def test_value_is_sum_of_limbs():
    assert frac([1.0, E60]) == 1 + Fraction(1, 2**60)
    assert frac([0.5, -(2.0**-80), 2.0**-140, 0.0]) == Fraction(1, 2) - Fraction(1, 2**80) + Fraction(1, 2**140)
    with pytest.raises(ValueError):
        frac([1.0, float("nan")])


def test_rounding_to_limbs_nonoverlapping():
    third = Fraction(1, 3)
    for L in (1, 2, 4):
        limbs = to_limbs_real(third, L)
        err = abs(frac(limbs) - third)
        # successive rounding: error at most half an ulp of the last limb, < 2^-(53L) * |x|
        assert err <= third * Fraction(1, 2 ** (53 * L - 1))
        for a, b in zip(limbs, limbs[1:]):
            assert abs(b) <= abs(a) * 2.0**-52


def test_exact_real_ops_hand_values():
    a = [1.0, E60]
    b = [1.0, -E60]
    assert exact_real("mul", a, b) == 1 - Fraction(1, 2**120)
    assert exact_real("add", a, b) == 2
    assert exact_real("sub", a, b) == Fraction(2, 2**60)
    assert exact_real("div", [3.0, 0.0], [4.0, 0.0]) == Fraction(3, 4)


def test_exact_complex_ops_hand_values():
    one_i = np.array([[1.0, 0.0], [1.0, 0.0]])  # 1 + i
    one_mi = np.array([[1.0, 0.0], [-1.0, 0.0]])  # 1 - i
    assert exact_complex("cmul", one_i, one_mi) == QC(2, 0)
    assert exact_complex("cdiv", one_i, one_mi) == QC(0, 1)
    two_i = np.array([[0.0, 0.0], [2.0, 0.0]])
    assert exact_complex("cinv", two_i, None) == QC(0, Fraction(-1, 2))
    # a - l*u with l = u = 1+i: (1+i)^2 = 2i
    assert exact_complex("cfms", one_i, one_i, one_i) == QC(1, -1)
    sre, sim = scale_complex("cmul", one_i, one_mi)
    assert (sre, sim) == (2, 2)
    assert cfrac(one_i) == QC(1, 1)


def test_err_units():
    L = 2
    exact = Fraction(1)
    u = Fraction(1, 2**106)
    assert err_units([1.0, 0.0], exact, Fraction(1), L) == 0.0
    assert err_units([1.0, 2.0**-106], exact, Fraction(1), L) == pytest.approx(1.0)
    assert err_units([1.0, 2.0**-103], exact, Fraction(2), L) == pytest.approx(float(Fraction(1, 2**103) / (2 * u)))


def test_rounding_keeps_precision_of_high_precision_inputs():
    # a value computed at high precision must not be re-rounded to the
    # caller's default mpmath precision when split into limbs
    import mpmath

    from oracle.numbers import to_limbs_complex

    with mpmath.workprec(400):
        v = mpmath.mpc(1, -2) / 3
    limbs = to_limbs_complex(v, 4)
    assert abs(frac(limbs[0]) - Fraction(1, 3)) < Fraction(1, 2**200)
    assert abs(frac(limbs[1]) + Fraction(2, 3)) < Fraction(1, 2**200)
