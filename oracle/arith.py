"""Exact results of the multiword operations (the arithmetic layer).

The paper runs every step in double-double or quad-double complex arithmetic
(Section 1; Section 2 quotes the ~8x cost of double doubles over doubles).
An operation on multiword inputs is checked against the exact rational result
of the same operation on the exact input values, with an error bound in units
of u_L = 2^(-53L) times a componentwise scale:

* real add/sub:      scale |a| + |b|
* real mul:          scale |a b|
* real div:          scale |a / b|
* complex add/sub:   per component, |a_re| + |b_re| (resp. im)
* complex mul:       re: |a_re b_re| + |a_im b_im|;  im: |a_re b_im| + |a_im b_re|
* complex fma a-l*u: re: |a_re| + |l_re u_re| + |l_im u_im|;  im likewise
* complex div/inv:   |a/b| (modulus of the exact quotient) for both components

Parity: exact by construction (Fraction arithmetic); pinned in
``tests/test_oracle_numbers_arith.py`` by hand-computed dyadic identities.
"""

from __future__ import annotations

from fractions import Fraction

from .numbers import QC, cfrac, frac

OPS_REAL = ("add", "sub", "mul", "div")
OPS_COMPLEX = ("cadd", "csub", "cmul", "cdiv", "cfms", "cinv")


def exact_real(op: str, a, b) -> Fraction:
    x, y = frac(a), frac(b)
    if op == "add":
        return x + y
    if op == "sub":
        return x - y
    if op == "mul":
        return x * y
    if op == "div":
        return x / y
    raise ValueError(op)


def scale_real(op: str, a, b) -> Fraction:
    x, y = frac(a), frac(b)
    if op in ("add", "sub"):
        return abs(x) + abs(y)
    if op == "mul":
        return abs(x * y)
    if op == "div":
        return abs(x / y)
    raise ValueError(op)


def exact_complex(op: str, a, b, c=None) -> QC:
    """Exact complex result.  ``cfms`` is ``a - b*c``; ``cinv`` is ``1/a``."""
    x = cfrac(a)
    if op == "cinv":
        return QC(1) / x
    y = cfrac(b)
    if op == "cadd":
        return x + y
    if op == "csub":
        return x - y
    if op == "cmul":
        return x * y
    if op == "cdiv":
        return x / y
    if op == "cfms":
        return x - y * cfrac(c)
    raise ValueError(op)


def _mod_upper(q: QC) -> Fraction:
    # |q| <= |re| + |im|; used as a rational stand-in for the modulus
    return abs(q.re) + abs(q.im)


def scale_complex(op: str, a, b, c=None):
    """(scale_re, scale_im) as Fractions for the error bound of ``op``."""
    x = cfrac(a)
    if op == "cinv":
        s = _mod_upper(QC(1) / x)
        return s, s
    y = cfrac(b)
    if op in ("cadd", "csub"):
        return abs(x.re) + abs(y.re), abs(x.im) + abs(y.im)
    if op == "cmul":
        return abs(x.re * y.re) + abs(x.im * y.im), abs(x.re * y.im) + abs(x.im * y.re)
    if op == "cdiv":
        s = _mod_upper(x / y)
        return s, s
    if op == "cfms":
        z = cfrac(c)
        return (
            abs(x.re) + abs(y.re * z.re) + abs(y.im * z.im),
            abs(x.im) + abs(y.re * z.im) + abs(y.im * z.re),
        )
    raise ValueError(op)


def err_units(result_limbs, exact: Fraction, scale: Fraction, L: int) -> float:
    """|result - exact| / (u_L * scale), as a float (0 when both sides are 0)."""
    d = abs(frac(result_limbs) - exact)
    if d == 0:
        return 0.0
    if scale == 0:
        return float("inf")
    return float(d / (scale * Fraction(1, 2 ** (53 * L))))
