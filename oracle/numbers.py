"""Exact values of multiword numbers and a small Gaussian-rational type.

A double-double (L=2) or quad-double (L=4) real is the unevaluated sum of its
L double limbs (Section 1 cites Dekker's floating-point technique and the
quad-double library of Hida, Li and Bailey for this representation).  Complex
numbers are stored ``[2][L]``: real limbs, then imaginary limbs.

Parity: these are definitions (exact rational value of a sum of doubles).
Pinned in ``tests/test_oracle_numbers_arith.py`` by hand-computed dyadic values.
"""

from __future__ import annotations

from fractions import Fraction
from typing import Iterable, Sequence

import mpmath
import numpy as np


def prec_bits(L: int) -> int:
    """Working precision of the oracle for an L-limb problem: 4*(53L)+64 bits."""
    return 4 * 53 * L + 64


def unit_roundoff(L: int) -> float:
    """u_L = 2^(-53L): half an ulp of an L-limb number relative to its value."""
    return 2.0 ** (-53 * L)


def frac(limbs: Iterable[float]) -> Fraction:
    """Exact value of a multiword real: the rational sum of its limbs."""
    s = Fraction(0)
    for h in np.asarray(limbs, dtype=np.float64).ravel():
        if not np.isfinite(h):
            raise ValueError("non-finite limb")
        s += Fraction(float(h))
    return s


class QC:
    """Gaussian rational re + i*im with exact Fraction parts."""

    __slots__ = ("re", "im")

    def __init__(self, re=0, im=0):
        self.re = Fraction(re)
        self.im = Fraction(im)

    def __add__(self, o):
        o = _qc(o)
        return QC(self.re + o.re, self.im + o.im)

    __radd__ = __add__

    def __sub__(self, o):
        o = _qc(o)
        return QC(self.re - o.re, self.im - o.im)

    def __rsub__(self, o):
        return _qc(o) - self

    def __neg__(self):
        return QC(-self.re, -self.im)

    def __mul__(self, o):
        o = _qc(o)
        return QC(self.re * o.re - self.im * o.im, self.re * o.im + self.im * o.re)

    __rmul__ = __mul__

    def conj(self):
        return QC(self.re, -self.im)

    def abs2(self) -> Fraction:
        return self.re * self.re + self.im * self.im

    def __truediv__(self, o):
        o = _qc(o)
        d = o.abs2()
        if d == 0:
            raise ZeroDivisionError("complex division by zero")
        p = self * o.conj()
        return QC(p.re / d, p.im / d)

    def __eq__(self, o):
        o = _qc(o)
        return self.re == o.re and self.im == o.im

    def __hash__(self):
        return hash((self.re, self.im))

    def __repr__(self):
        return f"QC({self.re}, {self.im})"

    def __pow__(self, e: int):
        assert e >= 0
        r = QC(1)
        for _ in range(e):
            r = r * self
        return r

    def to_mpc(self) -> mpmath.mpc:
        return mpmath.mpc(
            mpmath.mpf(self.re.numerator) / self.re.denominator,
            mpmath.mpf(self.im.numerator) / self.im.denominator,
        )


def _qc(x) -> QC:
    if isinstance(x, QC):
        return x
    if isinstance(x, complex):
        return QC(Fraction(x.real), Fraction(x.imag))
    return QC(Fraction(x), 0)


def cfrac(c: Sequence) -> QC:
    """Exact Gaussian rational of a ``[2][L]`` complex multiword number."""
    c = np.asarray(c, dtype=np.float64)
    return QC(frac(c[0]), frac(c[1]))


def mpf_of(limbs) -> mpmath.mpf:
    """mpf of a multiword real at the current mpmath precision (limbs summed exactly first)."""
    f = frac(limbs)
    return mpmath.mpf(f.numerator) / f.denominator


def mpc_of(c) -> mpmath.mpc:
    c = np.asarray(c, dtype=np.float64)
    return mpmath.mpc(mpf_of(c[0]), mpf_of(c[1]))


def vec_mpc(x) -> list:
    """``[n][2][L]`` array -> list of mpc."""
    return [mpc_of(x[v]) for v in range(len(x))]


def to_limbs_real(x, L: int) -> list:
    """Round a real (mpf or Fraction) to L nonoverlapping doubles by successive rounding."""
    if isinstance(x, Fraction):
        with mpmath.workprec(prec_bits(L) + 256):
            x = mpmath.mpf(x.numerator) / x.denominator
            return to_limbs_real(x, L)
    out = []
    with mpmath.workprec(max(mpmath.mp.prec, prec_bits(L)) + 64):
        r = mpmath.mpf(x)
        for _ in range(L):
            h = float(r)
            out.append(h)
            r = r - h
    return out


def to_limbs_complex(z, L: int) -> np.ndarray:
    if isinstance(z, QC):
        return np.array([to_limbs_real(z.re, L), to_limbs_real(z.im, L)])
    if isinstance(z, (int, float, complex)):
        z = complex(z)
        return np.array([to_limbs_real(mpmath.mpf(z.real), L), to_limbs_real(mpmath.mpf(z.imag), L)])
    # an mpc keeps its own precision: take its parts without re-rounding
    return np.array([to_limbs_real(z.real, L), to_limbs_real(z.imag, L)])


def mp_abs1(z) -> mpmath.mpf:
    """|Re z| + |Im z| (the 1-norm of a complex number)."""
    return abs(mpmath.re(z)) + abs(mpmath.im(z))
