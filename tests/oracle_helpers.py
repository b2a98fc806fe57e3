"""Small hand-built systems for the oracle pins (no oracle arithmetic here)."""

from fractions import Fraction

import numpy as np

from oracle.numbers import to_limbs_complex


def cl(z, L=2):
    """Complex number (python complex, Fraction pair or mpc) -> [2][L] limbs."""
    if isinstance(z, tuple):
        from oracle.numbers import QC

        return to_limbs_complex(QC(*z), L)
    if isinstance(z, complex) or isinstance(z, (int, float)):
        z = complex(z)
        return np.array([[z.real] + [0.0] * (L - 1), [z.imag] + [0.0] * (L - 1)])
    return to_limbs_complex(z, L)


def build(polys, n, L=2):
    """polys: list over i of list of (coef, exponent-list).  Returns exps, coefs, offsets."""
    exps, coefs, offs = [], [], [0]
    for terms in polys:
        for c, a in terms:
            assert len(a) == n
            exps.append(list(a))
            coefs.append(cl(c, L))
        offs.append(len(exps))
    return (
        np.array(exps, dtype=np.uint8).reshape(-1, n),
        np.array(coefs, dtype=np.float64).reshape(-1, 2, L),
        np.array(offs, dtype=np.int32),
    )


def point(vals, L=2):
    return np.stack([cl(v, L) for v in vals])


DYADIC = [(Fraction(3, 4), Fraction(1, 2)), (Fraction(-5, 8), Fraction(1, 16)), (Fraction(1, 2), Fraction(-3, 4)),
          (Fraction(7, 8), Fraction(1, 8)), (Fraction(-1, 4), Fraction(-1, 2)), (Fraction(9, 16), Fraction(5, 16))]
