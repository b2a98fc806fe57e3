"""Speedup and quality up (Section 2).

* speedup T_1 / T_p;
* quality Q = number of correct decimal places; quality up Q_p / Q_1 at a
  fixed time;
* the paper's estimate: with the multiword run on p cores taking T_hi and
  the lower-precision run on 1 core taking T_lo, and optimal speedup, the
  number of cores that brings the high-precision run down to T_lo is
  p* = (T_hi / T_lo) * p, rounded up; assuming y(p) = Q_p/Q_1 linear in p with
  y(1) = 1 and y(ceil(p*)) = Q_hi/Q_lo (2 for quad double over double
  double), the quality up at p cores is y(p) = 1 + (y* - 1)(p - 1)/(ceil(p*) - 1).

Parity: pinned by the worked example of Section 2 (cyclic 10-roots
refinement: 4.818 s DD on 1 core, 8.076 s QD on 8 cores -> 13.410, 14 cores,
y(8) = 1 + 7/13 ~ 1.538), stored in ``tests/golden/quality_up.json``.
"""

from __future__ import annotations

import math
from fractions import Fraction


def speedup(t1: float, tp: float) -> float:
    return t1 / tp


def cores_for_equal_time(t_lo_1core: float, t_hi_pcores: float, p: int):
    """(p* = T_hi/T_lo * p, ceil(p*))."""
    ps = t_hi_pcores / t_lo_1core * p
    return ps, math.ceil(ps)


def quality_up_estimate(t_lo_1core: float, t_hi_pcores: float, p: int, ratio_hi_lo: Fraction = Fraction(2)):
    """Linear-extrapolation quality up y(p) of Section 2, as an exact Fraction."""
    _, pc = cores_for_equal_time(t_lo_1core, t_hi_pcores, p)
    if pc <= 1:
        return Fraction(ratio_hi_lo)
    return 1 + (Fraction(ratio_hi_lo) - 1) * Fraction(p - 1, pc - 1)


def quality_up(q_p: float, q_1: float) -> float:
    return q_p / q_1
