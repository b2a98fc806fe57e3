"""Plain evaluation of a sparse system, its Jacobian, and the total-degree homotopy.

What is computed (Section 4: the array Y holds every polynomial value and all
partial derivatives needed for the Jacobian; Section 6: the derivative of a
monomial x^a with respect to x_v is a_v x^(a - e_v)):

    f_i(x)      = sum_j c_ij prod_v x_v^(a_ijv)
    df_i/dx_v   = sum_j c_ij a_ijv x_v^(a_ijv - 1) prod_{w != v} x_w^(a_ijw)

written out term by term from the exponent row, with exact powers of each
coordinate.  Nothing here uses the prefix/suffix (Speelpenning) products of
Section 6; every partial is formed on its own (``form="product"``) or, when
x_v != 0, as a_v * (c x^a) / x_v (``form="quotient"``), which is the same
definition rearranged and is used at large n for speed.

The homotopy is not printed in the paper (it only writes h(x,t)); the
total-degree homotopy used throughout is

    h_i(x,t) = t f_i(x) + (1-t) gamma (x_i^(d_i) - 1),   d_i = max_j sum_v a_ijv

Componentwise scales (used for tolerances and the residual):

    S_i   = sum_j |c_ij x^(a_ij)|
    S_iv  = sum_j |c_ij| a_ijv |x^(a_ij - e_v)|
    S^h_i = |t| S_i + |(1-t) gamma| (|x_i|^(d_i) + 1)
    S^h_iv= |t| S_iv + [i = v] |(1-t) gamma| d_i |x_i|^(d_i - 1)

Residual (reading of the unnamed norm in Algorithm 4.1):

    rho = max_i (|Re h_i| + |Im h_i|) / max_i S^h_i

Parity: pinned in ``tests/test_oracle_evaluate.py`` by closed forms
(Speelpenning's product, x^d - 1 at roots of unity, single monomials),
by Horner's rule at n = 1, by sympy differentiation of the expanded
polynomial at n = 2..3, and by central differences in high precision.  The
scales S, S_iv (and their homotopy forms) are pinned by exact rationals on a
two-term system at a dyadic point with rational moduli; the residual by
hand-computed rows (maximum over rows of |Re| + |Im|, divided by the largest
scale).
"""

from __future__ import annotations

from typing import Iterable, List, Optional, Sequence

import mpmath
import numpy as np

from .numbers import QC, cfrac, mpc_of, prec_bits, vec_mpc


def degrees(exps: np.ndarray, offsets: np.ndarray) -> List[int]:
    """d_i = max over the terms of polynomial i of the total degree sum_v a_ijv."""
    n = len(offsets) - 1
    tot = exps.astype(np.int64).sum(axis=1)
    return [int(tot[offsets[i] : offsets[i + 1]].max()) if offsets[i + 1] > offsets[i] else 0 for i in range(n)]


class EvalResult:
    """Values, Jacobian rows and scales for a subset of polynomials."""

    def __init__(self, rows, y, J, S, SJ):
        self.rows = list(rows)
        self.y = y  # list of mpc, one per row
        self.J = J  # list of lists of mpc
        self.S = S  # list of mpf
        self.SJ = SJ  # list of lists of mpf


def _limbs(x) -> int:
    """L of a multiword point array; a list of mpc counts as the widest (4 limbs)."""
    return x.shape[2] if isinstance(x, np.ndarray) else 4


def _point(x) -> list:
    """A point given as ``[n][2][L]`` limbs or as a list of mpc -> list of mpc."""
    if isinstance(x, np.ndarray):
        return vec_mpc(x)
    return [mpmath.mpc(v) for v in x]


def _powers(xv, emax: int):
    p = [mpmath.mpc(1)]
    for _ in range(emax):
        p.append(p[-1] * xv)
    return p


def eval_system(
    exps: np.ndarray,
    coefs: np.ndarray,
    offsets: np.ndarray,
    x: np.ndarray,
    rows: Optional[Iterable[int]] = None,
    prec: Optional[int] = None,
    form: str = "product",
) -> EvalResult:
    """f_i, df_i/dx_v and their scales at the point ``x``.

    ``x`` is ``[n][2][L]`` multiword limbs (taken at their exact value) or a
    list of mpc.  Computed in mpmath at ``prec`` bits (default 4*53L+64).
    ``rows`` selects polynomials (default all).
    """
    n = len(x)
    prec = prec or prec_bits(_limbs(x))
    rows = range(n) if rows is None else list(rows)
    emax = int(exps.max()) if exps.size else 0
    with mpmath.workprec(prec):
        X = _point(x)
        P = [_powers(X[v], emax) for v in range(n)]
        absP = [[abs(p) for p in P[v]] for v in range(n)]
        absX = [absP[v][1] if emax >= 1 else abs(X[v]) for v in range(n)]
        ys, Js, Ss, SJs = [], [], [], []
        for i in rows:
            y = mpmath.mpc(0)
            S = mpmath.mpf(0)
            J = [mpmath.mpc(0)] * n
            SJ = [mpmath.mpf(0)] * n
            for j in range(int(offsets[i]), int(offsets[i + 1])):
                a = [int(e) for e in exps[j]]
                c = mpc_of(coefs[j])
                act = [v for v in range(n) if a[v] > 0]
                mono = c
                for v in act:
                    mono = mono * P[v][a[v]]
                y += mono
                amono = abs(mono)
                S += amono
                ac = abs(c)
                for v in act:
                    if form == "product":
                        d = c * a[v] * P[v][a[v] - 1]
                        sd = ac * a[v] * absP[v][a[v] - 1]
                        for w in act:
                            if w != v:
                                d = d * P[w][a[w]]
                                sd = sd * absP[w][a[w]]
                    elif form == "quotient":
                        d = a[v] * mono / X[v]
                        sd = a[v] * amono / absX[v]
                    else:
                        raise ValueError(form)
                    J[v] = J[v] + d
                    SJ[v] = SJ[v] + sd
            ys.append(y)
            Js.append(J)
            Ss.append(S)
            SJs.append(SJ)
        return EvalResult(rows, ys, Js, Ss, SJs)


def homotopy_terms(gamma: np.ndarray, t: float, prec: int):
    """(1-t) * gamma, exactly from the FP64 t and the multiword gamma, as mpc."""
    with mpmath.workprec(prec):
        return (1 - mpmath.mpf(t)) * mpc_of(gamma)


def eval_homotopy(
    exps: np.ndarray,
    coefs: np.ndarray,
    offsets: np.ndarray,
    gamma: np.ndarray,
    t: float,
    x: np.ndarray,
    rows: Optional[Iterable[int]] = None,
    prec: Optional[int] = None,
    form: str = "product",
    deg: Optional[Sequence[int]] = None,
) -> EvalResult:
    """h(x,t) = t f(x) + (1-t) gamma g(x), g_i = x_i^(d_i) - 1, with Jacobian and scales."""
    n = len(x)
    prec = prec or prec_bits(_limbs(x))
    deg = list(deg) if deg is not None else degrees(exps, offsets)
    fr = eval_system(exps, coefs, offsets, x, rows=rows, prec=prec, form=form)
    with mpmath.workprec(prec):
        tt = mpmath.mpf(t)
        w = homotopy_terms(gamma, t, prec)
        aw = abs(w)
        X = _point(x)
        ys, Js, Ss, SJs = [], [], [], []
        for r, i in enumerate(fr.rows):
            d = deg[i]
            xd = X[i] ** d
            xd1 = X[i] ** (d - 1) if d >= 1 else mpmath.mpc(0)
            ys.append(tt * fr.y[r] + w * (xd - 1))
            J = [tt * fr.J[r][v] for v in range(n)]
            J[i] = J[i] + w * d * xd1
            Js.append(J)
            Ss.append(abs(tt) * fr.S[r] + aw * (abs(xd) + 1))
            SJ = [abs(tt) * fr.SJ[r][v] for v in range(n)]
            SJ[i] = SJ[i] + aw * d * abs(xd1)
            SJs.append(SJ)
        return EvalResult(fr.rows, ys, Js, Ss, SJs)


def residual(res: EvalResult) -> float:
    """rho = max_i (|Re h_i| + |Im h_i|) / max_i S_i, rounded to FP64."""
    num = max(abs(mpmath.re(y)) + abs(mpmath.im(y)) for y in res.y)
    den = max(res.S)
    if den == 0:
        return float(num)
    return float(num / den)


# --- exact evaluation over Gaussian rationals (tiny systems, pins) -----------------


def eval_system_exact(exps, coefs, offsets, x) -> tuple:
    """f and J as exact Gaussian rationals (``QC``) from the exact input values."""
    n = x.shape[0]
    X = [cfrac(x[v]) for v in range(n)]
    ys, Js = [], []
    for i in range(n):
        y = QC(0)
        J = [QC(0) for _ in range(n)]
        for j in range(int(offsets[i]), int(offsets[i + 1])):
            a = [int(e) for e in exps[j]]
            c = cfrac(coefs[j])
            mono = c
            for v in range(n):
                mono = mono * X[v] ** a[v]
            y = y + mono
            for v in range(n):
                if a[v] == 0:
                    continue
                d = c * a[v] * X[v] ** (a[v] - 1)
                for w in range(n):
                    if w != v:
                        d = d * X[w] ** a[w]
                J[v] = J[v] + d
        ys.append(y)
        Js.append(J)
    return ys, Js


def to_array(vals, L: int) -> np.ndarray:
    """list (or list of lists) of mpc -> FP64 complex numpy array (leading parts)."""
    return np.array(
        [[complex(v) for v in row] for row in vals] if isinstance(vals[0], list) else [complex(v) for v in vals]
    )
