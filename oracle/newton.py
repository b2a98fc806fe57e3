"""Newton's method on the homotopy at fixed t, in high precision.

Follows Algorithm 4.1: the residual is initialised to 1; while the residual is
above epsilon and fewer than Max_It iterations ran, evaluate h and its
Jacobian at z, compute the residual, solve J dz = -h by Gaussian elimination,
update z := z + dz and count the iteration.  On exit the corrector failed if
the last residual is >= epsilon.  (The update of the iteration that certified
the residual is kept, as in the algorithm.)

The linear solve is a library LU with partial pivoting (``mpmath.lu_solve``)
at 4*53L+64 bits; the matrix and right-hand side come from the plain
evaluation in ``oracle.evaluate``.

Parity: one step is pinned in ``tests/test_oracle_newton.py`` against
Cramer's rule in exact rationals (n = 2), against sympy's exact solve on a
3x3 Gaussian-rational system, and by quadratic convergence at a regular root.
``inv_norm_inf`` and ``cond_inf`` are pinned by the closed-form inverse of a
complex 2x2 matrix whose row and column sums differ.
"""

from __future__ import annotations

import dataclasses
from typing import List, Optional

import mpmath
import numpy as np

from .evaluate import eval_homotopy, residual
from .numbers import prec_bits, vec_mpc


@dataclasses.dataclass
class NewtonStep:
    z: list  # mpc list: z + dz
    dz: list  # mpc list
    rho: float  # residual at the input point
    h: list
    J: list


def newton_step(exps, coefs, offsets, gamma, t, x, prec=None, form="product", deg=None, L=None) -> NewtonStep:
    """One Newton iteration from ``x`` ([n][2][L] limbs, or a list of mpc)."""
    if prec is None:
        prec = prec_bits(L if L is not None else x.shape[2])
    r = eval_homotopy(exps, coefs, offsets, gamma, t, x, prec=prec, form=form, deg=deg)
    rho = residual(r)
    with mpmath.workprec(prec):
        A = mpmath.matrix(r.J)
        b = mpmath.matrix([-y for y in r.y])
        dz = mpmath.lu_solve(A, b)
        X = vec_mpc(x) if isinstance(x, np.ndarray) else [mpmath.mpc(v) for v in x]
        dzl = [dz[k] for k in range(len(X))]
        return NewtonStep([X[k] + dzl[k] for k in range(len(X))], dzl, rho, r.y, r.J)


def solve(J: list, rhs: list, prec: int) -> list:
    """x = J^{-1} rhs by mpmath.lu_solve."""
    with mpmath.workprec(prec):
        s = mpmath.lu_solve(mpmath.matrix(J), mpmath.matrix(rhs))
        return [s[k] for k in range(len(rhs))]


def inv_norm_inf(J: list, prec: int) -> float:
    """||J^{-1}||_inf (row sums of complex moduli of the inverse)."""
    with mpmath.workprec(prec):
        Ai = mpmath.inverse(mpmath.matrix(J))
        n = Ai.rows
        return float(max(sum(abs(Ai[i, j]) for j in range(n)) for i in range(n)))


def cond_inf(J: list, prec: int) -> float:
    """kappa_inf(J) = ||J||_inf ||J^{-1}||_inf (row sums of complex moduli)."""
    with mpmath.workprec(prec):
        A = mpmath.matrix(J)
        Ai = mpmath.inverse(A)
        n = A.rows

        def nrm(M):
            return max(sum(abs(M[i, j]) for j in range(n)) for i in range(n))

        return float(nrm(A) * nrm(Ai))


@dataclasses.dataclass
class NewtonRun:
    z: list  # mpc list, final iterate
    iterations: int
    success: bool
    residuals: List[float]


def newton(exps, coefs, offsets, gamma, t, x, eps, max_it, prec=None, form="product", deg=None) -> NewtonRun:
    """The loop of Algorithm 4.1 in high precision.

    Between iterations the iterate stays at full oracle precision (it is not
    rounded to L limbs).
    """
    L = x.shape[2]
    prec = prec or prec_bits(L)
    rho = 1.0
    i = 0
    res = []
    with mpmath.workprec(prec):
        z = vec_mpc(x)
    while rho > eps and i < max_it:
        st = newton_step(exps, coefs, offsets, gamma, t, z, prec=prec, form=form, deg=deg)
        rho = st.rho
        res.append(rho)
        z = st.z
        i += 1
    return NewtonRun(z, i, rho < eps, res)


def newton_tolerance(n: int, kappa: float, L: int, dz_inf: float, z_inf: float, jinv_inf: float = 0.0,
                     h_scale: float = 0.0) -> float:
    """Bound on ||z_kernel - z_oracle||_inf after one step from the same input bits.

    Three sources, added:
      * the elimination, backward stable: 8 n kappa u ||dz||;
      * the rounding of h in L-limb arithmetic, at most 64 u times its
        componentwise scale S (the bound the evaluation parity tests hold),
        carried into dz by J^{-1}: 64 u ||J^{-1}|| max_i S_i;
      * the final update z + dz: 2 u ||z||.
    """
    u = 2.0 ** (-53 * L)
    return 8 * n * kappa * u * dz_inf + 64 * u * jinv_inf * h_scale + 2 * u * z_inf
