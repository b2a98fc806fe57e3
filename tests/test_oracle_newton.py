"""Pins for the oracle's Newton step and the loop of Algorithm 4.1."""

from fractions import Fraction

import mpmath
import numpy as np
import pytest
import sympy

from oracle.newton import cond_inf, inv_norm_inf, newton, newton_step, newton_tolerance
from oracle.numbers import QC, vec_mpc
from synth.systems import CONFIGS, config_system
from tests.oracle_helpers import DYADIC, build, point

GAMMA = np.array([[1.0, 0.0], [0.0, 0.0]])


def qc(z):
    return QC(*z)


def test_linear_n2_one_step_equals_cramer():
    # f = A x + b is linear, so at t = 1 one Newton step from anywhere lands on
    # the solution; Cramer's rule gives it in exact rationals.
    A = [[DYADIC[0], DYADIC[1]], [DYADIC[2], DYADIC[3]]]
    b = [DYADIC[4], DYADIC[5]]
    polys = [[(A[i][0], [1, 0]), (A[i][1], [0, 1]), (b[i], [0, 0])] for i in range(2)]
    exps, coefs, offs = build(polys, 2)
    x0 = point([(Fraction(1, 3), 0), (0, Fraction(1, 5))])
    st = newton_step(exps, coefs, offs, GAMMA, 1.0, x0, prec=500)
    a11, a12, a21, a22 = (qc(A[0][0]), qc(A[0][1]), qc(A[1][0]), qc(A[1][1]))
    r1, r2 = -qc(b[0]), -qc(b[1])
    det = a11 * a22 - a12 * a21
    xs = [(r1 * a22 - a12 * r2) / det, (a11 * r2 - r1 * a21) / det]
    with mpmath.workprec(500):
        for k in range(2):
            assert abs(st.z[k] - xs[k].to_mpc()) < mpmath.mpf(2) ** -480


def test_linear_n3_matches_sympy_solve():
    n = 3
    rng = np.random.default_rng(7)
    A = [[(Fraction(int(rng.integers(-9, 10)), 8), Fraction(int(rng.integers(-9, 10)), 8)) for _ in range(n)] for _ in range(n)]
    b = [(Fraction(int(rng.integers(-9, 10)), 4), Fraction(int(rng.integers(-9, 10)), 4)) for _ in range(n)]
    polys = []
    for i in range(n):
        terms = [(A[i][v], [1 if w == v else 0 for w in range(n)]) for v in range(n)]
        terms.append((b[i], [0] * n))
        polys.append(terms)
    exps, coefs, offs = build(polys, n)
    st = newton_step(exps, coefs, offs, GAMMA, 1.0, point([(0, 0)] * n), prec=500)
    M = sympy.Matrix(n, n, lambda i, v: sympy.Rational(A[i][v][0]) + sympy.I * sympy.Rational(A[i][v][1]))
    rhs = sympy.Matrix(n, 1, lambda i, _: -(sympy.Rational(b[i][0]) + sympy.I * sympy.Rational(b[i][1])))
    sol = M.LUsolve(rhs)
    with mpmath.workprec(500):
        for k in range(n):
            ref = mpmath.mpc(sympy.re(sol[k]).evalf(160), sympy.im(sol[k]).evalf(160))
            assert abs(st.z[k] - ref) < mpmath.mpf(10) ** -140


def test_algorithm_4_1_loop_semantics():
    s = config_system(CONFIGS["n8_dd"])
    # residual initialised to 1: with eps >= 1 the loop body never runs and the
    # corrector reports failure (fail := residual >= eps)
    r = newton(s.exps, s.coefs, s.poly_offsets, s.gamma, 1.0, s.zstar, eps=1.0, max_it=5)
    assert r.iterations == 0 and not r.success
    r = newton(s.exps, s.coefs, s.poly_offsets, s.gamma, 1.0, s.zstar, eps=2.0, max_it=5)
    assert r.iterations == 0 and r.success
    # Max_It bounds the iterations; eps = 0 can never be met
    r = newton(s.exps, s.coefs, s.poly_offsets, s.gamma, 1.0, s.zstar, eps=0.0, max_it=2)
    assert r.iterations == 2 and not r.success


def test_quadratic_convergence_at_planted_root():
    s = config_system(CONFIGS["n8_dd"])
    x = np.array(s.zstar)
    x[:, :, 0] += 1e-4 * np.array([[1.0, -0.5]] * s.n)  # perturb the leading limbs
    x[:, :, 1] = 0.0
    r = newton(s.exps, s.coefs, s.poly_offsets, s.gamma, 1.0, x, eps=1e-220, max_it=8, prec=800)
    res = r.residuals
    assert res[0] > 1e-6
    # each residual roughly squares (order >= 1.7) until the precision floor
    for a, b in zip(res, res[1:]):
        if a < 1e-3 and b > 1e-200:
            assert np.log(b) <= 1.7 * np.log(a)
    assert res[-1] < 1e-150


def test_cond_inf_diagonal():
    J = [[mpmath.mpc(2), 0], [0, mpmath.mpc(0, 0.5)]]
    assert cond_inf(J, 200) == pytest.approx(4.0)


def _two_by_two():
    # J = [[a, b], [c, d]] with entries chosen so that row sums, column sums, the largest
    # modulus and the |Re| + |Im| norm of the inverse all differ
    a, b, c, d = mpmath.mpc(2, 0), mpmath.mpc(1, 1), mpmath.mpc(0, 3), mpmath.mpc(3, 4)
    return a, b, c, d


def test_inv_norm_inf_two_by_two_closed_form():
    # J^-1 = [[d, -b], [-c, a]] / det, so ||J^-1||_inf = max(|d| + |b|, |c| + |a|) / |det|
    with mpmath.workprec(300):
        a, b, c, d = _two_by_two()
        det = a * d - b * c
        expect = max(abs(d) + abs(b), abs(c) + abs(a)) / abs(det)
        got = inv_norm_inf([[a, b], [c, d]], 300)
        assert abs(got - float(expect)) <= 1e-15 * float(expect)
        # the column-sum norm differs on this matrix, so a transposed sum fails
        cols = max(abs(d) + abs(c), abs(b) + abs(a)) / abs(det)
        assert abs(float(cols) - got) > 1e-3


def test_cond_inf_two_by_two_closed_form():
    with mpmath.workprec(300):
        a, b, c, d = _two_by_two()
        det = a * d - b * c
        nJ = max(abs(a) + abs(b), abs(c) + abs(d))
        nI = max(abs(d) + abs(b), abs(c) + abs(a)) / abs(det)
        assert cond_inf([[a, b], [c, d]], 300) == pytest.approx(float(nJ * nI), rel=1e-15)


def test_newton_tolerance_terms():
    # 8 n kappa u ||dz|| + 64 u ||J^-1|| max S + 2 u ||z||, u = 2^(-53 L)
    u = 2.0 ** -106
    assert newton_tolerance(4, 10.0, 2, 0.5, 2.0) == pytest.approx(8 * 4 * 10.0 * u * 0.5 + 2 * u * 2.0, rel=1e-15)
    assert newton_tolerance(4, 10.0, 2, 0.5, 2.0, 3.0, 5.0) == pytest.approx(
        8 * 4 * 10.0 * u * 0.5 + 64 * u * 3.0 * 5.0 + 2 * u * 2.0, rel=1e-15)
