"""Pins for the oracle's plain evaluation of f, its Jacobian and the homotopy.

Each pin comes from outside the oracle: closed forms, Horner's rule, sympy's
symbolic differentiation, or central differences in high precision.
"""

from fractions import Fraction

import mpmath
import numpy as np
import pytest
import sympy

from oracle.evaluate import degrees, eval_homotopy, eval_system, eval_system_exact, residual
from oracle.numbers import QC, cfrac, mpc_of, vec_mpc
from synth.systems import CONFIGS, config_system, random_point, start_root
from tests.oracle_helpers import DYADIC, build, cl, point


def qc(z):
    return QC(*z)


@pytest.mark.parametrize("n", [2, 3, 5, 8])
def test_speelpenning_all_partials_equal_r_pow_n_minus_1(n):
    # f = prod_v x_v; with x_v = r for all v, every partial is r^(n-1) exactly
    exps, coefs, offs = build([[(1, [1] * n)]] + [[(1, [0] * n)]] * (n - 1), n)
    r = DYADIC[0]
    x = point([r] * n)
    ys, Js = eval_system_exact(exps, coefs, offs, x)
    rq = qc(r)
    expect = QC(1)
    for _ in range(n - 1):
        expect = expect * rq
    assert all(Js[0][v] == expect for v in range(n))
    assert ys[0] == expect * rq
    with mpmath.workprec(300):
        res = eval_system(exps, coefs, offs, x, rows=[0], prec=300)
        ref = mpmath.power(rq.to_mpc(), n - 1)
        for v in range(n):
            assert abs(res.J[0][v] - ref) < mpmath.mpf(2) ** -280


@pytest.mark.parametrize("n", [2, 4])
def test_speelpenning_distinct_values(n):
    # d/dx_m prod_v x_v = prod_{v != m} x_v (Speelpenning's example, Section 6)
    exps, coefs, offs = build([[(1, [1] * n)]] + [[(1, [0] * n)]] * (n - 1), n)
    vals = DYADIC[:n]
    ys, Js = eval_system_exact(exps, coefs, offs, point(vals))
    for m in range(n):
        e = QC(1)
        for v in range(n):
            if v != m:
                e = e * qc(vals[v])
        assert Js[0][m] == e


@pytest.mark.parametrize("d", [3, 7, 12])
def test_x_pow_d_minus_1_at_roots_of_unity(d):
    # f_i = x_i^d - 1 vanishes at exp(2 pi i k/d); J = diag(d x^(d-1))
    n, L = 3, 2
    polys = []
    for i in range(n):
        a = [0] * n
        a[i] = d
        polys.append([(1, a), (-1, [0] * n)])
    exps, coefs, offs = build(polys, n, L)
    x = start_root(np.array([d] * n), np.array([1, 2, d - 1]), L)
    res = eval_system(exps, coefs, offs, x, form="product")
    u = 2.0**-106
    with mpmath.workprec(400):
        X = vec_mpc(x)
        for i in range(n):
            assert abs(res.y[i]) <= 4 * d * u * res.S[i]
            for v in range(n):
                ref = d * mpmath.power(X[i], d - 1) if v == i else 0
                assert abs(res.J[i][v] - ref) < mpmath.mpf(2) ** -380


def test_single_monomial_partials_closed_form():
    # c x^a with a = (2, 0, 3): d/dx1 = 2 c x1 x3^3; d/dx2 = 0; d/dx3 = 3 c x1^2 x3^2
    c = (Fraction(1, 2), Fraction(-3, 4))
    exps, coefs, offs = build([[(c, [2, 0, 3])], [(1, [0, 0, 0])], [(1, [0, 0, 0])]], 3)
    x = DYADIC[:3]
    _, Js = eval_system_exact(exps, coefs, offs, point(x))
    C, X1, X3 = qc(c), qc(x[0]), qc(x[2])
    assert Js[0][0] == C * 2 * X1 * X3 * X3 * X3
    assert Js[0][1] == QC(0)
    assert Js[0][2] == C * 3 * X1 * X1 * X3 * X3


def test_n1_matches_horner():
    # n = 1: f(x) = sum_k c_k x^k; Horner's rule (the dense alternative of Section 6)
    cs = [(Fraction(1, 2), Fraction(1, 4)), (Fraction(-3, 8), 0), (0, Fraction(5, 16)), (Fraction(1, 8), Fraction(-1, 8))]
    polys = [[(c, [k]) for k, c in enumerate(cs)]]
    exps, coefs, offs = build(polys, 1)
    xv = (Fraction(5, 8), Fraction(-3, 8))
    ys, Js = eval_system_exact(exps, coefs, offs, point([xv]))
    X = qc(xv)
    p, dp = QC(0), QC(0)
    for c in reversed(cs):
        dp = dp * X + p
        p = p * X + qc(c)
    assert ys[0] == p
    assert Js[0][0] == dp


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_small_random_systems_match_sympy(seed):
    # n = 2 and 3: expand with sympy, differentiate symbolically, substitute exactly
    rng = np.random.default_rng(seed)
    n = 2 + seed % 2
    polys = []
    for i in range(n):
        terms = []
        for _ in range(4):
            a = list(rng.integers(0, 4, size=n))
            c = (Fraction(int(rng.integers(-8, 9)), 8), Fraction(int(rng.integers(-8, 9)), 8))
            terms.append((c, a))
        polys.append(terms)
    exps, coefs, offs = build(polys, n)
    xs = DYADIC[seed : seed + n]
    ys, Js = eval_system_exact(exps, coefs, offs, point(xs))
    X = sympy.symbols(f"x0:{n}")
    sub = {X[v]: sympy.Rational(xs[v][0]) + sympy.I * sympy.Rational(xs[v][1]) for v in range(n)}
    for i, terms in enumerate(polys):
        f = sum((sympy.Rational(c[0]) + sympy.I * sympy.Rational(c[1])) * sympy.prod([X[v] ** int(a[v]) for v in range(n)])
                for c, a in terms)
        fy = sympy.expand(f.subs(sub))
        assert sympy.re(fy) == ys[i].re and sympy.im(fy) == ys[i].im
        for v in range(n):
            dv = sympy.expand(sympy.diff(f, X[v]).subs(sub))
            assert sympy.re(dv) == Js[i][v].re and sympy.im(dv) == Js[i][v].im


def test_jacobian_matches_central_differences_on_config_system():
    s = config_system(CONFIGS["n8_dd"])
    x = random_point(s.n, s.L, seed=5, spread=0.1)
    res = eval_system(s.exps, s.coefs, s.poly_offsets, x, prec=700)
    with mpmath.workprec(700):
        X = vec_mpc(x)
        h = mpmath.mpf(2) ** -150
        for v in (0, 3, 7):
            Xp = list(X)
            Xm = list(X)
            Xp[v] += h
            Xm[v] -= h
            rp = eval_system(s.exps, s.coefs, s.poly_offsets, Xp, prec=700)
            rm = eval_system(s.exps, s.coefs, s.poly_offsets, Xm, prec=700)
            for i in range(s.n):
                fd = (rp.y[i] - rm.y[i]) / (2 * h)
                assert abs(fd - res.J[i][v]) <= mpmath.mpf(10) ** -60 * (1 + res.SJ[i][v])


def test_quotient_form_equals_product_form():
    s = config_system(CONFIGS["n8_dd"])
    x = random_point(s.n, s.L, seed=3, spread=0.2)
    a = eval_system(s.exps, s.coefs, s.poly_offsets, x, form="product")
    b = eval_system(s.exps, s.coefs, s.poly_offsets, x, form="quotient")
    with mpmath.workprec(500):
        for i in range(s.n):
            for v in range(s.n):
                assert abs(a.J[i][v] - b.J[i][v]) <= mpmath.mpf(10) ** -120 * (1 + a.SJ[i][v])


def test_homotopy_start_system_and_target_ends():
    s = config_system(CONFIGS["n8_dd"])
    deg = degrees(s.exps, s.poly_offsets)
    assert deg == [int(s.exps[s.poly_offsets[i]:s.poly_offsets[i + 1]].astype(int).sum(axis=1).max()) for i in range(s.n)]
    # t = 0: h = gamma (x^d - 1) vanishes at the start roots, J diagonal = gamma d x^(d-1)
    x0 = start_root(np.array(deg), np.arange(s.n), s.L)
    r0 = eval_homotopy(s.exps, s.coefs, s.poly_offsets, s.gamma, 0.0, x0)
    assert residual(r0) < 1e-29
    with mpmath.workprec(500):
        g = mpc_of(s.gamma)
        X = vec_mpc(x0)
        for i in range(s.n):
            for v in range(s.n):
                ref = g * deg[i] * mpmath.power(X[i], deg[i] - 1) if i == v else 0
                assert abs(r0.J[i][v] - ref) < mpmath.mpf(10) ** -120
    # t = 1: h = f; at the planted point the residual is at the coefficient rounding level
    r1 = eval_homotopy(s.exps, s.coefs, s.poly_offsets, s.gamma, 1.0, s.zstar)
    assert residual(r1) < 1e-29


def test_homotopy_t_derivative_and_x_derivative_by_differences():
    # dh/dt = f - gamma g and dh/dx_i (diagonal g part) checked by central differences
    s = config_system(CONFIGS["n8_dd"])
    x = random_point(s.n, s.L, seed=9, spread=0.05)
    t = 0.375
    with mpmath.workprec(600):
        ht = mpmath.mpf(2) ** -120
        rp = eval_homotopy(s.exps, s.coefs, s.poly_offsets, s.gamma, t + float(2.0**-40), x, prec=600)
        rm = eval_homotopy(s.exps, s.coefs, s.poly_offsets, s.gamma, t - float(2.0**-40), x, prec=600)
        f = eval_system(s.exps, s.coefs, s.poly_offsets, x, prec=600)
        g = mpc_of(s.gamma)
        X = vec_mpc(x)
        deg = degrees(s.exps, s.poly_offsets)
        for i in range(s.n):
            fd = (rp.y[i] - rm.y[i]) / (2 * mpmath.mpf(2) ** -40)
            # h is affine in t, so the central difference is exact up to rounding
            assert abs(fd - (f.y[i] - g * (mpmath.power(X[i], deg[i]) - 1))) < mpmath.mpf(10) ** -100
        r = eval_homotopy(s.exps, s.coefs, s.poly_offsets, s.gamma, t, x, prec=600)
        for v in (1, 6):
            Xp, Xm = list(X), list(X)
            Xp[v] += ht
            Xm[v] -= ht
            a = eval_homotopy(s.exps, s.coefs, s.poly_offsets, s.gamma, t, Xp, prec=600)
            b = eval_homotopy(s.exps, s.coefs, s.poly_offsets, s.gamma, t, Xm, prec=600)
            for i in range(s.n):
                fd = (a.y[i] - b.y[i]) / (2 * ht)
                assert abs(fd - r.J[i][v]) <= mpmath.mpf(10) ** -50 * (1 + r.SJ[i][v])


# --- componentwise scales and the residual (Algorithm 4.1, "Residual") -------------------
#
# Points and coefficients are dyadic with rational moduli (3/4 + i has modulus 5/4,
# (5 + 12 i)/16 has 13/16), so every scale is an exact rational written out by hand below.

X0 = (Fraction(3, 4), Fraction(1))           # |x0| = 5/4
X1 = (Fraction(5, 16), Fraction(12, 16))     # |x1| = 13/16
C1 = (Fraction(3, 4), Fraction(1))           # |c1| = 5/4
C2 = (Fraction(-2), Fraction(0))             # |c2| = 2
C3 = (Fraction(0), Fraction(-1, 2))          # |c3| = 1/2


def _two_term_system():
    # f_0 = c1 x0^2 x1 + c2 x1^3 ;  f_1 = c3 x0 + c2 (constant)
    return build([[(C1, [2, 1]), (C2, [0, 3])], [(C3, [1, 0]), (C2, [0, 0])]], 2)


def test_scales_of_a_two_term_system_are_the_exact_rationals():
    exps, coefs, offs = _two_term_system()
    x = point([X0, X1])
    a0, a1 = Fraction(5, 4), Fraction(13, 16)
    ac1, ac2, ac3 = Fraction(5, 4), Fraction(2), Fraction(1, 2)
    # S_i = sum_j |c_ij| |x^a_ij|  (a sum of moduli, not the modulus of the sum)
    S = [ac1 * a0**2 * a1 + ac2 * a1**3, ac3 * a0 + ac2]
    # S_iv = sum_j |c_ij| a_ijv |x^(a_ij - e_v)|  (the exponent factor included)
    SJ = [[ac1 * 2 * a0 * a1, ac1 * a0**2 + ac2 * 3 * a1**2], [ac3, Fraction(0)]]
    with mpmath.workprec(300):
        for form in ("product", "quotient"):
            r = eval_system(exps, coefs, offs, x, prec=300, form=form)
            for i in range(2):
                assert abs(r.S[i] - mpmath.mpf(S[i].numerator) / S[i].denominator) < mpmath.mpf(2) ** -280
                for v in range(2):
                    ref = mpmath.mpf(SJ[i][v].numerator) / SJ[i][v].denominator
                    assert abs(r.SJ[i][v] - ref) < mpmath.mpf(2) ** -280, (form, i, v)


def test_homotopy_scales_add_the_start_system_terms():
    # S^h_i = |t| S_i + |(1-t) gamma| (|x_i|^d_i + 1);  S^h_ii gains |(1-t) gamma| d_i |x_i|^(d_i-1)
    exps, coefs, offs = _two_term_system()
    x = point([X0, X1])
    gamma = cl((Fraction(3, 4), Fraction(1)))  # |gamma| = 5/4
    t = 0.25
    a0, a1 = Fraction(5, 4), Fraction(13, 16)
    ac1, ac2, ac3 = Fraction(5, 4), Fraction(2), Fraction(1, 2)
    d = [3, 1]
    w = (1 - Fraction(1, 4)) * Fraction(5, 4)
    S = [ac1 * a0**2 * a1 + ac2 * a1**3, ac3 * a0 + ac2]
    SJ = [[ac1 * 2 * a0 * a1, ac1 * a0**2 + ac2 * 3 * a1**2], [ac3, Fraction(0)]]
    ax = [a0, a1]
    Sh = [Fraction(1, 4) * S[i] + w * (ax[i] ** d[i] + 1) for i in range(2)]
    SJh = [[Fraction(1, 4) * SJ[i][v] + (w * d[i] * ax[i] ** (d[i] - 1) if i == v else 0) for v in range(2)]
           for i in range(2)]
    with mpmath.workprec(300):
        r = eval_homotopy(exps, coefs, offs, gamma, t, x, prec=300)
        for i in range(2):
            assert abs(r.S[i] - mpmath.mpf(Sh[i].numerator) / Sh[i].denominator) < mpmath.mpf(2) ** -280
            for v in range(2):
                ref = mpmath.mpf(SJh[i][v].numerator) / SJh[i][v].denominator
                assert abs(r.SJ[i][v] - ref) < mpmath.mpf(2) ** -280, (i, v)


def test_residual_is_max_one_norm_over_max_scale():
    # rho = max_i (|Re h_i| + |Im h_i|) / max_i S_i.  With h = (3 - 4i, 1 + i) and S = (10, 20):
    # 7/20.  A modulus (5) would give 1/4, a per-row ratio max(7/10, 2/20) 7/10, the sum of
    # the scales 7/30, the first row's scale 7/10.
    from oracle.evaluate import EvalResult

    with mpmath.workprec(200):
        res = EvalResult([0, 1], [mpmath.mpc(3, -4), mpmath.mpc(1, 1)], None, [mpmath.mpf(10), mpmath.mpf(20)], None)
        assert residual(res) == 0.35
        # the maximum is over rows: the second row dominates here
        res = EvalResult([0, 1], [mpmath.mpc(0.5, 0), mpmath.mpc(-2, 3)], None, [mpmath.mpf(40), mpmath.mpf(8)], None)
        assert residual(res) == 5.0 / 40.0
        # a zero scale leaves the absolute value
        res = EvalResult([0], [mpmath.mpc(-0.25, 0.5)], None, [mpmath.mpf(0)], None)
        assert residual(res) == 0.75


def test_residual_of_the_two_term_homotopy_by_hand():
    # at t = 1, h = f; every value at this dyadic point is an exact Gaussian rational
    exps, coefs, offs = _two_term_system()
    x = point([X0, X1])
    gamma = cl((Fraction(1), Fraction(0)))
    t = 1.0  # h = f
    x0, x1 = QC(*X0), QC(*X1)
    c1, c2, c3 = QC(*C1), QC(*C2), QC(*C3)
    f0 = c1 * x0 * x0 * x1 + c2 * x1 * x1 * x1
    f1 = c3 * x0 + c2
    one = [abs(f.re) + abs(f.im) for f in (f0, f1)]
    a0, a1 = Fraction(5, 4), Fraction(13, 16)
    S = [Fraction(5, 4) * a0**2 * a1 + 2 * a1**3, Fraction(1, 2) * a0 + 2]
    expect = max(one) / max(S)
    r = eval_homotopy(exps, coefs, offs, gamma, t, x, prec=300)
    assert residual(r) == pytest.approx(float(expect), rel=1e-15)
