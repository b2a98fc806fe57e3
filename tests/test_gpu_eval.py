"""Evaluation + Jacobian kernel vs the plain oracle, at the workload shapes
and on edge cases.  Tolerance: |value - oracle| <= tau * componentwise scale,
tau = 1e-30 (double double), 1e-60 (quad double), 1e-13 (double)."""

import mpmath
import numpy as np
import pytest

from oracle.evaluate import eval_homotopy as o_eval_homotopy
from oracle.evaluate import eval_system as o_eval_system
from synth.systems import CONFIGS, config_system, make_system, random_point
from tests.gpu_helpers import err_over_scale, say, start_power_bounds
from tests.oracle_helpers import build, point

pytestmark = pytest.mark.gpu

TAU = {1: 1e-13, 2: 1e-30, 4: 1e-60}


def check_eval(sysm, L, x, rows=None, form="product"):
    import paper_1109_0545_amd as q

    say("eval_jacobian n", sysm.n, "L", L, "rows", rows if rows is None else len(rows))
    S = q.System.from_synth(sysm, prec=sysm.L)
    y, J = q.eval_jacobian(S, x, L)
    s_eval = sysm.truncated(L) if L < sysm.L else sysm
    ref = o_eval_system(s_eval.exps, s_eval.coefs, s_eval.poly_offsets, x, rows=rows, form=form)
    worst = 0.0
    for r, i in enumerate(ref.rows):
        worst = max(worst, err_over_scale(y[i], ref.y[r], ref.S[r]))
        for v in range(sysm.n):
            worst = max(worst, err_over_scale(J[i, v], ref.J[r][v], ref.SJ[r][v]))
    say(f"  worst |d| / S = {worst:.3e} = {worst / 2.0 ** (-53 * L):.2f} u (bound {TAU[L]:.0e} = "
        f"{TAU[L] / 2.0 ** (-53 * L):.0f} u)")
    assert worst <= TAU[L], worst
    return worst


@pytest.mark.parametrize("L", [1, 2])
def test_eval_n8_all_rows(L):
    s = config_system(CONFIGS["n8_dd"])
    check_eval(s, L, random_point(s.n, L, seed=3, spread=0.3))


def test_eval_n32_dd_all_rows():
    s = config_system(CONFIGS["n32_dd"])
    check_eval(s, 2, random_point(s.n, 2, seed=4, spread=0.1), form="quotient")


def test_eval_n64_qd_sampled_rows():
    s = config_system(CONFIGS["n64_qd"])
    check_eval(s, 4, random_point(s.n, 4, seed=5, spread=0.05), rows=[0, 17, 63], form="quotient")


def test_eval_n64_qd_at_dd_precision_truncates():
    s = config_system(CONFIGS["n64_qd"])
    check_eval(s, 2, random_point(s.n, 2, seed=6, spread=0.05), rows=[1, 40], form="quotient")


def test_eval_n128_dd_sampled_rows():
    s = config_system(CONFIGS["n128_dd"])
    check_eval(s, 2, random_point(s.n, 2, seed=7, spread=0.02), rows=[0, 127], form="quotient")


@pytest.mark.parametrize("n,m,E,L,seed", [(1, 5, 6, 2, 1), (3, 7, 5, 4, 2), (5, 11, 3, 2, 3), (40, 9, 2, 2, 4),
                                          (17, 3, 4, 4, 5), (100, 6, 2, 2, 6)])
def test_eval_ragged_shapes(n, m, E, L, seed):
    # n not a power of two, m not a multiple of the monomial slots per workgroup
    s = make_system(n, m, E, L, seed)
    rows = None if n <= 40 else [0, n // 2, n - 1]
    check_eval(s, L, random_point(n, L, seed=seed + 10, spread=0.2), rows=rows,
               form="product" if n <= 17 else "quotient")


def test_eval_variable_term_counts_and_constants():
    # polynomials with 1, 2 and 9 terms; constant monomials; a zero exponent row
    import paper_1109_0545_amd as q

    polys = [
        [((0.5, -0.25), [0, 0, 0])],
        [((1, 0), [3, 0, 1]), ((-2, 1), [0, 0, 0])],
        [((k / 8, 1 - k / 8), [k % 3, (k * 2) % 4, k % 2]) for k in range(9)],
    ]
    from fractions import Fraction

    polys = [[((Fraction(c[0]).limit_denominator(64), Fraction(c[1]).limit_denominator(64)), a) for c, a in p]
             for p in polys]
    exps, coefs, offs = build(polys, 3, 2)
    from synth.systems import System

    s = System(3, 2, offs, exps, coefs, np.zeros((2, 2)), np.zeros((3, 2, 2)), np.zeros(3, np.int64),
               np.zeros(3, np.int32))
    check_eval(s, 2, point([(Fraction(3, 4), Fraction(-1, 2)), (Fraction(5, 8), 0), (0, Fraction(7, 8))]))


def zero_coordinate_system():
    """n = 7 with x_0 = x_3 = x_6 = 0 exactly: each monomial holds at most one of
    the zero coordinates (first, middle or last variable of the walk), with
    exponent 1 (its partial is the product of the other factors) or 2 (its
    partial vanishes), beside nonzero coordinates; some monomials hold none."""
    from fractions import Fraction

    n = 7
    polys = []
    for i in range(n):
        terms = []
        for k in range(8):
            a = [0] * n
            for v in (1, 2, 4, 5):
                a[v] = (i + k + v) % 3
            z = (0, 3, 6, None)[k % 4]
            if z is not None:
                a[z] = 1 + (k // 4 + i) % 2
            terms.append(((Fraction(k + 1, 8), Fraction(i - k, 16)), a))
        polys.append(terms)
    exps, coefs, offs = build(polys, n, 2)
    from synth.systems import System

    s = System(n, 2, offs, exps, coefs, np.zeros((2, 2)), np.zeros((n, 2, 2)), np.zeros(n, np.int64),
               np.zeros(n, np.int32))
    x = point([(0, 0), (Fraction(3, 4), Fraction(1, 8)), (Fraction(-5, 8), Fraction(1, 2)), (0, 0),
               (Fraction(7, 8), Fraction(-1, 4)), (Fraction(1, 2), Fraction(3, 8)), (0, 0)])
    return s, x


def test_eval_exact_zero_coordinates():
    # a zero factor inside the Speelpenning walk, against the plain product form
    s, x = zero_coordinate_system()
    check_eval(s, 2, x)


def test_speelpenning_closed_form_on_gpu():
    # f_0 = prod_v x_v at x_v = r: every partial is r^(n-1)
    import paper_1109_0545_amd as q
    from fractions import Fraction

    n = 48
    polys = [[((1, 0), [1] * n)]] + [[((1, 0), [0] * n)]] * (n - 1)
    exps, coefs, offs = build(polys, n, 2)
    S = q.System(n, offs, exps, coefs, 2)
    r = (Fraction(7, 8), Fraction(1, 4))
    x = point([r] * n)
    say("speelpenning n", n)
    y, J = q.eval_jacobian(S, x, 2)
    with mpmath.workprec(400):
        rc = mpmath.mpc(mpmath.mpf(7) / 8, mpmath.mpf(1) / 4)
        ref = rc ** (n - 1)
        from oracle.numbers import mpc_of

        for v in range(n):
            assert abs(mpc_of(J[0, v]) - ref) <= 1e-30 * abs(ref)


@pytest.mark.parametrize("t", [0.0, 0.37, 1.0])
def test_eval_homotopy_n32(t):
    import paper_1109_0545_amd as q

    s = config_system(CONFIGS["n32_dd"])
    S = q.System.from_synth(s)
    H = q.Homotopy(S, s.gamma)
    x = random_point(s.n, 2, seed=8, spread=0.05)
    say("eval_homotopy n32 t", t)
    y, J, sc = q.eval_homotopy(H, t, x, 2)
    rows = [0, 5, 31]
    ref = o_eval_homotopy(s.exps, s.coefs, s.poly_offsets, s.gamma, t, x, rows=rows, form="quotient")
    check_homotopy_rows(s, 2, t, x, ref, y, J, sc)


def check_homotopy_rows(s, L, t, x, ref, y, J, sc):
    """tau times the componentwise scale, plus the rounding bound of the
    start-system power (binary powering in working precision) on h_i and J_ii."""
    u = 2.0 ** (-53 * L)
    worst = 0.0  # |d| / (u S): the observed error in units of the componentwise scale
    for r, i in enumerate(ref.rows):
        bv, bd = start_power_bounds(L, t, s.gamma, x[i], int(s.degrees[i]))
        worst = max(worst, err_over_scale(y[i], ref.y[r], u * ref.S[r]))
        assert err_over_scale(y[i], ref.y[r], TAU[L] * ref.S[r] + bv) <= 1.0
        assert abs(sc[i] - float(ref.S[r])) <= 1e-12 * float(ref.S[r])
        for v in range(s.n):
            extra = bd if v == i else 0.0
            worst = max(worst, err_over_scale(J[i, v], ref.J[r][v], u * ref.SJ[r][v]))
            assert err_over_scale(J[i, v], ref.J[r][v], TAU[L] * ref.SJ[r][v] + extra) <= 1.0
    say(f"  homotopy rows: worst |d| / (u S) = {worst:.2f} (bound {TAU[L] / u:.0f} plus the start-power term)")


def test_eval_dev_variant_matches_host_variant():
    import torch

    import paper_1109_0545_amd as q

    s = config_system(CONFIGS["n32_dd"])
    S = q.System.from_synth(s)
    x = random_point(s.n, 2, seed=9, spread=0.1)
    say("eval_jacobian_dev n32")
    y, J = q.eval_jacobian(S, x, 2)
    xd = torch.from_numpy(x).cuda()
    yd = torch.zeros((s.n, 2, 2), dtype=torch.float64, device="cuda")
    Jd = torch.zeros((s.n, s.n, 2, 2), dtype=torch.float64, device="cuda")
    q.eval_jacobian_dev(S, xd, 2, yd, Jd, stream=torch.cuda.current_stream())
    torch.cuda.synchronize()
    assert np.array_equal(yd.cpu().numpy(), y) and np.array_equal(Jd.cpu().numpy(), J)


def test_eval_is_deterministic():
    import paper_1109_0545_amd as q

    s = config_system(CONFIGS["n64_dd"])
    S = q.System.from_synth(s)
    x = random_point(s.n, 2, seed=10, spread=0.05)
    say("eval determinism n64")
    a = q.eval_jacobian(S, x, 2)
    b = q.eval_jacobian(S, x, 2)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_eval_rejects_bad_precision_and_nonfinite():
    import paper_1109_0545_amd as q

    s = config_system(CONFIGS["n8_dd"])
    S = q.System.from_synth(s)
    with pytest.raises(q.QdpError):
        q.eval_jacobian(S, np.zeros((8, 2, 4)), 4)  # above the stored precision
    x = random_point(8, 2, seed=1)
    x[3, 1, 0] = np.inf
    with pytest.raises(q.QdpError) as e:
        q.eval_jacobian(S, x, 2)
    assert e.value.status == 4


@pytest.mark.parametrize("name,B,rows", [("n8_dd", 5, None), ("n32_dd", 3, [0, 13, 31]), ("n64_dd", 2, [0, 33, 63]),
                                         ("n64_qd", 2, [7, 63]), ("n64_qd", 8, [7, 63]), ("n128_dd", 1, [0, 127]),
                                         ("ragged", 2, [0, 50, 99])])
def test_eval_homotopy_batch_vs_oracle(name, B, rows):
    # B points in one launch; the monomials of a polynomial split over several
    # workgroups (the ragged system: 6 monomials over 4 parts, one part empty);
    # n64_qd at 8 points is not split and takes four variables per lane (the
    # first and last points checked against the oracle)
    import torch

    import paper_1109_0545_amd as q

    s = make_system(100, 6, 2, 2, 6) if name == "ragged" else config_system(CONFIGS[name])
    L, t = s.L, 0.43
    S = q.System.from_synth(s)
    H = q.Homotopy(S, s.gamma)
    xs = np.stack([random_point(s.n, L, seed=20 + b, spread=0.05) for b in range(B)])
    say("eval_homotopy_batch", name, "B", B)
    stream = torch.cuda.current_stream()
    xd = torch.from_numpy(xs).cuda()
    yd = torch.zeros((B, s.n, 2, L), dtype=torch.float64, device="cuda")
    Jd = torch.zeros((B, s.n, s.n, 2, L), dtype=torch.float64, device="cuda")
    Sd = torch.zeros((B, s.n), dtype=torch.float64, device="cuda")
    q.eval_homotopy_batch_dev(H, t, xd, B, L, yd, Jd, Sd, stream=stream)
    torch.cuda.synchronize()
    y, J, sc = yd.cpu().numpy(), Jd.cpu().numpy(), Sd.cpu().numpy()
    for b in (range(B) if B <= 5 else (0, B - 1)):
        ref = o_eval_homotopy(s.exps, s.coefs, s.poly_offsets, s.gamma, t, xs[b], rows=rows,
                              form="product" if s.n <= 8 else "quotient")
        check_homotopy_rows(s, L, t, xs[b], ref, y[b], J[b], sc[b])
    # the same launch again gives the same bits (fixed-order partial sums)
    y2 = torch.zeros_like(yd)
    J2 = torch.zeros_like(Jd)
    q.eval_homotopy_batch_dev(H, t, xd, B, L, y2, J2, None, stream=stream)
    torch.cuda.synchronize()
    assert torch.equal(y2, yd) and torch.equal(J2, Jd)
