"""Common-support systems (every polynomial sums the same monomials, the
workload of the paper's Table 1): the evaluation through the monomials'
partials and a dense coefficient product, against the oracle and against the
general sparse evaluation of the same polynomials.  Tolerances as in
test_gpu_eval (tau times the componentwise scale, plus the start-power
rounding bound) and test_gpu_newton (the oracle's step within the stated
Newton tolerance)."""

import mpmath
import numpy as np
import pytest

from oracle.evaluate import eval_homotopy as o_eval_homotopy
from oracle.evaluate import eval_system as o_eval_system
from oracle.numbers import mpc_of
from synth.systems import CONFIGS, System, config_system, make_system, random_point
from tests.gpu_helpers import err_over_scale, say
from tests.test_gpu_eval import TAU, check_homotopy_rows
from tests.test_gpu_newton import check_step

pytestmark = pytest.mark.gpu


def small_common(L, seed=11, n=8, m=12):
    return make_system(n, m, 2, L, seed, common=True)


def reordered(s: System) -> System:
    """The same polynomials with f_1's terms in reverse order (equal polynomials,
    no longer a common support: the general evaluation runs)."""
    m = int(s.poly_offsets[1])
    perm = np.arange(s.terms)
    perm[m : 2 * m] = perm[m : 2 * m][::-1]
    return System(s.n, s.L, s.poly_offsets.copy(), np.ascontiguousarray(s.exps[perm]),
                  np.ascontiguousarray(s.coefs[perm]), s.gamma.copy(), s.zstar.copy(), s.root_phase.copy(),
                  s.degrees.copy())


@pytest.mark.parametrize("L", [1, 2, 4])
def test_common_eval_jacobian_all_rows(L):
    import paper_1109_0545_amd as q

    s = small_common(L)
    x = random_point(s.n, L, seed=21, spread=0.2)
    say("common eval_jacobian n", s.n, "L", L)
    S = q.System.from_synth(s)
    y, J = q.eval_jacobian(S, x, L)
    ref = o_eval_system(s.exps, s.coefs, s.poly_offsets, x)
    for r, i in enumerate(ref.rows):
        assert err_over_scale(y[i], ref.y[r], ref.S[r]) <= TAU[L]
        for v in range(s.n):
            assert err_over_scale(J[i, v], ref.J[r][v], ref.SJ[r][v]) <= TAU[L]


@pytest.mark.parametrize("L", [2, 4])
def test_common_eval_homotopy_all_rows(L):
    import paper_1109_0545_amd as q

    s = small_common(L, seed=12)
    x = random_point(s.n, L, seed=22, spread=0.1)
    t = 0.37
    say("common eval_homotopy n", s.n, "L", L)
    H = q.Homotopy(q.System.from_synth(s), s.gamma)
    y, J, sc = q.eval_homotopy(H, t, x, L)
    ref = o_eval_homotopy(s.exps, s.coefs, s.poly_offsets, s.gamma, t, x)
    check_homotopy_rows(s, L, t, x, ref, y, J, sc)


def test_common_eval_table1_shape_sampled_rows():
    # 40 x 40, one support of 200 monomials of degree ~40 (exponents in {0,1,2})
    import paper_1109_0545_amd as q

    s = config_system(CONFIGS["c40_dd"])
    x = random_point(s.n, 2, seed=23, spread=0.02)
    t = 0.5
    say("common eval_homotopy c40_dd")
    H = q.Homotopy(q.System.from_synth(s), s.gamma)
    y, J, sc = q.eval_homotopy(H, t, x, 2)
    ref = o_eval_homotopy(s.exps, s.coefs, s.poly_offsets, s.gamma, t, x, rows=[0, 21, 39], form="quotient")
    check_homotopy_rows(s, 2, t, x, ref, y, J, sc)


def test_common_and_general_evaluation_agree():
    # the same polynomials, once with a shared support and once with f_1's
    # terms reordered (general path): equal within the evaluation tolerance
    import paper_1109_0545_amd as q

    s = small_common(2, seed=13, n=16, m=24)
    g = reordered(s)
    x = random_point(s.n, 2, seed=24, spread=0.1)
    say("common vs general n", s.n)
    Hs = q.Homotopy(q.System.from_synth(s), s.gamma)
    Hg = q.Homotopy(q.System.from_synth(g), g.gamma)
    ys, Js, ss = q.eval_homotopy(Hs, 0.6, x, 2)
    yg, Jg, sg = q.eval_homotopy(Hg, 0.6, x, 2)
    ref = o_eval_homotopy(s.exps, s.coefs, s.poly_offsets, s.gamma, 0.6, x)
    with mpmath.workprec(600):
        for r, i in enumerate(ref.rows):
            assert err_over_scale(ys[i], mpc_of(yg[i]), 2 * TAU[2] * ref.S[r]) <= 1.0
            for v in range(s.n):
                assert err_over_scale(Js[i, v], mpc_of(Jg[i, v]), 2 * TAU[2] * ref.SJ[r][v] + 1e-300) <= 1.0


def test_common_batch_matches_single_points():
    # the batched entry point (workspace scratch for B points, ragged B) gives
    # every point bit for bit what the single-point entry point gives
    import torch

    import paper_1109_0545_amd as q

    s = small_common(2, seed=14, n=12, m=20)
    H = q.Homotopy(q.System.from_synth(s), s.gamma)
    for B in (5, 3):
        xs = np.stack([random_point(s.n, 2, seed=30 + b, spread=0.1) for b in range(B)])
        say("common batch eval B", B)
        xd = torch.from_numpy(xs).cuda()
        y = torch.zeros((B, s.n, 2, 2), dtype=torch.float64, device="cuda")
        J = torch.zeros((B, s.n, s.n, 2, 2), dtype=torch.float64, device="cuda")
        sc = torch.zeros((B, s.n), dtype=torch.float64, device="cuda")
        q.eval_homotopy_batch_dev(H, 0.25, xd, B, 2, y, J, sc)
        torch.cuda.synchronize()
        for b in range(B):
            y1, J1, s1 = q.eval_homotopy(H, 0.25, xs[b], 2)
            assert np.array_equal(y.cpu().numpy()[b], y1)
            assert np.array_equal(J.cpu().numpy()[b], J1)
            assert np.array_equal(sc.cpu().numpy()[b], s1)


@pytest.mark.parametrize("L, mode", [(2, 0), (2, 1), (4, 0), (1, 0)])
def test_common_newton_step_matches_oracle(L, mode):
    import paper_1109_0545_amd as q

    s = small_common(L, seed=15)
    x = random_point(s.n, L, seed=25, spread=0.05)
    t = 0.5
    say("common newton step L", L, "mode", mode)
    H = q.Homotopy(q.System.from_synth(s), s.gamma)
    xg, info = q.newton_step(H, t, x, L, mode=mode, eps=0.0, max_it=1)
    check_step(s, x, t, L, xg, info, "product")


def test_common_newton_converges_to_planted_root():
    # t = 1: the target system itself; from 1e-6 off the planted root Newton
    # reaches it to double-double accuracy (the batched loop of Algorithm 4.1)
    import paper_1109_0545_amd as q

    s = config_system(CONFIGS["c40_dd"])
    H = q.Homotopy(q.System.from_synth(s), s.gamma)
    rng = np.random.default_rng(26)
    x = s.zstar.copy()
    x[:, :, 0] += 1e-6 * rng.standard_normal((s.n, 2))
    x[:, :, 1] = 0.0
    say("common newton c40 to planted root")
    xg, info = q.newton_step(H, 1.0, x, 2, eps=1e-28, max_it=8)
    assert info["success"] and not info["singular"] and info["iterations"] <= 6, info
    err = np.abs((xg[:, :, 0] - s.zstar[:, :, 0]) + (xg[:, :, 1] - s.zstar[:, :, 1])).max()
    assert err <= 1e-25, err


def dense_quadratic_common(n=3, seed=19):
    """n polynomials sharing the dense support of all monomials of degree <= 2
    (random unit-circle coefficients): the total-degree homotopy's 2^n paths all
    end at the 2^n (generically finite, distinct) roots."""
    import itertools

    rows = [e for e in itertools.product(range(3), repeat=n) if sum(e) <= 2]
    m = len(rows)
    rng = np.random.Generator(np.random.PCG64(seed))
    exps = np.array(rows * n, dtype=np.uint8)
    ang = rng.random(n * m) * 2 * np.pi
    coefs = np.zeros((n * m, 2, 2))
    coefs[:, 0, 0], coefs[:, 1, 0] = np.cos(ang), np.sin(ang)
    g = rng.random() * 2 * np.pi
    gamma = np.array([[np.cos(g), 0.0], [np.sin(g), 0.0]])
    return System(n, 2, (np.arange(n + 1) * m).astype(np.int32), exps, coefs, gamma,
                  np.zeros((n, 2, 2)), np.zeros(n, np.int64), np.full(n, 2, np.int32))


def test_common_track_paths_match_single_paths_and_end_at_roots():
    # Algorithm 3.1 on a common-support system: the batched tracker gives
    # every path exactly its single-path run, every path reaches t = 1 at a
    # root of f (scaled residual at the double-double level, evaluated by the
    # oracle at the end point), and the 2^n roots are distinct
    import itertools

    import paper_1109_0545_amd as q
    from oracle.evaluate import residual
    from synth.systems import start_root

    s = dense_quadratic_common()
    H = q.Homotopy(q.System.from_synth(s), s.gamma)
    ks = [np.array(k, np.int64) for k in itertools.product(range(2), repeat=s.n)]
    x0 = np.stack([start_root(s.degrees, k, 2) for k in ks])
    p = q.default_track_params(predictor=q.PRED_QUADRATIC, max_steps=20000)
    say("common track paths B", len(ks))
    zb, stb = q.track_paths(H, x0, 2, p)
    for b in range(len(ks)):
        z1, st1, _ = q.track_path(H, x0[b], 2, p)
        for f in ("fail", "succ_corrections", "corrections", "newton_iterations", "end_success"):
            assert stb[b][f] == st1[f], (b, f, stb[b], st1)
        assert np.array_equal(zb[b], z1), b
        assert not stb[b]["fail"] and stb[b]["end_success"], (b, stb[b])
        res = o_eval_system(s.exps, s.coefs, s.poly_offsets, zb[b])
        assert residual(res) <= 1e-26, (b, residual(res))
    ends = zb[:, :, :, 0]  # leading limbs
    for a in range(len(ks)):
        for b in range(a):
            assert np.abs(ends[a] - ends[b]).max() > 1e-6, (a, b)
