"""Newton corrector (eval + GE + back substitution + update) vs the oracle."""

import mpmath
import numpy as np
import pytest

from oracle.evaluate import eval_homotopy as o_eval_homotopy
from oracle.newton import cond_inf, inv_norm_inf, newton_step as o_newton_step, newton_tolerance
from oracle.numbers import mpc_of, to_limbs_complex
from synth.systems import CONFIGS, config_system, start_root
from tests.gpu_helpers import fixture, say, zss_mpc

pytestmark = pytest.mark.gpu


def limbs_point(vals, L):
    return np.stack([to_limbs_complex(mpmath.mpc(v), L) for v in vals])


def one_step_parity(name, L, t=0.5, form="product", mode=0):
    import paper_1109_0545_amd as q

    s = config_system(CONFIGS[name])
    s = s.truncated(L) if L < s.L else s
    fix = fixture(name)
    x = limbs_point([complex(a, b) for a, b in fix["x_half_f64"]], L)
    S = q.System.from_synth(s)
    H = q.Homotopy(S, s.gamma)
    say("newton one step", name, "L", L, "t", t, "mode", mode)
    xg, info = q.newton_step(H, t, x, L, mode=mode, eps=0.0, max_it=1)
    return check_step(s, x, t, L, xg, info, form)


def check_step(s, x, t, L, xg, info, form):
    """One GPU Newton iteration from x (result xg, info) against the oracle's step."""
    assert info["iterations"] == 1 and not info["success"] and not info["singular"]
    ref = o_newton_step(s.exps, s.coefs, s.poly_offsets, s.gamma, t, x, form=form)
    hs = o_eval_homotopy(s.exps, s.coefs, s.poly_offsets, s.gamma, t, x, form=form)
    with mpmath.workprec(600):
        kappa = cond_inf(ref.J, 300)
        jinv = inv_norm_inf(ref.J, 300)
        dzn = max(float(abs(d)) for d in ref.dz)
        zn = max(float(abs(z)) for z in ref.z)
        tol = newton_tolerance(s.n, kappa, L, dzn, zn, jinv, float(max(hs.S)))
        err = max(float(abs(mpc_of(xg[v]) - ref.z[v])) for v in range(s.n))
    say(f"  one step: |z_gpu - z_oracle| = {err:.3e}, bound {tol:.3e} (ratio {err / tol:.2e}), kappa {kappa:.3g}")
    assert err <= tol, (err, tol, kappa)
    # the residual agrees to FP64 unless it sits at the rounding floor of L limbs
    assert abs(info["residual_first"] - ref.rho) <= 1e-6 * ref.rho + 64 * s.n * 2.0 ** (-53 * L)
    return err, tol


def test_one_step_n8_dd():
    one_step_parity("n8_dd", 2)


def test_one_step_n8_f64():
    one_step_parity("n8_dd", 1)


def test_one_step_n32_dd():
    one_step_parity("n32_dd", 2, form="quotient")


def test_one_step_n64_qd():
    one_step_parity("n64_qd", 4, form="quotient")


def test_one_step_n64_dd():
    one_step_parity("n64_dd", 2, form="quotient")


@pytest.mark.parametrize("n", [48, 57, 64])
def test_elimination_sizes_and_batch(n):
    # sizes up to the largest matrix kept in LDS (odd and even n): a batch of
    # points, the first against the oracle, each bit for bit equal to its
    # single-point call
    import torch

    import paper_1109_0545_amd as q
    from synth.systems import make_system, random_point

    s = make_system(n, 12, 2, 2, 40 + n)
    S = q.System.from_synth(s)
    H = q.Homotopy(S, s.gamma)
    B, t = 3, 0.4
    xs = np.stack([random_point(n, 2, seed=60 + b, spread=0.05) for b in range(B)])
    say("elimination n", n, "B", B)
    stream = torch.cuda.current_stream()
    xd = torch.from_numpy(xs).cuda()
    q.newton_batch_dev(H, t, xd, B, 2, eps=0.0, max_it=1, stream=stream)
    infos = q.last_info_batch(H, 2, B, stream=stream)
    xg = xd.cpu().numpy()
    for b in range(B):
        x1, info1 = q.newton_step(H, t, xs[b], 2, eps=0.0, max_it=1)
        assert np.array_equal(xg[b], x1), b
        if b == 0:
            check_step(s, xs[b], t, 2, xg[b], infos[b], "quotient")


@pytest.mark.parametrize("name,L", [("n8_dd", 2), ("n32_dd", 2), ("n64_dd", 2), ("n64_qd", 4), ("n128_dd", 2)])
def test_one_step_mixed_precision(name, L):
    # FP64 factorization + refinement in the working precision: same bound as
    # the full elimination (the refinement reaches the working precision's level)
    one_step_parity(name, L, form="quotient", mode=1)


@pytest.mark.parametrize("name,L", [("n64_dd", 2), ("n128_dd", 2), ("n64_qd", 4)])
def test_mixed_precision_converges_to_target_root(name, L):
    import paper_1109_0545_amd as q

    fix = fixture(name)
    s = config_system(CONFIGS[name])
    S = q.System.from_synth(s)
    H = q.Homotopy(S, s.gamma)
    x = np.zeros((s.n, 2, L))
    x[:, :, 0] = s.zstar[:, :, 0]
    u = 2.0 ** (-53 * L)
    say("newton mixed converge", name)
    xg, info = q.newton_step(H, 1.0, x, L, mode=q.SOLVE_MIXED_IR, eps=64 * u, max_it=6)
    zss = zss_mpc(fix)
    with mpmath.workprec(600):
        err = max(float(abs(mpc_of(xg[v]) - zss[v])) for v in range(s.n))
    say(f"  |z - z**| = {err:.3e} = {err / u:.1f} u, refinements in the last step {info['refine_steps']}")
    assert info["success"] and info["refine_steps"] >= 1
    assert err <= 1e4 * u, err


@pytest.mark.parametrize("name,L,max_steps,floor", [("n32_dd", 2, 3, 1e-24), ("n64_qd", 4, 6, 1e-50)])
def test_mixed_precision_refinement_contracts(name, L, max_steps, floor):
    # the textbook iterative-refinement property: from a point off the root the
    # refinement of one Newton correction contracts (each step by about
    # kappa u64) and stops within its budget of steps, once its last relative
    # correction, or the next one predicted from the contraction, is at the
    # working precision's level; so the last correction itself lies well
    # below FP64 resolution (~1e-27 at n32 DD after two refinements, whose
    # predicted successor is ~1e-40)
    import paper_1109_0545_amd as q

    s = config_system(CONFIGS[name])
    S = q.System.from_synth(s)
    H = q.Homotopy(S, s.gamma)
    x = np.zeros((s.n, 2, L))
    x[:, :, 0] = s.zstar[:, :, 0] + 1e-6
    say("mixed refinement contraction", name)
    _, info = q.newton_step(H, 1.0, x, L, mode=q.SOLVE_MIXED_IR, eps=0.0, max_it=1)
    say(f"  {info['refine_steps']} refinements, last relative correction {info['refine_err']:.3e}")
    assert 1 <= info["refine_steps"] <= max_steps
    assert info["refine_err"] < floor


def test_mixed_precision_rejects_fp64():
    # the mixed mode refines in a working precision above the factorization's
    import paper_1109_0545_amd as q

    s = config_system(CONFIGS["n8_dd"])
    S = q.System.from_synth(s)
    H = q.Homotopy(S, s.gamma)
    with pytest.raises(q.QdpError) as e:
        q.newton_step(H, 1.0, np.zeros((s.n, 2, 1)), 1, mode=q.SOLVE_MIXED_IR)
    assert e.value.status == 5


def tiny_system(n, L, seed):
    """A dense system at n <= 2 (the random generator needs more distinct
    monomials than one or two variables of degree <= 2 allow): every
    polynomial has the constant, each x_v, and prod x_v^2, with unit-circle
    coefficients."""
    from synth.systems import System

    rng = np.random.Generator(np.random.PCG64(seed))
    rows = [[0] * n] + [[1 if k == v else 0 for k in range(n)] for v in range(n)] + [[2] * n]
    m = len(rows)
    exps = np.array([r for _ in range(n) for r in rows], dtype=np.uint8)
    ang = rng.uniform(0.0, 2 * np.pi, n * m + 1)
    coefs = np.zeros((n * m, 2, L))
    coefs[:, 0, 0], coefs[:, 1, 0] = np.cos(ang[:-1]), np.sin(ang[:-1])
    gamma = np.zeros((2, L))
    gamma[0, 0], gamma[1, 0] = np.cos(ang[-1]), np.sin(ang[-1])
    offsets = np.arange(0, n * m + 1, m, dtype=np.int32)
    return System(n, L, offsets, exps, coefs, gamma, np.zeros((n, 2, L)), np.zeros(n, dtype=np.int64),
                  np.full(n, 2 * n, dtype=np.int32))


@pytest.mark.parametrize("n,L", [(1, 2), (2, 2), (17, 4), (63, 2), (64, 2), (65, 2), (65, 4), (100, 2), (128, 4)])
def test_mixed_matches_full_across_sizes(n, L):
    # the two solve modes on random systems at the sizes where the mixed kernel
    # changes shape (one row, ragged tails, the last size with both factors in
    # LDS, the first with them in the global store, the largest): one Newton
    # step each from the same point; both are within the one-step bound of the
    # exact step, so they agree to twice that bound's working-precision scale
    import paper_1109_0545_amd as q
    from synth.systems import make_system, random_point

    s = tiny_system(n, L, 300 + n) if n <= 2 else make_system(n, min(n, 16), 2, L, 300 + n)
    S = q.System.from_synth(s)
    H = q.Homotopy(S, s.gamma)
    x = random_point(n, L, seed=400 + n, spread=0.05)
    say("mixed vs full n", n, "L", L)
    xf, inf_f = q.newton_step(H, 0.6, x, L, mode=q.SOLVE_FULL, eps=0.0, max_it=1)
    xm, inf_m = q.newton_step(H, 0.6, x, L, mode=q.SOLVE_MIXED_IR, eps=0.0, max_it=1)
    assert not inf_f["singular"] and not inf_m["singular"]
    assert inf_m["residual_first"] == inf_f["residual_first"]
    u = 2.0 ** (-53 * L)
    kappa = max(inf_f["cond_est"], 1.0)
    with mpmath.workprec(600):
        d = max(float(abs(mpc_of(xm[v]) - mpc_of(xf[v]))) for v in range(n))
        zn = max(float(abs(mpc_of(xf[v]))) for v in range(n))
        dzn = max(float(abs(mpc_of(xf[v]) - mpc_of(x[v]))) for v in range(n))
    bound = 64 * n * kappa * u * max(zn, dzn, 1.0)
    say(f"  |z_mixed - z_full| = {d:.3e}, bound {bound:.3e}, refinements {inf_m['refine_steps']}")
    assert d <= bound, (d, bound)
    assert inf_m["refine_steps"] >= 1


@pytest.mark.parametrize("name,L", [("n8_dd", 2), ("n32_dd", 2), ("n64_qd", 4), ("n64_dd", 2), ("n128_dd", 2)])
def test_converges_to_target_root(name, L):
    # at t = 1 (h = f) from the planted point cut to one limb, Newton reaches
    # the exact root z** of the stored system to working precision
    import paper_1109_0545_amd as q

    fix = fixture(name)
    s = config_system(CONFIGS[name])
    S = q.System.from_synth(s)
    H = q.Homotopy(S, s.gamma)
    x = np.zeros((s.n, 2, L))
    x[:, :, 0] = s.zstar[:, :, 0]
    say("newton converge", name)
    xg, info = q.newton_step(H, 1.0, x, L, eps=64 * 2.0 ** (-53 * L), max_it=6)
    zss = zss_mpc(fix)
    with mpmath.workprec(600):
        err = max(float(abs(mpc_of(xg[v]) - zss[v])) for v in range(s.n))
    assert info["success"] and 2 <= info["iterations"] <= 6
    assert err <= 1e4 * 2.0 ** (-53 * L), err


def test_loop_semantics_on_gpu():
    import paper_1109_0545_amd as q

    s = config_system(CONFIGS["n8_dd"])
    S = q.System.from_synth(s)
    H = q.Homotopy(S, s.gamma)
    x = s.zstar.copy()
    say("newton semantics")
    xg, info = q.newton_step(H, 1.0, x, 2, eps=1.0, max_it=5)
    assert info["iterations"] == 0 and not info["success"] and np.array_equal(xg, x)
    xg, info = q.newton_step(H, 1.0, x, 2, eps=2.0, max_it=5)
    assert info["iterations"] == 0 and info["success"]
    xg, info = q.newton_step(H, 1.0, x, 2, eps=0.0, max_it=3)
    assert info["iterations"] == 3 and not info["success"]
    xg, info = q.newton_step(H, 1.0, x, 2, eps=1e-10, max_it=0)
    assert info["iterations"] == 0 and not info["success"]


@pytest.mark.parametrize("name", ["n8_dd", "n64_dd"])
def test_singular_jacobian_is_reported(name):
    # t = 0: h = gamma (x^d - 1); at x = 0 the Jacobian gamma d x^(d-1) vanishes
    import paper_1109_0545_amd as q

    s = config_system(CONFIGS[name])
    S = q.System.from_synth(s)
    H = q.Homotopy(S, s.gamma)
    x = np.zeros((s.n, 2, 2))
    say("newton singular")
    xg, info = q.newton_step(H, 0.0, x, 2, eps=1e-10, max_it=4)
    assert info["singular"] == 1 and not info["success"] and info["iterations"] == 1
    assert np.array_equal(xg, x)


@pytest.mark.parametrize("name, prec, mode",
                         [("n8_dd", 2, 0), ("n32_dd", 2, 0), ("n32_dd", 2, 1), ("n64_qd", 4, 0), ("n64_dd", 2, 0),
                          ("n128_dd", 2, 0)])
def test_singular_later_column_is_reported(name, prec, mode):
    # t = 0: J = diag(gamma d_i x_i^(d_i - 1)); with one coordinate x_k = 0
    # (d_k >= 2) and the others on the unit circle, column k is the first
    # column without a nonzero pivot, found by the look-ahead step of column
    # k - 1 (a quarter in, the middle and the last column)
    import paper_1109_0545_amd as q

    s = config_system(CONFIGS[name])
    S = q.System.from_synth(s)
    H = q.Homotopy(S, s.gamma)
    cand = [k for k in range(s.n) if s.degrees[k] >= 2]
    for k in sorted({cand[len(cand) // 4], cand[len(cand) // 2], cand[-1]}):
        x = np.zeros((s.n, 2, prec))
        x[:, 0, 0] = 1.0
        x[k, 0, 0] = 0.0
        say(f"newton singular column {k} {name} mode {mode}")
        xg, info = q.newton_step(H, 0.0, x, prec, mode=mode, eps=1e-10, max_it=4)
        assert info["singular"] == 1 and not info["success"] and info["iterations"] == 1, (k, info)
        assert np.array_equal(xg, x)


def test_residual_sequence_matches_oracle():
    # four single iterations from a perturbed planted root at t = 1: every
    # residual agrees with the oracle's Newton run (quadratic convergence in
    # the oracle is pinned separately)
    import paper_1109_0545_amd as q
    from oracle.newton import newton

    s = config_system(CONFIGS["n32_dd"])
    S = q.System.from_synth(s)
    H = q.Homotopy(S, s.gamma)
    x = np.zeros((s.n, 2, 2))
    x[:, :, 0] = s.zstar[:, :, 0] + 1e-5
    ref = newton(s.exps, s.coefs, s.poly_offsets, s.gamma, 1.0, x, eps=0.0, max_it=4, form="quotient").residuals
    res = []
    say("newton residual sequence n32")
    for _ in range(4):
        x, info = q.newton_step(H, 1.0, x, 2, eps=0.0, max_it=1)
        res.append(info["residual_first"])
    for a, b in zip(res, ref):
        assert abs(a - b) <= 1e-6 * b + 1e-29, (res, ref)


@pytest.mark.parametrize("mode", [0, 1])
def test_batch_newton_each_point_matches_oracle(mode):
    # B points in one launch per kernel (evaluation split over workgroups,
    # one elimination workgroup per point); each point against the oracle
    import torch

    import paper_1109_0545_amd as q

    name, L, t, B = "n32_dd", 2, 0.5, 3
    s = config_system(CONFIGS[name])
    fix = fixture(name)
    base = [complex(a, b) for a, b in fix["x_half_f64"]]
    rng = np.random.Generator(np.random.PCG64(5))
    xs = np.stack([limbs_point([v * (1 + 1e-3 * b * complex(*rng.standard_normal(2))) for v in base], L)
                   for b in range(B)])
    S = q.System.from_synth(s)
    H = q.Homotopy(S, s.gamma)
    say("newton batch", name, "B", B, "mode", mode)
    stream = torch.cuda.current_stream()
    xd = torch.from_numpy(xs).cuda()
    q.newton_batch_dev(H, t, xd, B, L, mode=mode, eps=0.0, max_it=1, stream=stream)
    infos = q.last_info_batch(H, L, B, stream=stream)
    xg = xd.cpu().numpy()
    for b in range(B):
        check_step(s, xs[b], t, L, xg[b], infos[b], "quotient")


def test_batch_newton_points_run_their_own_loops():
    # a converged point stops after one iteration while the others continue:
    # every point's iteration count and success flag equal its single-point run
    import torch

    import paper_1109_0545_amd as q

    name, L, t = "n32_dd", 2, 1.0
    s = config_system(CONFIGS[name])
    fix = fixture(name)
    zss = [complex(mpc_of(np.array(v))) for v in fix["zss_limbs"]]
    pts = [limbs_point(zss, L), limbs_point([v * (1 + 1e-4) for v in zss], L),
           limbs_point([v * (1 + 3e-3j) for v in zss], L)]
    S = q.System.from_synth(s)
    H = q.Homotopy(S, s.gamma)
    say("newton batch loops", name)
    stream = torch.cuda.current_stream()
    xd = torch.from_numpy(np.stack(pts)).cuda()
    q.newton_batch_dev(H, t, xd, len(pts), L, eps=1e-24, max_it=6, stream=stream)
    infos = q.last_info_batch(H, L, len(pts), stream=stream)
    single = [q.newton_step(H, t, p, L, eps=1e-24, max_it=6)[1] for p in pts]
    for a, b in zip(infos, single):
        assert (a["iterations"], a["success"]) == (b["iterations"], b["success"]), (infos, single)
    assert infos[0]["success"] and infos[0]["iterations"] < infos[2]["iterations"] <= 6


@pytest.mark.parametrize("n,L", [(1, 2), (12, 4), (40, 1), (64, 1)])
def test_one_step_small_systems(n, L):
    # edge shapes of the elimination: n = 1 (no pivot chain), quad double
    # with the matrix in LDS, FP64 up to n = 64
    import paper_1109_0545_amd as q
    from synth.systems import make_system, random_point

    s = make_system(n, 3 if n == 1 else 6, 2, max(L, 2), 30 + n)
    s = s.truncated(L) if L < s.L else s
    x = random_point(n, L, seed=31 + n, spread=0.1)
    S = q.System.from_synth(s)
    H = q.Homotopy(S, s.gamma)
    say("newton small system n", n, "L", L)
    xg, info = q.newton_step(H, 0.3, x, L, eps=0.0, max_it=1)
    check_step(s, x, 0.3, L, xg, info, "product" if n <= 12 else "quotient")


@pytest.mark.parametrize("n,L", [(200, 2), (100, 4), (256, 1)])
def test_newton_converges_at_large_n(n, L):
    # beyond the oracle's reach: from a point near the planted root of a
    # system at t = 1, the Newton loop must converge (residual below the
    # working precision's floor within a few iterations, quadratically);
    # covers the elimination with four (n > 128) and two rows per lane and
    # quad double with the matrix in global memory
    import paper_1109_0545_amd as q
    from synth.systems import make_system

    s = make_system(n, 12, 2, max(L, 2), 50 + n)
    s = s.truncated(L) if L < s.L else s
    rng = np.random.Generator(np.random.PCG64(n))
    x = np.zeros((n, 2, L))
    x[:, :, 0] = s.zstar[:, :, 0] * (1.0 + 1e-7 * rng.standard_normal((n, 1)))
    S = q.System.from_synth(s)
    H = q.Homotopy(S, s.gamma)
    say("newton large n", n, "L", L)
    eps = {1: 1e-12, 2: 1e-26, 4: 1e-55}[L]
    xg, info = q.newton_step(H, 1.0, x, L, eps=eps, max_it=8)
    assert info["success"] and not info["singular"] and info["iterations"] <= 6, info
    _, info2 = q.newton_step(H, 1.0, xg, L, eps=0.0, max_it=1)
    assert info2["residual_first"] <= eps, info2
