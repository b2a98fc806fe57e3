"""The column-parallel eliminations (one workgroup per column of [A | -h], or
blocks of 16 columns per workgroup: Section 4's GE and Back_Subs spread over
compute units) against the one-workgroup-per-point kernels: bit for bit where
the latter is the register kernel (double double, n <= 64: same pivots, same
updates in the same order), within the one-step bound elsewhere; batches equal
single calls; singular and non-finite cases reported as the point kernels
report them."""

import mpmath
import numpy as np
import pytest

from oracle.numbers import mpc_of
from synth.systems import CONFIGS, config_system, make_system, random_point
from tests.gpu_helpers import say

pytestmark = pytest.mark.gpu


@pytest.fixture
def policy():
    import paper_1109_0545_amd as q

    yield q.set_elimination
    q.set_elimination(q.ELIM_AUTO)


def _system(n, L, seed):
    import paper_1109_0545_amd as q
    from tests.test_gpu_newton import tiny_system

    s = tiny_system(n, L, seed) if n <= 2 else make_system(n, min(n, 16), 2, L, seed)
    return s, q.Homotopy(q.System.from_synth(s), s.gamma)


def _step(q, H, x, L, policy_value, set_policy, max_it, t=0.6):
    set_policy(policy_value)
    return q.newton_step(H, t, x, L, eps=0.0, max_it=max_it)


@pytest.mark.parametrize("layout", ["columns", "blocks"])
@pytest.mark.parametrize("n", [1, 2, 8, 15, 16, 23, 24, 33, 48, 57, 64])
def test_columns_equal_register_kernel_bit_for_bit(n, layout, policy):
    # blocks of 16 columns, the last taking up to 24 with b: one workgroup up
    # to n = 23, two from n = 24 (the second with 9 columns), ragged last
    # blocks, and 16 + 16 + 16 + 17 at n = 64
    import paper_1109_0545_amd as q

    s, H = _system(n, 2, 500 + n)
    x = random_point(n, 2, seed=510 + n, spread=0.05)
    say(layout, "vs register kernel, DD n", n)
    xp, ip = _step(q, H, x, 2, q.ELIM_POINT, policy, 3)
    xc, ic = _step(q, H, x, 2, q.ELIM_COLUMNS if layout == "columns" else q.ELIM_BLOCKS, policy, 3)
    assert ic["iterations"] == 3 and not ic["singular"] and not ic["nonfinite"]
    assert np.array_equal(xp, xc)
    assert ip == ic, (ip, ic)


@pytest.mark.parametrize("n,L", [(1, 4), (12, 4), (17, 4), (40, 4), (64, 4), (65, 2), (100, 2), (127, 2), (128, 2)])
def test_blocks_equal_columns_bit_for_bit(n, L, policy):
    # the block and column layouts in quad double and, past n = 64 (two rows
    # per lane, the triangle read from device memory), double double: same
    # pivots, same updates, same substitution; the default takes one of them
    import paper_1109_0545_amd as q

    s, H = _system(n, L, 570 + n)
    x = random_point(n, L, seed=580 + n, spread=0.05)
    say("blocks vs columns n", n, "L", L)
    xc, ic = _step(q, H, x, L, q.ELIM_COLUMNS, policy, 2)
    xb, ib = _step(q, H, x, L, q.ELIM_BLOCKS, policy, 2)
    xa, ia = _step(q, H, x, L, q.ELIM_AUTO, policy, 2)
    assert ib["iterations"] == 2 and not ib["singular"] and not ib["nonfinite"]
    assert np.array_equal(xb, xc) and ib == ic, (ib, ic)
    assert np.array_equal(xa, xb) and ia == ib


@pytest.mark.parametrize("n,L", [(12, 4), (64, 4), (65, 2), (100, 2), (128, 2), (128, 4)])
def test_columns_agree_with_point_kernel(n, L, policy):
    # different pivot keys (the point kernel compares full FP64 magnitudes,
    # the column kernel 32-bit keys) can pick different pivots among near
    # ties: both steps are within the one-step bound of the exact step, so
    # they agree to twice that bound's working-precision scale
    import paper_1109_0545_amd as q

    s, H = _system(n, L, 520 + n)
    x = random_point(n, L, seed=530 + n, spread=0.05)
    say("columns vs point kernel n", n, "L", L)
    xp, ip = _step(q, H, x, L, q.ELIM_POINT, policy, 1)
    xc, ic = _step(q, H, x, L, q.ELIM_COLUMNS, policy, 1)
    xa, ia = _step(q, H, x, L, q.ELIM_AUTO, policy, 1)
    assert np.array_equal(xa, xc) and ia == ic  # the default takes columns or blocks here
    assert not ic["singular"] and not ic["nonfinite"] and ic["iterations"] == 1
    assert ic["residual_first"] == ip["residual_first"]
    u = 2.0 ** (-53 * L)
    kappa = max(ip["cond_est"], 1.0)
    with mpmath.workprec(600):
        d = max(float(abs(mpc_of(xc[v]) - mpc_of(xp[v]))) for v in range(n))
        zn = max(float(abs(mpc_of(xp[v]))) for v in range(n))
        dzn = max(float(abs(mpc_of(xp[v]) - mpc_of(x[v]))) for v in range(n))
    bound = 64 * n * kappa * u * max(zn, dzn, 1.0)
    say(f"  |z_columns - z_point| = {d:.3e}, bound {bound:.3e}")
    assert d <= bound, (d, bound)


@pytest.mark.parametrize("n,L,B,m,layout", [(57, 2, 3, 6, "columns"), (64, 4, 4, 2, "columns"),
                                            (128, 2, 2, 6, "columns"), (57, 2, 3, 6, "blocks"),
                                            (64, 2, 5, 6, "blocks"), (64, 4, 3, 2, "blocks"),
                                            (128, 2, 2, 6, "blocks")])
def test_columns_batch_equals_single_calls(n, L, B, m, layout, policy):
    # m monomials per polynomial, fewer than a workgroup part's minimum of two
    # wavefronts' worth (lanes per monomial: 16 here in double double, 32 in
    # quad double), so the evaluation is never split over workgroups (its
    # split depends on the batch size) and batch and single calls eliminate
    # the same matrices
    import torch

    import paper_1109_0545_amd as q

    s = make_system(n, m, 2, L, 540 + n)
    H = q.Homotopy(q.System.from_synth(s), s.gamma)
    xs = np.stack([random_point(n, L, seed=550 + b, spread=0.05) for b in range(B)])
    policy(q.ELIM_COLUMNS if layout == "columns" else q.ELIM_BLOCKS)
    say(layout, "batch n", n, "L", L, "B", B)
    stream = torch.cuda.current_stream()
    xd = torch.from_numpy(xs).cuda()
    q.newton_batch_dev(H, 0.4, xd, B, L, eps=0.0, max_it=2, stream=stream)
    infos = q.last_info_batch(H, L, B, stream=stream)
    xg = xd.cpu().numpy()
    for b in range(B):
        x1, i1 = q.newton_step(H, 0.4, xs[b], L, eps=0.0, max_it=2)
        assert np.array_equal(xg[b], x1), b
        assert infos[b] == i1, (b, infos[b], i1)


@pytest.mark.parametrize("layout", ["columns", "blocks"])
@pytest.mark.parametrize("name,prec", [("n8_dd", 2), ("n64_dd", 2), ("n64_qd", 4), ("n128_dd", 2)])
def test_columns_report_singular_columns(name, prec, layout, policy):
    # t = 0, x_k = 0 (d_k >= 2), the other coordinates on the unit circle:
    # column k is the first without a nonzero pivot (in the first, a middle
    # and the last block)
    import paper_1109_0545_amd as q

    s = config_system(CONFIGS[name])
    H = q.Homotopy(q.System.from_synth(s), s.gamma)
    cand = [k for k in range(s.n) if s.degrees[k] >= 2]
    policy(q.ELIM_COLUMNS if layout == "columns" else q.ELIM_BLOCKS)
    for k in sorted({cand[0], cand[len(cand) // 2], cand[-1]}):
        x = np.zeros((s.n, 2, prec))
        x[:, 0, 0] = 1.0
        x[k, 0, 0] = 0.0
        say(f"{layout} singular column {k} {name}")
        xg, info = q.newton_step(H, 0.0, x, prec, eps=1e-10, max_it=4)
        assert info["singular"] == 1 and not info["success"] and info["iterations"] == 1, (k, info)
        assert np.isinf(info["cond_est"])
        assert np.array_equal(xg, x)


@pytest.mark.parametrize("L", [2, 4])
def test_columns_report_nonfinite_residual(L, policy):
    # |x| = 1e100 with degrees up to 4: h overflows, the step is refused and
    # the point left unchanged, as the point kernels do
    import paper_1109_0545_amd as q

    s, H = _system(16, L, 560)
    x = np.zeros((16, 2, L))
    x[:, 0, 0] = 1e100
    out = {}
    for pol in (q.ELIM_POINT, q.ELIM_COLUMNS, q.ELIM_BLOCKS):
        policy(pol)
        say("columns non-finite h, policy", pol, "L", L)
        xg, info = q.newton_step(H, 0.5, x, L, eps=1e-10, max_it=3)
        assert info["nonfinite"] == 1 and not info["success"] and not info["singular"], info
        assert info["iterations"] == 1
        assert np.array_equal(xg, x)
        out[pol] = info
    assert np.isnan(out[q.ELIM_COLUMNS]["residual_first"])
