"""Path tracker (Algorithm 3.1) on the GPU: endpoints vs the oracle's exact
root z**, closed-form paths, invariants, failure forcing."""

import math
from fractions import Fraction

import mpmath
import numpy as np
import pytest

from oracle.numbers import mpc_of
from oracle.track import correct_digits
from synth.systems import CONFIGS, config_system, start_root
from tests.gpu_helpers import fixture, say, zss_mpc
from tests.test_oracle_track import branch, decoupled_system

pytestmark = pytest.mark.gpu


def track_config(name, L=None, **kw):
    import paper_1109_0545_amd as q

    fix = fixture(name)
    s = config_system(CONFIGS[name])
    L = L or s.L
    S = q.System.from_synth(s)
    H = q.Homotopy(S, s.gamma)
    x0 = start_root(np.array(fix["degrees"]), np.array(fix["start_k"]), L)
    p = q.default_track_params(**kw)
    say("track", name, "L", L, kw)
    z, st, _ = q.track_path(H, x0, L, p)
    return z, st, zss_mpc(fix)


def test_track_n8_dd_endpoint_digits():
    z, st, zss = track_config("n8_dd")
    assert not st["fail"] and st["t_final"] == 1.0
    assert st["corrections"] >= st["succ_corrections"] > 0
    assert correct_digits(z, zss) >= 28


def test_track_n32_dd_endpoint_digits():
    z, st, zss = track_config("n32_dd")
    assert not st["fail"]
    assert correct_digits(z, zss) >= 28


def test_track_n64_dd_and_qd_endpoint_digits():
    # the quality-up pair of the n = 64 workload: the same draws in double double and quad double
    z, st, zss = track_config("n64_dd")
    assert not st["fail"] and correct_digits(z, zss) >= 28
    z, st, zss = track_config("n64_qd")
    assert not st["fail"] and correct_digits(z, zss) >= 60


def test_track_decoupled_closed_form():
    import paper_1109_0545_amd as q

    d = [3, 4]
    c_turns = [Fraction(1, 7), Fraction(2, 5)]
    s = decoupled_system(d, c_turns, Fraction(3, 11))
    k = [1, 2]
    S = q.System.from_synth(s)
    H = q.Homotopy(S, s.gamma)
    say("track decoupled")
    z, st, _ = q.track_path(H, start_root(np.array(d), np.array(k), 2), 2)
    assert not st["fail"]
    g = complex(mpc_of(s.gamma))
    for i in range(2):
        ref = branch(d[i], k[i], complex(mpc_of(-s.coefs[2 * i + 1])), g, 1.0)
        with mpmath.workprec(300):
            zi = mpc_of(z[i])
            # the exact root of x^d = c_stored nearest the branch endpoint
            c = -mpc_of(s.coefs[2 * i + 1])
            roots = [mpmath.root(c, d[i], j) for j in range(d[i])]
            best = min(roots, key=lambda q_: abs(complex(q_) - ref))
            assert abs(zi - best) < 1e-29


def test_track_stop_criterion_forces_failure():
    import paper_1109_0545_amd as q

    s = config_system(CONFIGS["n8_dd"])
    S = q.System.from_synth(s)
    H = q.Homotopy(S, s.gamma)
    x0 = start_root(s.degrees, np.zeros(s.n, np.int64), 2)
    p = q.default_track_params(eps_path=0.0, max_it_path=1, lambda_min=0.009)
    say("track forced stop")
    z, st, _ = q.track_path(H, x0, 2, p)
    assert st["fail"] == 1 and st["t_final"] == 0.0 and st["corrections"] == 1 and st["succ_corrections"] == 0
    p = q.default_track_params(max_steps=3)
    z, st, _ = q.track_path(H, x0, 2, p)
    assert st["corrections"] == 3 and st["fail"] == 1


def test_track_step_log_and_invariants():
    import paper_1109_0545_amd as q

    fix = fixture("n8_dd")
    s = config_system(CONFIGS["n8_dd"])
    S = q.System.from_synth(s)
    H = q.Homotopy(S, s.gamma)
    x0 = start_root(np.array(fix["degrees"]), np.array(fix["start_k"]), 2)
    say("track log n8")
    z, st, log = q.track_path(H, x0, 2, log_cap=10000)
    assert len(log) == st["corrections"]
    acc = [r["lam"] for r in log if r["accepted"]]
    assert len(acc) == st["succ_corrections"]
    assert abs(math.fsum(acc) - 1.0) < 1e-12
    for lam in acc[:-1]:
        j = math.log2(lam / 0.01)
        assert j == round(j)
    assert st["min_step"] == min(acc)


def test_track_quadratic_predictor_endpoints():
    """The quadratic predictor (Section 5) reaches z** to double-double
    accuracy and needs no more Newton iterations than the secant predictor."""
    import paper_1109_0545_amd as q

    for name in ("n8_dd", "n32_dd"):
        z, st, zss = track_config(name, predictor=q.PRED_QUADRATIC)
        assert not st["fail"] and st["t_final"] == 1.0
        assert correct_digits(z, zss) >= 28
        _, sec, _ = track_config(name)
        say(name, "newton iterations quadratic", st["newton_iterations"], "secant", sec["newton_iterations"])
        assert st["newton_iterations"] <= sec["newton_iterations"]


def test_track_quadratic_predictions_match_oracle():
    """Step by step against the oracle tracker on the n = 8 workload: while both
    take the same steps, the predictor's displacement max_v |z'_v - z_v|
    (|re| + |im|) agrees with the oracle's interpolant through the last three
    accepted points (FP64 coefficients on the device: 1e-12 relative)."""
    import paper_1109_0545_amd as q
    from oracle.track import TrackParams, track_reference

    fix = fixture("n8_dd")
    s = config_system(CONFIGS["n8_dd"])
    S = q.System.from_synth(s)
    H = q.Homotopy(S, s.gamma)
    x0 = start_root(np.array(fix["degrees"]), np.array(fix["start_k"]), 2)
    say("track quadratic log n8")
    _, st, log = q.track_path(H, x0, 2, q.default_track_params(predictor=q.PRED_QUADRATIC), log_cap=10000)
    ref = track_reference(s, x0, TrackParams(predictor="quadratic"), record=True)
    same = 0
    for rec, (t, lam, tn, z, zq) in zip(log, ref.predictions):
        # equal states: same t and step (a differing accept decision shows up as a differing t)
        if rec["t"] != t or rec["lam"] != lam:
            break
        with mpmath.workprec(300):
            d = max(abs(mpmath.re(a - b)) + abs(mpmath.im(a - b)) for a, b in zip(zq, z))
        assert abs(rec["pred_dist"] - d) <= 1e-12 * d, (same, rec["pred_dist"], d)
        same += 1
    say("steps compared", same, "of", len(log), "oracle", len(ref.predictions))
    assert same >= min(30, len(ref.predictions))


@pytest.mark.parametrize("name,copies", [("n8_dd", 1), ("n32_dd", 4)])
def test_track_paths_batch_matches_single_paths(name, copies):
    """Several paths tracked together (one launch per kernel per round): every
    path's outcome, counts and end point equal its single-path run, for both
    predictors (the per-point kernels are the same at these batch sizes); the
    fixture path reaches z** to double-double accuracy."""
    import paper_1109_0545_amd as q

    fix = fixture(name)
    s = config_system(CONFIGS[name])
    S = q.System.from_synth(s)
    H = q.Homotopy(S, s.gamma)
    rng = np.random.Generator(np.random.PCG64(8))
    ks = [np.array(fix["start_k"])] * copies
    if copies == 1:  # other start roots: paths that converge elsewhere or fail
        ks += [rng.integers(0, s.degrees) for _ in range(4)]
    x0 = np.stack([start_root(s.degrees, k, 2) for k in ks])
    zss = zss_mpc(fix)
    for pred in (q.PRED_SECANT, q.PRED_QUADRATIC):
        p = q.default_track_params(predictor=pred, max_steps=20000)
        say("track paths", name, "B", len(ks), "predictor", pred)
        zb, stb = q.track_paths(H, x0, 2, p)
        singles = {}
        for b in range(len(ks)):
            key = tuple(ks[b])
            if key not in singles:
                singles[key] = q.track_path(H, x0[b], 2, p)
            z1, st1, _ = singles[key]
            for f in ("fail", "succ_corrections", "corrections", "newton_iterations", "end_success"):
                assert stb[b][f] == st1[f], (b, f, stb[b], st1)
            assert np.array_equal(zb[b], z1), b
        assert not stb[0]["fail"] and correct_digits(zb[0], zss) >= 28


def test_track_paths_rejects_unsupported_controls():
    import paper_1109_0545_amd as q

    s = config_system(CONFIGS["n8_dd"])
    S = q.System.from_synth(s)
    H = q.Homotopy(S, s.gamma)
    x0 = start_root(s.degrees, np.zeros(s.n, np.int64), 2)[None]
    with pytest.raises(q.QdpError) as e:
        q.track_paths(H, x0, 2, q.default_track_params(probe=1))
    assert e.value.status == 5
