"""Pins for the path oracle: closed-form paths, stationary paths, invariants, digits."""

import cmath
import json
import math
import os
from fractions import Fraction

import mpmath
import numpy as np
import pytest

from oracle.numbers import mpc_of, prec_bits, vec_mpc
from oracle.quality import cores_for_equal_time, quality_up_estimate, speedup
from oracle.track import F64Homotopy, TrackParams, correct_digits, extrapolate, refine_root, start_root_index, \
    track_f64, track_reference
from synth.systems import CONFIGS, System, config_system, start_root, unit_phasor

HERE = os.path.dirname(os.path.abspath(__file__))


def decoupled_system(d, c_turns, gamma_turns, L=2):
    """f_i = x_i^(d_i) - c_i with |c_i| = 1 (c_i = exp(2 pi i c_turns_i))."""
    n = len(d)
    exps, coefs, offs = [], [], [0]
    for i in range(n):
        a = [0] * n
        a[i] = d[i]
        exps.append(a)
        coefs.append(np.array([[1.0] + [0.0] * (L - 1), [0.0] * L]))
        exps.append([0] * n)
        coefs.append(-unit_phasor(Fraction(c_turns[i]), L))
        offs.append(len(exps))
    gamma = unit_phasor(Fraction(gamma_turns), L)
    return System(n, L, np.array(offs, dtype=np.int32), np.array(exps, dtype=np.uint8), np.array(coefs),
                  gamma, np.zeros((n, 2, L)), np.zeros(n, dtype=np.int64), np.array(d, dtype=np.int32))


def branch(d, k, c, gamma, t, grid=4000):
    """x(t) on the continuous branch of x^d = (t c + (1-t) gamma)/(t + (1-t) gamma) from exp(2 pi i k/d)."""
    ang = 0.0
    prev = None
    for s in np.linspace(0.0, t, grid):
        w = (s * c + (1 - s) * gamma) / (s + (1 - s) * gamma)
        a = cmath.phase(w)
        if prev is not None:
            da = a - prev
            da -= 2 * math.pi * round(da / (2 * math.pi))
            ang += da
        else:
            ang = a
        prev = a
    w = (t * c + (1 - t) * gamma) / (t + (1 - t) * gamma)
    return abs(w) ** (1.0 / d) * cmath.exp(1j * (ang + 2 * math.pi * k) / d)


def test_decoupled_target_closed_form_path():
    d = [3, 4]
    c_turns = [Fraction(1, 7), Fraction(2, 5)]
    s = decoupled_system(d, c_turns, Fraction(3, 11))
    k = [1, 2]
    x0 = start_root(np.array(d), np.array(k), s.L)
    r = track_reference(s, x0, record=True)
    assert not r.fail and r.t == 1.0
    g = complex(mpc_of(s.gamma))
    for t, z in r.history[1:]:
        for i in range(2):
            c = cmath.exp(2j * math.pi * float(c_turns[i]))
            ref = branch(d[i], k[i], c, g, t)
            assert abs(complex(z[i]) - ref) < 1e-9
    # endpoint: the branch value at t = 1, i.e. a d-th root of c, to DD accuracy
    for i in range(2):
        with mpmath.workprec(400):
            croot = mpmath.exp(2j * mpmath.pi * (mpmath.mpf(c_turns[i].numerator) / c_turns[i].denominator) / d[i])
            roots = [croot * mpmath.exp(2j * mpmath.pi * j / d[i]) for j in range(d[i])]
            ref = branch(d[i], k[i], cmath.exp(2j * math.pi * float(c_turns[i])), g, 1.0)
            best = min(roots, key=lambda q: abs(complex(q) - ref))
            assert abs(r.z[i] - best) < mpmath.mpf(10) ** -29


def test_extrapolate_reproduces_polynomial_paths():
    # z(t) = a + b t + c t^2 per coordinate, rational coefficients, exact arithmetic at 400 bits
    rng = np.random.Generator(np.random.PCG64(11))
    with mpmath.workprec(400):
        coef = [[mpmath.mpc(mpmath.mpf(int(rng.integers(-9, 10))) / 7, mpmath.mpf(int(rng.integers(-9, 10))) / 5)
                 for _ in range(3)] for _ in range(4)]

        def z(t, deg=2):
            t = mpmath.mpf(t)
            return [sum(cf[j] * t ** j for j in range(deg + 1)) for cf in coef]

        ts = [0.125, 0.25, 0.3125]
        tn = 0.4375
        tiny = mpmath.mpf(2) ** -380
        # three points reproduce a quadratic, two a line, one a constant
        assert max(abs(a - b) for a, b in zip(extrapolate(ts, [z(t) for t in ts], tn), z(tn))) < tiny
        assert max(abs(a - b) for a, b in zip(extrapolate(ts[1:], [z(t, 1) for t in ts[1:]], tn), z(tn, 1))) < tiny
        assert extrapolate(ts[2:], [z(ts[2])], tn) == z(ts[2])
        # the secant through the last two points misses a quadratic by c (t' - t_1)(t' - t_2)
        sec = extrapolate(ts[1:], [z(t) for t in ts[1:]], tn)
        gap = (mpmath.mpf(tn) - ts[1]) * (mpmath.mpf(tn) - ts[2])
        for v in range(4):
            assert abs(z(tn)[v] - sec[v] - coef[v][2] * gap) < tiny
        # the secant form used by the tracker: z + lam / (t - t_prev) (z - z_prev)
        zp, zc = z(ts[1]), z(ts[2])
        r = (mpmath.mpf(tn) - ts[2]) / (mpmath.mpf(ts[2]) - ts[1])
        assert max(abs(a - (c + r * (c - b))) for a, b, c in zip(sec, zp, zc)) < tiny


def test_quadratic_predictor_tracks_decoupled_closed_form_path():
    d = [3, 4]
    c_turns = [Fraction(1, 7), Fraction(2, 5)]
    s = decoupled_system(d, c_turns, Fraction(3, 11))
    k = [1, 2]
    x0 = start_root(np.array(d), np.array(k), s.L)
    r = track_reference(s, x0, TrackParams(predictor="quadratic"), record=True)
    assert not r.fail and r.t == 1.0
    g = complex(mpc_of(s.gamma))
    for t, z in r.history[1:]:
        for i in range(2):
            c = cmath.exp(2j * math.pi * float(c_turns[i]))
            assert abs(complex(z[i]) - branch(d[i], k[i], c, g, t)) < 1e-9
    # every prediction is the interpolant through the last (up to) three accepted points
    with mpmath.workprec(prec_bits(s.L)):
        acc = [(0.0, vec_mpc(x0))] + r.history
    for t, _, tn, z, zq in r.predictions:
        j = max(i for i, (ta, _) in enumerate(acc) if ta == t)
        pts = acc[max(0, j - 2): j + 1]
        assert z == pts[-1][1]
        with mpmath.workprec(300):
            ref = extrapolate([a for a, _ in pts], [b for _, b in pts], tn)
            assert max(abs(a - b) for a, b in zip(ref, zq)) < 1e-60
    # the quadratic predictor leaves smaller first Newton corrections than the secant on this smooth path
    sec = track_reference(s, x0, record=True)
    assert r.newton_iterations <= sec.newton_iterations


def test_stationary_path_when_target_is_start_system():
    d = [5, 3]
    s = decoupled_system(d, [Fraction(0), Fraction(0)], Fraction(2, 9))
    x0 = start_root(np.array(d), np.array([2, 1]), s.L)
    r = track_reference(s, x0, record=True)
    with mpmath.workprec(300):
        X0 = vec_mpc(x0)
        for _, z in r.history:
            assert max(abs(a - b) for a, b in zip(z, X0)) < 1e-30
        assert max(abs(a - b) for a, b in zip(r.z, X0)) < 1e-30


def test_tracker_invariants_on_config_n8():
    s = config_system(CONFIGS["n8_dd"])
    rr = refine_root(s, s.zstar)
    H = F64Homotopy(s)
    k, _ = start_root_index(H, np.array([complex(v) for v in rr.z]))
    r = track_reference(s, start_root(H.deg, k, s.L))
    assert not r.fail and r.t == 1.0
    assert r.corrections >= r.succ == len(r.steps)
    assert abs(math.fsum(r.steps) - 1.0) < 1e-12
    for lam in r.steps[:-1]:
        j = math.log2(lam / 0.01)
        assert j == round(j)  # every step (but the final clamp) is 0.01 * 2^j
    assert correct_digits(r.z, rr.z) >= 28


def test_stop_criterion_fails_path():
    s = config_system(CONFIGS["n8_dd"])
    H = F64Homotopy(s)
    x0 = start_root(H.deg, np.zeros(s.n, dtype=np.int64), s.L)
    # lambda_min above lambda0: the first failed correction stops the path with t < 1
    p = TrackParams(eps_path=0.0, max_it_path=1, lambda_min=0.009)
    r = track_reference(s, x0, p)
    assert r.fail and r.t < 1.0 and r.succ == 0 and r.corrections == 1


def test_refine_root_decoupled_closed_form():
    d = [3, 2]
    c_turns = [Fraction(1, 6), Fraction(1, 3)]
    s = decoupled_system(d, c_turns, Fraction(1, 5))
    guess = np.stack([unit_phasor(Fraction(c_turns[i]) / d[i] + Fraction(1, 10**6), s.L) for i in range(2)])
    rr = refine_root(s, guess)
    with mpmath.workprec(500):
        for i in range(2):
            # an exact root of the stored (rounded) coefficient c_i ...
            c_stored = -mpc_of(s.coefs[2 * i + 1])
            assert abs(mpmath.power(rr.z[i], d[i]) - c_stored) < mpmath.mpf(10) ** -150
            # ... next to the closed-form root of the unrounded one
            ref = mpmath.exp(2j * mpmath.pi * (mpmath.mpf(c_turns[i].numerator) / c_turns[i].denominator) / d[i])
            assert abs(rr.z[i] - ref) < mpmath.mpf(10) ** -30


def test_fp64_tracker_start_root_identification_decoupled():
    d = [4, 3]
    c_turns = [Fraction(1, 9), Fraction(4, 7)]
    s = decoupled_system(d, c_turns, Fraction(5, 13))
    H = F64Homotopy(s)
    k_true = [3, 1]
    g = complex(mpc_of(s.gamma))
    z1 = np.array([branch(d[i], k_true[i], cmath.exp(2j * math.pi * float(c_turns[i])), g, 1.0) for i in range(2)])
    k, _ = start_root_index(H, z1)
    assert list(k) == k_true
    x1, _ = track_f64(H, np.exp(2j * np.pi * np.array(k_true) / np.array(d)), 0.0, 1.0)
    assert np.max(np.abs(x1 - z1)) < 1e-10


def test_correct_digits():
    zss = [mpmath.mpc(1, 0), mpmath.mpc(0, 2)]
    z = np.array([[[1.0, 1e-20], [0.0, 0.0]], [[0.0, 0.0], [2.0, 0.0]]])
    assert correct_digits(z, zss) == 20
    z2 = np.array([[[1.0, 0.0], [0.0, 0.0]], [[0.0, 0.0], [2.0, 0.0]]])
    assert correct_digits(z2, zss) == 99


def test_quality_up_worked_example():
    with open(os.path.join(HERE, "golden", "quality_up.json")) as fh:
        g = json.load(fh)
    ps, pc = cores_for_equal_time(g["t_dd_1core"], g["t_qd_pcores"], g["p"])
    assert round(ps, 3) == g["p_star"]
    assert pc == g["cores"]
    y = quality_up_estimate(g["t_dd_1core"], g["t_qd_pcores"], g["p"])
    assert y == Fraction(g["y_num"], g["y_den"])
    assert round(float(y), 3) == g["y_rounded"]
    assert speedup(40.778, 6.177) == pytest.approx(6.602, abs=5e-4)
