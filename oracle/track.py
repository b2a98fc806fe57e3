"""Path tracking oracle: endpoint refinement, start-root identification, the
reference tracker loop, and correct decimal places.

* ``refine_root``: Newton in high precision at t = 1 from the planted point,
  giving the exact regular root z** of the stored system that a forward
  track must end at.  Quadratic convergence is checked (at least three
  iterations whose correction squares), which certifies a regular root.
* ``F64Homotopy`` / ``track_f64``: a plain FP64 predictor-corrector (tangent
  predictor, Newton corrector, step halving) on the same homotopy.  It is
  fixture tooling: tracked backward from z** (t: 1 -> 0) it names the root
  of the start system x_v^(d_v) = 1 whose forward path ends at z**; tracked
  forward from that start root it confirms the pair.  Regularity of the
  backward path follows from the random-gamma construction of the total
  degree homotopy (a standard fact of homotopy continuation, not stated in
  the paper).
* ``extrapolate``: the predictor, the interpolating polynomial through the
  last accepted points evaluated at the next t (two points: the secant
  predictor; three: the quadratic predictor of Section 5).
* ``track_reference``: the loop of Algorithm 3.1 (predict, correct with the
  Newton loop of Algorithm 4.1, step size control, step back on failure,
  stop criterion) in high precision, with the secant or the quadratic
  predictor.  The paper prints neither the predictor formula nor the
  step-size constants; the readings used are in ``TrackParams``.
* ``correct_digits``: the quality Q of Section 2 (number of correct decimal
  places) measured against z**.

Parity: ``refine_root`` is pinned by decoupled targets whose roots are known
in closed form; ``track_reference`` by the closed-form path of a decoupled
target (every accepted point lies on the branch x_i(t)^(d_i) =
((1-t) gamma + t c_i)/((1-t) gamma + t)), by the stationary path f = g, and
by the invariants (accepted steps sum to 1; corrections >= successes; every
step on the 0.01 * 2^j grid until the final clamp); ``extrapolate`` by exact
reproduction of polynomial paths of degree below the number of points.
"""

from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import mpmath
import numpy as np

from .evaluate import degrees, eval_homotopy, residual
from .newton import newton_step
from .numbers import mpc_of, prec_bits, vec_mpc


# --------------------------------------------------------------------- digits


def correct_digits(z, zss) -> int:
    """Q = floor(-log10( max_v |z_v - z**_v| / max(1, ||z**||_inf) )).

    ``z`` is ``[n][2][L]`` limbs or a list of mpc; ``zss`` a list of mpc.
    Returns 99 when the two agree to the oracle's precision.
    """
    with mpmath.workprec(4096):
        Z = vec_mpc(z) if isinstance(z, np.ndarray) else [mpmath.mpc(v) for v in z]
        err = max(abs(a - b) for a, b in zip(Z, zss))
        nrm = max(mpmath.mpf(1), max(abs(b) for b in zss))
        if err == 0:
            return 99
        return int(mpmath.floor(-mpmath.log10(err / nrm)))


# ------------------------------------------------------------ root refinement


@dataclasses.dataclass
class RefinedRoot:
    z: list  # mpc list
    corrections: List[float]  # ||dz||_inf per iteration (FP64)


def refine_root(sys, z0, prec: Optional[int] = None, max_it: int = 40) -> RefinedRoot:
    """Newton at t = 1 (h = f) in high precision from ``z0`` until ||dz|| <= 2^(-prec+16).

    ``z0`` is cut to its leading limb first, so that the certificate below sees
    the corrections shrink from ~1e-16 through several squarings.

    Raises if fewer than three quadratically contracting corrections are seen
    (the root would not be certified regular) or the iteration does not settle.
    """
    prec = prec or prec_bits(sys.L) + 128
    deg = degrees(sys.exps, sys.poly_offsets)
    z = np.ascontiguousarray(np.asarray(z0)[:, :, :1])
    hist: List[float] = []
    with mpmath.workprec(prec):
        tol = mpmath.mpf(2) ** (-prec + 16)
        for _ in range(max_it):
            st = newton_step(sys.exps, sys.coefs, sys.poly_offsets, sys.gamma, 1.0, z, prec=prec, form="quotient",
                             deg=deg, L=sys.L)
            d = max(abs(v) for v in st.dz)
            hist.append(float(d))
            z = st.z
            if d <= tol * max(1, max(abs(v) for v in z)):
                break
        else:
            raise RuntimeError("root refinement did not converge")
    # quadratic convergence: at least three steps whose correction roughly
    # squares (order >= 1.8), the last one possibly cut off by the precision
    floor = 2.0 ** (-prec + 24)
    quad = 0
    for a, b in zip(hist, hist[1:]):
        if 0 < a < 1e-3 and (b <= floor or math.log(b) <= 1.8 * math.log(a)):
            quad += 1
    if quad < 3:
        raise RuntimeError(f"root not certified regular: corrections {hist}")
    return RefinedRoot(z, hist)


# ------------------------------------------------------------- FP64 homotopy


class F64Homotopy:
    """h(x,t) = t f(x) + (1-t) gamma (x^d - 1) in numpy complex128 (leading precision)."""

    def __init__(self, sys):
        self.n = sys.n
        self.exps = sys.exps.astype(np.int64)
        lim = sys.coefs
        self.c = lim[:, 0, :].sum(axis=1) + 1j * lim[:, 1, :].sum(axis=1)
        self.gamma = sys.gamma[0].sum() + 1j * sys.gamma[1].sum()
        self.off = np.asarray(sys.poly_offsets, dtype=np.int64)
        self.deg = np.array(degrees(sys.exps, sys.poly_offsets), dtype=np.int64)
        self.emax = int(self.exps.max())

    def f_and_jac(self, x):
        n = self.n
        P = x[:, None] ** np.arange(self.emax + 1)[None, :]
        M = np.prod(P[np.arange(n)[None, :], self.exps], axis=1)
        cm = self.c * M
        f = np.add.reduceat(cm, self.off[:-1])
        J = np.add.reduceat(cm[:, None] * self.exps, self.off[:-1], axis=0) / x[None, :]
        return f, J

    def eval(self, x, t):
        f, Jf = self.f_and_jac(x)
        xd = x ** self.deg
        g = xd - 1
        dg = self.deg * x ** (self.deg - 1)
        h = t * f + (1 - t) * self.gamma * g
        J = t * Jf
        J[np.diag_indices(self.n)] += (1 - t) * self.gamma * dg
        ht = f - self.gamma * g
        return h, J, ht


def track_f64(H: F64Homotopy, x0, t0: float, t1: float, dt0: float = 0.01, dt_max: float = 0.05,
              dt_min: float = 1e-9, tol: float = 1e-11, max_steps: int = 200000):
    """Tangent-predictor / Newton-corrector FP64 tracker from (x0, t0) to t1.

    Accepts a step when three or fewer Newton iterations bring the relative
    correction below ``tol`` with contraction at every iteration and the first
    correction stays below 2% of max(1, |x|); otherwise halves the step.
    Returns (x at t1, number of accepted steps) or raises if the step
    underflows.
    """
    x = np.array(x0, dtype=np.complex128)
    t = t0
    sgn = 1.0 if t1 > t0 else -1.0
    dt = dt0
    ok_run = 0
    steps = 0
    while (t1 - t) * sgn > 0:
        if steps > max_steps:
            raise RuntimeError("FP64 tracker: too many steps")
        h_ = min(dt, abs(t1 - t))
        tn = t1 if h_ >= abs(t1 - t) else t + sgn * h_
        # tangent predictor: dx/dt = -J^{-1} dh/dt (midpoint / RK2)
        try:
            _, J, ht = H.eval(x, t)
            k1 = -np.linalg.solve(J, ht)
            xm = x + 0.5 * (tn - t) * k1
            _, Jm, htm = H.eval(xm, 0.5 * (t + tn))
            k2 = -np.linalg.solve(Jm, htm)
            xp = x + (tn - t) * k2
        except np.linalg.LinAlgError:
            xp = None
        good = False
        if xp is not None and np.all(np.isfinite(xp)):
            scale = max(1.0, float(np.max(np.abs(xp))))
            prev = None
            y = xp
            for it in range(4):
                hh, JJ, _ = H.eval(y, tn)
                try:
                    d = np.linalg.solve(JJ, -hh)
                except np.linalg.LinAlgError:
                    break
                nd = float(np.max(np.abs(d)))
                if it == 0 and nd > 0.02 * scale:
                    break
                if prev is not None and nd > 0.5 * prev:
                    break
                y = y + d
                prev = nd
                if nd <= tol * scale:
                    good = True
                    break
        if good:
            x, t = y, tn
            steps += 1
            ok_run += 1
            if ok_run >= 3:
                dt = min(2 * dt, dt_max)
                ok_run = 0
        else:
            dt *= 0.5
            ok_run = 0
            if dt < dt_min:
                raise RuntimeError(f"FP64 tracker: step underflow at t={t}")
    return x, steps


def start_root_index(H: F64Homotopy, zss_f64, **kw):
    """Track backward from the target root to t = 0; return (k, x0) with
    x0_v ~ exp(2 pi i k_v / d_v)."""
    x0, _ = track_f64(H, zss_f64, 1.0, 0.0, **kw)
    k = np.round(np.angle(x0) * H.deg / (2 * np.pi)).astype(np.int64) % H.deg
    root = np.exp(2j * np.pi * k / H.deg)
    if np.max(np.abs(root - x0)) > 1e-6:
        raise RuntimeError("backward track did not end at a start root")
    return k, x0


# -------------------------------------------------------- reference tracker


@dataclasses.dataclass
class TrackParams:
    """Step-size control readings (the paper names the controls, not the constants).

    lambda0: initial step; shrink/expand: factors on failure / after
    ``expand_after`` consecutive successes; lambda_max caps the step;
    lambda_min and max_steps make up the stop criterion; eps_path / max_it_path
    drive the corrector along the path; eps_end / max_it_end the refinement at
    t = 1 (which also stops when the residual stops decreasing).
    """

    lambda0: float = 0.01
    lambda_min: float = 0.01 * 2.0 ** -30
    lambda_max: float = 0.08
    shrink: float = 0.5
    expand: float = 2.0
    expand_after: int = 3
    eps_path: float = 1e-10
    max_it_path: int = 4
    eps_end: float = 0.0  # 0 selects 64 u_L
    max_it_end: int = 10
    max_steps: int = 2_000_000
    predictor: str = "secant"  # or "quadratic"


@dataclasses.dataclass
class TrackResult:
    z: list
    t: float
    fail: bool
    succ: int
    corrections: int
    newton_iterations: int
    steps: List[float]  # accepted step sizes
    history: List[tuple] = dataclasses.field(default_factory=list)  # accepted (t, z)
    predictions: List[tuple] = dataclasses.field(default_factory=list)  # every correction: (t, lam, t', z, z')


def extrapolate(ts, zs, tn):
    """Value at ``tn`` of the interpolating polynomial through the points
    (ts[j], zs[j]) (one coordinate list per point), in Lagrange form:
    z' = sum_j l_j(tn) z_j with l_j(tn) = prod_{k != j} (tn - t_k)/(t_j - t_k).
    One point gives the constant predictor, two the secant (linear
    extrapolation), three the quadratic predictor.  Runs at the caller's
    working precision."""
    m = len(ts)
    T = [mpmath.mpf(v) for v in ts]
    tn = mpmath.mpf(tn)
    w = []
    for j in range(m):
        lj = mpmath.mpf(1)
        for k in range(m):
            if k != j:
                lj *= (tn - T[k]) / (T[j] - T[k])
        w.append(lj)
    return [mpmath.fsum(w[j] * zs[j][v] for j in range(m)) for v in range(len(zs[0]))]


def _limbs_point(z: list, L: int) -> np.ndarray:
    from .numbers import to_limbs_complex

    return np.stack([to_limbs_complex(v, L) for v in z])


def track_reference(sys, z0: np.ndarray, p: TrackParams = TrackParams(), round_limbs: bool = True,
                    record: bool = False) -> TrackResult:
    """Algorithm 3.1 with the secant or the quadratic predictor, in high precision.

    Predictor (reading of the unprinted predictors): with the step
    lam = min(lambda, 1 - t), predict t' = t + lam (t' = 1 when the step
    reaches the end) and z' = ``extrapolate`` through the last accepted
    points: two for the secant predictor, i.e. z' = z + (lam / (t - t_prev))
    (z - z_prev), three for the quadratic one (two while only two exist);
    before the second accepted point the predictor is constant (z' = z).
    Corrector: the Newton loop of Algorithm 4.1 with eps_path, max_it_path.
    Step size control: on success accept and, after ``expand_after``
    consecutive successes, lambda := min(expand * lambda, lambda_max); on
    failure step back (keep t, z) and lambda := shrink * lambda.
    Stop when lambda < lambda_min or the number of corrections reaches
    max_steps.  The path fails when it stops with t < 1 (the comment of
    Algorithm 3.1; its printed formula is garbled).  At t = 1 the endpoint is
    refined with eps_end / max_it_end.
    With ``round_limbs`` every accepted point is rounded to L limbs, as a
    multiword implementation stores it.
    """
    L = sys.L
    prec = prec_bits(L)
    deg = degrees(sys.exps, sys.poly_offsets)
    eps_end = p.eps_end or 64 * 2.0 ** (-53 * L)
    with mpmath.workprec(prec):
        z = vec_mpc(z0)
        t = 0.0
        pts = [(0.0, z)]  # accepted points, newest last, at most the predictor's order + 1
        order = {"secant": 2, "quadratic": 3}[p.predictor]
        preds: List[tuple] = []
        lam = p.lambda0
        run = 0
        succ = corr = nit = 0
        steps: List[float] = []
        hist: List[tuple] = []
        stop = False
        while t < 1.0 and not stop:
            step = min(lam, 1.0 - t)
            tn = 1.0 if t + step >= 1.0 else t + step
            zq = extrapolate([a for a, _ in pts], [b for _, b in pts], tn)
            if record:
                preds.append((t, step, tn, list(z), list(zq)))
            # Newton loop (Algorithm 4.1)
            rho, it = 1.0, 0
            y = zq
            while rho > p.eps_path and it < p.max_it_path:
                st = newton_step(sys.exps, sys.coefs, sys.poly_offsets, sys.gamma, tn, y, prec=prec, deg=deg, L=L)
                rho = st.rho
                y = st.z
                it += 1
                if not all(mpmath.isfinite(v) for v in y):
                    rho = math.inf
                    break
            nit += it
            corr += 1
            if rho < p.eps_path:
                if round_limbs:
                    y = vec_mpc(_limbs_point(y, L))
                z, t = y, tn
                pts = (pts + [(t, z)])[-order:]
                succ += 1
                steps.append(step)
                if record:
                    hist.append((t, list(z)))
                run += 1
                if run >= p.expand_after:
                    lam = min(lam * p.expand, p.lambda_max)
                    run = 0
            else:
                lam = lam * p.shrink
                run = 0
            stop = lam < p.lambda_min or corr >= p.max_steps
        if t >= 1.0:
            rho_prev = math.inf
            rho, it = 1.0, 0
            while rho > eps_end and it < p.max_it_end:
                st = newton_step(sys.exps, sys.coefs, sys.poly_offsets, sys.gamma, 1.0, z, prec=prec, deg=deg, L=L)
                rho = st.rho
                z = st.z
                it += 1
                if rho >= rho_prev:
                    break
                rho_prev = rho
            nit += it
            if round_limbs:
                z = vec_mpc(_limbs_point(z, L))
        return TrackResult(z, t, t < 1.0, succ, corr, nit, steps, hist, preds)
