"""Random sparse polynomial systems shaped like the paper's dimension / degree sweeps.

A system has ``n`` polynomials in ``n`` variables.  Polynomial ``i`` owns the
terms ``poly_offsets[i] .. poly_offsets[i+1]-1``; term ``j`` has a dense
exponent row ``exps[j, :]`` (one byte per variable, zero = absent) and a
complex coefficient ``coefs[j]`` stored as ``[2][L]`` doubles: the L limbs of
the real part (largest first), then the L limbs of the imaginary part.  A
multiword number is the exact sum of its limbs.

Workloads (Section 7 sweeps dimension and degree; the generator the paper
used is not published):

* exponents iid uniform in ``{0..E}`` per (monomial, variable), duplicate
  monomials of one polynomial redrawn;
* coefficients uniform on the unit circle, rounded to L limbs;
* a planted root ``z*`` on the unit torus so that the total-degree homotopy
  has a regular finite endpoint to track to.  The planting uses integer
  phase arithmetic: with ``z*_v = exp(2 pi i r_v / 2^32)`` every monomial of
  ``z*`` is the unit phasor ``exp(2 pi i p / 2^32)`` with the integer phase
  ``p = sum_v a_v r_v mod 2^32``; the coefficients of polynomial ``i`` are
  shifted by the minimal-norm correction that makes the phasor-weighted sum
  vanish.  No monomial product is formed here.

Random draws use ``numpy.random.Generator(PCG64(seed))`` in a fixed order:
exponents ``[n][m][n]``, coefficient angles ``[n][m]``, the angle of gamma,
root phases ``[n]``, then redraws of duplicate exponent rows.

Common-support workloads (the system of the paper's Table 1: 40 polynomials
in 40 variables sharing one support of 200 monomials, average degree 40 and
at most 80, i.e. exponents uniform in {0,1,2}): one support ``[m][n]`` is
drawn in place of ``[n][m][n]`` and every polynomial uses its rows in the
same order; the other draws and the planting are as above.
"""

from __future__ import annotations

import dataclasses
from typing import Dict, List, Optional

import mpmath
import numpy as np

# bits used for the transcendental constants before rounding to limbs
_PREC_BITS = 480
PHASE_BITS = 32


def limbs_of(x, L: int) -> List[float]:
    """Round the real number ``x`` (mpf / int / Fraction-like) to ``L`` doubles.

    Successive round-to-nearest: ``h_0 = fl(x)``, ``h_1 = fl(x - h_0)``, ...
    The result is nonoverlapping (|h_{k+1}| <= ulp(h_k)/2).
    """
    out = []
    with mpmath.workprec(_PREC_BITS + 64):
        r = mpmath.mpf(x)
        for _ in range(L):
            h = float(r)
            out.append(h)
            r = r - h
    return out


def unit_phasor(turns, L: int) -> np.ndarray:
    """``exp(2 pi i * turns)`` as ``[2][L]`` limbs; ``turns`` is an mpf/float/Fraction."""
    with mpmath.workprec(_PREC_BITS):
        if hasattr(turns, "denominator") and not isinstance(turns, (int, float)):
            turns = mpmath.mpf(turns.numerator) / turns.denominator
        a = 2 * mpmath.pi * mpmath.mpf(turns)
        re, im = mpmath.cos(a), mpmath.sin(a)
        return np.array([limbs_of(re, L), limbs_of(im, L)], dtype=np.float64)


@dataclasses.dataclass(frozen=True)
class Config:
    """One workload shape: n equations/variables, m monomials per polynomial,
    exponents uniform in {0..E}, L limbs per real component."""

    name: str
    n: int
    m: int
    E: int
    L: int
    seed: int
    common: bool = False  # every polynomial has the same m exponent rows


CONFIGS: Dict[str, Config] = {
    "n8_dd": Config("n8_dd", 8, 8, 2, 2, 0),
    "n32_dd": Config("n32_dd", 32, 32, 3, 2, 1),
    "n64_qd": Config("n64_qd", 64, 64, 4, 4, 2),
    "n64_dd": Config("n64_dd", 64, 64, 4, 2, 2),  # same draws as n64_qd, DD limbs
    "n128_dd": Config("n128_dd", 128, 128, 3, 2, 3),
    # the paper's Table 1 shape: common support of 200 monomials, degree 40 on average
    "c40_dd": Config("c40_dd", 40, 200, 2, 2, 4, common=True),
}


@dataclasses.dataclass
class System:
    n: int
    L: int
    poly_offsets: np.ndarray  # int32 [n+1]
    exps: np.ndarray  # uint8 [terms][n]
    coefs: np.ndarray  # float64 [terms][2][L]
    gamma: np.ndarray  # float64 [2][L]
    zstar: np.ndarray  # float64 [n][2][L]; planted root rounded to L limbs
    root_phase: np.ndarray  # int64 [n]; z*_v = exp(2 pi i root_phase_v / 2^32)
    degrees: np.ndarray  # int32 [n]; total degree of f_i

    @property
    def terms(self) -> int:
        return int(self.poly_offsets[-1])

    def poly_terms(self, i: int) -> range:
        return range(int(self.poly_offsets[i]), int(self.poly_offsets[i + 1]))

    def truncated(self, L: int) -> "System":
        """The same system with every multiword number cut to its first L limbs."""
        assert L <= self.L
        return System(
            self.n,
            L,
            self.poly_offsets.copy(),
            self.exps.copy(),
            np.ascontiguousarray(self.coefs[:, :, :L]),
            np.ascontiguousarray(self.gamma[:, :L]),
            np.ascontiguousarray(self.zstar[:, :, :L]),
            self.root_phase.copy(),
            self.degrees.copy(),
        )


def _dedupe(rng, exps: np.ndarray, E: int) -> None:
    n, m, _ = exps.shape
    for i in range(n):
        while True:
            seen = set()
            dup = []
            for j in range(m):
                key = exps[i, j].tobytes()
                if key in seen:
                    dup.append(j)
                seen.add(key)
            if not dup:
                break
            for j in dup:
                exps[i, j] = rng.integers(0, E + 1, size=exps.shape[2], dtype=np.int64)


def make_system(
    n: int, m: int, E: int, L: int, seed: int, plant: bool = True, common: bool = False
) -> System:
    """Draw one random system (see module docstring for the recipe)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    if common:
        support = rng.integers(0, E + 1, size=(1, m, n), dtype=np.int64)
    else:
        exps = rng.integers(0, E + 1, size=(n, m, n), dtype=np.int64)
    theta_c = rng.random((n, m))
    theta_g = rng.random()
    phase = rng.integers(0, 2**PHASE_BITS, size=n, dtype=np.int64)
    if common:
        _dedupe(rng, support, E)
        exps = np.repeat(support, n, axis=0)
    else:
        _dedupe(rng, exps, E)

    coefs = np.zeros((n * m, 2, L))
    with mpmath.workprec(_PREC_BITS):
        two_pi = 2 * mpmath.pi
        for i in range(n):
            cs = []
            us = []
            for j in range(m):
                a = two_pi * mpmath.mpf(float(theta_c[i, j]))
                cs.append(mpmath.mpc(mpmath.cos(a), mpmath.sin(a)))
                if plant:
                    p = int(np.dot(exps[i, j], phase)) % (2**PHASE_BITS)
                    b = two_pi * mpmath.mpf(p) / 2**PHASE_BITS
                    us.append(mpmath.mpc(mpmath.cos(b), mpmath.sin(b)))
            if plant:
                s = mpmath.fsum(c * u for c, u in zip(cs, us))
                shift = s / m
                cs = [c - shift * mpmath.conj(u) for c, u in zip(cs, us)]
            for j, c in enumerate(cs):
                coefs[i * m + j, 0] = limbs_of(c.real, L)
                coefs[i * m + j, 1] = limbs_of(c.imag, L)

    gamma = unit_phasor(mpmath.mpf(float(theta_g)), L)
    zstar = np.stack(
        [unit_phasor(mpmath.mpf(int(p)) / 2**PHASE_BITS, L) for p in phase]
    )
    exps_u8 = exps.reshape(n * m, n).astype(np.uint8)
    degrees = exps.sum(axis=2).max(axis=1).astype(np.int32)
    offsets = (np.arange(n + 1) * m).astype(np.int32)
    return System(n, L, offsets, exps_u8, coefs, gamma, zstar, phase, degrees)


def config_system(cfg: Config, plant: bool = True) -> System:
    return make_system(cfg.n, cfg.m, cfg.E, cfg.L, cfg.seed, plant=plant, common=cfg.common)


def start_root(degrees: np.ndarray, k: np.ndarray, L: int) -> np.ndarray:
    """Root of the start system ``x_v^{d_v} = 1``: ``x_v = exp(2 pi i k_v / d_v)``, ``[n][2][L]``."""
    from fractions import Fraction

    return np.stack(
        [unit_phasor(Fraction(int(kv) % int(d), int(d)), L) for kv, d in zip(k, degrees)]
    )


def random_point(
    n: int, L: int, seed: int, radius: float = 1.0, spread: float = 0.0
) -> np.ndarray:
    """Random point ``[n][2][L]`` near the circle of the given radius.

    Modulus ``radius * exp(spread * N(0,1))``, uniform argument; the modulus and
    angle are drawn in FP64 and the complex value is rounded to L limbs.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    ang = rng.random(n)
    mod = radius * np.exp(spread * rng.standard_normal(n))
    out = np.zeros((n, 2, L))
    with mpmath.workprec(_PREC_BITS):
        for v in range(n):
            a = 2 * mpmath.pi * mpmath.mpf(float(ang[v]))
            r = mpmath.mpf(float(mod[v]))
            out[v, 0] = limbs_of(r * mpmath.cos(a), L)
            out[v, 1] = limbs_of(r * mpmath.sin(a), L)
    return out


def random_unit_scalar(seed: int, L: int) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    return unit_phasor(mpmath.mpf(float(rng.random())), L)


def random_limbs(shape, L: int, seed: int, exp_spread: int = 0) -> np.ndarray:
    """Random nonoverlapping multiword reals ``shape + [L]``.

    Each value is ``sign * 2^e * (1 + u)`` with ``u`` carrying ``53*L`` random
    bits and ``e`` uniform in ``[-exp_spread, exp_spread]``; rounded to limbs
    exactly (the value has at most ``53*L`` significant bits).
    """
    from fractions import Fraction

    rng = np.random.Generator(np.random.PCG64(seed))
    size = int(np.prod(shape)) if len(shape) else 1
    out = np.zeros((size, L))
    nbits = 53 * L
    for idx in range(size):
        mant = (1 << (nbits - 1)) | int.from_bytes(rng.bytes((nbits + 7) // 8), "little") % (
            1 << (nbits - 1)
        )
        e = int(rng.integers(-exp_spread, exp_spread + 1)) if exp_spread else 0
        sgn = -1 if rng.random() < 0.5 else 1
        val = Fraction(sgn * mant, 1 << (nbits - 1)) * (Fraction(2) ** e)
        out[idx] = limbs_of(mpmath.mpf(val.numerator) / val.denominator, L)
    return out.reshape(tuple(shape) + (L,))


def optional(x: Optional[np.ndarray]) -> Optional[np.ndarray]:
    return None if x is None else np.ascontiguousarray(x)
