// Multiword floating point on gfx950: double (L=1), double-double (L=2) and
// quad-double (L=4) reals and complexes, built from FP64 error-free
// transformations.
//
// The paper runs its path tracker in double-double and quad-double complex
// arithmetic (Section 1, citing Dekker's technique and the quad-double
// algorithms of Hida, Li and Bailey; Section 2 quotes the ~8x cost of double
// doubles over doubles).  The building blocks here are the published ones:
//   * TwoSum (Knuth): s + e = a + b exactly, 6 flops, no ordering condition;
//   * FastTwoSum (Dekker): same with 3 flops when |a| >= |b| (or a == 0);
//   * TwoProd with the hardware FMA: p + e = a * b exactly, 2 flops.
// Double-double follows the "sloppy" add and the FMA-based product; the
// complex product sums both real products exactly before one normalisation.
// Quad-double accumulates partial products level by level (terms of order
// u^k at level k, u = 2^-53) with TwoSum carries, keeps levels 0..3 exactly,
// approximates level 4, and renormalises with a bottom-up then top-down
// TwoSum pass.  Every result is accurate to a few units of 2^(-53L) relative
// to the componentwise scale of the operation (|a|+|b| for sums, |a||b| for
// products), which is the bound the tests check against exact rationals.
//
// Must be compiled with -ffp-contract=off (no silent FMA contraction).

#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#pragma clang fp contract(off)

#define MW_DEV __device__ __forceinline__

namespace mw {

// ---------------------------------------------------------------- EFTs

MW_DEV double two_sum(double a, double b, double &e) {
  double s = a + b;
  double bb = s - a;
  e = (a - (s - bb)) + (b - bb);
  return s;
}

MW_DEV double fast_two_sum(double a, double b, double &e) {
  double s = a + b;
  e = b - (s - a);
  return s;
}

MW_DEV double two_prod(double a, double b, double &e) {
  double p = a * b;
  e = __builtin_fma(a, b, -p);
  return p;
}

// ---------------------------------------------------------------- real types

template <int L> struct R { double v[L]; };
template <int L> struct C { R<L> re, im; };

template <int L> MW_DEV R<L> rzero() {
  R<L> r;
#pragma unroll
  for (int k = 0; k < L; ++k) r.v[k] = 0.0;
  return r;
}
template <int L> MW_DEV R<L> rfrom(double a) {
  R<L> r = rzero<L>();
  r.v[0] = a;
  return r;
}
template <int L> MW_DEV R<L> rneg(const R<L> &a) {
  R<L> r;
#pragma unroll
  for (int k = 0; k < L; ++k) r.v[k] = -a.v[k];
  return r;
}
// multiply by a power of two (exact)
template <int L> MW_DEV R<L> rldexp(const R<L> &a, int e) {
  R<L> r;
#pragma unroll
  for (int k = 0; k < L; ++k) r.v[k] = ldexp(a.v[k], e);
  return r;
}

// ---- quad-double helpers

// renormalise five level-ordered terms into four limbs
MW_DEV void renorm5(double &x0, double &x1, double &x2, double &x3, double x4) {
  double e;
  // bottom-up: x0 becomes the rounded sum, the others the carried errors
  x3 = two_sum(x3, x4, x4);
  x2 = two_sum(x2, x3, x3);
  x1 = two_sum(x1, x2, x2);
  x0 = two_sum(x0, x1, x1);
  // top-down: make consecutive limbs nonoverlapping; zeros move down
  x1 = two_sum(x1, x2, x2);
  x2 = two_sum(x2, x3, x3);
  x3 = two_sum(x3, x4, e);
  (void)e;
}

MW_DEV void renorm4(double &x0, double &x1, double &x2, double &x3) {
  x2 = two_sum(x2, x3, x3);
  x1 = two_sum(x1, x2, x2);
  x0 = two_sum(x0, x1, x1);
  x1 = two_sum(x1, x2, x2);
  x2 = two_sum(x2, x3, x3);
}

// ---------------------------------------------------------------- add

template <int L> MW_DEV R<L> radd(const R<L> &a, const R<L> &b);

template <> MW_DEV R<1> radd<1>(const R<1> &a, const R<1> &b) {
  R<1> r;
  r.v[0] = a.v[0] + b.v[0];
  return r;
}

// double-double sum: exact sum of the leading limbs, the trailing limbs added
// into its error, one normalisation (error ~ u^2 (|a| + |b|))
template <> MW_DEV R<2> radd<2>(const R<2> &a, const R<2> &b) {
  double e;
  double s = two_sum(a.v[0], b.v[0], e);
  e += a.v[1] + b.v[1];
  R<2> r;
  r.v[0] = fast_two_sum(s, e, r.v[1]);
  return r;
}

// quad-double sum, level by level
template <> MW_DEV R<4> radd<4>(const R<4> &a, const R<4> &b) {
  double e0, e1, e2, f0, f1, g0;
  double s0 = two_sum(a.v[0], b.v[0], e0);  // e0: level 1
  double s1 = two_sum(a.v[1], b.v[1], e1);  // e1: level 2
  double s2 = two_sum(a.v[2], b.v[2], e2);  // e2: level 3
  double s3 = a.v[3] + b.v[3];              // level 3 (error level 4, dropped)
  s1 = two_sum(s1, e0, f0);                 // f0: level 2
  s2 = two_sum(s2, e1, f1);                 // f1: level 3
  s2 = two_sum(s2, f0, g0);                 // g0: level 3
  s3 = s3 + (e2 + (f1 + g0));
  renorm4(s0, s1, s2, s3);
  R<4> r;
  r.v[0] = s0; r.v[1] = s1; r.v[2] = s2; r.v[3] = s3;
  return r;
}

template <int L> MW_DEV R<L> rsub(const R<L> &a, const R<L> &b) { return radd<L>(a, rneg<L>(b)); }

// ---------------------------------------------------------------- mul

template <int L> MW_DEV R<L> rmul(const R<L> &a, const R<L> &b);

template <> MW_DEV R<1> rmul<1>(const R<1> &a, const R<1> &b) {
  R<1> r;
  r.v[0] = a.v[0] * b.v[0];
  return r;
}

template <> MW_DEV R<2> rmul<2>(const R<2> &a, const R<2> &b) {
  double e;
  double p = two_prod(a.v[0], b.v[0], e);
  e = __builtin_fma(a.v[0], b.v[1], e);
  e = __builtin_fma(a.v[1], b.v[0], e);
  R<2> r;
  r.v[0] = fast_two_sum(p, e, r.v[1]);
  return r;
}

template <> MW_DEV R<4> rmul<4>(const R<4> &a, const R<4> &b) {
  const double *x = a.v, *y = b.v;
  double q00, q01, q10, q02, q11, q20;
  double p00 = two_prod(x[0], y[0], q00);  // level 0, error level 1
  double p01 = two_prod(x[0], y[1], q01);  // level 1, errors level 2
  double p10 = two_prod(x[1], y[0], q10);
  double p02 = two_prod(x[0], y[2], q02);  // level 2, errors level 3
  double p11 = two_prod(x[1], y[1], q11);
  double p20 = two_prod(x[2], y[0], q20);
  // level 1: p01 + p10 + q00
  double r1, r2;
  double s1 = two_sum(p01, p10, r1);
  s1 = two_sum(s1, q00, r2);
  // level 2: p02 + p11 + p20 + q01 + q10 + r1 + r2
  double u1, u2, u3, u4, u5, u6;
  double s2 = two_sum(p02, p11, u1);
  s2 = two_sum(s2, p20, u2);
  s2 = two_sum(s2, q01, u3);
  s2 = two_sum(s2, q10, u4);
  s2 = two_sum(s2, r1, u5);
  s2 = two_sum(s2, r2, u6);
  // level 3: plain sums (errors at level 4)
  double s3 = ((x[0] * y[3] + x[3] * y[0]) + (x[1] * y[2] + x[2] * y[1])) +
              ((q02 + q11) + q20) + ((u1 + u2) + (u3 + u4)) + (u5 + u6);
  // level 4: leading level-4 products
  double s4 = __builtin_fma(x[1], y[3], __builtin_fma(x[2], y[2], x[3] * y[1]));
  double s0 = p00;
  renorm5(s0, s1, s2, s3, s4);
  R<4> r;
  r.v[0] = s0; r.v[1] = s1; r.v[2] = s2; r.v[3] = s3;
  return r;
}

// multiword times a double (exact small integers and powers of two included)
template <int L> MW_DEV R<L> rmul_d(const R<L> &a, double b);

template <> MW_DEV R<1> rmul_d<1>(const R<1> &a, double b) {
  R<1> r;
  r.v[0] = a.v[0] * b;
  return r;
}
template <> MW_DEV R<2> rmul_d<2>(const R<2> &a, double b) {
  double e;
  double p = two_prod(a.v[0], b, e);
  e = __builtin_fma(a.v[1], b, e);
  R<2> r;
  r.v[0] = fast_two_sum(p, e, r.v[1]);
  return r;
}
template <> MW_DEV R<4> rmul_d<4>(const R<4> &a, double b) {
  double q0, q1, q2;
  double p0 = two_prod(a.v[0], b, q0);
  double p1 = two_prod(a.v[1], b, q1);
  double p2 = two_prod(a.v[2], b, q2);
  double p3 = a.v[3] * b;
  double r1, r2, r3;
  double s1 = two_sum(p1, q0, r1);        // level 1; r1 level 2
  double s2 = two_sum(p2, q1, r2);        // level 2; r2 level 3
  s2 = two_sum(s2, r1, r3);               // r3 level 3
  double s3 = p3 + (q2 + (r2 + r3));
  double s4 = __builtin_fma(a.v[3], b, -p3);
  double s0 = p0;
  renorm5(s0, s1, s2, s3, s4);
  R<4> r;
  r.v[0] = s0; r.v[1] = s1; r.v[2] = s2; r.v[3] = s3;
  return r;
}

// ---------------------------------------------------------------- division

// long division: q_k = (remainder leading limb) / b_0, remainder -= q_k * b
template <int L> MW_DEV R<L> rdiv(const R<L> &a, const R<L> &b) {
  if constexpr (L == 1) {
    R<1> r;
    r.v[0] = a.v[0] / b.v[0];
    return r;
  } else {
    double q[L + 1];
    R<L> rem = a;
#pragma unroll
    for (int k = 0; k <= L; ++k) {
      q[k] = rem.v[0] / b.v[0];
      if (k < L) rem = rsub<L>(rem, rmul_d<L>(b, q[k]));
    }
    R<L> r;
    if constexpr (L == 2) {
      double e;
      double s = fast_two_sum(q[0], q[1], e);
      e += q[2];
      r.v[0] = fast_two_sum(s, e, r.v[1]);
    } else {
      double x0 = q[0], x1 = q[1], x2 = q[2], x3 = q[3];
      renorm5(x0, x1, x2, x3, q[4]);
      r.v[0] = x0; r.v[1] = x1; r.v[2] = x2; r.v[3] = x3;
    }
    return r;
  }
}

template <int L> MW_DEV double rabs_hi(const R<L> &a) { return __builtin_fabs(a.v[0]); }

// ---------------------------------------------------------------- complex

template <int L> MW_DEV C<L> czero() { return C<L>{rzero<L>(), rzero<L>()}; }
template <int L> MW_DEV C<L> cone() { return C<L>{rfrom<L>(1.0), rzero<L>()}; }
template <int L> MW_DEV C<L> cneg(const C<L> &a) { return C<L>{rneg<L>(a.re), rneg<L>(a.im)}; }
template <int L> MW_DEV C<L> cconj(const C<L> &a) { return C<L>{a.re, rneg<L>(a.im)}; }
template <int L> MW_DEV C<L> cadd(const C<L> &a, const C<L> &b) {
  return C<L>{radd<L>(a.re, b.re), radd<L>(a.im, b.im)};
}
template <int L> MW_DEV C<L> csub(const C<L> &a, const C<L> &b) {
  return C<L>{rsub<L>(a.re, b.re), rsub<L>(a.im, b.im)};
}
template <int L> MW_DEV C<L> cmul_d(const C<L> &a, double s) {
  return C<L>{rmul_d<L>(a.re, s), rmul_d<L>(a.im, s)};
}
template <int L> MW_DEV C<L> cmul_r(const C<L> &a, const R<L> &s) {
  return C<L>{rmul<L>(a.re, s), rmul<L>(a.im, s)};
}

// double-double complex product: each component sums its two exact leading
// products with TwoSum, folds the product errors and the cross terms into the
// tail with FMAs, then normalises once.
MW_DEV R<2> dd_dot2(const R<2> &a, const R<2> &b, const R<2> &c, const R<2> &d, double sgn) {
  // a*b + sgn * c*d
  double e1, e2, t;
  double p1 = two_prod(a.v[0], b.v[0], e1);
  double p2 = two_prod(sgn * c.v[0], d.v[0], e2);
  double s = two_sum(p1, p2, t);
  t = t + (e1 + e2);
  t = __builtin_fma(a.v[0], b.v[1], t);
  t = __builtin_fma(a.v[1], b.v[0], t);
  t = __builtin_fma(sgn * c.v[0], d.v[1], t);
  t = __builtin_fma(sgn * c.v[1], d.v[0], t);
  R<2> r;
  r.v[0] = fast_two_sum(s, t, r.v[1]);
  return r;
}

template <int L> MW_DEV C<L> cmul(const C<L> &a, const C<L> &b) {
  if constexpr (L == 1) {
    C<1> r;
    r.re.v[0] = __builtin_fma(a.re.v[0], b.re.v[0], -(a.im.v[0] * b.im.v[0]));
    r.im.v[0] = __builtin_fma(a.re.v[0], b.im.v[0], a.im.v[0] * b.re.v[0]);
    return r;
  } else if constexpr (L == 2) {
    return C<2>{dd_dot2(a.re, b.re, a.im, b.im, -1.0), dd_dot2(a.re, b.im, a.im, b.re, 1.0)};
  } else {
    return C<L>{rsub<L>(rmul<L>(a.re, b.re), rmul<L>(a.im, b.im)),
                radd<L>(rmul<L>(a.re, b.im), rmul<L>(a.im, b.re))};
  }
}

// double-double a + x1*y1 + x2*y2: both leading products exact, both sums
// exact (TwoSum), every error and cross term folded into the tail, one
// normalisation
MW_DEV R<2> dd_fms3(const R<2> &a, const R<2> &x1, const R<2> &y1, const R<2> &x2, const R<2> &y2) {
  double e1, e2, t1, t2;
  double p1 = two_prod(x1.v[0], y1.v[0], e1);
  double p2 = two_prod(x2.v[0], y2.v[0], e2);
  double s = two_sum(a.v[0], p1, t1);
  s = two_sum(s, p2, t2);
  double t = a.v[1] + ((t1 + t2) + (e1 + e2));
  t = __builtin_fma(x1.v[0], y1.v[1], t);
  t = __builtin_fma(x1.v[1], y1.v[0], t);
  t = __builtin_fma(x2.v[0], y2.v[1], t);
  t = __builtin_fma(x2.v[1], y2.v[0], t);
  R<2> r;
  r.v[0] = fast_two_sum(s, t, r.v[1]);
  return r;
}

// a - l*u
template <int L> MW_DEV C<L> cfms(const C<L> &a, const C<L> &l, const C<L> &u) {
  if constexpr (L == 2) {
    // re: a.re - l.re u.re + l.im u.im ; im: a.im - l.re u.im - l.im u.re
    return C<2>{dd_fms3(a.re, rneg<2>(l.re), u.re, l.im, u.im), dd_fms3(a.im, rneg<2>(l.re), u.im, rneg<2>(l.im), u.re)};
  } else if constexpr (L == 1) {
    C<1> r;
    r.re.v[0] = __builtin_fma(l.im.v[0], u.im.v[0], __builtin_fma(-l.re.v[0], u.re.v[0], a.re.v[0]));
    r.im.v[0] = __builtin_fma(-l.im.v[0], u.re.v[0], __builtin_fma(-l.re.v[0], u.im.v[0], a.im.v[0]));
    return r;
  } else {
    return csub<L>(a, cmul<L>(l, u));
  }
}

// 1/p: an FP64 seed conj(p)/|p|^2 (with a power-of-two prescale against
// overflow), then Newton's iteration inv <- inv + inv (1 - p inv), which
// doubles the number of correct bits per step (one step for double double,
// two for quad double).
template <int L> MW_DEV C<L> cinv(const C<L> &a) {
  double m = fmax(__builtin_fabs(a.re.v[0]), __builtin_fabs(a.im.v[0]));
  int ex = 0;
  if (m > 0.0 && m < __builtin_inf()) (void)frexp(m, &ex);
  const C<L> p{rldexp<L>(a.re, -ex), rldexp<L>(a.im, -ex)};
  const double pr = p.re.v[0], pi = p.im.v[0];
  // 1/|p|^2 with |p| in [1/2, sqrt 2): the hardware reciprocal estimate and two
  // FP64 Newton steps (each squares the relative error, down to FP64 rounding;
  // the double-double correction below squares what is left)
  const double q2 = __builtin_fma(pr, pr, pi * pi);
  double r0 = __builtin_amdgcn_rcp(q2);
  r0 = __builtin_fma(r0, __builtin_fma(-q2, r0, 1.0), r0);
  r0 = __builtin_fma(r0, __builtin_fma(-q2, r0, 1.0), r0);
  const double i0r = pr * r0, i0i = -pi * r0;
  C<L> inv;
  if constexpr (L == 1) {
    inv.re.v[0] = i0r;
    inv.im.v[0] = i0i;
  } else {
    // q = p * inv0 with inv0 an FP64 complex, to double-double accuracy
    double e1, e2, t, u;
    double qr = two_sum(two_prod(pr, i0r, e1), two_prod(-pi, i0i, e2), t);
    t = t + (e1 + e2);
    t = __builtin_fma(p.re.v[1], i0r, t);
    t = __builtin_fma(-p.im.v[1], i0i, t);
    double qi = two_sum(two_prod(pr, i0i, e1), two_prod(pi, i0r, e2), u);
    u = u + (e1 + e2);
    u = __builtin_fma(p.re.v[1], i0i, u);
    u = __builtin_fma(p.im.v[1], i0r, u);
    // e = 1 - q (1 - qr is exact: qr is within a few ulps of 1)
    const double er = (1.0 - qr) - t;
    const double ei = -(qi + u);
    const double dr = __builtin_fma(i0r, er, -(i0i * ei));
    const double di = __builtin_fma(i0r, ei, i0i * er);
    C<2> d2;
    d2.re.v[0] = two_sum(i0r, dr, d2.re.v[1]);
    d2.im.v[0] = two_sum(i0i, di, d2.im.v[1]);
    if constexpr (L == 2) {
      inv = d2;
    } else {
      inv = czero<L>();
      inv.re.v[0] = d2.re.v[0];
      inv.re.v[1] = d2.re.v[1];
      inv.im.v[0] = d2.im.v[0];
      inv.im.v[1] = d2.im.v[1];
      const C<L> e = csub<L>(cone<L>(), cmul<L>(p, inv));
      inv = cadd<L>(inv, cmul<L>(inv, e));
    }
  }
  inv.re = rldexp<L>(inv.re, -ex);
  inv.im = rldexp<L>(inv.im, -ex);
  return inv;
}

template <int L> MW_DEV C<L> cdiv(const C<L> &a, const C<L> &b) { return cmul<L>(a, cinv<L>(b)); }

// |re| + |im| of the leading limbs (pivot key and residual norm)
template <int L> MW_DEV double cabs1_hi(const C<L> &a) {
  return __builtin_fabs(a.re.v[0]) + __builtin_fabs(a.im.v[0]);
}
// FP64 modulus of the leading limbs
template <int L> MW_DEV double cabs_hi(const C<L> &a) { return hypot(a.re.v[0], a.im.v[0]); }

template <int L> MW_DEV bool cfinite(const C<L> &a) {
  bool ok = true;
#pragma unroll
  for (int k = 0; k < L; ++k) ok = ok && __builtin_isfinite(a.re.v[k]) && __builtin_isfinite(a.im.v[k]);
  return ok;
}

// ---------------------------------------------------------------- memory
// A complex multiword number in memory: [re limbs (L)][im limbs (L)] doubles.

template <int L> MW_DEV C<L> cload(const double *p) {
  C<L> r;
#pragma unroll
  for (int k = 0; k < L; ++k) {
    r.re.v[k] = p[k];
    r.im.v[k] = p[L + k];
  }
  return r;
}
// load keeping only the first L of LS stored limbs (precision truncation)
template <int L> MW_DEV C<L> cload_trunc(const double *p, int LS) {
  C<L> r;
#pragma unroll
  for (int k = 0; k < L; ++k) {
    r.re.v[k] = p[k];
    r.im.v[k] = p[LS + k];
  }
  return r;
}
template <int L> MW_DEV void cstore(double *p, const C<L> &a) {
#pragma unroll
  for (int k = 0; k < L; ++k) {
    p[k] = a.re.v[k];
    p[L + k] = a.im.v[k];
  }
}

// A complex multiword number split into limb planes: limb k of the real part
// at p[k*ps], limb k of the imaginary part at p[(L+k)*ps].  Consecutive
// elements of a plane are consecutive doubles, so a wavefront reading
// consecutive elements touches consecutive LDS banks.
template <int L> MW_DEV C<L> pload(const double *p, size_t ps) {
  C<L> r;
#pragma unroll
  for (int k = 0; k < L; ++k) {
    r.re.v[k] = p[k * ps];
    r.im.v[k] = p[(L + k) * ps];
  }
  return r;
}
template <int L> MW_DEV void pstore(double *p, size_t ps, const C<L> &a) {
#pragma unroll
  for (int k = 0; k < L; ++k) {
    p[k * ps] = a.re.v[k];
    p[(L + k) * ps] = a.im.v[k];
  }
}

// power x^e for e >= 0 by binary powering; both products of a step are
// formed every time (they are independent, so they overlap) and the one the
// exponent bit does not ask for is dropped
template <int L> MW_DEV C<L> cpow(const C<L> &x, int e) {
  C<L> r = cone<L>();
  C<L> b = x;
  while (e > 0) {
    const C<L> rb = cmul<L>(r, b);
    const C<L> bb = cmul<L>(b, b);
    if (e & 1) r = rb;
    b = bb;
    e >>= 1;
  }
  return r;
}

// cross-lane shuffles of a complex multiword value
template <int L> MW_DEV C<L> cshfl(const C<L> &a, int src, int width) {
  C<L> r;
#pragma unroll
  for (int k = 0; k < L; ++k) {
    r.re.v[k] = __shfl(a.re.v[k], src, width);
    r.im.v[k] = __shfl(a.im.v[k], src, width);
  }
  return r;
}
template <int L> MW_DEV C<L> cshfl_up(const C<L> &a, unsigned d, int width) {
  C<L> r;
#pragma unroll
  for (int k = 0; k < L; ++k) {
    r.re.v[k] = __shfl_up(a.re.v[k], d, width);
    r.im.v[k] = __shfl_up(a.im.v[k], d, width);
  }
  return r;
}
template <int L> MW_DEV C<L> cshfl_down(const C<L> &a, unsigned d, int width) {
  C<L> r;
#pragma unroll
  for (int k = 0; k < L; ++k) {
    r.re.v[k] = __shfl_down(a.re.v[k], d, width);
    r.im.v[k] = __shfl_down(a.im.v[k], d, width);
  }
  return r;
}
template <int L> MW_DEV C<L> cshfl_xor(const C<L> &a, int m, int width) {
  C<L> r;
#pragma unroll
  for (int k = 0; k < L; ++k) {
    r.re.v[k] = __shfl_xor(a.re.v[k], m, width);
    r.im.v[k] = __shfl_xor(a.im.v[k], m, width);
  }
  return r;
}

template <int L> MW_DEV C<L> cselect(bool c, const C<L> &a, const C<L> &b) {
  C<L> r;
#pragma unroll
  for (int k = 0; k < L; ++k) {
    r.re.v[k] = c ? a.re.v[k] : b.re.v[k];
    r.im.v[k] = c ? a.im.v[k] : b.im.v[k];
  }
  return r;
}

}  // namespace mw
