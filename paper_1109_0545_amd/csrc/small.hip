// Small kernels around the Newton loop: state reset, the secant predictor,
// and the multiword arithmetic test entry.

#include "common.hpp"
#include "ge_kernel.hpp"
#include "ctl_features.hpp"

namespace qdp {
using namespace mw;

// Algorithm 4.1 initialises the residual to 1 and loops while it exceeds eps
// and fewer than Max_It iterations ran.
// mask (nullable): points with mask[b] == 0 start inactive (their kernels return at once)
__global__ void k_init_state(NewtonState *states, int B, double eps, int max_it, const int *mask) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  NewtonState *s = states + b;
  s->iterations = 0;
  s->success = (1.0 < eps) ? 1 : 0;
  s->singular = 0;
  s->nonfinite = 0;
  s->max_it = max_it;
  s->eps = eps;
  s->rho = 1.0;
  s->rho_first = 1.0;
  s->cond_est = 0.0;
  s->dz_norm = 0.0;
  s->refine_err = 0.0;
  s->refine_steps = 0;
  s->pad = 0;
  s->dz_first = 0.0;
  s->xnorm = 0.0;
  s->active = (1.0 > eps && max_it > 0 && (!mask || mask[b])) ? 1 : 0;
}

hipError_t launch_init_state(NewtonState *st, int B, double eps, int max_it, const int *mask, hipStream_t s) {
  hipLaunchKernelGGL(k_init_state, dim3((B + 63) / 64), dim3(64), 0, s, st, B, eps, max_it, mask);
  return hipGetLastError();
}

// Predictor: z' = z + c1 (z_prev - z) + c2 (z_prev2 - z), the coefficients
// formed on the host in FP64 from the parameter values:
//   constant   (one accepted point):   c1 = c2 = 0;
//   secant     (two points):           c1 = -(t' - t)/(t - t_prev), c2 = 0
//              (linear extrapolation through the last two accepted points);
//   quadratic  (three points, Section 5): c1, c2 the Lagrange weights of the
//              parabola through (t_prev2, z_prev2), (t_prev, z_prev), (t, z)
//              evaluated at t', coordinate by coordinate;
//   blends of the secant and quadratic coefficients (learned controller).
// Writing z' as z plus weighted differences keeps the small increments
// accurate.  One workgroup; aux[0] gets ||z' - z||_inf (leading limbs).
template <int L>
__global__ __launch_bounds__(256) void k_predict(int n, const double *x, const double *xp, const double *xpp,
                                                 double c1, double c2, double *out, double *aux) {
  __shared__ double red[4];
  double m = 0.0;
  for (int v = threadIdx.x; v < n; v += 256) {
    const C<L> z = cload<L>(x + (size_t)v * 2 * L);
    C<L> d = czero<L>();
    if (c1 != 0.0) d = cmul_d<L>(csub<L>(cload<L>(xp + (size_t)v * 2 * L), z), c1);
    if (c2 != 0.0) d = cadd<L>(d, cmul_d<L>(csub<L>(cload<L>(xpp + (size_t)v * 2 * L), z), c2));
    cstore<L>(out + (size_t)v * 2 * L, cadd<L>(z, d));
    m = fmax(m, cabs1_hi<L>(d));
  }
  for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0 && aux) aux[0] = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
}

hipError_t launch_predict(int L, int n, const double *x, const double *xprev, const double *xprev2, double c1,
                          double c2, double *xpred, double *aux, hipStream_t s) {
  dim3 g(1), b(256);
  switch (L) {
    case 1: hipLaunchKernelGGL(k_predict<1>, g, b, 0, s, n, x, xprev, xprev2, c1, c2, xpred, aux); break;
    case 2: hipLaunchKernelGGL(k_predict<2>, g, b, 0, s, n, x, xprev, xprev2, c1, c2, xpred, aux); break;
    case 4: hipLaunchKernelGGL(k_predict<4>, g, b, 0, s, n, x, xprev, xprev2, c1, c2, xpred, aux); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Predictor for a batch of paths: point b of xw gets x_b + c1[b] (xp_b - x_b)
// + c2[b] (xpp_b - x_b) where mask[b] != 0 (see k_predict).  Points are
// n complex values apart; grid (ceil(n / 64), B).
template <int L>
__global__ __launch_bounds__(64) void k_predict_batch(int n, const double *x, const double *xp, const double *xpp,
                                                      const double *cf, const int *mask, int B, double *xw) {
  const int b = blockIdx.y, v = blockIdx.x * 64 + threadIdx.x;
  if (v >= n || !mask[b]) return;
  const size_t o = ((size_t)b * n + v) * 2 * L;
  const double c1 = cf[b], c2 = cf[B + b];
  const C<L> z = cload<L>(x + o);
  C<L> d = czero<L>();
  if (c1 != 0.0) d = cmul_d<L>(csub<L>(cload<L>(xp + o), z), c1);
  if (c2 != 0.0) d = cadd<L>(d, cmul_d<L>(csub<L>(cload<L>(xpp + o), z), c2));
  cstore<L>(xw + o, cadd<L>(z, d));
}

hipError_t launch_predict_batch(int L, int n, int B, const double *x, const double *xp, const double *xpp,
                                const double *cf, const int *mask, double *xw, hipStream_t s) {
  dim3 g((n + 63) / 64, B), b(64);
  switch (L) {
    case 1: hipLaunchKernelGGL(k_predict_batch<1>, g, b, 0, s, n, x, xp, xpp, cf, mask, B, xw); break;
    case 2: hipLaunchKernelGGL(k_predict_batch<2>, g, b, 0, s, n, x, xp, xpp, cf, mask, B, xw); break;
    case 4: hipLaunchKernelGGL(k_predict_batch<4>, g, b, 0, s, n, x, xp, xpp, cf, mask, B, xw); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Acceptance for a batch of paths: where acc[b] != 0, (xpp, xp, x) <- (xp, x, xw)
// for point b (each element read before any write of it).
__global__ void k_accept_batch(size_t per_point, const int *acc, double *x, double *xp, double *xpp,
                               const double *xw, size_t count) {
  const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= count || !acc[q / per_point]) return;
  const double a = xp[q], c = x[q], w = xw[q];
  xpp[q] = a;
  xp[q] = c;
  x[q] = w;
}

hipError_t launch_accept_batch(int L, int n, int B, const int *acc, double *x, double *xp, double *xpp,
                               const double *xw, hipStream_t s) {
  const size_t per = (size_t)n * 2 * L, count = per * B;
  hipLaunchKernelGGL(k_accept_batch, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, per, acc, x, xp, xpp,
                     xw, count);
  return hipGetLastError();
}

// Least-squares weight of the quadratic term for a corrected point: with the
// secant prediction z_s and the quadratic prediction z_q (coefficients as in
// k_predict) and d = z_q - z_s, e = z_corr - z_s: aux[1] = Re <d, e>,
// aux[2] = <d, d> (leading limbs, fixed order), so w* = aux[1]/aux[2]
// minimises |z_s + w d - z_corr|.
template <int L>
__global__ __launch_bounds__(256) void k_blend_label(int n, const double *x, const double *xp, const double *xpp,
                                                     const double *xc, double s1, double q1, double q2,
                                                     double *aux) {
  __shared__ double ra[256], rb[256];
  double a = 0.0, b = 0.0;
  for (int v = threadIdx.x; v < n; v += 256) {
    const C<L> z = cload<L>(x + (size_t)v * 2 * L);
    const C<L> dp = csub<L>(cload<L>(xp + (size_t)v * 2 * L), z);
    const C<L> dpp = csub<L>(cload<L>(xpp + (size_t)v * 2 * L), z);
    const C<L> d = cadd<L>(cmul_d<L>(dp, q1 - s1), cmul_d<L>(dpp, q2));
    const C<L> e = csub<L>(csub<L>(cload<L>(xc + (size_t)v * 2 * L), z), cmul_d<L>(dp, s1));
    const double dr = d.re.v[0], di = d.im.v[0], er = e.re.v[0], ei = e.im.v[0];
    a += dr * er + di * ei;
    b += dr * dr + di * di;
  }
  ra[threadIdx.x] = a;
  rb[threadIdx.x] = b;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      ra[threadIdx.x] += ra[threadIdx.x + w];
      rb[threadIdx.x] += rb[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    aux[1] = ra[0];
    aux[2] = rb[0];
  }
}

hipError_t launch_blend_label(int L, int n, const double *x, const double *xprev, const double *xprev2,
                              const double *xcorr, double s1, double q1, double q2, double *aux, hipStream_t s) {
  dim3 g(1), b(256);
  switch (L) {
    case 1: hipLaunchKernelGGL(k_blend_label<1>, g, b, 0, s, n, x, xprev, xprev2, xcorr, s1, q1, q2, aux); break;
    case 2: hipLaunchKernelGGL(k_blend_label<2>, g, b, 0, s, n, x, xprev, xprev2, xcorr, s1, q1, q2, aux); break;
    case 4: hipLaunchKernelGGL(k_blend_label<4>, g, b, 0, s, n, x, xprev, xprev2, xcorr, s1, q1, q2, aux); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// The controller's features of the state a corrector stage leads to if the
// Newton test accepts it: the host-known part in `h`, the stage's Newton
// results from its state and the predictor distance from aux[0].
__global__ void k_ctl_features(CtlFeatIn h, const NewtonState *st, const double *aux, float *f) {
  h.iters = st->iterations;
  h.rho_first = st->rho_first;
  h.rho_last = st->rho;
  h.cond = st->cond_est;
  h.dz_first = st->dz_first;
  h.znorm = st->xnorm;
  h.pred_dist = aux[0];
  ctl_features(h, f);
}

hipError_t launch_ctl_features(const CtlFeatIn &h, const NewtonState *st, const double *aux, float *f,
                               hipStream_t s) {
  hipLaunchKernelGGL(k_ctl_features, dim3(1), dim3(1), 0, s, h, st, aux, f);
  return hipGetLastError();
}

__global__ void k_stage_readback(const NewtonState *st, const double *aux, const float *pout, StageReadback *rb) {
  const int t = threadIdx.x;
  if (t == 0) rb->st = *st;
  if (t < 4) rb->aux[t] = aux[t];
  if (t < 8) rb->pout[t] = pout ? pout[t] : 0.0f;
}

hipError_t launch_stage_readback(const NewtonState *st, const double *aux, const float *pout, StageReadback *rb,
                                 hipStream_t s) {
  hipLaunchKernelGGL(k_stage_readback, dim3(1), dim3(64), 0, s, st, aux, pout, rb);
  return hipGetLastError();
}

__global__ void k_copy(double *dst, const double *src, size_t count) {
  const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < count) dst[q] = src[q];
}

hipError_t launch_copy(double *dst, const double *src, size_t count, hipStream_t s) {
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, dst, src, count);
  return hipGetLastError();
}

// ---- arithmetic test entry

template <int L>
__global__ void k_arith(int op, int64_t count, const double *a, const double *b, const double *c, double *out) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= count) return;  // count is a multiple of 64 for op 16: whole wavefronts stay
  if (op == 16) {
    // the elimination's pivot search over each group of 64 elements (one wavefront)
    const C<L> x = cload<L>(a + q * 2 * L);
    const unsigned long long best = wave_max_u64(pack_key(cabs1_hi<L>(x), (int)(threadIdx.x & 63)));
    out[q * L] = packed_nonzero(best) ? (double)unpack_row(best) : -1.0;
#pragma unroll
    for (int k = 1; k < L; ++k) out[q * L + k] = 0.0;
    return;
  }
  if (op < 10) {
    R<L> x, y, r;
#pragma unroll
    for (int k = 0; k < L; ++k) {
      x.v[k] = a[q * L + k];
      y.v[k] = b[q * L + k];
    }
    switch (op) {
      case 0: r = radd<L>(x, y); break;
      case 1: r = rsub<L>(x, y); break;
      case 2: r = rmul<L>(x, y); break;
      default: r = rdiv<L>(x, y); break;
    }
#pragma unroll
    for (int k = 0; k < L; ++k) out[q * L + k] = r.v[k];
  } else {
    const C<L> x = cload<L>(a + q * 2 * L);
    C<L> r;
    if (op == 15) {
      r = cinv<L>(x);
    } else {
      const C<L> y = cload<L>(b + q * 2 * L);
      switch (op) {
        case 10: r = cadd<L>(x, y); break;
        case 11: r = csub<L>(x, y); break;
        case 12: r = cmul<L>(x, y); break;
        case 13: r = cdiv<L>(x, y); break;
        default: r = cfms<L>(x, y, cload<L>(c + q * 2 * L)); break;
      }
    }
    cstore<L>(out + q * 2 * L, r);
  }
}

hipError_t launch_arith(int op, int L, int64_t count, const double *a, const double *b, const double *c,
                        double *out, hipStream_t s) {
  dim3 g((unsigned)((count + 255) / 256)), bl(256);
  switch (L) {
    case 1: hipLaunchKernelGGL(k_arith<1>, g, bl, 0, s, op, count, a, b, c, out); break;
    case 2: hipLaunchKernelGGL(k_arith<2>, g, bl, 0, s, op, count, a, b, c, out); break;
    case 4: hipLaunchKernelGGL(k_arith<4>, g, bl, 0, s, op, count, a, b, c, out); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace qdp
