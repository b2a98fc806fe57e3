// Small kernels around the Newton loop: state reset, the secant predictor,
// and the multiword arithmetic test entry.

#include "common.hpp"

namespace qdp {
using namespace mw;

// Algorithm 4.1 initialises the residual to 1 and loops while it exceeds eps
// and fewer than Max_It iterations ran.
__global__ void k_init_state(NewtonState *s, double eps, int max_it) {
  if (threadIdx.x != 0) return;
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
  s->active = (1.0 > eps && max_it > 0) ? 1 : 0;
}

hipError_t launch_init_state(NewtonState *st, double eps, int max_it, hipStream_t s) {
  hipLaunchKernelGGL(k_init_state, dim3(1), dim3(64), 0, s, st, eps, max_it);
  return hipGetLastError();
}

// Secant predictor: z' = z + w r (z - z_prev) with r = (t' - t)/(t - t_prev)
// (w = 1 is the secant through the last two accepted points; a learned
// controller may blend it towards the constant predictor w = 0); constant
// predictor before the second accepted point.  One workgroup; aux[0] gets
// ||z' - z||_inf (|Re| + |Im| of the leading limbs).
template <int L>
__global__ __launch_bounds__(256) void k_predict(int n, const double *x, const double *xp, double r, int have_prev,
                                                 double *out, double *aux) {
  __shared__ double red[4];
  double m = 0.0;
  for (int v = threadIdx.x; v < n; v += 256) {
    const C<L> z = cload<L>(x + (size_t)v * 2 * L);
    C<L> o = z;
    if (have_prev) {
      const C<L> d = cmul_d<L>(csub<L>(z, cload<L>(xp + (size_t)v * 2 * L)), r);
      o = cadd<L>(z, d);
      m = fmax(m, cabs1_hi<L>(d));
    }
    cstore<L>(out + (size_t)v * 2 * L, o);
  }
  for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0 && aux) aux[0] = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
}

hipError_t launch_predict(int L, int n, const double *x, const double *xprev, double r, int have_prev,
                          double *xpred, double *aux, hipStream_t s) {
  dim3 g(1), b(256);
  switch (L) {
    case 1: hipLaunchKernelGGL(k_predict<1>, g, b, 0, s, n, x, xprev, r, have_prev, xpred, aux); break;
    case 2: hipLaunchKernelGGL(k_predict<2>, g, b, 0, s, n, x, xprev, r, have_prev, xpred, aux); break;
    case 4: hipLaunchKernelGGL(k_predict<4>, g, b, 0, s, n, x, xprev, r, have_prev, xpred, aux); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Best secant weight for a corrected point: with d = z - z_prev and
// e = z_corr - z, aux[1] = Re <d, e> and aux[2] = <d, d> (leading limbs, fixed
// order), so that w* = aux[1] / (r aux[2]) minimises |z + w r d - z_corr|.
template <int L>
__global__ __launch_bounds__(256) void k_blend_label(int n, const double *x, const double *xp, const double *xc,
                                                     double *aux) {
  __shared__ double ra[256], rb[256];
  double a = 0.0, b = 0.0;
  for (int v = threadIdx.x; v < n; v += 256) {
    const C<L> z = cload<L>(x + (size_t)v * 2 * L);
    const C<L> d = csub<L>(z, cload<L>(xp + (size_t)v * 2 * L));
    const C<L> e = csub<L>(cload<L>(xc + (size_t)v * 2 * L), z);
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

hipError_t launch_blend_label(int L, int n, const double *x, const double *xprev, const double *xcorr, double *aux,
                              hipStream_t s) {
  switch (L) {
    case 1: hipLaunchKernelGGL(k_blend_label<1>, dim3(1), dim3(256), 0, s, n, x, xprev, xcorr, aux); break;
    case 2: hipLaunchKernelGGL(k_blend_label<2>, dim3(1), dim3(256), 0, s, n, x, xprev, xcorr, aux); break;
    case 4: hipLaunchKernelGGL(k_blend_label<4>, dim3(1), dim3(256), 0, s, n, x, xprev, xcorr, aux); break;
    default: return hipErrorInvalidValue;
  }
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
  if (q >= count) return;
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
