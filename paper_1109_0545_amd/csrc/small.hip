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
  s->active = (1.0 > eps && max_it > 0) ? 1 : 0;
}

hipError_t launch_init_state(NewtonState *st, double eps, int max_it, hipStream_t s) {
  hipLaunchKernelGGL(k_init_state, dim3(1), dim3(64), 0, s, st, eps, max_it);
  return hipGetLastError();
}

// Secant predictor: z' = z + r (z - z_prev) with r = (t' - t)/(t - t_prev);
// constant predictor (z' = z) before the second accepted point.
template <int L>
__global__ void k_predict(int n, const double *x, const double *xp, double r, int have_prev, double *out) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const C<L> z = cload<L>(x + (size_t)v * 2 * L);
  C<L> o = z;
  if (have_prev) {
    const C<L> zp = cload<L>(xp + (size_t)v * 2 * L);
    o = cadd<L>(z, cmul_d<L>(csub<L>(z, zp), r));
  }
  cstore<L>(out + (size_t)v * 2 * L, o);
}

hipError_t launch_predict(int L, int n, const double *x, const double *xprev, double r, int have_prev,
                          double *xpred, hipStream_t s) {
  dim3 g((n + 255) / 256), b(256);
  switch (L) {
    case 1: hipLaunchKernelGGL(k_predict<1>, g, b, 0, s, n, x, xprev, r, have_prev, xpred); break;
    case 2: hipLaunchKernelGGL(k_predict<2>, g, b, 0, s, n, x, xprev, r, have_prev, xpred); break;
    case 4: hipLaunchKernelGGL(k_predict<4>, g, b, 0, s, n, x, xprev, r, have_prev, xpred); break;
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
