// Mixed-precision Newton correction for double-double systems: the Jacobian
// is factored in FP64 and the correction is refined against the
// double-double residual (iterative refinement).
//
// The paper solves the Newton system by Gaussian elimination in the working
// precision (Algorithm 4.1, GE and Back_Subs).  Here, per Newton iteration:
//   1. A64 = fl64(J) (the leading limbs, which are limb planes 0 and 2 of the
//      double-double [A | b] buffer), factored by partial-pivoting
//      elimination in FP64 together with b64 = fl64(b), b = -h;
//   2. dz = U^{-1} L^{-1} P b64, kept in double double;
//   3. up to R times: r = b - J dz in double double (J, b the full
//      double-double evaluation), c = U^{-1} L^{-1} P fl64(r) by forward and
//      back substitution with the stored FP64 factors, dz += c (double
//      double); stop early once ||c|| <= 2^-104 ||dz||;
//   4. z += dz.
// With kappa(J) u64 << 1 each refinement gains about -log10(kappa u64)
// digits, down to the double-double level.  The residual, the pivot choice
// and every error-free transformation stay in FP64 hardware arithmetic.

#include "ge_kernel.hpp"

namespace qdp {
using namespace mw;

struct MixedArgs {
  int n;
  double *ab;     // double-double [A | -h], column-major, 4 limb planes of n(n+1)
  double *scale;  // [n]
  double *x;      // [n][2][2] double-double point, updated in place
  double *lu;     // FP64 workspace of 2 planes of n(n+1) (used when the factors do not fit in LDS)
  NewtonState *st;
  int max_refine;
};

template <int NT, bool IN_LDS>
__global__ __launch_bounds__(NT) void k_mixed(MixedArgs a) {
  // point b of a batch: every array advances by its per-point size
  {
    const size_t b = blockIdx.x, ps = (size_t)a.n * (a.n + 1);
    if (a.st) a.st += b;
    a.ab += b * 4 * ps;
    if (a.scale) a.scale += b * a.n;
    if (a.x) a.x += b * a.n * 4;
    if (a.lu) a.lu += b * 2 * ps;
  }
  if (a.st && !a.st->active) return;
  extern __shared__ double smem[];
  const int n = a.n;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const size_t PS = (size_t)n * (n + 1);
  const int nch = NT / n < 16 ? NT / n : 16;       // chunks actually used
  const int cw = (n + nch - 1) / nch;               // columns per chunk

  // ---- LDS carve-up
  size_t off = 0;
  double *M64 = IN_LDS ? smem : a.lu;  // FP64 [A | b]: planes re, im (PS apart)
  if (IN_LDS) off += 2 * PS;
  ElimLds<1> el;
  el.invp = reinterpret_cast<C<1> *>(smem + off);
  off += 2 * (size_t)n;
  double *dz = smem + off;  // double-double correction, 4 planes of n
  off += 4 * (size_t)n;
  double *yv = smem + off;  // FP64 work vector, 2 planes of n
  off += 2 * (size_t)n;
  double *part = smem + off;  // double-double partial products, 4 planes of 16*n
  off += 4 * 16 * (size_t)n;
  double *redbuf = smem + off;
  off += 16;
  el.list0 = reinterpret_cast<int *>(smem + off);
  el.list1 = el.list0 + n;
  el.perm = el.list1 + n;
  el.ctl = el.perm + n;

  // ---- residual, FP64 copy of [A | b]
  bool bad = false;
  const double rho = residual_of<2, NT>(a.ab + (size_t)n * n, PS, n, a.scale, redbuf, bad);
  for (size_t q = tid; q < PS; q += NT) {
    M64[q] = a.ab[q];               // re, leading limb
    M64[PS + q] = a.ab[2 * PS + q];  // im, leading limb
  }
  __syncthreads();

  double pmax = 0.0, pmin = __builtin_inf();
  const bool ok = eliminate<1, NT>(M64, PS, n, el, bad, pmax, pmin);
  if (ok) scale_upper<1, NT>(M64, PS, n, el.perm, el.invp);  // U rows / pivots; the multipliers stay
  __syncthreads();

  // ---- first correction from the eliminated right-hand side
  if (ok && wave == 0)
    back_substitute<1>(M64, PS, n, el.perm, el.invp, yv,
                       [&](int i) { return pload<1>(M64 + (size_t)n * n + el.perm[i], PS); });
  __syncthreads();
  if (ok)
    for (int v = tid; v < n; v += NT) {
      const C<1> c = pload<1>(yv + v, n);
      C<2> d = czero<2>();
      d.re.v[0] = c.re.v[0];
      d.im.v[0] = c.im.v[0];
      pstore<2>(dz + v, n, d);
    }
  __syncthreads();

  // ---- iterative refinement
  int steps = 0;
  double rel = 0.0;
  for (int it = 0; ok && it < a.max_refine; ++it) {
    // partial products sum_k J(i,k) dz_k over column chunks
    {
      const int i = tid % n, c = tid / n;
      if (c < nch) {
        C<2> acc = czero<2>();
        const int k0 = c * cw, k1 = min(n, k0 + cw);
        for (int k = k0; k < k1; ++k)
          acc = cadd<2>(acc, cmul<2>(pload<2>(a.ab + (size_t)k * n + i, PS), pload<2>(dz + k, n)));
        pstore<2>(part + (size_t)c * n + i, (size_t)16 * n, acc);
      }
    }
    __syncthreads();
    // r_i = b_i - sum_c part[c][i] in fixed order; FP64 copy in pivot order for the solve
    for (int i = tid; i < n; i += NT) {
      C<2> s = pload<2>(part + i, (size_t)16 * n);
      for (int c = 1; c < nch; ++c) s = cadd<2>(s, pload<2>(part + (size_t)c * n + i, (size_t)16 * n));
      const C<2> r = csub<2>(pload<2>(a.ab + (size_t)n * n + i, PS), s);
      C<1> r64;
      r64.re.v[0] = r.re.v[0] + r.re.v[1];
      r64.im.v[0] = r.im.v[0] + r.im.v[1];
      pstore<1>(part + i, (size_t)16 * n, r64);  // reuse chunk 0 as the FP64 residual (row order)
    }
    __syncthreads();
    if (wave == 0) {
      // forward substitution with the stored multipliers, in pivot order
      for (int i = lane; i < n; i += 64) pstore<1>(yv + i, n, pload<1>(part + el.perm[i], (size_t)16 * n));
      for (int j = 0; j < n; ++j) {
        const int owner = j & 63;
        C<1> yj = czero<1>();
        if (lane == owner) yj = pload<1>(yv + j, n);
        yj = cbcast<1>(yj, owner);
        for (int i = j + 1 + ((lane - (j + 1)) & 63); i < n; i += 64)
          pstore<1>(yv + i, n, cfms<1>(pload<1>(yv + i, n), pload<1>(M64 + (size_t)j * n + el.perm[i], PS), yj));
      }
      back_substitute<1>(M64, PS, n, el.perm, el.invp, yv, [&](int i) { return pload<1>(yv + i, n); });
    }
    __syncthreads();
    double cm = 0.0, zm = 0.0;
    for (int v = tid; v < n; v += NT) {
      const C<1> c = pload<1>(yv + v, n);
      C<2> d = pload<2>(dz + v, n);
      C<2> c2 = czero<2>();
      c2.re.v[0] = c.re.v[0];
      c2.im.v[0] = c.im.v[0];
      d = cadd<2>(d, c2);
      pstore<2>(dz + v, n, d);
      cm = fmax(cm, cabs1_hi<1>(c));
      zm = fmax(zm, cabs1_hi<2>(d));
    }
    cm = block_max<NT>(cm, redbuf);
    zm = block_max<NT>(zm, redbuf);
    ++steps;
    rel = zm > 0.0 ? cm / zm : 0.0;
    if (rel <= 0x1p-104) break;  // uniform: every thread holds the same block maxima
  }

  // ---- update and bookkeeping
  double dmax = 0.0, xmax = 0.0;
  if (ok)
    for (int v = tid; v < n; v += NT) {
      const C<2> d = pload<2>(dz + v, n);
      double *xp = a.x + (size_t)v * 4;
      const C<2> xn = cadd<2>(cload<2>(xp), d);
      cstore<2>(xp, xn);
      dmax = fmax(dmax, cabs1_hi<2>(d));
      xmax = fmax(xmax, cabs1_hi<2>(xn));
    }
  dmax = block_max<NT>(dmax, redbuf);
  xmax = block_max<NT>(xmax, redbuf);
  if (tid == 0 && a.st) {
    newton_bookkeeping(a.st, rho, !ok, bad, dmax, pmax, pmin, xmax);
    a.st->refine_steps = steps;
    a.st->refine_err = rel;
  }
}

size_t mixed_lds_bytes(int n, bool in_lds) {
  size_t d = (in_lds ? 2 * (size_t)n * (n + 1) : 0) + 2 * (size_t)n + 4 * (size_t)n + 2 * (size_t)n +
             4 * 16 * (size_t)n + 16;
  return d * sizeof(double) + (3 * (size_t)n + 8) * sizeof(int) + 64;
}

hipError_t launch_mixed_solve(int n, int B, double *ab, double *scale, double *x, NewtonState *st, double *lu,
                              double * /*work*/, int refinements, hipStream_t s) {
  if (B < 1) return hipErrorInvalidValue;
  constexpr int NT = 1024;
  MixedArgs a{n, ab, scale, x, lu, st, refinements};
  const bool fit = mixed_lds_bytes(n, true) <= 160 * 1024;
  const size_t lds = mixed_lds_bytes(n, fit);
  hipError_t e;
  if (fit) {
    e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_mixed<NT, true>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_mixed<NT, true>), dim3(B), dim3(NT), lds, s, a);
  } else {
    e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_mixed<NT, false>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_mixed<NT, false>), dim3(B), dim3(NT), lds, s, a);
  }
  return hipGetLastError();
}

}  // namespace qdp
