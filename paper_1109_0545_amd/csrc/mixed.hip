// Mixed-precision Newton correction: the Jacobian factored in FP64 (its
// leading limbs), the correction refined against the double-double or
// quad-double residual (iterative refinement).
//
// The paper solves the Newton system by Gaussian elimination in the working
// precision (Section 4, GE and Back_Subs in Algorithm 4.1).  Here, per Newton
// iteration and point, in one workgroup:
//   1. A64 = fl64([A | b]) (limb planes 0 and L of the working-precision
//      buffer, b = -h) is eliminated in registers with partial pivoting on the
//      FP64 keys by the counter-synchronized kernel of ge_reg.hpp; each
//      finished column's U part goes into a packed upper triangle in pivot
//      order scaled by that column's pivot inverse (U(i,c) / U(c,c)), its
//      multipliers are kept by row, and column n becomes y = L^-1 P b64;
//   2. dz = (LU)^-1 P fl64(b);
//   3. up to R times: r = b - J dz in the working precision (J and b the full
//      evaluation), c = (LU)^-1 P fl64(r) with the FP64 factors, dz += c; stop
//      once rho_k = ||c_k|| / ||dz|| <= 2^(-52 L), or once the next correction,
//      predicted as rho_k times the observed contraction rho_k / rho_(k-1),
//      falls below it (the error left in dz is about that next correction);
//   4. z += dz.
// With kappa(J) u64 << 1 each refinement gains about -log10(kappa u64)
// digits, up to the working precision's level.  The residual, the pivot
// choice and every error-free transformation stay in FP64 hardware
// arithmetic.
//
// Applying (LU)^-1 P: forward and back substitution on one wavefront (lane i
// holds entry i of the pivot-order vector, the current column's value travels
// by lane reads, the next columns' entries are loaded PF steps ahead, with a
// clamped address and a select instead of a branch).  Up to n = 64 both
// triangles stay in LDS (the multipliers are repacked once, from row order
// into a packed lower triangle in pivot order); at n = 128 they do not fit
// together, so the elimination writes them to a global workspace
// (L2-resident) and each correction first copies its triangle into LDS with
// the whole workgroup.
// (An explicit FP64 inverse X = U^-1 L^-1 P with one matrix-vector product per
// correction was measured slower at n = 64: forming X is n^3 work on one CU,
// ~57 us, against ~5 us per pair of substitutions.)
// The residual runs on every thread: row i = t mod n, the columns in NCH
// chunks, the chunks' partial sums added per row in a fixed order.

#include "ge_reg.hpp"

namespace qdp {
using namespace mw;

struct MixedArgs {
  int n;
  const double *ab;     // [B] working-precision [A | -h], column-major, 2L limb planes of n(n+1)
  const double *scale;  // [B][n] (nullable)
  double *x;            // [B][n][2][L] point, updated in place
  double *lu;           // [B] global factor store for n > 64 (mixed_ws_doubles each)
  NewtonState *st;      // [B]
  int max_refine;
};

// column chunks of the residual: as many as the workgroup has rows of threads
// for, at most 16; their partial sums (2L n chunks doubles) fit the region
// they share (2 n^2 doubles up to n = 64, a staged triangle beyond)
__host__ __device__ inline int mixed_chunks(int NT, int n, int L) {
  const int c = NT / n;
  return c < 1 ? 1 : (c > 16 ? 16 : c);
}

// LDS layout (double offsets; the int arrays at `ints`):
//   mult [KRING][2][RMAX], invp [2][RMAX], pmag [RMAX], misc [16] (elimination)
//   dz [2L][RMAX]   working-precision correction, by variable
//   yv [2][RMAX]    FP64 right-hand side of a correction
//   red [16]        reductions
//   n <= 64: tr: U' [2][TZ] then L' [2][TZ] (TZ = n(n-1)/2 + 1, the last entry
//            of a plane zero); big [2][n][n]: the
//            multipliers by row during the elimination, then the residual's
//            partial sums
//   n > 64:  tr: one staged triangle, or the residual's partial sums
//   ints: ctl [RMAX] int2, pub, rd [32], pos [RMAX] (pivot step of each row)
struct MixedLayout {
  size_t mult, invp, pmag, misc, dz, yv, red, tr, big, ints, bytes;
};
__host__ __device__ inline MixedLayout mixed_layout(int L, int RMAX, int NT, int n, bool resident) {
  MixedLayout o{};
  const size_t TS = ge_reg_tri_doubles(n);
  const size_t part = (size_t)2 * L * mixed_chunks(NT, n, L) * n;
  size_t d = 0;
  o.mult = d;
  d += (size_t)KRING * 2 * RMAX;
  o.invp = d;
  d += 2 * (size_t)RMAX;
  o.pmag = d;
  d += RMAX;
  o.misc = d;
  d += 16;
  o.dz = d;
  d += (size_t)2 * L * RMAX;
  o.yv = d;
  d += 2 * (size_t)RMAX;
  o.red = d;
  d += 16;
  o.tr = d;
  if (resident) {
    d += 4 * (TS + 1);
    o.big = d;
    const size_t lr = (size_t)2 * n * n;
    d += lr > part ? lr : part;
  } else {
    d += 2 * (TS + 1) > part ? 2 * (TS + 1) : part;
    o.big = o.tr;
  }
  o.ints = d;
  o.bytes = d * sizeof(double) + (2 * (size_t)RMAX + 33 + RMAX) * sizeof(int);
  return o;
}

// global doubles per point for n > 64: the multipliers by row [2][n][n], then U' [2][n(n-1)/2]
__host__ __device__ size_t mixed_ws_doubles(int n) {
  return n > 64 ? 2 * (size_t)n * n + 2 * ge_reg_tri_doubles(n) : 0;
}

// packed lower triangle in pivot order: column c holds rows c+1..n-1
__device__ __forceinline__ size_t lcol(int c, int n) { return (size_t)c * n - (size_t)c * (c + 1) / 2; }

// The substitutions keep the columns of the next PF steps in registers (a
// ring indexed at compile time: the loop is unrolled PF times; unrolled
// completely at n <= 64 the compiler spilled), so each column's LDS load is
// issued PF steps before its use.  The triangles in LDS have planes of
// TZ = n(n-1)/2 + 1 doubles whose last entry is zero: a lane outside the
// column reads that entry, so a load needs neither a branch nor a select (a
// select right after the load would wait for it there).
constexpr int PF = 4;
template <int RPL>
__device__ __forceinline__ void masked_load(C<1> (&v)[RPL], const double *base, const int (&idx)[RPL],
                                            const bool (&in)[RPL], size_t TZ) {
#pragma unroll
  for (int u = 0; u < RPL; ++u) v[u] = pload<1>(base + (in[u] ? idx[u] : (int)TZ - 1), TZ);
}
// y <- L'^-1 y (unit lower, packed by columns), pivot order
template <int RPL, int NMAX>
__device__ __forceinline__ void lower_solve(C<1> (&y)[RPL], const double *lp, int n, size_t TZ) {
  const int lane = threadIdx.x & 63;
  auto colL = [&](int c, C<1>(&v)[RPL]) {  // zero for c >= n-1
    int idx[RPL];
    bool in[RPL];
#pragma unroll
    for (int u = 0; u < RPL; ++u) {
      const int i = lane + 64 * u;
      in[u] = i > c && i < n;
      idx[u] = (int)lcol(c, n) + (i - c - 1);
    }
    masked_load<RPL>(v, lp, idx, in, TZ);
  };
  C<1> buf[PF][RPL];
#pragma unroll
  for (int k = 0; k < PF; ++k) colL(k, buf[k]);
  auto step = [&](int c, C<1>(&b)[RPL]) {
    const C<1> yc = reg_row<1, RPL>(y, c);
#pragma unroll
    for (int u = 0; u < RPL; ++u) y[u] = cfms<1>(y[u], b[u], yc);  // zero up to row c
    colL(c + PF, b);
  };
  int c0 = 0;
  for (; c0 + PF < n; c0 += PF) {  // full groups: steps c0..c0+PF-1 all < n-1
#pragma unroll
    for (int k = 0; k < PF; ++k) step(c0 + k, buf[k]);
  }
#pragma unroll
  for (int k = 0; k < PF; ++k)
    if (c0 + k + 1 < n) step(c0 + k, buf[k]);  // wave-uniform
}
// y <- U''^-1 y with U' (y_i -= U'(i,c) y_c for i < c, c = n-1..1); the
// division by U(c,c) is left to the caller
template <int RPL, int NMAX>
__device__ __forceinline__ void upper_solve(C<1> (&y)[RPL], const double *up, int n, size_t TZ) {
  const int lane = threadIdx.x & 63;
  auto colU = [&](int c, C<1>(&v)[RPL]) {  // zero for c <= 0
    int idx[RPL];
    bool in[RPL];
#pragma unroll
    for (int u = 0; u < RPL; ++u) {
      const int i = lane + 64 * u;
      in[u] = i < c;
      idx[u] = c * (c - 1) / 2 + i;
    }
    masked_load<RPL>(v, up, idx, in, TZ);
  };
  C<1> buf[PF][RPL];
#pragma unroll
  for (int k = 0; k < PF; ++k) colU(n - 1 - k, buf[k]);
  auto step = [&](int c, C<1>(&b)[RPL]) {
    const C<1> yc = reg_row<1, RPL>(y, c);
#pragma unroll
    for (int u = 0; u < RPL; ++u) {
      if (64 * u >= c) break;  // wave-uniform: no row of this slot is above c
      y[u] = cfms<1>(y[u], b[u], yc);
    }
    colU(c - PF, b);
  };
  // step m handles column c = n - 1 - m
  int m0 = 0;
  for (; m0 + PF < n; m0 += PF) {  // full groups: columns n-1-m0..n-PF-m0, all > 0
#pragma unroll
    for (int k = 0; k < PF; ++k) step(n - 1 - m0 - k, buf[k]);
  }
#pragma unroll
  for (int k = 0; k < PF; ++k)
    if (m0 + k + 1 < n) step(n - 1 - m0 - k, buf[k]);  // wave-uniform
}

template <int L, int NW, int NMAX>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu((NW + 3) / 4, (NW + 3) / 4)))
void k_mixed(MixedArgs a) {
  using S = RegShape<NW, NMAX>;
  constexpr int RPL = S::RPL, RMAX = S::RMAX, CPW = S::CPW, NT = S::NT, E2 = 2 * L;
  constexpr bool RES = NMAX <= 64;  // factors and X resident in LDS
  const int n = a.n;
  const size_t b = blockIdx.x;
  NewtonState *const nst = a.st ? a.st + b : nullptr;
  if (nst && !nst->active) return;
  const size_t PS = (size_t)n * (n + 1), NN = (size_t)n * n;
  const size_t TS = ge_reg_tri_doubles(n), TZ = TS + 1;
  const double *const ab = a.ab + b * E2 * PS;
  const double *const bvec = ab + NN;  // column n: b = -h
  const double *const scale = a.scale ? a.scale + b * n : nullptr;
  double *const xpt = a.x + b * (size_t)n * E2;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

  const MixedLayout lo = mixed_layout(L, RMAX, NT, n, RES);
  extern __shared__ double smem[];
  double *const mult = smem + lo.mult;
  double *const invp = smem + lo.invp;
  double *const pmag = smem + lo.pmag;
  double *const misc = smem + lo.misc;
  double *const dz = smem + lo.dz;
  double *const yv = smem + lo.yv;
  double *const red = smem + lo.red;
  double *const upl = smem + lo.tr;              // U' in LDS (n > 64: the staged triangle)
  double *const lpl = upl + (RES ? 2 * TZ : 0);  // L' in LDS (n > 64: the staged triangle)
  double *const big = smem + lo.big;             // n <= 64: multipliers by row; the residual's partial sums
  double *const part = big;
  int2 *const ctl = reinterpret_cast<int2 *>(smem + lo.ints);
  int *const pub = reinterpret_cast<int *>(ctl + RMAX);
  int *const rd = pub + 1;
  int *const pos = rd + 32;
  // multipliers by row (column c at c n + r, planes NN apart) and U' during
  // the elimination: LDS up to n = 64, else the global workspace
  double *const gws = RES ? nullptr : a.lu + b * mixed_ws_doubles(n);
  double *const lrow = RES ? big : gws;
  double *const ust = RES ? upl : gws + 2 * NN;

  // ---- FP64 copy of [A | b] into registers: column wave + NW s, rows lane + 64 u
  C<1> A[CPW][RPL];
#pragma unroll
  for (int s = 0; s < CPW; ++s) {
    const int c = wave + NW * s;
#pragma unroll
    for (int u = 0; u < RPL; ++u) {
      const int r = lane + 64 * u;
      C<1> v = czero<1>();
      if (c <= n && r < n) {
        v.re.v[0] = ab[(size_t)c * n + r];
        v.im.v[0] = ab[(size_t)L * PS + (size_t)c * n + r];
      }
      A[s][u] = v;
    }
  }
  // ---- residual of h (column n, before elimination) by its owner
  if (wave == n % NW) {
    double hb = 0.0, sb = 0.0;
    bool fin = true;
#pragma unroll
    for (int s = 0; s < CPW; ++s)
      if (s == n / NW) {
#pragma unroll
        for (int u = 0; u < RPL; ++u)
          if (lane + 64 * u < n) {
            hb = fmax(hb, cabs1_hi<1>(A[s][u]));
            fin = fin && cfinite<1>(A[s][u]);
          }
      }
    for (int r = lane; r < n; r += 64) sb = fmax(sb, scale ? scale[r] : 1.0);
    hb = wave_max_f64(hb);
    sb = wave_max_f64(sb);
    const bool bad = __ballot(!fin) != 0ull;
    if (lane == 0) {
      misc[0] = bad ? __builtin_nan("") : (sb > 0.0 ? hb / sb : hb);
      misc[1] = bad ? 1.0 : 0.0;
    }
  }

  // ---- FP64 elimination: U' (pivot rows, pivot order) and the multipliers
  // (by row) of each finished column into the factor store
  int mypos[RPL];
  const RegElimLds lds{mult, invp, pmag, ctl, pub, rd};
  const bool ok = reg_eliminate<1, NW, NMAX>(
      A, mypos, n, misc + 1, lds,
      [&](int c, const C<1>(&col)[RPL], const C<1> &inv, int p, const int(&rp)[RPL]) __attribute__((always_inline)) {
#pragma unroll
        for (int u = 0; u < RPL; ++u) {
          const int r = lane + 64 * u;
          if (r < n) {
            if (rp[u] < c)
              pstore<1>(ust + (size_t)c * (c - 1) / 2 + rp[u], RES ? TZ : TS, cmul<1>(col[u], inv));
            else if (r != p)
              pstore<1>(lrow + (size_t)c * n + r, NN, col[u]);
          }
        }
      });
  const bool bad = misc[1] != 0.0;
  if (ok && wave == n % NW) {
    // y = L^-1 P b64 (column n, slot 0 of its owner) in pivot order
#pragma unroll
    for (int u = 0; u < RPL; ++u)
      if (lane + 64 * u < n) pstore<1>(yv + mypos[u], RMAX, A[0][u]);
  }
  if (wave == 0) {
#pragma unroll
    for (int u = 0; u < RPL; ++u)
      if (lane + 64 * u < n) pos[lane + 64 * u] = mypos[u];  // pivot step of every row
    // the zero closing each plane of U' (resident; L' gets its own when staged)
    if (RES && lane < 2) upl[lane * TZ + TS] = 0.0;
  }
  __syncthreads();

  // L' from the multipliers by row (every thread), eight elements in flight;
  // the closing zero of each plane (the region may have held partial sums)
  auto stage_lower = [&](double *dst) {
    if (tid < 2) dst[tid * TZ + TS] = 0.0;
    for (size_t t0 = tid; t0 < NN; t0 += 8 * (size_t)NT) {
      C<1> v[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const size_t t = t0 + (size_t)k * NT;
        v[k] = t < NN ? pload<1>(lrow + t, NN) : czero<1>();
      }
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const size_t t = t0 + (size_t)k * NT;
        if (t < NN) {
          const int c = (int)(t / n), r = (int)(t - (size_t)c * n);
          const int i = pos[r];
          if (i > c) pstore<1>(dst + lcol(c, n) + (i - c - 1), TZ, v[k]);
        }
      }
    }
  };
  auto stage_upper = [&](double *dst) {
    if (tid < 2) dst[tid * TZ + TS] = 0.0;
    for (size_t t0 = tid; t0 < TS; t0 += 8 * (size_t)NT) {
      C<1> v[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const size_t t = t0 + (size_t)k * NT;
        v[k] = t < TS ? pload<1>(ust + t, TS) : czero<1>();
      }
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const size_t t = t0 + (size_t)k * NT;
        if (t < TS) pstore<1>(dst + t, TZ, v[k]);
      }
    }
  };
  auto widen = [](const C<1> &v) {
    C<L> w = czero<L>();
    w.re.v[0] = v.re.v[0];
    w.im.v[0] = v.im.v[0];
    return w;
  };
  // the pivot-order right-hand side from yv into lanes (wavefront 0)
  auto load_yv = [&](C<1>(&y)[RPL]) {
#pragma unroll
    for (int u = 0; u < RPL; ++u) y[u] = lane + 64 * u < n ? pload<1>(yv + lane + 64 * u, RMAX) : czero<1>();
  };

  // ---- first correction: dz = U^-1 y by back substitution (L' stays
  // resident in LDS up to n = 64, staged per correction beyond)
  if (ok) {
    if constexpr (RES)
      stage_lower(lpl);
    else
      stage_upper(upl);
  }
  __syncthreads();
  if (ok && wave == 0) {
    C<1> y[RPL];
    load_yv(y);
    upper_solve<RPL, NMAX>(y, upl, n, TZ);
#pragma unroll
    for (int u = 0; u < RPL; ++u) {
      const int i = lane + 64 * u;
      if (i < n) pstore<L>(dz + i, RMAX, widen(cmul<1>(y[u], pload<1>(invp + i, RMAX))));
    }
  }

  // ---- refinements: r = b - J dz, c = (LU)^-1 P fl64(r), dz += c
  const int nch = mixed_chunks(NT, n, L);
  const int cw = (n + nch - 1) / nch;
  const double eps_r = L == 2 ? 0x1p-104 : 0x1p-208;
  int steps = 0;
  double rel = 0.0, rel_prev = 0.0;
  for (int it = 0; ok && it < a.max_refine; ++it) {
    __syncthreads();  // dz complete; the staged triangle read
    {
      // r = b - J dz: partial sums over column chunks (loads of RB columns
      // issued together; two in quad double, whose operands take twice the
      // registers), then per row in order
      constexpr int RB = L == 4 ? 2 : 4;
      const int i = tid % n, ch = tid / n;
      if (ch < nch) {
        C<L> acc = czero<L>();
        const int k0 = ch * cw, k1 = min(n, k0 + cw);
        for (int kb = k0; kb < k1; kb += RB) {
          C<L> jv[RB], dv[RB];
#pragma unroll
          for (int q = 0; q < RB; ++q) {
            const int k = kb + q < k1 ? kb + q : k0;
            jv[q] = pload<L>(ab + (size_t)k * n + i, PS);
            dv[q] = pload<L>(dz + k, RMAX);
          }
#pragma unroll
          for (int q = 0; q < RB; ++q)
            if (kb + q < k1) acc = cadd<L>(acc, cmul<L>(jv[q], dv[q]));
        }
        pstore<L>(part + (size_t)ch * n + i, (size_t)nch * n, acc);
      }
      __syncthreads();
      for (int r = tid; r < n; r += NT) {
        C<L> s = pload<L>(part + r, (size_t)nch * n);
        for (int c = 1; c < nch; ++c) s = cadd<L>(s, pload<L>(part + (size_t)c * n + r, (size_t)nch * n));
        const C<L> rr = csub<L>(pload<L>(bvec + r, PS), s);
        C<1> r64;
        r64.re.v[0] = rr.re.v[0] + rr.re.v[1];
        r64.im.v[0] = rr.im.v[0] + rr.im.v[1];
        pstore<1>(yv + pos[r], RMAX, r64);  // pivot order
      }
    }
    __syncthreads();
    C<1> y[RPL];
    if constexpr (RES) {
      if (wave == 0) {
        load_yv(y);
        lower_solve<RPL, NMAX>(y, lpl, n, TZ);
        upper_solve<RPL, NMAX>(y, upl, n, TZ);
      }
    } else {
      stage_lower(lpl);
      __syncthreads();
      if (wave == 0) {
        load_yv(y);
        lower_solve<RPL, NMAX>(y, lpl, n, TZ);
      }
      __syncthreads();  // the lower triangle read
      stage_upper(upl);
      __syncthreads();
      if (wave == 0) upper_solve<RPL, NMAX>(y, upl, n, TZ);
    }
    if (wave == 0) {
#pragma unroll
      for (int u = 0; u < RPL; ++u) {
        const int i = lane + 64 * u;
        if (i < n) y[u] = cmul<1>(y[u], pload<1>(invp + i, RMAX));
      }
    }
    // dz += c; the size of the step against the correction so far
    if (wave == 0) {
      double cm = 0.0, zm = 0.0;
#pragma unroll
      for (int u = 0; u < RPL; ++u) {
        const int v = lane + 64 * u;
        if (v < n) {
          const C<L> d = cadd<L>(pload<L>(dz + v, RMAX), widen(y[u]));
          pstore<L>(dz + v, RMAX, d);
          cm = fmax(cm, cabs1_hi<1>(y[u]));
          zm = fmax(zm, cabs1_hi<L>(d));
        }
      }
      cm = wave_max_f64(cm);
      zm = wave_max_f64(zm);
      if (lane == 0) {
        red[0] = cm;
        red[1] = zm;
      }
    }
    __syncthreads();
    ++steps;
    rel = red[1] > 0.0 ? red[0] / red[1] : 0.0;
    // uniform: every thread reads the same values
    if (rel <= eps_r || (steps >= 2 && rel * rel <= eps_r * rel_prev)) break;
    rel_prev = rel;
  }
  __syncthreads();

  // ---- update and bookkeeping
  double dmax = 0.0, xmax = 0.0;
  if (ok)
    for (int v = tid; v < n; v += NT) {
      const C<L> d = pload<L>(dz + v, RMAX);
      double *xp = xpt + (size_t)v * E2;
      const C<L> xn = cadd<L>(cload<L>(xp), d);
      cstore<L>(xp, xn);
      dmax = fmax(dmax, cabs1_hi<L>(d));
      xmax = fmax(xmax, cabs1_hi<L>(xn));
    }
  dmax = block_max<NT>(dmax, red + 2);
  xmax = block_max<NT>(xmax, red + 2);
  if (wave != 0) return;
  const int last = *pub - 1;
  double pmx = 0.0, pmn = __builtin_inf();
  for (int j = lane; j <= last; j += 64) {
    pmx = fmax(pmx, pmag[j]);
    pmn = fmin(pmn, pmag[j]);
  }
  pmx = wave_max_f64(pmx);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) pmn = fmin(pmn, __shfl_xor(pmn, off, 64));
  if (lane == 0 && nst) {
    newton_bookkeeping(nst, misc[0], !ok, bad, dmax, pmx, pmn, xmax);
    nst->refine_steps = steps;
    nst->refine_err = rel;
  }
}

size_t mixed_lds_bytes(int L, int n) {
  return n <= 64 ? mixed_layout(L, 64, 1024, n, true).bytes : mixed_layout(L, 128, 512, n, false).bytes;
}

template <int L, int NW, int NMAX>
static hipError_t launch_mixed_L(int n, int B, const MixedArgs &a, hipStream_t s) {
  const size_t lds = mixed_layout(L, RegShape<NW, NMAX>::RMAX, 64 * NW, n, NMAX <= 64).bytes;
  if (lds > 160 * 1024) return hipErrorInvalidValue;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_mixed<L, NW, NMAX>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_mixed<L, NW, NMAX>), dim3(B), dim3(64 * NW), lds, s, a);
  return hipGetLastError();
}

hipError_t launch_mixed_solve(int L, int n, int B, const double *ab, const double *scale, double *x,
                              NewtonState *st, double *lu, int refinements, hipStream_t s) {
  if (B < 1 || n < 1 || n > 128 || refinements < 0 || !ab || !x) return hipErrorInvalidValue;
  if (n > 64 && !lu) return hipErrorInvalidValue;
  const MixedArgs a{n, ab, scale, x, lu, st, refinements};
  if (L == 2) return n <= 64 ? launch_mixed_L<2, 16, 64>(n, B, a, s) : launch_mixed_L<2, 8, 128>(n, B, a, s);
  if (L == 4) return n <= 64 ? launch_mixed_L<4, 16, 64>(n, B, a, s) : launch_mixed_L<4, 8, 128>(n, B, a, s);
  return hipErrorInvalidValue;
}

}  // namespace qdp
