// Residual, Gaussian elimination with partial pivoting on [A b], back
// substitution and the update z := z + dz of one Newton iteration
// (Algorithm 4.1 and the description of GE / Back_Subs in Section 4).
//
// Section 4 selects as pivot the largest number in the current column, then
// lets every thread update its own rows, then solves the triangular system.
// Here one workgroup owns the whole system: the augmented matrix sits in LDS
// when it fits (n <= 64 in double-double), otherwise in global memory (L2).
// The matrix is column-major (column k holds a_{rk} for all rows r, the
// right-hand side b = -h is column n), so a wavefront reading one column
// reads consecutive addresses.  Rows are never swapped: the not-yet-pivoted
// rows form a list that is compacted each step (double-buffered), and each
// elimination step spreads the remaining rows times remaining columns over
// all threads with one barrier per step.  The pivot key is |Re| + |Im| of the
// leading limb (FP64), ties to the lowest row index; every wavefront finds the
// pivot on its own, so no extra barrier is needed.  The inverse of each pivot
// is kept for the back substitution, which one wavefront runs column by
// column with register shuffles.

#pragma once
#include "common.hpp"

namespace qdp {
using namespace mw;

template <int L> struct GeArgs {
  int n;
  double *ab;     // column-major (n+1) x n complex, element (r,k) at (k*n + r)*2L
  double *scale;  // [n] FP64 componentwise scale of h (nullable -> 1)
  double *x;      // [n][2][L] current point, updated in place
  double *dz;     // [n][2][L] correction out (nullable)
  NewtonState *st;
};

template <int NT> __device__ double block_max(double v, double *buf) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  __syncthreads();
  if (lane == 0) buf[wave] = v;
  __syncthreads();
  double r = buf[0];
  for (int w = 1; w < NT / 64; ++w) r = fmax(r, buf[w]);
  return r;
}

template <int L, int NT, bool IN_LDS>
__global__ __launch_bounds__(NT) void k_ge(GeArgs<L> a) {
  if (a.st && !a.st->active) return;
  extern __shared__ double smem[];
  const int n = a.n;
  const int tid = threadIdx.x, lane = tid & 63;
  constexpr int E2 = 2 * L;

  // LDS carve-up
  size_t off = 0;
  double *Mlds = smem;
  if (IN_LDS) off += (size_t)n * (n + 1) * E2;
  C<L> *invp = reinterpret_cast<C<L> *>(smem + off);
  off += (size_t)n * E2;
  C<L> *bb = reinterpret_cast<C<L> *>(smem + off);
  off += (size_t)n * E2;
  double *redbuf = smem + off;
  off += 16;
  int *act0 = reinterpret_cast<int *>(smem + off);
  int *act1 = act0 + n;
  int *perm = act1 + n;
  int *flags = perm + n;  // [0] singular

  double *M = IN_LDS ? Mlds : a.ab;
  auto at = [&](int r, int k) -> double * { return M + ((size_t)k * n + r) * E2; };

  if (IN_LDS) {
    const size_t tot = (size_t)n * (n + 1) * E2;
    for (size_t q = tid; q < tot; q += NT) Mlds[q] = a.ab[q];
  }
  for (int r = tid; r < n; r += NT) act0[r] = r;
  if (tid == 0) flags[0] = 0;
  __syncthreads();

  // ---- residual rho = max_i |h_i|_1 / max_i S_i (leading limbs, FP64)
  double hb = 0.0, sb = 0.0;
  for (int r = tid; r < n; r += NT) {
    const C<L> b = cload<L>(at(r, n));
    hb = fmax(hb, cabs1_hi<L>(b));
    if (!cfinite<L>(b)) hb = __builtin_nan("");
    sb = fmax(sb, a.scale ? a.scale[r] : 1.0);
  }
  // NaN must survive the max: encode it as +inf for the reduction
  const double hb_r = block_max<NT>(__builtin_isnan(hb) ? __builtin_inf() : hb, redbuf);
  const double sb_r = block_max<NT>(sb, redbuf);
  const double rho = (hb_r == __builtin_inf()) ? __builtin_nan("") : (sb_r > 0.0 ? hb_r / sb_r : hb_r);

  // ---- elimination
  double pmax = 0.0, pmin = __builtin_inf();
  int *cur = act0, *nxt = act1;
  bool singular = !(rho == rho);  // NaN residual: skip the solve
  for (int j = 0; j < n && !singular; ++j) {
    const int K = n - j;
    // pivot search (every wavefront, identical result)
    double best = -1.0;
    int bestr = 0x7fffffff, bests = 0;
    for (int s = lane; s < K; s += 64) {
      const int r = cur[s];
      const double key = cabs1_hi<L>(cload<L>(at(r, j)));
      const double kk = (key == key) ? key : -1.0;
      if (kk > best || (kk == best && r < bestr)) {
        best = kk;
        bestr = r;
        bests = s;
      }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const double ob = __shfl_xor(best, o, 64);
      const int orr = __shfl_xor(bestr, o, 64);
      const int os = __shfl_xor(bests, o, 64);
      if (ob > best || (ob == best && orr < bestr)) {
        best = ob;
        bestr = orr;
        bests = os;
      }
    }
    if (!(best > 0.0)) {  // zero (or NaN) column: singular
      singular = true;
      break;
    }
    const int p = bestr;
    const C<L> inv = cinv<L>(cload<L>(at(p, j)));
    pmax = fmax(pmax, best);
    pmin = fmin(pmin, best);
    if (tid == 0) {
      invp[j] = inv;
      perm[j] = p;
    }
    const int R = K - 1;
    if (R > 0) {
      // compacted list without p: slot s -> row (cur[s] == p ? cur[K-1] : cur[s])
      for (int s = tid; s < R; s += NT) {
        const int r = cur[s];
        nxt[s] = (r == p) ? cur[K - 1] : r;
      }
      const int P = NT / R > 0 ? NT / R : 1;
      for (int q = tid; q < R * P; q += NT) {
        const int s = q % R, ph = q / R;
        int r = cur[s];
        if (r == p) r = cur[K - 1];
        const C<L> l = cmul<L>(cload<L>(at(r, j)), inv);
        for (int k = j + 1 + ph; k <= n; k += P) {
          double *e = at(r, k);
          cstore<L>(e, cfms<L>(cload<L>(e), l, cload<L>(at(p, k))));
        }
      }
    }
    __syncthreads();
    int *tmp = cur;
    cur = nxt;
    nxt = tmp;
  }

  // ---- back substitution (one wavefront) and update
  if (!singular && tid < 64) {
    for (int i = lane; i < n; i += 64) bb[i] = cload<L>(at(perm[i], n));
    for (int j = n - 1; j >= 0; --j) {
      C<L> dj = czero<L>();
      if (lane == (j & 63)) dj = cmul<L>(bb[j], invp[j]);
      dj = cshfl<L>(dj, j & 63, 64);
      for (int i = lane; i < j; i += 64) bb[i] = cfms<L>(bb[i], cload<L>(at(perm[i], j)), dj);
      if (lane == (j & 63)) bb[j] = dj;
    }
  }
  __syncthreads();
  double dmax = 0.0;
  if (!singular) {
    for (int v = tid; v < n; v += NT) {
      const C<L> d = bb[v];
      if (a.dz) cstore<L>(a.dz + (size_t)v * E2, d);
      if (a.x) {
        double *xp = a.x + (size_t)v * E2;
        cstore<L>(xp, cadd<L>(cload<L>(xp), d));
      }
      dmax = fmax(dmax, cabs1_hi<L>(d));
    }
  }
  dmax = block_max<NT>(dmax, redbuf);
  if (tid == 0 && a.st) {
    NewtonState *s = a.st;
    s->iterations += 1;
    if (s->iterations == 1) s->rho_first = rho;
    s->rho = rho;
    s->dz_norm = dmax;
    s->cond_est = (pmin > 0.0 && pmin < __builtin_inf()) ? pmax / pmin : __builtin_inf();
    if (singular && rho == rho) s->singular = 1;
    if (!(rho == rho)) s->nonfinite = 1;
    s->success = (rho < s->eps) ? 1 : 0;
    s->active = (!singular && rho > s->eps && s->iterations < s->max_it) ? 1 : 0;
  }
}

}  // namespace qdp
