// Residual, Gaussian elimination with partial pivoting on [A b], back
// substitution and the update z := z + dz of one Newton iteration
// (Algorithm 4.1 and the description of GE / Back_Subs in Section 4).
//
// Section 4 lets one thread pick the pivot (the largest number in the
// current column) while the others wait, then every thread updates its own
// rows, with a barrier per column.  On one CDNA4 workgroup the pivot search
// and the pivot's inverse would then sit on the critical path of every
// column, so this kernel looks one column ahead:
//   * during step j, wavefront 0 updates column j+1 of every remaining row
//     first, finds the pivot of column j+1 in registers (largest |Re|+|Im| of
//     the leading limb, ties to the lowest row), forms its inverse and
//     publishes both in LDS;
//   * meanwhile the other wavefronts update columns j+2..n (the right-hand
//     side b = -h is column n);
//   * one barrier per column.
// The augmented matrix is column-major and split into limb planes (a
// wavefront reading one column reads consecutive doubles of each plane, so
// LDS accesses hit consecutive banks); it sits in LDS when it fits, else in
// global memory.
// Rows are never swapped: the not-yet-pivoted rows form an ordered list,
// compacted each step without reordering (double-buffered).  The pivot
// inverses are kept for the back substitution, which one wavefront runs
// column by column with register shuffles.
#pragma once
#include "common.hpp"

namespace qdp {
using namespace mw;

// One workgroup per point of a batch: point b's arrays start b times the
// per-point size after point 0's.
template <int L> struct GeArgs {
  int n;
  double *ab;     // [B] column-major (n+1) x n complex in 2L limb planes: limb c of (r,k) at c*n(n+1) + k*n + r
  double *scale;  // [B][n] FP64 componentwise scale of h (nullable -> 1)
  double *x;      // [B][n][2][L] current point, updated in place (nullable)
  double *dz;     // [B][n][2][L] correction out (nullable)
  NewtonState *st;  // [B] (nullable)
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

// Pack a nonnegative FP64 pivot key and a row index into one 64-bit word
// whose unsigned order is (key descending, then row ascending), so that the
// argmax over a wavefront is a max over one word.  The key contributes the
// high word of its FP64 bit pattern (sign, exponent, 20 mantissa bits), which
// is monotone for nonnegative doubles; keys within a relative 1e-6 of each
// other tie and go to the lowest row, which partial pivoting tolerates.
// 0 = no candidate (NaN or no row); a high word of zero marks a zero column.
__device__ inline unsigned long long pack_key(double key, int row) {
  const bool ok = key == key && key >= 0.0;
  const unsigned int kb = ok ? (unsigned int)(__double_as_longlong(key) >> 32) + 1u : 0u;
  return ((unsigned long long)kb << 32) | (unsigned int)(0x7fffffff - row);
}
__device__ inline int unpack_row(unsigned long long w) { return 0x7fffffff - (int)(w & 0xffffffffu); }
__device__ inline bool packed_nonzero(unsigned long long w) { return (w >> 32) > 1u; }

__device__ inline unsigned long long wave_max_u64(unsigned long long w) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const unsigned long long ow = __shfl_xor(w, o, 64);
    w = ow > w ? ow : w;
  }
  return w;
}

// broadcast lane `src` (wave-uniform) of a complex multiword value
template <int L> __device__ inline C<L> cbcast(const C<L> &a, int src) {
  C<L> r;
#pragma unroll
  for (int k = 0; k < L; ++k) {
    r.re.v[k] = __shfl(a.re.v[k], src, 64);
    r.im.v[k] = __shfl(a.im.v[k], src, 64);
  }
  return r;
}

// Shared state of one elimination in LDS.
template <int L> struct ElimLds {
  C<L> *invp;  // [n] pivot inverses
  int *list0, *list1;
  int *perm;   // [n] pivot row of each column
  int *ctl;    // [4] parity-indexed control words (see eliminate)
};

// Gaussian elimination with partial pivoting of the column-major matrix M
// (n rows, n+1 columns, 2L limb planes PS apart), one workgroup of NT
// threads; the last column is the right-hand side and is eliminated too.
// Multipliers are stored in place of the eliminated entries; perm[j] is the
// pivot row of column j and invp[j] the inverse of its pivot.  Returns false
// when a column has no nonzero pivot.  Must be called by every thread.
//
// Wavefront 0 looks one column ahead: during step j it updates column j+1 of
// every remaining row, finds that column's pivot (largest |Re|+|Im| of the
// leading limb; see pack_key), forms its inverse and stores the multipliers
// of column j+1, and publishes pivot row / list slot / inverse / singular
// flag in parity-indexed LDS words (ctl[j & 1] = slot of the pivot of column
// j in the list of step j, ctl[2 + (j & 1)] = column j has no nonzero pivot),
// while the other wavefronts update columns j+2..n.  One barrier per column.
template <int L, int NT>
__device__ bool eliminate(double *M, size_t PS, int n, const ElimLds<L> &e, bool bad, double &pmax, double &pmin) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  auto at = [&](int r, int k) -> double * { return M + (size_t)k * n + r; };
  C<L> *invp = e.invp;
  int *perm = e.perm, *ctl = e.ctl;
  for (int r = tid; r < n; r += NT) e.list0[r] = r;

  // ---- column 0: pivot and multipliers (wavefront 0)
  if (wave == 0) {
    unsigned long long best = 0;
    for (int s = lane; s < n; s += 64) {
      const unsigned long long w = pack_key(cabs1_hi<L>(pload<L>(at(s, 0), PS)), s);
      best = w > best ? w : best;
    }
    best = wave_max_u64(best);
    const bool sing = !packed_nonzero(best) || bad;
    const int p0 = unpack_row(best);
    if (!sing) {
      const C<L> pv = pload<L>(at(p0, 0), PS);
      const C<L> inv = cinv<L>(pv);
      for (int s = lane; s < n; s += 64)
        if (s != p0) pstore<L>(at(s, 0), PS, cmul<L>(pload<L>(at(s, 0), PS), inv));
      if (lane == 0) {
        invp[0] = inv;
        const double k = cabs1_hi<L>(pv);
        pmax = k;
        pmin = k;
      }
    }
    if (lane == 0) {
      ctl[2] = sing ? 1 : 0;
      ctl[0] = p0;  // the initial list is the identity: slot = row
      perm[0] = p0;
    }
  }
  __syncthreads();

  int *cur = e.list0, *nxt = e.list1;
  bool singular = ctl[2] != 0;
  int steps_done = 0;
  for (int j = 0; j < n && !singular; ++j) {
    const int K = n - j;  // rows in the list (the pivot row included)
    const int R = K - 1;  // rows to update
    const int p = perm[j];
    const int pos = ctl[j & 1];
    // slot s of the rows to update -> row (the list without the pivot, order kept)
    auto row_of = [&](int s) { return cur[s + (s >= pos ? 1 : 0)]; };
    if (R > 0) {
      if (wave == 0) {
        // look-ahead: update column j+1, choose its pivot, store its multipliers
        const C<L> up = pload<L>(at(p, j + 1), PS);
        unsigned long long best = 0;
        constexpr int RPL = 4;  // rows per lane kept in registers (n <= 256)
        C<L> vals[RPL];
        int rows[RPL];
#pragma unroll
        for (int u = 0; u < RPL; ++u) {
          const int s = lane + 64 * u;
          rows[u] = -1;
          vals[u] = czero<L>();
          if (s < R) {
            const int r = row_of(s);
            const C<L> v = cfms<L>(pload<L>(at(r, j + 1), PS), pload<L>(at(r, j), PS), up);
            vals[u] = v;
            rows[u] = r;
            nxt[s] = r;
            const unsigned long long w = pack_key(cabs1_hi<L>(v), r);
            best = w > best ? w : best;
          }
        }
        best = wave_max_u64(best);
        const bool sing = !packed_nonzero(best);
        const int p1 = unpack_row(best);
        // the lane holding the pivot value broadcasts it
        int owner = 0, ou = 0;
#pragma unroll
        for (int u = 0; u < RPL; ++u) {
          const unsigned long long m = __ballot(rows[u] == p1);
          if (m) {
            owner = __builtin_ffsll(m) - 1;
            ou = u;
          }
        }
        C<L> pv = vals[0];
#pragma unroll
        for (int u = 1; u < RPL; ++u)
          if (ou == u) pv = vals[u];
        pv = cbcast<L>(pv, owner);
        if (!sing) {
          const C<L> inv = cinv<L>(pv);
#pragma unroll
          for (int u = 0; u < RPL; ++u)
            if (rows[u] >= 0) pstore<L>(at(rows[u], j + 1), PS, rows[u] == p1 ? vals[u] : cmul<L>(vals[u], inv));
          if (lane == 0) {
            invp[j + 1] = inv;
            const double k = cabs1_hi<L>(pv);
            pmax = fmax(pmax, k);
            pmin = fmin(pmin, k);
          }
        }
        if (lane == 0) {
          ctl[2 + ((j + 1) & 1)] = sing ? 1 : 0;
          ctl[(j + 1) & 1] = ou * 64 + owner;
          perm[j + 1] = p1;
        }
      } else {
        // trailing update of columns j+2..n: items (column, row slot) in
        // column-major order spread evenly over wavefronts 1..
        const int ncol = n - j - 1;
        if (ncol > 0) {
          constexpr int T = NT - 64;
          const int items = R * ncol;
          const int t = tid - 64;
          if (t < items) {
            const int dk = T / R, ds = T - dk * R;
            int s = t % R, k = j + 2 + t / R;
            for (int q = t; q < items; q += T) {
              const int r = row_of(s);
              double *ep = at(r, k);
              pstore<L>(ep, PS, cfms<L>(pload<L>(ep, PS), pload<L>(at(r, j), PS), pload<L>(at(p, k), PS)));
              s += ds;
              k += dk;
              if (s >= R) {
                s -= R;
                k += 1;
              }
            }
          }
        }
      }
    }
    __syncthreads();
    singular = (R > 0) && ctl[2 + ((j + 1) & 1)] != 0;
    steps_done = j + 1;
    int *tmp = cur;
    cur = nxt;
    nxt = tmp;
  }
  return !singular && steps_done == n;
}

// Back substitution by wavefront 0 on the eliminated matrix: returns through
// the limb planes of `out` (n elements, plane stride n) the solution of the
// upper triangle (rows perm[0..n-1]) with right-hand side rhs_of(i) for the
// pivot-ordered index i.
template <int L, typename Rhs>
__device__ void back_substitute(const double *M, size_t PS, int n, const int *perm, const C<L> *invp, double *out,
                                Rhs rhs_of) {
  const int lane = threadIdx.x & 63;
  auto at = [&](int r, int k) -> const double * { return M + (size_t)k * n + r; };
  for (int i = lane; i < n; i += 64) pstore<L>(out + i, n, rhs_of(i));
  for (int j = n - 1; j >= 0; --j) {
    const int owner = j & 63;
    C<L> dj = czero<L>();
    if (lane == owner) dj = cmul<L>(pload<L>(out + j, n), invp[j]);
    dj = cbcast<L>(dj, owner);
    for (int i = lane; i < j; i += 64)
      pstore<L>(out + i, n, cfms<L>(pload<L>(out + i, n), pload<L>(at(perm[i], j), PS), dj));
    if (lane == owner) pstore<L>(out + j, n, dj);
  }
}

template <int L, int NT>
__device__ double residual_of(const double *bcol, size_t PS, int n, const double *scale, double *redbuf, bool &bad) {
  const int tid = threadIdx.x;
  double hb = 0.0, sb = 0.0;
  for (int r = tid; r < n; r += NT) {
    const C<L> b = pload<L>(bcol + r, PS);
    hb = fmax(hb, cabs1_hi<L>(b));
    if (!cfinite<L>(b)) hb = __builtin_inf();
    sb = fmax(sb, scale ? scale[r] : 1.0);
  }
  const double hb_r = block_max<NT>(hb, redbuf);
  const double sb_r = block_max<NT>(sb, redbuf);
  bad = !(hb_r < __builtin_inf());
  return bad ? __builtin_nan("") : (sb_r > 0.0 ? hb_r / sb_r : hb_r);
}

__device__ inline void newton_bookkeeping(NewtonState *s, double rho, bool singular, bool bad, double dmax,
                                          double pmax, double pmin, double xmax) {
  s->iterations += 1;
  if (s->iterations == 1) {
    s->rho_first = rho;
    s->dz_first = dmax;
  }
  s->xnorm = xmax;
  s->rho = rho;
  s->dz_norm = dmax;
  s->cond_est = (pmin > 0.0 && pmin < __builtin_inf()) ? pmax / pmin : __builtin_inf();
  if (singular && !bad) s->singular = 1;
  if (bad) s->nonfinite = 1;
  s->success = (rho < s->eps) ? 1 : 0;
  s->active = (!singular && rho > s->eps && s->iterations < s->max_it) ? 1 : 0;
}

template <int L, int NT, bool IN_LDS>
__global__ __launch_bounds__(NT) void k_ge(GeArgs<L> a) {
  const int n = a.n;
  const size_t b = blockIdx.x;
  NewtonState *const nst = a.st ? a.st + b : nullptr;
  if (nst && !nst->active) return;
  double *const ab = a.ab + b * 2 * L * (size_t)n * (n + 1);
  const double *const scale = a.scale ? a.scale + b * n : nullptr;
  double *const xpt = a.x ? a.x + b * n * 2 * L : nullptr;
  double *const dzp = a.dz ? a.dz + b * n * 2 * L : nullptr;
  extern __shared__ double smem[];
  const int tid = threadIdx.x, wave = tid >> 6;
  constexpr int E2 = 2 * L;

  // ---- LDS carve-up
  size_t off = 0;
  double *Mlds = smem;
  if (IN_LDS) off += (size_t)n * (n + 1) * E2;
  ElimLds<L> el;
  el.invp = reinterpret_cast<C<L> *>(smem + off);
  off += (size_t)n * E2;
  double *bb = smem + off;  // [n] back-substitution vector, limb planes of n
  off += (size_t)n * E2;
  double *redbuf = smem + off;  // [16]
  off += 16;
  el.list0 = reinterpret_cast<int *>(smem + off);
  el.list1 = el.list0 + n;
  el.perm = el.list1 + n;
  el.ctl = el.perm + n;

  double *M = IN_LDS ? Mlds : ab;
  const size_t PS = (size_t)n * (n + 1);  // plane size
  if (IN_LDS) {
    const size_t tot = PS * E2;
    for (size_t q = tid; q < tot; q += NT) Mlds[q] = ab[q];
  }
  __syncthreads();

  bool bad = false;
  const double rho = residual_of<L, NT>(M + (size_t)n * n, PS, n, scale, redbuf, bad);
  double pmax = 0.0, pmin = __builtin_inf();
  const bool ok = eliminate<L, NT>(M, PS, n, el, bad, pmax, pmin);
  if (ok && wave == 0)
    back_substitute<L>(M, PS, n, el.perm, el.invp, bb,
                       [&](int i) { return pload<L>(M + (size_t)n * n + el.perm[i], PS); });
  __syncthreads();
  double dmax = 0.0, xmax = 0.0;
  if (ok) {
    for (int v = tid; v < n; v += NT) {
      const C<L> d = pload<L>(bb + v, n);
      if (dzp) cstore<L>(dzp + (size_t)v * E2, d);
      if (xpt) {
        double *xp = xpt + (size_t)v * E2;
        const C<L> xn = cadd<L>(cload<L>(xp), d);
        cstore<L>(xp, xn);
        xmax = fmax(xmax, cabs1_hi<L>(xn));
      }
      dmax = fmax(dmax, cabs1_hi<L>(d));
    }
  }
  dmax = block_max<NT>(dmax, redbuf);
  xmax = block_max<NT>(xmax, redbuf);
  if (tid == 0 && nst) newton_bookkeeping(nst, rho, !ok, bad, dmax, pmax, pmin, xmax);
}

}  // namespace qdp
