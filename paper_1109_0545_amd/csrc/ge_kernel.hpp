// Residual, Gaussian elimination with partial pivoting on [A b], back
// substitution and the update z := z + dz of one Newton iteration
// (Algorithm 4.1 and the description of GE / Back_Subs in Section 4).
//
// In Section 4 a single thread chooses the pivot row by magnitude within the
// column while the other threads wait; then all threads update their rows,
// and the threads synchronise once per column.  On one CDNA4 workgroup the pivot search
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
// inverses are kept for the back substitution: every thread scales the rows
// of U by them, then one wavefront runs the substitution column by column
// with lane reads.
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

// One butterfly step of a wavefront maximum on a 64-bit key: each lane takes
// the larger of its key and the key of the lane the DPP control names.
template <int CTRL> __device__ inline unsigned long long dpp_max_step(unsigned long long w) {
  const int lo = (int)(unsigned)w, hi = (int)(unsigned)(w >> 32);
  const unsigned olo = (unsigned)__builtin_amdgcn_update_dpp(lo, lo, CTRL, 0xf, 0xf, false);
  const unsigned ohi = (unsigned)__builtin_amdgcn_update_dpp(hi, hi, CTRL, 0xf, 0xf, false);
  const unsigned long long o = ((unsigned long long)ohi << 32) | olo;
  return o > w ? o : w;
}

// Maximum over a full wavefront (all 64 lanes active), returned in every
// lane: butterflies inside each row of 16 lanes with DPP (lane xor 1, lane
// xor 2, the half-row mirror, the row mirror), then the four row maxima read
// into scalars.  No LDS round trip.
__device__ inline unsigned long long wave_max_u64(unsigned long long w) {
  w = dpp_max_step<0xB1>(w);   // quad_perm [1,0,3,2]
  w = dpp_max_step<0x4E>(w);   // quad_perm [2,3,0,1]
  w = dpp_max_step<0x141>(w);  // row_half_mirror
  w = dpp_max_step<0x140>(w);  // row_mirror
  unsigned long long m = 0;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)w, 16 * r);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(w >> 32), 16 * r);
    const unsigned long long v = ((unsigned long long)hi << 32) | lo;
    m = v > m ? v : m;
  }
  return m;
}

// value of lane `src` (the same in every lane) in every lane
__device__ inline double rdlane(double v, int src) {
  const long long b = __double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, src);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), src);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// broadcast lane `src` (wave-uniform) of a complex multiword value
template <int L> __device__ inline C<L> cbcast(const C<L> &a, int src) {
  C<L> r;
#pragma unroll
  for (int k = 0; k < L; ++k) {
    r.re.v[k] = rdlane(a.re.v[k], src);
    r.im.v[k] = rdlane(a.im.v[k], src);
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

// rows of the matrix a lane of wavefront 0 owns: lane + 64 u, u < RPL; RPL = 1
// for n <= 64 keeps the look-ahead state small, 4 covers n <= 256
constexpr int kRowsPerLane = 4;

// Gaussian elimination with partial pivoting of the column-major matrix M
// (n rows, n+1 columns, 2L limb planes PS apart), one workgroup of NT
// threads; the last column is the right-hand side and is eliminated too.
// Multipliers are stored in place of the eliminated entries; perm[j] is the
// pivot row of column j and invp[j] the inverse of its pivot.  Returns false
// when a column has no nonzero pivot.  Must be called by every thread.
//
// Wavefront 0 looks one column ahead and keeps its state in registers: lane l
// owns rows l + 64u with an "not yet pivot" flag and the multiplier of the
// last pivot column.  During step j it updates column j+1 of its rows, finds
// that column's pivot (largest |Re|+|Im| of the leading limb; see pack_key)
// with a DPP maximum, forms the pivot's inverse, stores the multipliers of
// column j+1 and writes the list of rows the next step updates, while the
// other wavefronts update columns j+2..n of the rows of this step's list.
// Pivot row, inverse and a singular flag go to LDS (parity-indexed: ctl[2 +
// (j & 1)] = column j has no nonzero pivot).  One barrier per column.
template <int L, int NT, int RPL = kRowsPerLane>
__device__ bool eliminate(double *M, size_t PS, int n, const ElimLds<L> &e, bool bad, double &pmax, double &pmin) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  auto at = [&](int r, int k) -> double * { return M + (size_t)k * n + r; };
  C<L> *invp = e.invp;
  int *perm = e.perm, *ctl = e.ctl;
  const unsigned long long below = (1ull << lane) - 1ull;  // lanes under this one

  bool act[RPL];    // wavefront 0: row lane + 64u not yet a pivot row
  C<L> mul[RPL];    // wavefront 0: its multiplier of the last pivot column
  int p = 0;        // wavefront 0: pivot row of the current column

  // wavefront 0, after the pivot p1 of a column is chosen among the values v:
  // multipliers (or, for the pivot row, the U entry) stored in column k,
  // flags updated, and the ordered list of the remaining rows written to out
  auto publish = [&](C<L> (&v)[RPL], int k, int p1, bool sing, const C<L> &inv, int *out) {
#pragma unroll
    for (int u = 0; u < RPL; ++u) {
      if (64 * u >= n) break;  // wave-uniform: no row in this slot
      const int r = lane + 64 * u;
      if (act[u]) {
        if (r == p1) {
          pstore<L>(at(r, k), PS, v[u]);
          act[u] = false;
        } else if (!sing) {
          mul[u] = cmul<L>(v[u], inv);
          pstore<L>(at(r, k), PS, mul[u]);
        }
      }
    }
    int base = 0;
#pragma unroll
    for (int u = 0; u < RPL; ++u) {
      if (64 * u >= n) break;
      const unsigned long long m = __ballot(act[u]);
      if (act[u]) out[base + __popcll(m & below)] = lane + 64 * u;
      base += __popcll(m);
    }
  };
  // the pivot row's value, from the lane that holds it (a per-lane select,
  // not an index into v: an indexed register array would go to scratch)
  auto pivot_value = [&](C<L> (&v)[RPL], int p1) {
    C<L> pv = czero<L>();
#pragma unroll
    for (int u = 0; u < RPL; ++u) pv = cselect<L>(lane + 64 * u == p1, v[u], pv);
    return cbcast<L>(pv, p1 & 63);
  };

  // wavefront 0 carries the column-to-column dependence chain: it issues
  // first when the SIMD it shares with update wavefronts has a choice
  if (wave == 0) __builtin_amdgcn_s_setprio(3);

  // ---- column 0: pivot and multipliers (wavefront 0)
  if (wave == 0) {
    unsigned long long best = 0;
    C<L> v[RPL];
#pragma unroll
    for (int u = 0; u < RPL; ++u) {
      const int r = lane + 64 * u;
      act[u] = r < n;
      v[u] = czero<L>();
      if (act[u]) {
        v[u] = pload<L>(at(r, 0), PS);
        const unsigned long long w = pack_key(cabs1_hi<L>(v[u]), r);
        best = w > best ? w : best;
      }
    }
    best = wave_max_u64(best);
    const bool sing = !packed_nonzero(best) || bad;
    p = unpack_row(best);
    const C<L> pv = pivot_value(v, p);
    const C<L> inv = sing ? czero<L>() : cinv<L>(pv);
    publish(v, 0, p, sing, inv, e.list0);
    if (lane == 0) {
      invp[0] = inv;
      const double k = cabs1_hi<L>(pv);
      pmax = k;
      pmin = k;
      ctl[2] = sing ? 1 : 0;
      perm[0] = p;
    }
  }
  __syncthreads();

  int *cur = e.list0, *nxt = e.list1;
  bool singular = ctl[2] != 0;
  int steps_done = 0;
  for (int j = 0; j < n && !singular; ++j) {
    const int R = n - 1 - j;  // rows this step updates: not yet pivot rows
    if (R > 0) {
      if (wave == 0) {
        // look-ahead: column j+1 of every remaining row, its pivot, multipliers
        const C<L> up = pload<L>(at(p, j + 1), PS);
        unsigned long long best = 0;
        C<L> v[RPL];
#pragma unroll
        for (int u = 0; u < RPL; ++u) {
          const int r = lane + 64 * u;
          v[u] = czero<L>();
          if (64 * u < n && act[u]) {
            v[u] = cfms<L>(pload<L>(at(r, j + 1), PS), mul[u], up);
            const unsigned long long w = pack_key(cabs1_hi<L>(v[u]), r);
            best = w > best ? w : best;
          }
        }
        best = wave_max_u64(best);
        const bool sing = !packed_nonzero(best);
        const int p1 = unpack_row(best);
        const C<L> pv = pivot_value(v, p1);
        const C<L> inv = sing ? czero<L>() : cinv<L>(pv);
        publish(v, j + 1, p1, sing, inv, nxt);
        if (lane == 0) {
          invp[j + 1] = inv;
          const double k = cabs1_hi<L>(pv);
          pmax = fmax(pmax, k);
          pmin = fmin(pmin, k);
          ctl[2 + ((j + 1) & 1)] = sing ? 1 : 0;
          perm[j + 1] = p1;
        }
        p = p1;
      } else {
        // trailing update of columns j+2..n: each thread keeps one row (and
        // its multiplier) and takes every CPR-th column, two at a time with
        // both loads issued first; lanes of a wavefront share columns, so the
        // pivot row's entry is a broadcast read
        const int ncol = n - j - 1;
        const int pj = perm[j];
        if (ncol > 0) {
          constexpr int T = NT - 64;
          const int t = tid - 64;
          const int CPR = T / R;
          if (t < CPR * R) {
            const int sl = t % R, c = t / R;
            const int r = cur[sl];
            const C<L> lr = pload<L>(at(r, j), PS);
            constexpr int UN = 2;
            for (int k = j + 2 + c; k <= n; k += UN * CPR) {
              C<L> av[UN], uv[UN];
#pragma unroll
              for (int w = 0; w < UN; ++w) {
                const int kk = k + w * CPR;
                if (kk <= n) {
                  av[w] = pload<L>(at(r, kk), PS);
                  uv[w] = pload<L>(at(pj, kk), PS);
                }
              }
#pragma unroll
              for (int w = 0; w < UN; ++w) {
                const int kk = k + w * CPR;
                if (kk <= n) pstore<L>(at(r, kk), PS, cfms<L>(av[w], lr, uv[w]));
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
  if (wave == 0) __builtin_amdgcn_s_setprio(0);
  return !singular && steps_done == n;
}

// Rows of U scaled by their pivot inverses: U(i, k) / U(i, i) for i < k < n
// in place (the right-hand-side column n is left as it is), by every thread
// of the workgroup, one column per group of lanes (consecutive lanes take
// consecutive pivot rows of one column).  Takes the product by the pivot
// inverse out of the back substitution's column-to-column chain.
template <int L, int NT>
__device__ void scale_upper(double *M, size_t PS, int n, const int *perm, const C<L> *invp) {
  for (int q = threadIdx.x; q < n * n; q += NT) {
    const int k = q / n, i = q - k * n;
    if (i < k) {
      double *p = M + (size_t)k * n + perm[i];
      pstore<L>(p, PS, cmul<L>(pload<L>(p, PS), invp[i]));
    }
  }
}

// Back substitution by wavefront 0 on the eliminated matrix whose U rows were
// scaled by scale_upper: returns through the limb planes of `out` (n
// elements, plane stride n) the solution of the upper triangle (rows
// perm[0..n-1]) with right-hand side rhs_of(i) for the pivot-ordered index i.
// With y_i = rhs_i / U(i, i) and U' the scaled rows, x_j = y_j - sum_{k > j}
// U'(j, k) x_k: lane l keeps y_l, y_{l+64}, ... in registers, and once x_j is
// final (column j's turn) it travels by lane reads to every lane, which
// subtracts U'(i, j) x_j from its rows i < j.
template <int L, typename Rhs, int RPL = kRowsPerLane>
__device__ void back_substitute(const double *M, size_t PS, int n, const int *perm, const C<L> *invp, double *out,
                                Rhs rhs_of) {
  const int lane = threadIdx.x & 63;
  auto at = [&](int r, int k) -> const double * { return M + (size_t)k * n + r; };
  C<L> b[RPL];
  int pr[RPL];
#pragma unroll
  for (int u = 0; u < RPL; ++u) {
    const int i = lane + 64 * u;
    b[u] = czero<L>();
    pr[u] = 0;
    if (i < n) {
      b[u] = cmul<L>(rhs_of(i), invp[i]);
      pr[u] = perm[i];
    }
  }
  for (int j = n - 1; j >= 0; --j) {
    C<L> bj = czero<L>();
#pragma unroll
    for (int u = 0; u < RPL; ++u) bj = cselect<L>(lane + 64 * u == j, b[u], bj);
    const C<L> xj = cbcast<L>(bj, j & 63);
#pragma unroll
    for (int u = 0; u < RPL; ++u) {
      if (64 * u >= j) break;  // wave-uniform: no row of this slot is above j
      const int i = lane + 64 * u;
      if (i < j) b[u] = cfms<L>(b[u], pload<L>(at(pr[u], j), PS), xj);
    }
  }
#pragma unroll
  for (int u = 0; u < RPL; ++u) {
    const int i = lane + 64 * u;
    if (i < n) pstore<L>(out + i, n, b[u]);
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

template <int L, int NT, bool IN_LDS, int RPL>
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
  const bool ok = eliminate<L, NT, RPL>(M, PS, n, el, bad, pmax, pmin);
  if (ok) scale_upper<L, NT>(M, PS, n, el.perm, el.invp);  // ok is the same in every thread
  __syncthreads();
  auto rhs = [&](int i) { return pload<L>(M + (size_t)n * n + el.perm[i], PS); };
  if (ok && wave == 0) back_substitute<L, decltype(rhs), RPL>(M, PS, n, el.perm, el.invp, bb, rhs);
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
