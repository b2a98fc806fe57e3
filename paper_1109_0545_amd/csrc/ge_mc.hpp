// Gaussian elimination with partial pivoting and back substitution of one
// point's Newton system (Section 4, GE and Back_Subs; the solve of
// Algorithm 4.1) spread over n+1 workgroups, one per column of [A | b], for
// the systems whose elimination keeps one compute unit busy for a long time
// (quad double, and double double past 64 rows): one point then runs on
// n+1 compute units instead of one.
//
// Workgroup c (one wavefront) holds column c in registers, lane l rows
// l + 64u.  Step j of the elimination needs from column j's workgroup only
// the pivot row and the multipliers of column j; they go through a per-point
// global workspace, published with a release fence and a 64-bit flag
// (agent scope, so workgroups on different XCDs see them):
//   * workgroup c takes the steps j < c in order: waits for column j's flag,
//     reads its pivot row p and multipliers (zero in the rows the step leaves
//     alone, pivot rows included) and applies a - l u with u its own entry in
//     row p (a lane read);
//   * after step c-1 its column is final below the pivot rows: it chooses
//     the pivot (the same 32-bit DPP maximum, ties and candidate rules as the
//     register kernel), forms the inverse and the multipliers, publishes
//     them, then stores its U part scaled by the pivot inverses,
//     U(k, c) / U(k, k), into a packed triangle and raises a second flag;
//   * workgroup n (the right-hand side) forms the residual of h from its
//     column before the first step, takes all n steps, scales y by the pivot
//     inverses, waits for every column's triangle and back-substitutes
//     column by column (x_j by a lane read, a fused multiply-subtract in
//     every lane above j, the next columns loaded ahead), then updates x and
//     the Newton state exactly as the one-workgroup kernels do.
// The chain from one pivot to the next crosses compute units once per column
// (publish, flag, read: ~1.2 us measured on MI355X), so this pays where a
// column's trailing update costs more than that on one compute unit.
// The arithmetic is that of the register kernel step for step (the same
// updates in the same order, the same pivot choice and scaled substitution),
// so the two agree bit for bit where both apply.
//
// Flags hold a tag (magic high word, launch counter low word): a stale flag
// from an earlier launch, or from other data in the workspace, never matches
// the current launch, so the workspace is never cleared.  All workgroups of
// a launch must be resident at once (the launcher caps points x (n+1)); every
// wait is bounded by the shader wall clock, and a wait past its limit ends
// the elimination with the point marked non-finite instead of hanging.
#pragma once
#include "ge_reg.hpp"

namespace qdp {

constexpr unsigned long long kMcOk = 0x9E3779B9ull << 32;    // | launch counter
constexpr unsigned long long kMcFail = 0x7F4A7C15ull << 32;  // | launch counter
constexpr unsigned long long kMcWaitTicks = 20000000ull;       // 0.2 s of the 100 MHz wall clock

// Wait (lane 0 polls, the wavefront follows) until *f == tag; false after
// the time limit.  The acquire fence after it makes the publisher's data
// visible.
__device__ inline bool mc_wait(const unsigned long long *f, unsigned long long tag, bool spin) {
  int ok = 1;
  if ((threadIdx.x & 63) == 0) {
    const unsigned long long t0 = wall_clock64();
    for (int it = 0; __hip_atomic_load(f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != tag; ++it) {
      if ((it & 63) == 63 && wall_clock64() - t0 > kMcWaitTicks) {
        ok = 0;
        break;
      }
      if (!spin) __builtin_amdgcn_s_sleep(1);
    }
  }
  ok = __builtin_amdgcn_readfirstlane(__shfl(ok, 0, 64));
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  return ok != 0;
}
__device__ inline void mc_raise(unsigned long long *f, unsigned long long v) {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  if ((threadIdx.x & 63) == 0) __hip_atomic_store(f, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// grid (n+1, B), 64 threads; ws: B per-point workspaces of ge_mc_doubles(L, n)
template <int L, int RPL, int PF = 4>
__global__ __launch_bounds__(64) void k_ge_mc(GeArgs<L> a, double *ws, unsigned epoch) {
  constexpr int RMAX = 64 * RPL, E2 = 2 * L;
  constexpr int RB = RPL == 1 ? 6 : 7;
  const int n = a.n, c = blockIdx.x;
  const size_t b = blockIdx.y;
  NewtonState *const nst = a.st ? a.st + b : nullptr;
  if (nst && !nst->active) return;
  const size_t PS = (size_t)n * (n + 1);
  const double *const ab = a.ab + b * E2 * PS;
  const int lane = threadIdx.x;
  const unsigned long long tag = kMcOk | epoch, tag_fail = kMcFail | epoch;

  double *const mult = ws + b * ge_mc_doubles(L, n);
  const size_t TT = mc_tri_doubles(n);
  double *const tri = mult + (size_t)n * E2 * RMAX;
  double *const invp = tri + E2 * TT;
  double *const pmag = invp + E2 * RMAX;
  int2 *const ctl = reinterpret_cast<int2 *>(pmag + RMAX);
  unsigned long long *const pub = reinterpret_cast<unsigned long long *>(pmag + 2 * RMAX);
  unsigned long long *const fin = pub + RMAX;

  C<L> v[RPL];
  int pos[RPL];  // pivot step of row lane + 64u (n while not yet a pivot row)
  bool act[RPL];
#pragma unroll
  for (int u = 0; u < RPL; ++u) {
    const int r = lane + 64 * u;
    v[u] = r < n ? pload<L>(ab + (size_t)c * n + r, PS) : czero<L>();
    pos[u] = n;
    act[u] = r < n;
  }

  // residual of h (column n before the elimination)
  double rho = 0.0;
  bool bad = false;
  if (c == n) {
    const double *const scale = a.scale ? a.scale + b * n : nullptr;
    double hb = 0.0, sb = 0.0;
    bool fin_ok = true;
#pragma unroll
    for (int u = 0; u < RPL; ++u)
      if (lane + 64 * u < n) {
        hb = fmax(hb, cabs1_hi<L>(v[u]));
        fin_ok = fin_ok && cfinite<L>(v[u]);
      }
    for (int r = lane; r < n; r += 64) sb = fmax(sb, scale ? scale[r] : 1.0);
    hb = wave_max_f64(hb);
    sb = wave_max_f64(sb);
    bad = __ballot(!fin_ok) != 0ull;
    rho = bad ? __builtin_nan("") : (sb > 0.0 ? hb / sb : hb);
  }

  // ---- steps j < c
  bool ok = true, late = false;
  int last = c < n ? c : n - 1;  // last column whose pivot this workgroup reads or makes
  for (int j = 0; j < c; ++j) {
    if (!mc_wait(pub + j, tag, j + 1 == c)) {
      ok = false;
      late = true;
      break;
    }
    const int2 cj = ctl[j];
    const int sgj = __builtin_amdgcn_readfirstlane(cj.y);
    const int p = __builtin_amdgcn_readfirstlane(cj.x);
    if (sgj != 0) {
      ok = false;
      last = j;
      break;
    }
    const double *const mj = mult + (size_t)j * E2 * RMAX;
    C<L> l[RPL];
#pragma unroll
    for (int u = 0; u < RPL; ++u) l[u] = pload<L>(mj + lane + 64 * u, RMAX);
    const C<L> uv = reg_row<L, RPL>(v, p);
#pragma unroll
    for (int u = 0; u < RPL; ++u) {
      v[u] = cfms<L>(v[u], l[u], uv);
      const int r = lane + 64 * u;
      if (r == p) pos[u] = j;
      act[u] = act[u] && r != p;
    }
  }

  if (c < n) {
    // ---- pivot of column c, its multipliers published; then the scaled U part
    if (ok) {
      unsigned best = 0;
      double key[RPL];
      C<L> own_inv[RPL];
#pragma unroll
      for (int u = 0; u < RPL; ++u) {
        key[u] = cabs1_hi<L>(v[u]);
        best = max(best, pack_key32<RB>(key[u], lane + 64 * u, act[u]));
        own_inv[u] = cinv<L>(v[u]);
      }
      best = wave_umax32(best);
      const bool sg = (best >> RB) <= 1u;
      const int p = sg ? 0 : RMAX - 1 - (int)(best & (RMAX - 1));
      const C<L> inv = sg ? czero<L>() : reg_row<L, RPL>(own_inv, p);
      double pkey = key[0];
#pragma unroll
      for (int u = 1; u < RPL; ++u)
        if ((p >> 6) == u) pkey = key[u];
      pkey = sg ? 0.0 : rdlane(pkey, p & 63);
      double *const mc = mult + (size_t)c * E2 * RMAX;
#pragma unroll
      for (int u = 0; u < RPL; ++u) {
        const int r = lane + 64 * u;
        const bool upd = !sg && act[u] && r != p;
        pstore<L>(mc + r, RMAX, upd ? cmul<L>(v[u], inv) : czero<L>());
      }
      if (lane == 0) {
        ctl[c] = make_int2(p, sg ? 1 : 0);
        pstore<L>(invp + c, RMAX, inv);
        pmag[c] = pkey;
      }
      mc_raise(pub + c, tag);
      if (!sg) {
#pragma unroll
        for (int u = 0; u < RPL; ++u)
          if (pos[u] < c)
            pstore<L>(tri + (size_t)c * (c - 1) / 2 + pos[u], TT, cmul<L>(v[u], pload<L>(invp + pos[u], RMAX)));
      }
    }
    mc_raise(fin + c, late ? tag_fail : tag);
    return;
  }

  // ---- workgroup n: y scaled by the pivot inverses, in pivot order
  __shared__ double ys[E2 * RMAX];
  if (bad) ok = false;
  if (ok) {
#pragma unroll
    for (int u = 0; u < RPL; ++u)
      if (pos[u] < n) pstore<L>(ys + pos[u], RMAX, cmul<L>(v[u], pload<L>(invp + pos[u], RMAX)));
    // every column's triangle part stored
    bool all = true;
#pragma unroll
    for (int u = 0; u < RPL; ++u) {
      const int cc = lane + 64 * u;
      if (cc < n) {
        const unsigned long long t0 = wall_clock64();
        unsigned long long f;
        int it = 0;
        while ((f = __hip_atomic_load(fin + cc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) != tag && f != tag_fail) {
          if ((++it & 63) == 0 && wall_clock64() - t0 > kMcWaitTicks) break;
          __builtin_amdgcn_s_sleep(1);
        }
        all = all && f == tag;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    if (__ballot(!all) != 0ull) {
      ok = false;
      late = true;
    }
  }
  if (late) bad = true;
  __syncthreads();

  // ---- back substitution: x_j = y_j - sum_{k > j} U'(j, k) x_k
  double *const xpt = a.x ? a.x + b * n * E2 : nullptr;
  double *const dzp = a.dz ? a.dz + b * n * E2 : nullptr;
  double dmax = 0.0, xmax = 0.0;
  if (ok) {
    C<L> bb[RPL];
#pragma unroll
    for (int u = 0; u < RPL; ++u) {
      const int k = lane + 64 * u;
      bb[u] = k < n ? pload<L>(ys + k, RMAX) : czero<L>();
    }
    auto col_of = [&](int j, C<L> (&uc)[RPL]) __attribute__((always_inline)) {
#pragma unroll
      for (int u = 0; u < RPL; ++u) {
        const int k = lane + 64 * u;
        uc[u] = (j >= 1 && k < j) ? pload<L>(tri + (size_t)j * (j - 1) / 2 + k, TT) : czero<L>();
      }
    };
    C<L> ring[PF][RPL];
#pragma unroll
    for (int q = 0; q < PF; ++q) col_of(n - 1 - q, ring[q]);
    for (int j0 = n - 1; j0 > 0; j0 -= PF) {
#pragma unroll
      for (int q = 0; q < PF; ++q) {
        const int j = j0 - q;
        if (j < 1) break;
        const C<L> xj = reg_row<L, RPL>(bb, j);
#pragma unroll
        for (int u = 0; u < RPL; ++u) {
          if (64 * u >= j) break;  // wave-uniform: no row of this slot is above j
          bb[u] = cfms<L>(bb[u], ring[q][u], xj);  // zero from row j on
        }
        col_of(j - PF, ring[q]);
      }
    }
#pragma unroll
    for (int u = 0; u < RPL; ++u) {
      const int k = lane + 64 * u;
      if (k < n) {
        const C<L> d = bb[u];
        if (dzp) cstore<L>(dzp + (size_t)k * E2, d);
        if (xpt) {
          double *xp = xpt + (size_t)k * E2;
          const C<L> xn = cadd<L>(cload<L>(xp), d);
          cstore<L>(xp, xn);
          xmax = fmax(xmax, cabs1_hi<L>(xn));
        }
        dmax = fmax(dmax, cabs1_hi<L>(d));
      }
    }
  }
  dmax = wave_max_f64(dmax);
  xmax = wave_max_f64(xmax);
  if (bad) last = 0;
  double pmx = 0.0, pmn = __builtin_inf();
  for (int j = lane; j <= last; j += 64) {
    pmx = fmax(pmx, pmag[j]);
    pmn = fmin(pmn, pmag[j]);
  }
  pmx = wave_max_f64(pmx);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) pmn = fmin(pmn, __shfl_xor(pmn, off, 64));
  if (lane == 0 && nst) newton_bookkeeping(nst, rho, !ok, bad, dmax, pmx, pmn, xmax);
}

}  // namespace qdp
