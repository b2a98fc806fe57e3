// Gaussian elimination with partial pivoting and back substitution of one
// point's Newton system (Section 4, GE and Back_Subs; the solve of
// Algorithm 4.1) in blocks of WB consecutive columns, one block per
// workgroup (double double up to n = 128, quad double up to n = 64; RPL = 2
// rows per lane past n = 64): the register kernel's elimination (ge_reg.hpp)
// inside each block, device-memory hand-offs between blocks, so that the
// trailing updates of one point spread over several compute units while the
// pivot chain crosses a compute unit only once per block.
//
// Workgroup g holds columns g WB .. g WB + WB - 1 of [A | b]; the last one
// holds the rest, up to NW x CPW columns, ending with b = -h (column n), so
// that b does not sit alone in a block of its own.  Column c0 + w + NW s is
// in slot s of column wavefront w (lane = row); one more wavefront forwards.
//   * Steps of earlier blocks: the forwarding wavefront waits for their
//     device flags (several steps per poll when they are already raised),
//     reads pivot rows and multipliers from device memory and places them in
//     the workgroup's LDS ring of multiplier vectors, raising the LDS
//     step counter; the column wavefronts cannot tell these steps from their
//     own.
//   * Steps of the block's own columns: as in the register kernel (the owner
//     of the next column updates it first, pivots, publishes to the ring and
//     the counter, then updates the rest; no barrier per column), and the
//     owner also writes the multipliers, pivot row, inverse and magnitude to
//     device memory and raises the column's device flag for later blocks.
//   * Each finished column's U part (pivot rows, pivot order) goes to a
//     packed triangle in device memory; a block raises its flag when all of
//     its columns are stored.
//   * The workgroup holding column n waits for every block (its forwarding
//     wavefront, idle by then, waits for their flags and, in double double,
//     gathers their columns early), copies the triangle into LDS scaled by
//     the pivot inverses, and one wavefront back-substitutes as the register
//     kernel does (past n = 64 the triangle does not fit: it is read from
//     device memory, scaled as it arrives, the next four columns in flight,
//     as the column-parallel kernel does).
// Same pivots, same updates in the same order and the same substitution as
// the register kernel and the column-parallel kernel, so they agree bit for
// bit.  The workspace and its tags are those of the column-parallel kernel
// (ge_mc.hpp); all workgroups of a launch must be resident at once, and
// device-memory waits are bounded.
#pragma once
#include "ge_mc.hpp"

namespace qdp {

// LDS of one block workgroup, in doubles (then ints):
//   ring [KR][2L][R]      multipliers of the last KR steps (KR = 8, 4 in quad
//                         double, whose gathered triangle takes 129 KB at n = 64)
//   tri  [2L][TT]         (last block, n <= 64) scaled U, packed by columns;
//                         past n = 64 it is read from device memory instead
//   rhs  [2L][R]          (last block) scaled right-hand side, pivot order
//   ctl  [R] int2         pivot row and flag of every step (flag 2: a device
//                         wait ran out of time)
//   pub, rd[NW]           steps in the ring; steps read by each column wavefront
// (R = 64 rows, 128 past n = 64)
__host__ __device__ inline constexpr int mcb_ring(int L) { return L == 4 ? 4 : KRING; }
// Blocks of one point: WB columns each, the last up to WB + X (X = NW x CPW -
// WB, its spare slots) so that b joins the last full block.
__host__ __device__ inline int mcb_blocks(int n, int WB, int X) {
  const int rest = n + 1 - X;
  return rest <= WB ? 1 : (rest + WB - 1) / WB;
}
__host__ __device__ inline size_t ge_mcb_lds_bytes(int L, int n, int NW) {
  const size_t R = (size_t)mc_rows(n);
  const size_t d = (size_t)(mcb_ring(L) * 2 * L + 2 * L) * R + (n <= 64 ? 2 * (size_t)L * mc_tri_doubles(n) : 0);
  return d * sizeof(double) + R * sizeof(int2) + (size_t)(2 + NW) * sizeof(int);
}

template <int L, int NW, int CPW, int K = 4, int RPL = 1, int WB = NW * CPW>
__global__ __launch_bounds__(64 * (NW + 1)) void k_ge_mcb(GeArgs<L> a, double *ws, unsigned epoch) {
  constexpr int RMAX = 64 * RPL, E2 = 2 * L, KR = mcb_ring(L);
  static_assert(WB <= NW * CPW, "a block fits in the slots");
  constexpr bool TRI_LDS = RPL == 1;  // the gathered triangle fits in LDS
  // the forwarding wavefront gathers the earlier blocks' columns while this
  // block eliminates (double double; a quad-double entry's scaling is a
  // ~330-instruction product that slows the pivot chain sharing its SIMD)
  constexpr bool EARLY_GATHER = TRI_LDS && L <= 2;
  const int n = a.n, g = blockIdx.x;
  const size_t b = blockIdx.y;
  NewtonState *const nst = a.st ? a.st + b : nullptr;
  if (nst && !nst->active) return;
  const size_t PS = (size_t)n * (n + 1);
  const double *const ab = a.ab + b * E2 * PS;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int G = mcb_blocks(n, WB, NW * CPW - WB);  // workgroups of the point
  const int c0 = g * WB, ncols = g == G - 1 ? n + 1 - c0 : WB;
  const bool last_wg = g == G - 1;  // holds column n
  const unsigned long long tag = kMcOk | epoch, tag_fail = kMcFail | epoch;

  // device workspace (layout of ge_mc_doubles; fin holds one flag per block)
  double *const gmult = ws + b * ge_mc_doubles(L, n);
  const size_t TT = mc_tri_doubles(n);
  double *const gtri = gmult + (size_t)n * E2 * RMAX;
  double *const ginvp = gtri + E2 * TT;
  double *const gpmag = ginvp + E2 * RMAX;
  int2 *const gctl = reinterpret_cast<int2 *>(gpmag + RMAX);
  unsigned long long *const gpub = reinterpret_cast<unsigned long long *>(gpmag + 2 * RMAX);
  unsigned long long *const gfin = gpub + RMAX;

  extern __shared__ double smem[];
  double *const ring = smem;
  double *const ltri = ring + KR * E2 * RMAX;
  double *const rhs = ltri + (TRI_LDS ? E2 * TT : 0);
  int2 *const ctl = reinterpret_cast<int2 *>(rhs + E2 * RMAX);
  int *const pub = reinterpret_cast<int *>(ctl + RMAX);
  int *const rd = pub + 1;
  __shared__ double s_rho;
  __shared__ int s_bad, s_late, s_fins;

  // ---- columns into registers
  C<L> A[CPW][RPL];
  int live = 0;
  if (wave < NW) {
#pragma unroll
    for (int s = 0; s < CPW; ++s) {
      const int lc = wave + NW * s;
#pragma unroll
      for (int u = 0; u < RPL; ++u) {
        const int r = lane + 64 * u;
        A[s][u] = (lc < ncols && r < n) ? pload<L>(ab + (size_t)(c0 + lc) * n + r, PS) : czero<L>();
      }
    }
    live = wave < ncols ? (ncols - 1 - wave) / NW + 1 : 0;
  }
  // residual of h by the owner of column n
  if (tid == 0) {
    s_bad = 0;
    s_late = 0;
    s_fins = 1;
  }
  if (tid < NW) rd[tid] = 0;
  if (tid == 0) *pub = 0;
  __syncthreads();
  if (last_wg && wave == (n - c0) % NW) {
    const int sn = (n - c0) / NW;
    double hb = 0.0, sb = 0.0;
    bool fin_ok = true;
#pragma unroll
    for (int s = 0; s < CPW; ++s)
      if (s == sn) {
#pragma unroll
        for (int u = 0; u < RPL; ++u)
          if (lane + 64 * u < n) {
            hb = fmax(hb, cabs1_hi<L>(A[s][u]));
            fin_ok = fin_ok && cfinite<L>(A[s][u]);
          }
      }
    const double *const scale = a.scale ? a.scale + b * n : nullptr;
    for (int r = lane; r < n; r += 64) sb = fmax(sb, scale ? scale[r] : 1.0);
    hb = wave_max_f64(hb);
    sb = wave_max_f64(sb);
    const bool bad = __ballot(!fin_ok) != 0ull;
    if (lane == 0) {
      s_rho = bad ? __builtin_nan("") : (sb > 0.0 ? hb / sb : hb);
      s_bad = bad ? 1 : 0;
    }
  }

  int mypos[RPL];  // pivot step of row lane + 64u (n while not yet a pivot row)
  bool act[RPL];
#pragma unroll
  for (int u = 0; u < RPL; ++u) {
    mypos[u] = n;
    act[u] = lane + 64 * u < n;
  }
  bool stop = false;

  // a column's device publication (multipliers, pivot row, inverse,
  // magnitude, flag) and its U part, unscaled, into the device triangle
  auto publish_device = [&](int col, const C<L>(&v)[RPL], const bool(&upd)[RPL], int p, const C<L> &inv, double pk)
                            __attribute__((always_inline)) {
    const bool sg = pk == 0.0;
#pragma unroll
    for (int u = 0; u < RPL; ++u) {
      const int r = lane + 64 * u;
      pstore<L>(gmult + (size_t)col * E2 * RMAX + r, RMAX, (upd[u] && !sg && r != p) ? v[u] : czero<L>());
    }
    if (lane == 0) {
      gctl[col] = make_int2(p, sg ? 1 : 0);
      pstore<L>(ginvp + col, RMAX, inv);
      gpmag[col] = pk;
    }
    mc_raise(gpub + col, tag);
  };
  auto store_u = [&](int col, const C<L>(&v)[RPL]) __attribute__((always_inline)) {
#pragma unroll
    for (int u = 0; u < RPL; ++u)
      if (mypos[u] < col) pstore<L>(gtri + (size_t)col * (col - 1) / 2 + mypos[u], TT, v[u]);
  };
  // packed index q = c (c - 1) / 2 + i of the triangle, i < c: entry scaled by
  // the pivot inverse of row i, into LDS
  auto gather_entry = [&](int q) __attribute__((always_inline)) {
    int c = (int)((1.0 + sqrt(1.0 + 8.0 * q)) * 0.5);
    while (c * (c - 1) / 2 > q) --c;
    while ((c + 1) * c / 2 <= q) ++c;
    const int i = q - c * (c - 1) / 2;
    pstore<L>(ltri + q, TT, cmul<L>(pload<L>(gtri + q, TT), pload<L>(ginvp + i, RMAX)));
  };
  auto retire_slot0 = [&]() __attribute__((always_inline)) {
#pragma unroll
    for (int s = 0; s + 1 < CPW; ++s)
#pragma unroll
      for (int u = 0; u < RPL; ++u) A[s][u] = A[s + 1][u];
#pragma unroll
    for (int u = 0; u < RPL; ++u) A[CPW - 1][u] = czero<L>();
    --live;
  };

  if (wave == NW) {
    // ---- forwarding wavefront: steps 0..c0-1 from device memory into the ring
    int j = 0;
    while (j < c0) {
      if (!mc_wait(gpub + j, tag, true)) {
        // out of time: a failure entry stops the column wavefronts
        const int need = j - KR + 1;
        int rdl = lane < NW ? __hip_atomic_load(rd + lane, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) : need;
        while (__ballot(rdl < need) != 0ull)
          rdl = lane < NW ? __hip_atomic_load(rd + lane, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) : need;
        if (lane == 0) {
          ctl[j] = make_int2(0, 2);
          s_late = 1;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        if (lane == 0) __hip_atomic_store(pub, j + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        break;
      }
      // the steps after j already raised (up to K in all)
      const bool rdy = lane >= 1 && lane < K && j + lane < c0 &&
                       __hip_atomic_load(gpub + j + lane, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == tag;
      const unsigned long long nr = ~(__ballot(rdy) | 1ull);
      const int r = nr ? __builtin_ctzll(nr) : K;  // leading raised flags, >= 1
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      C<L> lk[K][RPL];
      const int2 ck = lane < r ? gctl[j + lane] : make_int2(0, 0);
#pragma unroll
      for (int k = 0; k < K; ++k)
        if (k < r)
#pragma unroll
          for (int u = 0; u < RPL; ++u) lk[k][u] = pload<L>(gmult + (size_t)(j + k) * E2 * RMAX + lane + 64 * u, RMAX);
      bool sing = false;
#pragma unroll
      for (int k = 0; k < K; ++k) {
        if (k >= r || sing) break;
        const int jj = j + k;
        const int px = __builtin_amdgcn_readlane(ck.x, k), py = __builtin_amdgcn_readlane(ck.y, k);
        const int need = jj - KR + 1;
        int rdl = lane < NW ? __hip_atomic_load(rd + lane, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) : need;
        while (__ballot(rdl < need) != 0ull)
          rdl = lane < NW ? __hip_atomic_load(rd + lane, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) : need;
#pragma unroll
        for (int u = 0; u < RPL; ++u) pstore<L>(ring + (jj % KR) * E2 * RMAX + lane + 64 * u, RMAX, lk[k][u]);
        if (lane == 0) ctl[jj] = make_int2(px, py);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        if (lane == 0) __hip_atomic_store(pub, jj + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        sing = py != 0;
      }
      if (sing) break;
      j += r;
    }
    if (last_wg) {
      // idle from here on: wait for the other blocks' flags (every block
      // raises its flag, also after a stop), then gather their triangle
      // columns into LDS while this block eliminates its own
      bool all = true;
      if (lane < G - 1) {
        const unsigned long long t0 = wall_clock64();
        unsigned long long f;
        int it = 0;
        while ((f = __hip_atomic_load(gfin + lane, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) != tag && f != tag_fail) {
          if ((++it & 63) == 0 && wall_clock64() - t0 > kMcWaitTicks) break;
          __builtin_amdgcn_s_sleep(1);
        }
        all = f == tag;
      }
      const bool fins = __ballot(!all) == 0ull;
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      if (lane == 0) s_fins = fins ? 1 : 0;
      if constexpr (EARLY_GATHER) {
        if (fins)
          for (int q = lane; q < c0 * (c0 - 1) / 2; q += 64) gather_entry(q);
      }
    }
  } else {
    // ---- column wavefronts
    auto published = [&]() {
      return __builtin_amdgcn_readfirstlane(__hip_atomic_load(pub, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP));
    };
    const int jend = c0 + ncols - 1;  // steps 0..jend-1 touch this block
    if (c0 == 0 && wave == 0) {
      // column 0: pivoted before any step
      C<L> inv;
      double pk;
      int p0;
      reg_pivot<L, RPL>(A[0], act, 0, ring, ctl, inv, pk, p0);
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
      if (lane == 0) __hip_atomic_store(pub, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      publish_device(0, A[0], act, p0, inv, pk);
      retire_slot0();
    }
    bool hasdef = false;
    int pdef = 0;
    C<L> ldef[RPL];
#pragma unroll
    for (int u = 0; u < RPL; ++u) ldef[u] = czero<L>();
    auto apply = [&](const C<L> (&lm)[RPL], int ps) __attribute__((always_inline)) {
      apply_live<L, RPL, CPW>(A, live, lm, ps);
    };
    // the owner wavefront of column c in this block, or -1
    auto owner_of = [&](int c) { return (c >= c0 && c <= jend && c < n) ? (c - c0) % NW : -1; };
    for (int j = 0; j < jend; ++j) {
      const int j1 = j + 1;
      const bool owner = owner_of(j1) == wave;
      while (published() <= j)
        if (!owner) __builtin_amdgcn_s_sleep(1);
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
      const int2 cj = ctl[j];
      C<L> l[RPL];
#pragma unroll
      for (int u = 0; u < RPL; ++u) l[u] = pload<L>(ring + (j % KR) * E2 * RMAX + lane + 64 * u, RMAX);
      const int sgj = __builtin_amdgcn_readfirstlane(cj.y);
      const int p = __builtin_amdgcn_readfirstlane(cj.x);
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
      if (lane == 0) __hip_atomic_store(rd + wave, j + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      if (sgj != 0) {
        stop = true;
        break;
      }
      bool upd[RPL];  // rows this step updates
#pragma unroll
      for (int u = 0; u < RPL; ++u) {
        const int r = lane + 64 * u;
        if (r == p) mypos[u] = j;
        upd[u] = act[u] && r != p;
        l[u] = cselect<L>(upd[u], l[u], czero<L>());
      }
      if (owner) {
        __builtin_amdgcn_s_setprio(2);
        const int need = j1 - KR + 1;
        int rdl = lane < NW ? __hip_atomic_load(rd + lane, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) : need;
        const C<L> uv = reg_row<L, RPL>(A[0], p);
#pragma unroll
        for (int u = 0; u < RPL; ++u) A[0][u] = cfms<L>(A[0][u], l[u], uv);
        while (__ballot(rdl < need) != 0ull)
          rdl = lane < NW ? __hip_atomic_load(rd + lane, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) : need;
        C<L> inv;
        double pk;
        int pn;
        reg_pivot<L, RPL>(A[0], upd, j1, ring + (j1 % KR) * E2 * RMAX, ctl, inv, pk, pn);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        if (lane == 0) __hip_atomic_store(pub, j1 + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        __builtin_amdgcn_s_setprio(0);
        publish_device(j1, A[0], upd, pn, inv, pk);
        store_u(j1, A[0]);
        retire_slot0();
        if (hasdef) {
          apply(ldef, pdef);
          hasdef = false;
        }
        apply(l, p);
      } else if (j1 + 1 < n && owner_of(j1 + 1) == wave) {
        const C<L> uv = reg_row<L, RPL>(A[0], p);
#pragma unroll
        for (int u = 0; u < RPL; ++u) {
          A[0][u] = cfms<L>(A[0][u], l[u], uv);
          ldef[u] = l[u];
        }
        hasdef = true;
        pdef = p;
      } else {
        apply(l, p);
      }
#pragma unroll
      for (int u = 0; u < RPL; ++u) act[u] = upd[u];
    }
    // this wavefront's device stores before the block's flag
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  }
  __syncthreads();
  if (!last_wg) {
    if (tid == 0) __hip_atomic_store(gfin + g, s_late ? tag_fail : tag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return;
  }

  // ---- last block: every block's triangle, scaled into LDS; back substitution
  const bool bad = s_bad != 0;
  bool ok = !stop;
  int last = n - 1;
  {
    // the stopping step, as every column wavefront saw it (the owner of
    // column n took every step)
    __shared__ int s_stop;
    if (tid == 0) s_stop = -1;
    __syncthreads();
    if (stop && lane == 0) atomicMax(&s_stop, 0);
    __syncthreads();
    ok = s_stop < 0 && s_late == 0;
  }
  if (!ok) {
    // the first step with a nonzero flag in the ring's control array
    for (int j = 0; j < n; ++j)
      if (ctl[j].y != 0) {
        last = j;
        break;
      }
  }
  // the other blocks' flags, as the forwarding wavefront saw them (all
  // raised, or one failed or ran out of time)
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  if (!s_fins) {
    ok = false;
    last = 0;
    if (tid == 0) s_late = 1;
    __syncthreads();
  }
  if (ok) {
    // right-hand side (column n, slot 0 of its owner) in pivot order, scaled;
    // this block's own triangle columns scaled by the pivot inverses (the
    // earlier blocks' columns are in LDS already)
    if (wave == (n - c0) % NW)
#pragma unroll
      for (int u = 0; u < RPL; ++u)
        if (mypos[u] < n) pstore<L>(rhs + mypos[u], RMAX, cmul<L>(A[0][u], pload<L>(ginvp + mypos[u], RMAX)));
    if constexpr (TRI_LDS) {
      const int ntri = n * (n - 1) / 2;
      for (int q = (EARLY_GATHER ? c0 * (c0 - 1) / 2 : 0) + tid; q < ntri; q += 64 * (NW + 1)) gather_entry(q);
    }
  }
  __syncthreads();
  if (wave != 0) return;
  const bool late = s_late != 0;
  const bool badx = bad || late;
  if (badx) ok = false;

  double *const xpt = a.x ? a.x + b * n * E2 : nullptr;
  double *const dzp = a.dz ? a.dz + b * n * E2 : nullptr;
  double dmax = 0.0, xmax = 0.0;
  if (ok) {
    C<L> bb[RPL];
#pragma unroll
    for (int u = 0; u < RPL; ++u) {
      const int k = lane + 64 * u;
      bb[u] = k < n ? pload<L>(rhs + k, RMAX) : czero<L>();
    }
    if constexpr (TRI_LDS) {
      auto col_of = [&](int j) -> C<L> {
        return (j >= 1 && lane < j) ? pload<L>(ltri + (size_t)j * (j - 1) / 2 + lane, TT) : czero<L>();
      };
      C<L> ucur = col_of(n - 1);
      for (int j = n - 1; j > 0; --j) {
        const C<L> unext = col_of(j - 1);
        const C<L> xj = cbcast<L>(bb[0], j);
        bb[0] = cfms<L>(bb[0], ucur, xj);  // ucur is zero from row j on
        ucur = unext;
      }
    } else {
      // the triangle from device memory, scaled by this lane's pivot
      // inverses as it arrives (the same products as a scaled copy), the
      // next PF columns in flight
      constexpr int PF = 4;
      C<L> invk[RPL];
#pragma unroll
      for (int u = 0; u < RPL; ++u) {
        const int k = lane + 64 * u;
        invk[u] = k < n ? pload<L>(ginvp + k, RMAX) : czero<L>();
      }
      auto col_of = [&](int j, C<L>(&uc)[RPL]) __attribute__((always_inline)) {
#pragma unroll
        for (int u = 0; u < RPL; ++u) {
          const int k = lane + 64 * u;
          uc[u] = (j >= 1 && k < j) ? pload<L>(gtri + (size_t)j * (j - 1) / 2 + k, TT) : czero<L>();
        }
      };
      C<L> ring_u[PF][RPL];
#pragma unroll
      for (int q = 0; q < PF; ++q) col_of(n - 1 - q, ring_u[q]);
      for (int j0 = n - 1; j0 > 0; j0 -= PF) {
#pragma unroll
        for (int q = 0; q < PF; ++q) {
          const int j = j0 - q;
          if (j < 1) break;
          const C<L> xj = reg_row<L, RPL>(bb, j);
#pragma unroll
          for (int u = 0; u < RPL; ++u) {
            if (64 * u >= j) break;  // wave-uniform: no row of this slot is above j
            bb[u] = cfms<L>(bb[u], cmul<L>(ring_u[q][u], invk[u]), xj);  // zero from row j on
          }
          col_of(j - PF, ring_u[q]);
        }
      }
    }
#pragma unroll
    for (int u = 0; u < RPL; ++u) {
      const int k = lane + 64 * u;
      if (k < n) {
        if (dzp) cstore<L>(dzp + (size_t)k * E2, bb[u]);
        if (xpt) {
          double *xp = xpt + (size_t)k * E2;
          const C<L> xn = cadd<L>(cload<L>(xp), bb[u]);
          cstore<L>(xp, xn);
          xmax = fmax(xmax, cabs1_hi<L>(xn));
        }
        dmax = fmax(dmax, cabs1_hi<L>(bb[u]));
      }
    }
  }
  dmax = wave_max_f64(dmax);
  xmax = wave_max_f64(xmax);
  if (badx) last = 0;
  double pmx = 0.0, pmn = __builtin_inf();
  for (int j = lane; j <= last; j += 64) {
    pmx = fmax(pmx, gpmag[j]);
    pmn = fmin(pmn, gpmag[j]);
  }
  pmx = wave_max_f64(pmx);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) pmn = fmin(pmn, __shfl_xor(pmn, off, 64));
  if (lane == 0 && nst) newton_bookkeeping(nst, s_rho, !ok, badx, dmax, pmx, pmn, xmax);
}

}  // namespace qdp
