// Register-resident Gaussian elimination with partial pivoting and back
// substitution of one point's Newton system (Section 4, GE and Back_Subs;
// the solve of Algorithm 4.1), for systems whose augmented matrix fits in
// the vector registers of one workgroup.
//
// Layout: NW wavefronts; column c of [A | b] (n rows, n+1 columns, b = -h in
// column n) belongs to wavefront c mod NW, which keeps it in register slot
// c / NW; lane l holds rows l + 64u, u < RPL.  Step j of the elimination then
// needs from other wavefronts only the multipliers of column j (one LDS
// vector per step, double-buffered); the pivot row's entry of a column is in
// the owner's own lane and travels by lane reads, so the trailing update
// never touches LDS.  No barrier per column: the wavefronts meet through
// counters in LDS.
//   * The owner of column j+1 updates that column with column j's
//     multipliers as soon as they are published, chooses its pivot (largest
//     |Re|+|Im| of the leading limb, ties to the lowest row, with a DPP
//     wavefront maximum), forms the pivot's inverse and the multipliers and
//     publishes them into a ring of KRING multiplier vectors, then raises the
//     published-column counter.
//   * Every wavefront takes the steps in order: it waits until column j is
//     published, reads its multipliers, records that it has read them (a
//     counter per wavefront; a publisher waits until every wavefront has read
//     the ring entry it reuses), and updates its columns j+1..n.  The owner
//     of the next look-ahead column applies a step to that column alone and
//     the rest after its look-ahead, so its pivot work starts as early as
//     possible.
// The chain of pivot steps (one wavefront at a time) then overlaps the bulk
// update instead of waiting for the slowest wavefront at every column.
// Rows are never swapped: each lane keeps a flag for rows not yet used as a
// pivot row, and the pivot column of rows already used.
//
// A column is final once its pivot is chosen: its owner then retires it, at
// the start of the next step, by storing its U part (pivot rows, in pivot
// order) into a packed upper triangle in LDS (column k holds pivot-order rows
// 0..k-1) and shifting its remaining columns down one slot.  So a
// wavefront's live columns are always its slots 0..K-1, slot 0 is its next
// look-ahead column, and a step's update is one straight-line block over the
// live slots.  After the last column the triangle and the right-hand side
// are scaled by the pivot inverses (U(i,k)/U(i,i)); one wavefront then runs
// the back substitution column by column: the value x_j travels by lane reads
// and every lane above j applies one fused multiply-subtract, the next
// column's entries loaded one step ahead.
#pragma once
#include "ge_kernel.hpp"

namespace qdp {
using namespace mw;

// Shape of one instantiation: NW wavefronts, at most NMAX rows.
template <int NW, int NMAX> struct RegShape {
  static constexpr int NT = 64 * NW;
  static constexpr int RPL = (NMAX + 63) / 64;     // rows per lane
  static constexpr int RMAX = 64 * RPL;
  static constexpr int CPW = (NMAX + 1 + NW - 1) / NW;  // column slots per wavefront
};

// LDS of one register elimination (doubles; then ints):
//   mult [KRING][2L][RMAX] multipliers of the last KRING pivot columns
//   invp [2L][RMAX]     pivot inverses by column
//   rhs  [2L][RMAX]     scaled right-hand side, pivot order
//   pmag [RMAX]         |Re|+|Im| of each pivot's leading limb
//   misc [16]           residual, non-finite flag
//   tri  [2L][n(n-1)/2] scaled U, packed by columns
//   ctl  [RMAX] int2    pivot row of column j and its zero-pivot flag (read together)
//   sync [32] int       published-column counter, then columns read by each wavefront
constexpr int KRING = 8;
__host__ __device__ inline size_t ge_reg_tri_doubles(int n) { return n > 1 ? (size_t)n * (n - 1) / 2 : 1; }
__host__ __device__ inline size_t ge_reg_lds_doubles(int L, int RMAX, int n) {
  return (size_t)(KRING * 2 * L + 2 * L + 2 * L) * RMAX + RMAX + 16 + 2 * L * ge_reg_tri_doubles(n);
}
__host__ __device__ inline size_t ge_reg_lds_bytes(int L, int RMAX, int n) {
  return ge_reg_lds_doubles(L, RMAX, n) * sizeof(double) + (2 * (size_t)RMAX + 32) * sizeof(int);
}

// Entry of row `row` (wave-uniform) from a column held as RPL lane slots.
template <int L, int RPL> __device__ __forceinline__ C<L> reg_row(const C<L> (&v)[RPL], int row) {
  C<L> pv = v[0];
#pragma unroll
  for (int u = 1; u < RPL; ++u)
    if ((row >> 6) == u) pv = v[u];  // wave-uniform
  return cbcast<L>(pv, row & 63);
}

// Wavefront maximum of a nonnegative double, in every lane.
__device__ inline double wave_max_f64(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

// Maximum over a full wavefront of a 32-bit key, in lane 63 (read out as a
// scalar): butterflies inside each row of 16 lanes (lane xor 1, xor 2, the
// half-row mirror, the row mirror), then the row broadcasts of lanes 15 and
// 31 into the rows above.  A lane reading outside the wavefront or a row left
// out by the row mask sees 0, the identity of the maximum, so each level is
// one max instruction with the lane permutation on its operand.
template <int CTRL, int ROWS> __device__ inline unsigned dpp_umax(unsigned w) {
  return max(w, (unsigned)__builtin_amdgcn_update_dpp(0, (int)w, CTRL, ROWS, 0xf, true));
}
__device__ inline unsigned wave_umax32(unsigned w) {
  w = dpp_umax<0xB1, 0xf>(w);   // quad_perm [1,0,3,2]
  w = dpp_umax<0x4E, 0xf>(w);   // quad_perm [2,3,0,1]
  w = dpp_umax<0x141, 0xf>(w);  // row_half_mirror
  w = dpp_umax<0x140, 0xf>(w);  // row_mirror
  w = dpp_umax<0x142, 0xa>(w);  // row_bcast:15 into rows 1 and 3
  w = dpp_umax<0x143, 0xc>(w);  // row_bcast:31 into rows 2 and 3
  return (unsigned)__builtin_amdgcn_readlane((int)w, 63);
}

// Pivot key of a row for a 32-bit maximum: the high word of the FP64 key
// (sign, exponent, 20 mantissa bits; monotone for nonnegative doubles) with
// its low RB bits dropped, plus one, above the row index stored as RMAX-1-r
// (so equal keys go to the lowest row).  Keys within a relative 2^(RB-20) of
// each other tie, which partial pivoting tolerates.  0 = no candidate (not a
// candidate row, or a NaN key); key part 1 = a zero (or subnormal) entry.
template <int RB> __device__ inline unsigned pack_key32(double key, int row, bool cand) {
  const bool ok = cand && key == key && key >= 0.0;
  const unsigned hi = (unsigned)(__double_as_longlong(key) >> 32);
  return ok ? (((hi >> RB) + 1u) << RB) | (unsigned)((1 << RB) - 1 - row) : 0u;
}

// Pivot of a column held in registers among the rows `cand`: largest
// |Re|+|Im| of the leading limb (see pack_key32), then its inverse and the
// multipliers v_r / pivot, which replace the candidates' entries (the pivot
// row keeps its entry, the diagonal of U) and go to `mbuf`.  Every lane
// inverts its own entry while the maximum runs (one pass of the SIMD; the two
// chains are independent), so the pivot's inverse is one lane read.  Lane 0
// records the pivot row and zero-pivot flag (one 8-byte store); the inverse,
// the pivot's magnitude and its row are returned for the caller to record
// (after it has published the column).  Called by one whole wavefront.
template <int L, int RPL>
__device__ __forceinline__ void reg_pivot(C<L> (&v)[RPL], const bool (&cand)[RPL], int col, double *mbuf, int2 *ctl,
                                          C<L> &inv_out, double &pkey_out, int &p_out) {
  constexpr int RMAX = 64 * RPL;
  constexpr int RB = RPL == 1 ? 6 : (RPL == 2 ? 7 : 8);
  const int lane = threadIdx.x & 63;
  unsigned best = 0;
  double key[RPL];
  C<L> own_inv[RPL];
#pragma unroll
  for (int u = 0; u < RPL; ++u) {
    key[u] = cabs1_hi<L>(v[u]);
    best = max(best, pack_key32<RB>(key[u], lane + 64 * u, cand[u]));
    own_inv[u] = cinv<L>(v[u]);  // other lanes' values (zeros included) are unused
  }
  best = wave_umax32(best);
  const bool sg = (best >> RB) <= 1u;  // no candidate, or the largest entry is zero
  const int p = sg ? 0 : RMAX - 1 - (int)(best & (RMAX - 1));
  const C<L> inv = sg ? czero<L>() : reg_row<L, RPL>(own_inv, p);
  double pkey = key[0];
#pragma unroll
  for (int u = 1; u < RPL; ++u)
    if ((p >> 6) == u) pkey = key[u];  // wave-uniform
  pkey = sg ? 0.0 : rdlane(pkey, p & 63);
  if (!sg) {
#pragma unroll
    for (int u = 0; u < RPL; ++u) {
      const int r = lane + 64 * u;
      if (cand[u] && r != p) {
        const C<L> m = cmul<L>(v[u], inv);
        v[u] = m;
        pstore<L>(mbuf + r, RMAX, m);
      }
    }
  }
  if (lane == 0) ctl[col] = make_int2(p, sg ? 1 : 0);
  inv_out = inv;
  pkey_out = pkey;
  p_out = p;
}
// the pivot's inverse and magnitude into their LDS arrays (lane 0)
template <int L, int RMAX>
__device__ __forceinline__ void reg_record(int col, const C<L> &inv, double pkey, double *invp, double *pmag) {
  if ((threadIdx.x & 63) == 0) {
    pstore<L>(invp + col, RMAX, inv);
    pmag[col] = pkey;
  }
}

// The live slots 0..K-1 of a wavefront's columns updated with one step's
// multipliers lm (zero in rows the step leaves alone) and pivot row ps: one
// straight-line block per K, so the independent columns' products
// interleave.  No lane mask: a - 0 u is a exactly, so rows with a zero
// multiplier (pivot rows, the U part) keep their values bit for bit.
template <int L, int RPL, int CPW, int K>
__device__ __forceinline__ void apply_prefix(C<L> (&A)[CPW][RPL], const C<L> (&lm)[RPL], int ps) {
#pragma unroll
  for (int s = 0; s < K; ++s) {
    const C<L> uv = reg_row<L, RPL>(A[s], ps);
#pragma unroll
    for (int u = 0; u < RPL; ++u) A[s][u] = cfms<L>(A[s][u], lm[u], uv);
  }
}
template <int L, int RPL, int CPW, int K = CPW>
__device__ __forceinline__ void apply_live(C<L> (&A)[CPW][RPL], int live, const C<L> (&lm)[RPL], int ps) {
  if constexpr (K > 0) {
    if (live == K)
      apply_prefix<L, RPL, CPW, K>(A, lm, ps);
    else
      apply_live<L, RPL, CPW, K - 1>(A, live, lm, ps);
  }
}

// LDS arrays of the elimination loop (layout above).
struct RegElimLds {
  double *mult;  // [KRING][2L][RMAX] multiplier ring
  double *invp;  // [2L][RMAX]
  double *pmag;  // [RMAX]
  int2 *ctl;     // [RMAX]
  int *pub;      // columns published
  int *rd;       // [NW] columns read by each wavefront
};

// The elimination of [A | b] held in registers (column wave + NW s in slot
// s, rows lane + 64 u), called by every thread of the workgroup: wavefront 0
// pivots column 0, one barrier (after it, *badflag != 0 stops the
// elimination before any step), then the steps as described at the top of
// this file.  retire(c, col, inv, p, pos) receives each column c < n in the
// registers of its owner once its pivot (row p, inverse inv) is chosen, with
// pos[u] the pivot step of row lane + 64u for the steps before c (n for rows
// not yet pivot rows); the column then leaves the slots.  On return
// mypos[u] = pivot step of row lane + 64u (n for none), column n is in
// slot 0 of its owner, and invp/pmag/ctl hold the columns examined (the
// published counter says how many).  Returns false if a column had no
// nonzero pivot (or *badflag was set).
template <int L, int NW, int NMAX, int CPW, int RPL, class Retire>
__device__ __forceinline__ bool reg_eliminate(C<L> (&A)[CPW][RPL], int (&mypos_out)[RPL], int n,
                                              const double *badflag, const RegElimLds &m, Retire &&retire) {
  using S = RegShape<NW, NMAX>;
  static_assert(CPW == S::CPW && RPL == S::RPL, "register array of this shape");
  constexpr int RMAX = S::RMAX, E2 = 2 * L;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // kept local and copied out at the end: held through the caller's
  // reference, the compiler allocated the loop ~10 more registers and the
  // n = 64 double-double elimination ran 10% slower (measured)
  int mypos[RPL];
  bool act[RPL];  // row not yet a pivot row
#pragma unroll
  for (int u = 0; u < RPL; ++u) {
    act[u] = lane + 64 * u < n;
    mypos[u] = n;
  }
  int live = wave <= n ? (n - wave) / NW + 1 : 0;  // columns this wavefront still holds
  // retire slot 0 (column c, final): handed to the caller, the other slots
  // shift down
  auto retire_slot0 = [&](int c, const C<L> &inv, int p) __attribute__((always_inline)) {
    retire(c, A[0], inv, p, mypos);
#pragma unroll
    for (int s = 0; s + 1 < CPW; ++s)
#pragma unroll
      for (int u = 0; u < RPL; ++u) A[s][u] = A[s + 1][u];
#pragma unroll
    for (int u = 0; u < RPL; ++u) A[CPW - 1][u] = czero<L>();
    --live;
  };
  // ---- pivot of column 0 (wave 0, slot 0), retired at once (a later stop
  // discards it)
  if (wave == 0) {
    C<L> inv0;
    double pk;
    int p0;
    reg_pivot<L, RPL>(A[0], act, 0, m.mult, m.ctl, inv0, pk, p0);
    reg_record<L, RMAX>(0, inv0, pk, m.invp, m.pmag);
    retire_slot0(0, inv0, p0);
  }
  if (tid < NW) m.rd[tid] = 0;
  if (tid == 0) *m.pub = 1;
  __syncthreads();

  // ---- elimination: step j applies column j's multipliers to columns j+1..n
  auto published = [&]() {
    return __builtin_amdgcn_readfirstlane(__hip_atomic_load(m.pub, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP));
  };
  bool stop = *badflag != 0.0;
  bool hasdef = false;  // step deferred on the slots past slot 0 (next look-ahead owner)
  int pdef = 0;
  C<L> ldef[RPL];
#pragma unroll
  for (int u = 0; u < RPL; ++u) ldef[u] = czero<L>();
  auto apply = [&](const C<L> (&lm)[RPL], int ps) __attribute__((always_inline)) {
    apply_live<L, RPL, CPW>(A, live, lm, ps);
  };
  for (int j = 0; j + 1 < n && !stop; ++j) {
    // wait for column j, read its pivot row, flag and multipliers (every row;
    // rows this step leaves alone are zeroed below), record the read
    const int j1 = j + 1;
    const bool owner = wave == j1 % NW;  // runs the look-ahead of column j+1: polls without sleeping
    while (published() <= j)
      if (!owner) __builtin_amdgcn_s_sleep(1);
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    const int2 cj = m.ctl[j];
    const double *const mj = m.mult + (j % KRING) * E2 * RMAX;
    C<L> l[RPL];
#pragma unroll
    for (int u = 0; u < RPL; ++u) l[u] = pload<L>(mj + lane + 64 * u, RMAX);
    const int sgj = __builtin_amdgcn_readfirstlane(cj.y);
    const int p = __builtin_amdgcn_readfirstlane(cj.x);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");  // the reads above have completed
    if (lane == 0) __hip_atomic_store(m.rd + wave, j + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    if (sgj != 0) {  // column j has no nonzero pivot
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
      // look-ahead: column j+1 (slot 0, steps 0..j-1 applied) updated by
      // step j, its pivot and multipliers published, the column retired;
      // then the steps this wavefront still owes its other columns
      __builtin_amdgcn_s_setprio(2);
      // the ring entry this column reuses must have been read by every
      // wavefront: the counters are loaded before the product, checked after
      const int need = j1 - KRING + 1;
      int rdl = lane < NW ? __hip_atomic_load(m.rd + lane, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) : need;
      const C<L> uv = reg_row<L, RPL>(A[0], p);
#pragma unroll
      for (int u = 0; u < RPL; ++u) A[0][u] = cfms<L>(A[0][u], l[u], uv);
      while (__ballot(rdl < need) != 0ull)
        rdl = lane < NW ? __hip_atomic_load(m.rd + lane, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) : need;
      C<L> inv;
      double pk;
      int pn;
      reg_pivot<L, RPL>(A[0], upd, j1, m.mult + (j1 % KRING) * E2 * RMAX, m.ctl, inv, pk, pn);
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");  // multipliers and flags before the counter
      if (lane == 0) __hip_atomic_store(m.pub, j1 + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      __builtin_amdgcn_s_setprio(0);
      reg_record<L, RMAX>(j1, inv, pk, m.invp, m.pmag);
      retire_slot0(j1, inv, pn);
      if (hasdef) {
        apply(ldef, pdef);
        hasdef = false;
      }
      apply(l, p);
    } else if (j1 + 1 < n && wave == (j1 + 1) % NW) {
      // next look-ahead owner: this step on its look-ahead column only; the
      // other columns get it after that look-ahead
      const C<L> uv = reg_row<L, RPL>(A[0], p);
#pragma unroll
      for (int u = 0; u < RPL; ++u) A[0][u] = cfms<L>(A[0][u], l[u], uv);
      hasdef = true;
      pdef = p;
#pragma unroll
      for (int u = 0; u < RPL; ++u) ldef[u] = l[u];
    } else {
      apply(l, p);  // every live column is j+2..n
    }
#pragma unroll
    for (int u = 0; u < RPL; ++u) act[u] = upd[u];
  }
  if (!stop) {
    // the last pivot column's flag (published by the last look-ahead; for
    // n = 1, column 0)
    while (published() < n) __builtin_amdgcn_s_sleep(1);
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    const int2 cl = m.ctl[n - 1];
    stop = __builtin_amdgcn_readfirstlane(cl.y) != 0;
    const int pl = __builtin_amdgcn_readfirstlane(cl.x);
#pragma unroll
    for (int u = 0; u < RPL; ++u)
      if (lane + 64 * u == pl) mypos[u] = n - 1;
  }
#pragma unroll
  for (int u = 0; u < RPL; ++u) mypos_out[u] = mypos[u];
  return !stop;
}

// NW / 4 wavefronts share a SIMD: the compiler may use that SIMD's whole
// register file instead of spilling to reach a higher occupancy nothing uses
template <int L, int NW, int NMAX>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu((NW + 3) / 4, (NW + 3) / 4)))
void k_ge_reg(GeArgs<L> a) {
  using S = RegShape<NW, NMAX>;
  constexpr int RPL = S::RPL, RMAX = S::RMAX, CPW = S::CPW, E2 = 2 * L;
  const int n = a.n;
  const size_t b = blockIdx.x;
  NewtonState *const nst = a.st ? a.st + b : nullptr;
  if (nst && !nst->active) return;
  const size_t PS = (size_t)n * (n + 1);
  const double *const ab = a.ab + b * E2 * PS;
  const double *const scale = a.scale ? a.scale + b * n : nullptr;
  double *const xpt = a.x ? a.x + b * n * E2 : nullptr;
  double *const dzp = a.dz ? a.dz + b * n * E2 : nullptr;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

  extern __shared__ double smem[];
  double *const mult = smem;
  double *const invp = mult + KRING * E2 * RMAX;
  double *const rhs = invp + E2 * RMAX;
  double *const pmag = rhs + E2 * RMAX;
  double *const misc = pmag + RMAX;
  double *const tri = misc + 16;
  const size_t TS = ge_reg_tri_doubles(n);
  int2 *const ctl = reinterpret_cast<int2 *>(tri + E2 * TS);
  int *const pub = reinterpret_cast<int *>(ctl + RMAX);  // columns published
  int *const rd = pub + 1;                               // [NW] columns read by each wavefront

  // ---- the matrix into registers: column wave + NW s, rows lane + 64 u
  C<L> A[CPW][RPL];
#pragma unroll
  for (int s = 0; s < CPW; ++s) {
    const int c = wave + NW * s;
#pragma unroll
    for (int u = 0; u < RPL; ++u) {
      const int r = lane + 64 * u;
      A[s][u] = (c <= n && r < n) ? pload<L>(ab + (size_t)c * n + r, PS) : czero<L>();
    }
  }
  // ---- residual of h (the right-hand side column, before elimination) by its owner
  if (wave == n % NW) {
    double hb = 0.0, sb = 0.0;
    bool fin = true;
#pragma unroll
    for (int s = 0; s < CPW; ++s)
      if (s == n / NW) {
#pragma unroll
        for (int u = 0; u < RPL; ++u)
          if (lane + 64 * u < n) {
            hb = fmax(hb, cabs1_hi<L>(A[s][u]));
            fin = fin && cfinite<L>(A[s][u]);
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
  // ---- elimination; each finished column's U part (pivot rows, pivot
  // order mypos < c) goes into the packed triangle
  int mypos[RPL];  // pivot column of row lane + 64u (n while not yet a pivot row)
  const RegElimLds lds{mult, invp, pmag, ctl, pub, rd};
  const bool ok = reg_eliminate<L, NW, NMAX>(A, mypos, n, misc + 1, lds,
                                             [&](int c, const C<L>(&col)[RPL], const C<L> &, int, const int(&pos)[RPL])
                                                 __attribute__((always_inline)) {
#pragma unroll
                                               for (int u = 0; u < RPL; ++u)
                                                 if (pos[u] < c)
                                                   pstore<L>(tri + (size_t)c * (c - 1) / 2 + pos[u], TS, col[u]);
                                             });
  const bool bad = misc[1] != 0.0;

  // ---- right-hand side (column n, slot 0 of its owner) in pivot order, then
  // the triangle and the right-hand side scaled by the pivot inverses
  if (ok && wave == n % NW) {
#pragma unroll
    for (int u = 0; u < RPL; ++u)
      if (mypos[u] < n) pstore<L>(rhs + mypos[u], RMAX, A[0][u]);
  }
  __syncthreads();
  if (ok) {
    const int ntri = n * (n - 1) / 2;
    for (int q = tid; q < ntri + n; q += S::NT) {
      int i, c;
      double *e;
      if (q < ntri) {
        // q = c (c - 1) / 2 + i, 0 <= i < c
        c = (int)((1.0 + sqrt(1.0 + 8.0 * q)) * 0.5);
        while (c * (c - 1) / 2 > q) --c;
        while ((c + 1) * c / 2 <= q) ++c;
        i = q - c * (c - 1) / 2;
        e = tri + q;
      } else {
        i = q - ntri;
        e = rhs + i;
      }
      const size_t st = q < ntri ? TS : (size_t)RMAX;
      pstore<L>(e, st, cmul<L>(pload<L>(e, st), pload<L>(invp + i, RMAX)));
    }
  }
  __syncthreads();
  if (wave != 0) return;

  // ---- back substitution (wavefront 0): x_j = y_j - sum_{k > j} U'(j, k) x_k
  double dmax = 0.0, xmax = 0.0;
  if (ok) {
    C<L> bb[RPL];
#pragma unroll
    for (int u = 0; u < RPL; ++u) {
      const int i = lane + 64 * u;
      bb[u] = i < n ? pload<L>(rhs + i, RMAX) : czero<L>();
    }
    auto col_of = [&](int j, C<L> (&uc)[RPL]) {
#pragma unroll
      for (int u = 0; u < RPL; ++u) {
        const int i = lane + 64 * u;
        uc[u] = i < j ? pload<L>(tri + (size_t)j * (j - 1) / 2 + i, TS) : czero<L>();
      }
    };
    C<L> ucur[RPL];
    col_of(n - 1, ucur);
    for (int j = n - 1; j > 0; --j) {
      C<L> unext[RPL];
      col_of(j - 1, unext);
      const C<L> xj = reg_row<L, RPL>(bb, j);
#pragma unroll
      for (int u = 0; u < RPL; ++u) {
        if (64 * u >= j) break;  // wave-uniform: no row of this slot is above j
        bb[u] = cfms<L>(bb[u], ucur[u], xj);  // ucur is zero from row j on
      }
#pragma unroll
      for (int u = 0; u < RPL; ++u) ucur[u] = unext[u];
    }
    // bb at pivot-order index i is the correction of variable i
#pragma unroll
    for (int u = 0; u < RPL; ++u) {
      const int v = lane + 64 * u;
      if (v < n) {
        const C<L> d = bb[u];
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
  }
  dmax = wave_max_f64(dmax);
  xmax = wave_max_f64(xmax);
  // pivot magnitudes of the columns examined
  const int last = *pub - 1;
  double pmx = 0.0, pmn = __builtin_inf();
  for (int j = lane; j <= last; j += 64) {
    pmx = fmax(pmx, pmag[j]);
    pmn = fmin(pmn, pmag[j]);
  }
  pmx = wave_max_f64(pmx);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) pmn = fmin(pmn, __shfl_xor(pmn, off, 64));
  if (lane == 0 && nst) newton_bookkeeping(nst, misc[0], !ok, bad, dmax, pmx, pmn, xmax);
}

}  // namespace qdp
