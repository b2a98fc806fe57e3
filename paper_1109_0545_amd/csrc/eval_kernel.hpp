// Evaluation of a sparse polynomial system and its full Jacobian, fused with
// the total-degree homotopy blend.
//
// What is computed is the array Y of Section 4 (every polynomial value and
// every partial derivative); how each monomial is differentiated follows the
// reverse-mode (Speelpenning) products of Section 6: with g_v = x_v^(a_v) the
// factor of variable v, the partial of c * prod_v g_v with respect to x_v is
//     c * (product of the factors before v) * (product of the factors after v)
//       * a_v x_v^(a_v - 1),
// for any fixed order of the variables.  Powers x_v^e and e x_v^(e-1) come
// from a table built once per evaluation in LDS (the common factor x^(a-1) of
// Section 6 folded into the table), so each variable of a monomial costs four
// complex products, as the paper's scheme.
//
// Mapping on CDNA4: one workgroup per polynomial, or, when that leaves the
// chip idle, the monomials of a polynomial split over up to eight
// workgroups that store partial rows, added in part order by a second small
// kernel (see EvalSplit); blockIdx.y selects the point of a batch.  A monomial is spread over
// LM lanes of a wavefront and lane g owns the CH variables g, g+LM, g+2LM, ...
// (interleaved, so that neighbouring lanes read neighbouring table entries).
// The order used for the prefix/suffix products is lane-major: a lane first
// forms the suffix products of its own variables, the LM lanes then combine
// their chunk products by a butterfly of wavefront shuffles into the product
// over the other lanes, and each lane walks its variables forward once.  A lane keeps
// the running sums of its CH Jacobian entries in registers over all the
// monomials it visits; the per-polynomial reduction is a fixed-order shuffle
// butterfly then a fixed-order LDS sum across wavefronts (no atomics: results
// are bit-reproducible).  Tables and the reduction buffer are stored as limb
// planes so that a wavefront's LDS accesses hit consecutive banks.
#pragma once
#include "common.hpp"

namespace qdp {
using namespace mw;

template <int L> struct EvalArgs {
  DevSystem s;
  const double *x;  // [B][n][2][L] at the compute precision, points bx doubles apart
  long bx;
  HomArgs h;
  EvalOut o;
  const NewtonState *gate;  // [B] or nullptr
  int P;                    // workgroups per polynomial
  double *part;             // P > 1: partial rows [B][n][P] records (part_record)
};

// doubles of one partial-row record: n+1 complex values, then the scale sum
__host__ __device__ inline size_t part_record(int n, int L) { return (size_t)(n + 1) * 2 * L + 1; }
__host__ __device__ inline size_t part_scale_at(int n, int L) { return (size_t)(n + 1) * 2 * L; }
// doubles per point of a split evaluation with P parts: the n x P partial
// records, then the start-system powers (x_i^(d_i - 1), x_i^(d_i)) of every row
__host__ __device__ inline size_t part_point_doubles(int n, int L, int P) {
  return (size_t)n * P * part_record(n, L) + (size_t)4 * L * n;
}

// Start-system powers of row i: pd1 = x_i^(d-1), pd = x_i^d by binary
// powering in working precision (relative error about d units of the last
// place); d = 0 gives pd1 = 0, pd = 1.
template <int L> __device__ void start_powers(const double *xi_p, int d, C<L> &pd1, C<L> &pd) {
  const C<L> xi = cload<L>(xi_p);
  if (d >= 1) {
    pd1 = cpow<L>(xi, d - 1);
    pd = cmul<L>(pd1, xi);
  } else {
    pd1 = czero<L>();
    pd = cone<L>();
  }
}

// Homotopy blend and store of column col of row i of point b: s is the sum
// over the monomials of f_i (col < n: the partial with respect to x_col;
// col = n: the value, S its componentwise scale sum); pd1, pd the start-system
// powers of row i (start_powers).
template <int L>
__device__ void eval_finish(const EvalArgs<L> &a, int b, int i, int col, C<L> s, double S, const C<L> &pd1,
                            const C<L> &pd) {
  const int n = a.s.n;
  const double t = a.h.tb ? a.h.tb[b] : a.h.t;
  if (col < n) {
    C<L> Jv = s;
    if (a.h.homotopy) {
      Jv = cmul_d<L>(s, t);
      if (col == i) {
        const C<L> g = cload<L>(a.h.gamma);
        double e1;
        R<L> omt = rzero<L>();
        omt.v[0] = two_sum(1.0, -t, e1);
        if (L > 1) omt.v[1] = e1;
        const C<L> w = cmul_r<L>(g, omt);
        const int d = a.s.deg[i];
        if (d >= 1) Jv = cadd<L>(Jv, cmul<L>(w, cmul_d<L>(pd1, (double)d)));
      }
    }
    pstore<L>(a.o.J + (size_t)b * a.o.bJ + (size_t)i * a.o.rsJ + (size_t)col * a.o.csJ, a.o.psJ, Jv);
  } else {
    C<L> hv = s;
    if (a.h.homotopy) {
      const C<L> g = cload<L>(a.h.gamma);
      double e1;
      R<L> omt = rzero<L>();
      omt.v[0] = two_sum(1.0, -t, e1);
      if (L > 1) omt.v[1] = e1;
      const C<L> w = cmul_r<L>(g, omt);
      C<L> gm = pd;
      gm.re = rsub<L>(gm.re, rfrom<L>(1.0));
      hv = cadd<L>(cmul_d<L>(s, t), cmul<L>(w, gm));
      S = fabs(t) * S + cabs_hi<L>(w) * (cabs_hi<L>(pd) + 1.0);
    }
    if (a.o.ysign < 0) hv = cneg<L>(hv);
    pstore<L>(a.o.y + (size_t)b * a.o.by + (size_t)i * a.o.sy, a.o.psy, hv);
    if (a.o.scale) a.o.scale[(size_t)b * a.o.bS + i] = S;
  }
}

// Second stage of a split evaluation: row i of point b is the sum of its P
// partial rows in part order, then blended (with the start-system powers the
// first stage's extra workgroup formed) and stored.
// Row of workgroup slot s < n.  Workgroups go to the eight XCDs in turn (slot
// s to XCD s mod 8), and each XCD has its own L2; with n a multiple of 8 the
// rows are dealt so that the XCD of slot s holds the n/8 consecutive rows
// (s mod 8) n/8 ..: the rows that share a cache line of a column of [A | -h]
// are then written through one L2, which merges them into whole lines, and
// the parts of a split row (slot part n + s) share the XCD of its sum.
__device__ inline int eval_row_of_slot(int s, int n) {
  if (n & 7) return s;
  const int R = n >> 3;
  return (s & 7) * R + (s >> 3);
}

template <int L>
__global__ __launch_bounds__(256) void k_eval_sum(EvalArgs<L> a) {
  const int b = blockIdx.y, i = eval_row_of_slot(blockIdx.x, a.s.n);
  if (a.gate && !a.gate[b].active) return;
  const int n = a.s.n;
  const size_t rec = part_record(n, L);
  const double *pt = a.part + (size_t)b * part_point_doubles(n, L, a.P);
  const double *rows = pt + (size_t)i * a.P * rec;
  // the start-system powers, formed by k_eval's extra workgroup
  C<L> pd1 = czero<L>(), pd = cone<L>();
  if (a.h.homotopy) {
    const double *pw = pt + (size_t)n * a.P * rec + (size_t)i * 4 * L;
    pd1 = cload<L>(pw);
    pd = cload<L>(pw + 2 * L);
  }
  for (int col = threadIdx.x; col <= n; col += 256) {
    // every load first (the parts are independent), then the fixed-order sum
    C<L> v[kMaxEvalParts];
#pragma unroll
    for (int p = 0; p < kMaxEvalParts; ++p)
      v[p] = p < a.P ? cload<L>(rows + (size_t)p * rec + (size_t)col * 2 * L) : czero<L>();
    C<L> s = v[0];
#pragma unroll
    for (int p = 1; p < kMaxEvalParts; ++p)
      if (p < a.P) s = cadd<L>(s, v[p]);
    double S = 0.0;
    if (col == n)
      for (int p = 0; p < a.P; ++p) S += rows[(size_t)p * rec + part_scale_at(n, L)];
    eval_finish<L>(a, b, i, col, s, S, pd1, pd);
  }
}

// row stride (doubles) of a table plane: a multiple of 32 so that lanes with
// consecutive variables read consecutive banks whatever their exponents
__host__ __device__ inline int table_stride(int n) { return (n + 31) & ~31; }

// Power tables of one point in LDS, by threads tid = start, start + step, ...:
// Gt[e][v] = x_v^e and Qt[e][v] = e x_v^(e-1) for e <= E1 - 1 (limb planes
// tps apart, rows nv apart).  The derivative table folds the common factor
// x^(a-1) of Section 6 into a lookup.
template <int L>
__device__ void power_tables(const double *x, int n, int E1, int nv, size_t tps, double *Gt, double *Qt, int start,
                             int step) {
  for (int v = start; v < n; v += step) {
    const C<L> xv = cload<L>(x + (size_t)v * 2 * L);
    C<L> p = cone<L>();
    pstore<L>(Gt + v, tps, p);
    pstore<L>(Qt + v, tps, czero<L>());
    for (int e = 1; e < E1; ++e) {
      pstore<L>(Qt + (size_t)e * nv + v, tps, cmul_d<L>(p, (double)e));
      p = cmul<L>(p, xv);
      pstore<L>(Gt + (size_t)e * nv + v, tps, p);
    }
  }
}

// Speelpenning's products for one monomial c x^a spread over LM lanes of a
// wavefront, lane gl owning the variables gl + k LM (k < CH, exponents ex[k]):
// emit(k, d) receives d = c * (partial of x^a with respect to that variable)
// for each of the lane's variables; the return value is c x^a (in every lane
// of the group).  gval(v, e) / qval(v, e) read x_v^e and e x_v^(e-1) (one and
// zero past the last variable).  UNIT: c = 1, its product is not formed.
//
// Each lane forms the suffix products of its own variables (the last one is
// one and is not formed); the LM lanes combine their chunk products by a
// butterfly of xor shuffles: after the exchange at distance d a lane holds
// the product over its aligned block of 2d lanes (blk) and that product
// without its own chunk (others); the lane then walks its variables forward
// from c * others.  Four complex products per variable, as in Section 6.
template <int L, int CH, int LM, bool UNIT, class GV, class QV, class Emit>
__device__ __forceinline__ C<L> monomial_walk(const int (&ex)[CH], const C<L> &coef, int gl, GV gval, QV qval,
                                              Emit emit) {
  C<L> sfx[CH];
  C<L> chunk = gval(gl + (CH - 1) * LM, ex[CH - 1]);
  if constexpr (CH > 1) {
    sfx[CH - 2] = chunk;
#pragma unroll
    for (int k = CH - 3; k >= 0; --k) sfx[k] = cmul<L>(sfx[k + 1], gval(gl + (k + 1) * LM, ex[k + 1]));
    chunk = cmul<L>(sfx[0], gval(gl, ex[0]));
  }
  C<L> run = UNIT ? cone<L>() : coef;
  if constexpr (LM > 1) {
    C<L> blk = chunk, others = cshfl_xor<L>(chunk, 1, LM);
    blk = cmul<L>(blk, others);
#pragma unroll
    for (int d = 2; d < LM; d <<= 1) {
      const C<L> p = cshfl_xor<L>(blk, d, LM);
      others = cmul<L>(others, p);
      blk = cmul<L>(blk, p);
    }
    run = UNIT ? others : cmul<L>(run, others);
  }
  // run = c * (all factors before v) * (all factors of the other lanes)
#pragma unroll
  for (int k = 0; k < CH; ++k) {
    const int v = gl + k * LM;
    const C<L> d = k < CH - 1 ? cmul<L>(cmul<L>(run, sfx[k]), qval(v, ex[k])) : cmul<L>(run, qval(v, ex[k]));
    emit(k, d);
    run = cmul<L>(run, gval(v, ex[k]));
  }
  return run;
}

// NT threads work on monomials.  With one part per polynomial (P = 1, the
// batched case) thread 0 forms the start-system powers in the workgroup's
// tail: a chain of dependent products that the other workgroups sharing the
// compute unit cover (an extra wavefront for it cost a workgroup slot per CU:
// measured 33% slower at 256 points); a split evaluation (few points, many
// parts per polynomial) gets one extra workgroup per point that forms them for
// every row while the parts run (in k_eval_sum they were a serial tail; one
// evaluation at n = 64 measured 22.3 -> 18.8 us in double double, 89.5 -> 79.7
// us in quad double).  The register budget
// is that of NT + 64 threads (five wavefronts), which keeps three
// four-wavefront workgroups per CU.
template <int L, int CH, int LM, int NT>
__global__ __launch_bounds__(NT + 64) void k_eval(EvalArgs<L> a) {
  constexpr int G = 64 / LM;  // monomials per wavefront at a time
  constexpr int W = NT / 64;  // wavefronts on monomials
  constexpr int SLOTS = W * G;
  const int b = blockIdx.y;
  if (a.gate && !a.gate[b].active) return;
  const double *x = a.x + (size_t)b * a.bx;
  const int n = a.s.n;
  if (a.P > 1 && (int)blockIdx.x == n * a.P) {
    // split evaluation: the extra workgroup of a point forms the start-system
    // powers of every row (a chain of ~2 log2 d products per row) while the
    // parts run, for k_eval_sum
    if (a.h.homotopy) {
      double *pw = a.part + (size_t)b * part_point_doubles(n, L, a.P) + (size_t)n * a.P * part_record(n, L);
      for (int r = threadIdx.x; r < n; r += NT) {
        C<L> q1, q;
        start_powers<L>(x + (size_t)r * 2 * L, a.s.deg[r], q1, q);
        cstore<L>(pw + (size_t)r * 4 * L, q1);
        cstore<L>(pw + (size_t)r * 4 * L + 2 * L, q);
      }
    }
    return;
  }

  extern __shared__ double smem[];
  const int E1 = a.s.emax + 1;
  const int nv = table_stride(n);
  const size_t tps = (size_t)E1 * nv;  // plane size of one table
  double *Gt = smem;                   // x_v^e          plane c at Gt + c*tps + e*nv + v
  double *Qt = smem + 2 * L * tps;     // e x_v^(e-1)
  const int tid = threadIdx.x;
  __shared__ double powbuf[4 * L];

  // ---- power tables
  for (int v = tid; v < n; v += NT) {
    const C<L> xv = cload<L>(x + (size_t)v * 2 * L);
    C<L> p = cone<L>();
    pstore<L>(Gt + v, tps, p);
    pstore<L>(Qt + v, tps, czero<L>());
    for (int e = 1; e < E1; ++e) {
      pstore<L>(Qt + (size_t)e * nv + v, tps, cmul_d<L>(p, (double)e));
      p = cmul<L>(p, xv);
      pstore<L>(Gt + (size_t)e * nv + v, tps, p);
    }
  }
  __syncthreads();

  // part-major slots: part p of row i in slot p n + s(i), on the XCD of row i's sum
  const int part = blockIdx.x / n, i = eval_row_of_slot(blockIdx.x - part * n, n);
  const int m0 = a.s.offsets[i], m1 = a.s.offsets[i + 1];
  const int chunk = (m1 - m0 + a.P - 1) / a.P;
  const int t0 = min(m1, m0 + part * chunk), t1 = min(m1, t0 + chunk);
  const int lane = tid & 63, wave = tid >> 6;
  const int grp = lane / LM, gl = lane % LM;
  const int slot = wave * G + grp;
  const int LS = a.s.LS;

  C<L> acc[CH];
#pragma unroll
  for (int k = 0; k < CH; ++k) acc[k] = czero<L>();
  C<L> accv = czero<L>();
  double accS = 0.0;

  // table offsets e * nv + v with a 24-bit multiply (e <= 255, nv < 2^16)
  auto gval = [&](int v, int e) -> C<L> { return v < n ? pload<L>(Gt + __umul24(e, nv) + v, tps) : cone<L>(); };
  auto qval = [&](int v, int e) -> C<L> { return v < n ? pload<L>(Qt + __umul24(e, nv) + v, tps) : czero<L>(); };

  for (int base = t0; base < t1; base += SLOTS) {
    const int j = base + slot;
    const bool valid = j < t1;
    const int jj = valid ? j : t0;
    const uint8_t *er = a.s.exps + (size_t)jj * a.s.npad + gl;
    int ex[CH];
#pragma unroll
    for (int k = 0; k < CH; ++k) ex[k] = er[k * LM];
    const C<L> coef = cload_trunc<L>(a.s.coefs + (size_t)jj * 2 * LS, LS);

    // the walk of monomial_walk written out here: through the shared function
    // the compiler scheduled this kernel 3-10% slower (measured)
    // suffix products of this lane's variables (exclusive; sfx[CH-1] = 1 is
    // never formed), and the product of all of them
    C<L> sfx[CH];
    C<L> chunk = gval(gl + (CH - 1) * LM, ex[CH - 1]);
    if constexpr (CH > 1) {
      sfx[CH - 2] = chunk;
#pragma unroll
      for (int k = CH - 3; k >= 0; --k) sfx[k] = cmul<L>(sfx[k + 1], gval(gl + (k + 1) * LM, ex[k + 1]));
      chunk = cmul<L>(sfx[0], gval(gl, ex[0]));
    }

    // product of the other LM - 1 lanes' chunk products by a butterfly: after
    // the exchange at distance d a lane holds the product over its aligned
    // block of 2d lanes (blk) and that product without its own chunk (others)
    C<L> run = coef;
    if constexpr (LM > 1) {
      C<L> blk = chunk, others = cshfl_xor<L>(chunk, 1, LM);
      blk = cmul<L>(blk, others);
#pragma unroll
      for (int d = 2; d < LM; d <<= 1) {
        const C<L> p = cshfl_xor<L>(blk, d, LM);
        others = cmul<L>(others, p);
        blk = cmul<L>(blk, p);
      }
      run = cmul<L>(run, others);
    }

    // walk this lane's variables: run = c * (all factors before v)
    //                                   * (all factors of the other lanes)
#pragma unroll
    for (int k = 0; k < CH; ++k) {
      const int v = gl + k * LM;
      const C<L> d = k < CH - 1 ? cmul<L>(cmul<L>(run, sfx[k]), qval(v, ex[k])) : cmul<L>(run, qval(v, ex[k]));
      if (valid) acc[k] = cadd<L>(acc[k], d);
      run = cmul<L>(run, gval(v, ex[k]));
    }
    // lane 0 of the group now holds c * x^a (the monomial value)
    if (valid && gl == 0) {
      accv = cadd<L>(accv, run);
      accS += cabs_hi<L>(run);
    }
  }

  // ---- reduction over the monomial groups of a wavefront (fixed butterfly)
#pragma unroll
  for (int off = LM; off < 64; off <<= 1) {
#pragma unroll
    for (int k = 0; k < CH; ++k) acc[k] = cadd<L>(acc[k], cshfl_xor<L>(acc[k], off, 64));
    accv = cadd<L>(accv, cshfl_xor<L>(accv, off, 64));
    accS += __shfl_xor(accS, off, 64);
  }
  __syncthreads();  // tables no longer needed: reuse LDS for the cross-wave sum
  const int rn = n + 1;
  const size_t rps = (size_t)W * rn;  // plane size of the reduction buffer [W][n+1]
  double *red = smem;
  double *redS = smem + 2 * L * rps;
  if (lane < LM) {
#pragma unroll
    for (int k = 0; k < CH; ++k) {
      const int v = gl + k * LM;
      if (v < n) pstore<L>(red + (size_t)wave * rn + v, rps, acc[k]);
    }
    if (lane == 0) {
      pstore<L>(red + (size_t)wave * rn + n, rps, accv);
      redS[wave] = accS;
    }
  }
  __syncthreads();

  // ---- fixed-order sum over wavefronts; one part: blend and store; several
  // parts: store this part's row for k_eval_sum
  if (a.P == 1) {
    if (tid == 0 && a.h.homotopy) {
      C<L> q1, q;
      start_powers<L>(x + (size_t)i * 2 * L, a.s.deg[i], q1, q);
      cstore<L>(powbuf, q1);
      cstore<L>(powbuf + 2 * L, q);
    }
    __syncthreads();  // a.P is the same in every thread
    C<L> pd1 = czero<L>(), pd = cone<L>();
    if (a.h.homotopy) {
      pd1 = cload<L>(powbuf);
      pd = cload<L>(powbuf + 2 * L);
    }
    for (int col = tid; col <= n; col += NT) {
      C<L> s = pload<L>(red + col, rps);
      for (int w = 1; w < W; ++w) s = cadd<L>(s, pload<L>(red + (size_t)w * rn + col, rps));
      double S = 0.0;
      if (col == n)
        for (int w = 0; w < W; ++w) S += redS[w];
      eval_finish<L>(a, b, i, col, s, S, pd1, pd);
    }
    return;
  }
  const size_t rec = part_record(n, L);
  double *mine = a.part + (size_t)b * part_point_doubles(n, L, a.P) + ((size_t)i * a.P + part) * rec;
  for (int col = tid; col <= n; col += NT) {
    C<L> s = pload<L>(red + col, rps);
    for (int w = 1; w < W; ++w) s = cadd<L>(s, pload<L>(red + (size_t)w * rn + col, rps));
    cstore<L>(mine + (size_t)col * 2 * L, s);
  }
  if (tid == 0) {
    double S = 0.0;
    for (int w = 0; w < W; ++w) S += redS[w];
    mine[part_scale_at(n, L)] = S;
  }
}

// LDS of the evaluation kernel with NT threads: two power tables of 2L limb
// planes [emax+1][n rounded up to 32], or the cross-wave reduction buffer of
// 2L planes [NT/64][n+1] plus NT/64 scale sums, whichever is larger
inline size_t eval_lds_bytes_nt(int L, const DevSystem &s, int NT) {
  const size_t nv = ((size_t)s.n + 31) & ~(size_t)31;
  const size_t tables = 2 * 2 * (size_t)L * (s.emax + 1) * nv;
  const size_t W = NT / 64;
  const size_t red = 2 * (size_t)L * W * (s.n + 1) + W;
  return (tables > red ? tables : red) * sizeof(double);
}

inline int next_pow2(int v) {
  int p = 1;
  while (p < v) p <<= 1;
  return p;
}

template <int L, int CH, int NT>
hipError_t launch_eval_lm(int LM, const EvalArgs<L> &a, int B, hipStream_t st) {
  dim3 grid(a.s.n * a.P + (a.P > 1 ? 1 : 0), B), block(NT);  // + the start-power workgroup of a split
  const size_t lds = eval_lds_bytes_nt(L, a.s, NT);
  if (lds > 64 * 1024) {
    hipError_t e = hipSuccess;
    switch (LM) {
#define QDP_ATTR(X)                                                                                   \
  case X:                                                                                             \
    e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_eval<L, CH, X, NT>),                    \
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);                    \
    break;
      QDP_ATTR(1) QDP_ATTR(2) QDP_ATTR(4) QDP_ATTR(8) QDP_ATTR(16) QDP_ATTR(32) QDP_ATTR(64)
#undef QDP_ATTR
    }
    if (e != hipSuccess) return e;
  }
  switch (LM) {
#define QDP_LM(X) \
  case X: hipLaunchKernelGGL((k_eval<L, CH, X, NT>), grid, block, lds, st, a); break;
    QDP_LM(1) QDP_LM(2) QDP_LM(4) QDP_LM(8) QDP_LM(16) QDP_LM(32) QDP_LM(64)
#undef QDP_LM
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Launch for one precision: LM lanes per monomial from CH variables per lane;
// the split P doubles while fewer than 512 workgroups would run and every
// part keeps at least one wavefront's worth of monomials.  256 threads: with
// 150-250 registers per lane several such workgroups share a compute unit
// and overlap each other's table and reduction phases, which measured faster
// than 512 threads (same at n = 128 double double, 12% at n = 64 quad double)
// and than 128 (20-40%).
template <int L, int CH>
hipError_t launch_eval_T(const DevSystem &s, const double *x, long bx, int B, const HomArgs &h, const EvalOut &o,
                         const NewtonState *gate, const EvalSplit &sp, hipStream_t st) {
  const int LM = next_pow2((s.n + CH - 1) / CH);
  if (LM > 64 || B < 1) return hipErrorInvalidValue;
  const int G = 64 / LM;
  int P = 1;
  if (sp.part)
    while (2 * P <= sp.max_parts && (long)s.n * B * P < 512 && (s.maxm + 2 * P - 1) / (2 * P) >= G) P *= 2;
  EvalArgs<L> a{s, x, bx, h, o, gate, P, sp.part};
  // a split part with at most half of a 256-thread workgroup's monomial
  // slots (one path at n <= 64 in double double) runs on 128 threads: no
  // idle wavefronts in the walk, half the reduction (measured 3% faster)
  const int per_part = (s.maxm + P - 1) / P;
  hipError_t e = (P > 1 && L == 2 && CH == 4 && per_part <= 2 * G) ? launch_eval_lm<L, CH, 128>(LM, a, B, st)
                                                                    : launch_eval_lm<L, CH, 256>(LM, a, B, st);
  if (e != hipSuccess || P == 1) return e;
  hipLaunchKernelGGL(k_eval_sum<L>, dim3(s.n, B), dim3(256), 0, st, a);
  return hipGetLastError();
}

// ---------------------------------------------------------------- common support
// Systems whose polynomials all sum the same M monomials with their own
// coefficients, f_i = sum_m C[i][m] x^(a_m) (the common-support workload of
// the paper's Table 1).  The monomials' partials and values V[m][k] (k < n:
// partial with respect to x_k; k = n: the value) are formed once per point
// by Speelpenning's products (k_supp_v), and the evaluation is the dense
// complex product Y[i][k] = sum_m C[i][m] V[m][k] (k_supp_gemm), blended and
// stored exactly like the sparse evaluation.  The support is the exponent
// rows [0, M) (those of f_0; every polynomial has the same rows).


template <int L> struct SuppArgs {
  DevSystem s;  // s.supp = M
  const double *x;
  long bx;
  HomArgs h;
  EvalOut o;
  const NewtonState *gate;
  double *V;  // [B] points of supp_v_doubles each: V, then the start-system powers
};

// one group of LM lanes per support monomial; blockIdx.y = point.  The last
// workgroup of a point forms the start-system powers of every row instead
// (one chain per thread), stored after V for the product kernel.
template <int L, int CH, int LM, int NT>
__global__ __launch_bounds__(NT) void k_supp_v(SuppArgs<L> a) {
  constexpr int G = 64 / LM, W = NT / 64, SLOTS = W * G;
  const int b = blockIdx.y;
  if (a.gate && !a.gate[b].active) return;
  const double *x = a.x + (size_t)b * a.bx;
  extern __shared__ double smem[];
  const int n = a.s.n, M = a.s.supp;
  if (blockIdx.x == gridDim.x - 1) {
    double *P = a.V + (size_t)b * supp_v_doubles(M, n, L) + supp_pow_offset(M, n, L);
    if (a.h.homotopy)
      for (int i = threadIdx.x; i < n; i += NT) {
        C<L> q1, q;
        start_powers<L>(x + (size_t)i * 2 * L, a.s.deg[i], q1, q);
        cstore<L>(P + (size_t)i * 4 * L, q1);
        cstore<L>(P + (size_t)i * 4 * L + 2 * L, q);
      }
    return;
  }
  const int E1 = a.s.emax + 1;
  const int nv = table_stride(n);
  const size_t tps = (size_t)E1 * nv;
  double *Gt = smem, *Qt = smem + 2 * L * tps;
  const int tid = threadIdx.x;
  power_tables<L>(x, n, E1, nv, tps, Gt, Qt, tid, NT);
  __syncthreads();
  const int lane = tid & 63, wave = tid >> 6, grp = lane / LM, gl = lane % LM;
  const int m = blockIdx.x * SLOTS + wave * G + grp;
  if (m >= M) return;  // whole groups leave together: the shuffles stay inside a group
  auto gval = [&](int v, int e) -> C<L> { return v < n ? pload<L>(Gt + __umul24(e, nv) + v, tps) : cone<L>(); };
  auto qval = [&](int v, int e) -> C<L> { return v < n ? pload<L>(Qt + __umul24(e, nv) + v, tps) : czero<L>(); };
  const uint8_t *er = a.s.exps + (size_t)m * a.s.npad + gl;
  int ex[CH];
#pragma unroll
  for (int k = 0; k < CH; ++k) ex[k] = er[k * LM];
  double *Vm = a.V + (size_t)b * supp_v_doubles(M, n, L) + (size_t)m * 2 * L * (n + 1);
  const size_t vps = (size_t)n + 1;
  const C<L> val = monomial_walk<L, CH, LM, true>(ex, cone<L>(), gl, gval, qval, [&](int k, const C<L> &d) {
    const int v = gl + k * LM;
    if (v < n) pstore<L>(Vm + v, vps, d);
  });
  if (gl == 0) pstore<L>(Vm + n, vps, val);
}

constexpr int kSuppCols = 16;   // output columns per workgroup
constexpr int kSuppParts = 32;  // monomial parts per column, added by a fixed tree

// blockIdx = (row i, column block, point); thread (part p, column k): the
// part's sum over m of C[i][m] V[m][k], then the parts by a fixed pairwise
// tree, the blend and the store
template <int L>
__global__ __launch_bounds__(kSuppCols * kSuppParts) void k_supp_gemm(SuppArgs<L> a) {
  const int i = blockIdx.x, b = blockIdx.z;
  if (a.gate && !a.gate[b].active) return;
  const int n = a.s.n, M = a.s.supp, LS = a.s.LS;
  const int kl = threadIdx.x % kSuppCols, p = threadIdx.x / kSuppCols;
  const int k = blockIdx.y * kSuppCols + kl;
  constexpr int RP = kSuppCols * kSuppParts;  // plane stride of the part sums
  __shared__ double red[2 * L * RP];
  __shared__ double redS[kSuppParts];
  const int chunk = (M + kSuppParts - 1) / kSuppParts;
  const int m0 = min(M, p * chunk), m1 = min(M, m0 + chunk);
  C<L> acc = czero<L>();
  double S = 0.0;
  if (k <= n) {
    const double *V = a.V + (size_t)b * supp_v_doubles(M, n, L) + k;
    const double *Ci = a.s.coefs + (size_t)a.s.offsets[i] * 2 * LS;
    const size_t vps = (size_t)n + 1, vm = 2 * (size_t)L * vps;
    // U monomials' loads issued together (the sum is a dependent chain; the
    // loads are not), then their terms added in order
    constexpr int U = L >= 4 ? 4 : 8;
    for (int m = m0; m < m1; m += U) {
      C<L> cb[U], vb[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int mm = m + u < m1 ? m + u : m1 - 1;  // a valid address; its term is not added
        cb[u] = cload_trunc<L>(Ci + (size_t)mm * 2 * LS, LS);
        vb[u] = pload<L>(V + (size_t)mm * vm, vps);
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (m + u < m1) {
          acc = cfms<L>(acc, cneg<L>(cb[u]), vb[u]);  // acc + c v
          if (k == n) S += cabs_hi<L>(cb[u]) * cabs_hi<L>(vb[u]);
        }
    }
  }
  pstore<L>(red + p * kSuppCols + kl, RP, acc);
  if (k == n) redS[p] = S;
#pragma unroll
  for (int w = kSuppParts / 2; w >= 1; w >>= 1) {
    __syncthreads();
    if (p < w) {
      const C<L> o = pload<L>(red + (p + w) * kSuppCols + kl, RP);
      acc = cadd<L>(acc, o);
      pstore<L>(red + p * kSuppCols + kl, RP, acc);
    }
  }
  if (p != 0 || k > n) return;
  double SS = 0.0;
  if (k == n)
    for (int q = 0; q < kSuppParts; ++q) SS += redS[q];
  C<L> pd1 = czero<L>(), pd = cone<L>();
  if (a.h.homotopy) {
    const double *P = a.V + (size_t)b * supp_v_doubles(M, n, L) + supp_pow_offset(M, n, L) + (size_t)i * 4 * L;
    pd1 = cload<L>(P);
    pd = cload<L>(P + 2 * L);
  }
  const C<L> sum = acc;
  const EvalArgs<L> ea{a.s, a.x, a.bx, a.h, a.o, a.gate, 1, nullptr};
  eval_finish<L>(ea, b, i, k, sum, SS, pd1, pd);
}

// Common-support evaluation of B points: V and the start powers into the
// caller's scratch (B * supp_v_doubles), then the product.
template <int L, int CH>
hipError_t launch_supp_T(const DevSystem &s, const double *x, long bx, int B, const HomArgs &h, const EvalOut &o,
                         const NewtonState *gate, double *V, hipStream_t st) {
  const int LM = next_pow2((s.n + CH - 1) / CH);
  if (LM > 64 || B < 1 || s.supp < 1 || !V) return hipErrorInvalidValue;
  constexpr int NT = 128;
  SuppArgs<L> a{s, x, bx, h, o, gate, V};
  const int slots = (NT / 64) * (64 / LM);
  const dim3 grid((s.supp + slots - 1) / slots + 1, B);  // + the start-power workgroup
  const size_t nv = ((size_t)s.n + 31) & ~(size_t)31;
  const size_t lds = 2 * 2 * (size_t)L * (s.emax + 1) * nv * sizeof(double);
  switch (LM) {
#define QDP_SV(X)                                                                                       \
  case X:                                                                                               \
    if (lds > 64 * 1024) {                                                                              \
      hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_supp_v<L, CH, X, NT>),        \
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);         \
      if (e != hipSuccess) return e;                                                                    \
    }                                                                                                   \
    hipLaunchKernelGGL((k_supp_v<L, CH, X, NT>), grid, dim3(NT), lds, st, a);                           \
    break;
    QDP_SV(1) QDP_SV(2) QDP_SV(4) QDP_SV(8) QDP_SV(16) QDP_SV(32) QDP_SV(64)
#undef QDP_SV
    default:
      return hipErrorInvalidValue;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const dim3 g2(s.n, (s.n + 1 + kSuppCols - 1) / kSuppCols, B);
  hipLaunchKernelGGL(k_supp_gemm<L>, g2, dim3(kSuppCols * kSuppParts), 0, st, a);
  return hipGetLastError();
}

}  // namespace qdp
