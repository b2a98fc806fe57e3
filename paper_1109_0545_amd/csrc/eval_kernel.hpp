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
// Mapping on CDNA4: one workgroup per polynomial; a monomial is spread over
// LM lanes of a wavefront and lane g owns the CH variables g, g+LM, g+2LM, ...
// (interleaved, so that neighbouring lanes read neighbouring table entries).
// The order used for the prefix/suffix products is lane-major: a lane first
// forms the suffix products of its own variables, the LM lanes then combine
// their chunk products with Hillis-Steele scans in both directions (wavefront
// shuffles), and each lane walks its variables forward once.  A lane keeps
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
  const double *x;  // [n][2][L] at the compute precision
  HomArgs h;
  EvalOut o;
  const NewtonState *gate;
};

// row stride (doubles) of a table plane: a multiple of 32 so that lanes with
// consecutive variables read consecutive banks whatever their exponents
__host__ __device__ inline int table_stride(int n) { return (n + 31) & ~31; }

template <int L, int CH, int LM, int NT>
__global__ __launch_bounds__(NT) void k_eval(EvalArgs<L> a) {
  constexpr int G = 64 / LM;  // monomials per wavefront at a time
  constexpr int W = NT / 64;  // wavefronts
  constexpr int SLOTS = W * G;
  if (a.gate && !a.gate->active) return;

  extern __shared__ double smem[];
  const int n = a.s.n;
  const int E1 = a.s.emax + 1;
  const int nv = table_stride(n);
  const size_t tps = (size_t)E1 * nv;  // plane size of one table
  double *Gt = smem;                   // x_v^e          plane c at Gt + c*tps + e*nv + v
  double *Qt = smem + 2 * L * tps;     // e x_v^(e-1)
  const int tid = threadIdx.x;

  // ---- power tables
  for (int v = tid; v < n; v += NT) {
    const C<L> xv = cload<L>(a.x + (size_t)v * 2 * L);
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

  const int i = blockIdx.x;
  const int t0 = a.s.offsets[i], t1 = a.s.offsets[i + 1];
  const int lane = tid & 63, wave = tid >> 6;
  const int grp = lane / LM, gl = lane % LM;
  const int slot = wave * G + grp;
  const int LS = a.s.LS;

  C<L> acc[CH];
#pragma unroll
  for (int k = 0; k < CH; ++k) acc[k] = czero<L>();
  C<L> accv = czero<L>();
  double accS = 0.0;

  auto gval = [&](int v, int e) -> C<L> { return v < n ? pload<L>(Gt + (size_t)e * nv + v, tps) : cone<L>(); };
  auto qval = [&](int v, int e) -> C<L> { return v < n ? pload<L>(Qt + (size_t)e * nv + v, tps) : czero<L>(); };

  for (int base = t0; base < t1; base += SLOTS) {
    const int j = base + slot;
    const bool valid = j < t1;
    const int jj = valid ? j : t0;
    const uint8_t *er = a.s.exps + (size_t)jj * a.s.npad + gl;
    int ex[CH];
#pragma unroll
    for (int k = 0; k < CH; ++k) ex[k] = er[k * LM];
    const C<L> coef = cload_trunc<L>(a.s.coefs + (size_t)jj * 2 * LS, LS);

    // suffix products of this lane's variables (exclusive), and their product
    C<L> sfx[CH];
    sfx[CH - 1] = cone<L>();
#pragma unroll
    for (int k = CH - 2; k >= 0; --k) sfx[k] = cmul<L>(sfx[k + 1], gval(gl + (k + 1) * LM, ex[k + 1]));
    const C<L> chunk = cmul<L>(sfx[0], gval(gl, ex[0]));

    // inclusive scans of chunk products over the LM lanes of this monomial
    C<L> fw = chunk, bw = chunk;
#pragma unroll
    for (int d = 1; d < LM; d <<= 1) {
      C<L> y = cshfl_up<L>(fw, d, LM);
      C<L> z = cshfl_down<L>(bw, d, LM);
      fw = cselect<L>(gl >= d, cmul<L>(y, fw), fw);
      bw = cselect<L>(gl + d < LM, cmul<L>(bw, z), bw);
    }
    C<L> pre = cshfl_up<L>(fw, 1, LM);
    C<L> suf = cshfl_down<L>(bw, 1, LM);
    if (LM == 1 || gl == 0) pre = cone<L>();
    if (LM == 1 || gl == LM - 1) suf = cone<L>();

    // walk this lane's variables: run = c * (all factors before v)
    //                                   * (all factors of later lanes)
    C<L> run = cmul<L>(cmul<L>(coef, pre), suf);
#pragma unroll
    for (int k = 0; k < CH; ++k) {
      const int v = gl + k * LM;
      C<L> d = cmul<L>(cmul<L>(run, sfx[k]), qval(v, ex[k]));
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

  // ---- fixed-order sum over wavefronts, homotopy blend, store
  for (int col = tid; col <= n; col += NT) {
    C<L> s = pload<L>(red + col, rps);
    for (int w = 1; w < W; ++w) s = cadd<L>(s, pload<L>(red + (size_t)w * rn + col, rps));
    if (col < n) {
      C<L> Jv = s;
      if (a.h.homotopy) {
        Jv = cmul_d<L>(s, a.h.t);
        if (col == i) {
          const C<L> g = cload<L>(a.h.gamma);
          double e1;
          R<L> omt = rzero<L>();
          omt.v[0] = two_sum(1.0, -a.h.t, e1);
          if (L > 1) omt.v[1] = e1;
          const C<L> w = cmul_r<L>(g, omt);
          const int d = a.s.deg[i];
          const C<L> xi = cload<L>(a.x + (size_t)i * 2 * L);
          if (d >= 1) {
            C<L> p1 = cpow<L>(xi, d - 1);
            Jv = cadd<L>(Jv, cmul<L>(w, cmul_d<L>(p1, (double)d)));
          }
        }
      }
      pstore<L>(a.o.J + (size_t)i * a.o.rsJ + (size_t)col * a.o.csJ, a.o.psJ, Jv);
    } else {
      C<L> hv = s;
      double S = 0.0;
      for (int w = 0; w < W; ++w) S += redS[w];
      if (a.h.homotopy) {
        const C<L> g = cload<L>(a.h.gamma);
        double e1;
        R<L> omt = rzero<L>();
        omt.v[0] = two_sum(1.0, -a.h.t, e1);
        if (L > 1) omt.v[1] = e1;
        const C<L> w = cmul_r<L>(g, omt);
        const int d = a.s.deg[i];
        const C<L> xi = cload<L>(a.x + (size_t)i * 2 * L);
        const C<L> pd = cpow<L>(xi, d);
        C<L> gm = pd;
        gm.re = rsub<L>(gm.re, rfrom<L>(1.0));
        hv = cadd<L>(cmul_d<L>(s, a.h.t), cmul<L>(w, gm));
        S = fabs(a.h.t) * S + cabs_hi<L>(w) * (cabs_hi<L>(pd) + 1.0);
      }
      if (a.o.ysign < 0) hv = cneg<L>(hv);
      pstore<L>(a.o.y + (size_t)i * a.o.sy, a.o.psy, hv);
      if (a.o.scale) a.o.scale[i] = S;
    }
  }
}

}  // namespace qdp
