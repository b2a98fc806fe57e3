// Evaluation of a sparse polynomial system and its full Jacobian, fused with
// the total-degree homotopy blend.
//
// What is computed is the array Y of Section 4 (every polynomial value and
// every partial derivative); how each monomial is differentiated follows the
// reverse-mode (Speelpenning) products of Section 6: with g_v = x_v^(a_v) the
// factor of variable v, the partial of c * prod_v g_v with respect to x_v is
//     c * (prod_{w<v} g_w) * (prod_{w>v} g_w) * a_v x_v^(a_v - 1),
// i.e. a prefix product times a suffix product times a derivative factor.
// Powers x_v^e and e x_v^(e-1) come from a table built once per evaluation in
// LDS (the common factor x^(a-1) of Section 6 folded into the table), so each
// variable of a monomial costs four complex products, as the paper's scheme.
//
// Mapping on CDNA4: one workgroup per polynomial; a monomial is spread over
// LM lanes of a wavefront, each lane owning C consecutive variables (dense
// exponent rows, coalesced byte loads).  Within a lane the suffix products of
// its chunk are formed sequentially; across the LM lanes the chunk products
// are combined by a Hillis-Steele scan in both directions (wavefront
// shuffles); each lane then walks its chunk forward once.  A lane keeps the
// running sums of its C Jacobian entries in registers over all monomials it
// visits; the per-polynomial reduction is a fixed-order shuffle butterfly then
// a fixed-order LDS sum across wavefronts (no atomics: results are
// bit-reproducible).  The homotopy blend and the b = -h column are written
// directly in the layout the eliminator reads.

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

template <int L, int CH, int LM, int NT>
__global__ __launch_bounds__(NT) void k_eval(EvalArgs<L> a) {
  constexpr int G = 64 / LM;   // monomials per wavefront at a time
  constexpr int W = NT / 64;   // wavefronts
  constexpr int SLOTS = W * G;
  if (a.gate && !a.gate->active) return;

  extern __shared__ double smem[];
  const int n = a.s.n;
  const int E1 = a.s.emax + 1;
  C<L> *Gt = reinterpret_cast<C<L> *>(smem);  // [n][E1] x^e
  C<L> *Qt = Gt + n * E1;                     // [n][E1] e x^(e-1)
  const int tid = threadIdx.x;

  // ---- power tables
  for (int v = tid; v < n; v += NT) {
    C<L> xv = cload<L>(a.x + (size_t)v * 2 * L);
    C<L> p = cone<L>();
    Gt[v * E1] = p;
    Qt[v * E1] = czero<L>();
    for (int e = 1; e < E1; ++e) {
      Qt[v * E1 + e] = cmul_d<L>(p, (double)e);
      p = cmul<L>(p, xv);
      Gt[v * E1 + e] = p;
    }
  }
  __syncthreads();

  const int i = blockIdx.x;
  const int t0 = a.s.offsets[i], t1 = a.s.offsets[i + 1];
  const int lane = tid & 63, wave = tid >> 6;
  const int grp = lane / LM, gl = lane % LM;
  const int slot = wave * G + grp;
  const int v0 = gl * CH;
  const int LS = a.s.LS;

  C<L> acc[CH];
#pragma unroll
  for (int k = 0; k < CH; ++k) acc[k] = czero<L>();
  C<L> accv = czero<L>();
  double accS = 0.0;

  auto gval = [&](int v, int e) -> C<L> { return v < n ? Gt[v * E1 + e] : cone<L>(); };
  auto qval = [&](int v, int e) -> C<L> { return v < n ? Qt[v * E1 + e] : czero<L>(); };

  for (int base = t0; base < t1; base += SLOTS) {
    const int j = base + slot;
    const bool valid = j < t1;
    const int jj = valid ? j : t0;
    const uint8_t *er = a.s.exps + (size_t)jj * a.s.npad + v0;
    int ex[CH];
#pragma unroll
    for (int k = 0; k < CH; ++k) ex[k] = er[k];
    const C<L> coef = cload_trunc<L>(a.s.coefs + (size_t)jj * 2 * LS, LS);

    // suffix products inside the chunk (exclusive), and the chunk product
    C<L> sfx[CH];
    sfx[CH - 1] = cone<L>();
#pragma unroll
    for (int k = CH - 2; k >= 0; --k) sfx[k] = cmul<L>(sfx[k + 1], gval(v0 + k + 1, ex[k + 1]));
    const C<L> chunk = cmul<L>(sfx[0], gval(v0, ex[0]));

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

    // walk the chunk: running = c * prefix(all before v) * suffix(all after chunk)
    C<L> run = cmul<L>(cmul<L>(coef, pre), suf);
#pragma unroll
    for (int k = 0; k < CH; ++k) {
      C<L> d = cmul<L>(cmul<L>(run, sfx[k]), qval(v0 + k, ex[k]));
      if (valid) acc[k] = cadd<L>(acc[k], d);
      run = cmul<L>(run, gval(v0 + k, ex[k]));
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
  C<L> *red = reinterpret_cast<C<L> *>(smem);  // [W][n+1]
  double *redS = reinterpret_cast<double *>(red + W * (n + 1));
  if (lane < LM) {
#pragma unroll
    for (int k = 0; k < CH; ++k)
      if (v0 + k < n) red[wave * (n + 1) + v0 + k] = acc[k];
    if (lane == 0) {
      red[wave * (n + 1) + n] = accv;
      redS[wave] = accS;
    }
  }
  __syncthreads();

  // ---- fixed-order sum over wavefronts, homotopy blend, store
  for (int col = tid; col <= n; col += NT) {
    C<L> s = red[col];
    for (int w = 1; w < W; ++w) s = cadd<L>(s, red[w * (n + 1) + col]);
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
      cstore<L>(a.o.J + ((size_t)i * a.o.rsJ + (size_t)col * a.o.csJ) * 2 * L, Jv);
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
      cstore<L>(a.o.y + (size_t)i * a.o.sy * 2 * L, hv);
      if (a.o.scale) a.o.scale[i] = S;
    }
  }
}

}  // namespace qdp
