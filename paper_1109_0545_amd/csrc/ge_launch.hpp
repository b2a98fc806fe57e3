// Elimination launcher shared by the per-precision translation units: the
// column-parallel kernel (ge_mc.hpp) when the caller chose it (GeMc), else
// the register-resident kernel (ge_reg.hpp) when the augmented matrix fits in
// one workgroup's registers, else the LDS / global-memory kernel
// (ge_kernel.hpp).
#pragma once
#include "ge_mcb.hpp"

namespace qdp {

size_t ge_lds_bytes(int L, int n, bool in_lds);

template <int L, int NW, int NMAX>
static hipError_t launch_ge_reg(int n, int B, const GeArgs<L> &a, hipStream_t s) {
  const size_t lds = ge_reg_lds_bytes(L, RegShape<NW, NMAX>::RMAX, n);
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_ge_reg<L, NW, NMAX>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_ge_reg<L, NW, NMAX>), dim3(B), dim3(64 * NW), lds, s, a);
  return hipGetLastError();
}

// eight column wavefronts, 16 columns per block (two slots each; in double
// double with one row per lane a third slot lets the last block take up to
// 24 columns, so that b joins the last full block: at n = 64, 4 blocks
// instead of 5, 95.2 -> 92.5 us; with two rows per lane, or in quad double,
// the third slot measured slower: n = 128 DD 302.6 against 292.3 us, n = 64
// QD 583 against 508 us); the forwarding wavefront takes up to 4 raised
// steps per poll (2 in quad double, for registers); RPL rows per lane (2 past
// n = 64)
template <int L, int RPL>
static hipError_t launch_ge_mcb(int n, int B, const GeArgs<L> &a, const GeMc &mc, hipStream_t s) {
  constexpr int NW = 8, WB = 16, CPW = (L == 2 && RPL == 1) ? 3 : 2, K = L == 4 ? 2 : 4;
  const size_t lds = ge_mcb_lds_bytes(L, n, NW);
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_ge_mcb<L, NW, CPW, K, RPL, WB>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_ge_mcb<L, NW, CPW, K, RPL, WB>), dim3(mcb_blocks(n, WB, NW * CPW - WB), B),
                     dim3(64 * (NW + 1)), lds, s, a, mc.ws, mc.epoch);
  return hipGetLastError();
}

template <int L>
static hipError_t launch_ge_L(int n, int B, double *ab, double *scale, double *x, double *dz, NewtonState *st,
                              const GeMc &mc, hipStream_t s) {
  GeArgs<L> a{n, ab, scale, x, dz, st};
  if constexpr (L == 2 || L == 4) {
    if (mc.ws && mc.blocks) {
      if (n < 1 || n > (L == 2 ? 128 : 64)) return hipErrorInvalidValue;
      if (n <= 64) return launch_ge_mcb<L, 1>(n, B, a, mc, s);
      if constexpr (L == 2) return launch_ge_mcb<L, 2>(n, B, a, mc, s);
    }
  }
  if constexpr (L == 2 || L == 4) {
    if (mc.ws) {
      if (n < 1 || n > 128) return hipErrorInvalidValue;
      if (n <= 64)
        hipLaunchKernelGGL((k_ge_mc<L, 1>), dim3(n + 1, B), dim3(64), 0, s, a, mc.ws, mc.epoch);
      else
        hipLaunchKernelGGL((k_ge_mc<L, 2>), dim3(n + 1, B), dim3(64), 0, s, a, mc.ws, mc.epoch);
      return hipGetLastError();
    }
  }
  // quad double keeps the LDS kernel: its pivot step (inverse and products in
  // four limbs) is long enough that the register kernel measured slower
  if constexpr (L == 1) {
    if (n <= 64) return launch_ge_reg<1, 16, 64>(n, B, a, s);
    if (n <= 128) return launch_ge_reg<1, 8, 128>(n, B, a, s);
  } else if constexpr (L == 2) {
    if (n <= 16) return launch_ge_reg<2, 4, 16>(n, B, a, s);
    if (n <= 32) return launch_ge_reg<2, 8, 32>(n, B, a, s);
    if (n <= 64) return launch_ge_reg<2, 16, 64>(n, B, a, s);
  }
  constexpr int NT = (L == 4) ? 512 : 1024;
  const bool fit = ge_lds_bytes(L, n, true) <= 160 * 1024;
  // look-ahead rows per lane: 1 up to n = 64, 2 up to 128, 4 up to 256
  const int rpl = n <= 64 ? 1 : (n <= 128 ? 2 : 4);
  const size_t lds = ge_lds_bytes(L, n, fit);
  if (fit) {
    const void *k = rpl == 1 ? reinterpret_cast<const void *>(&k_ge<L, NT, true, 1>)
                  : rpl == 2 ? reinterpret_cast<const void *>(&k_ge<L, NT, true, 2>)
                             : reinterpret_cast<const void *>(&k_ge<L, NT, true, 4>);
    hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
#define QDP_GE(FIT, RPL) hipLaunchKernelGGL((k_ge<L, NT, FIT, RPL>), dim3(B), dim3(NT), lds, s, a)
  if (fit) {
    if (rpl == 1) QDP_GE(true, 1);
    else if (rpl == 2) QDP_GE(true, 2);
    else QDP_GE(true, 4);
  } else {
    if (rpl == 1) QDP_GE(false, 1);
    else if (rpl == 2) QDP_GE(false, 2);
    else QDP_GE(false, 4);
  }
#undef QDP_GE
  return hipGetLastError();
}

}  // namespace qdp
