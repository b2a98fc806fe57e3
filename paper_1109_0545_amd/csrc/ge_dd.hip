// Elimination launchers, one precision per file.
#include "ge_kernel.hpp"

namespace qdp {

size_t ge_lds_bytes(int L, int n, bool in_lds);

template <int L>
static hipError_t launch_ge_L(int n, int B, double *ab, double *scale, double *x, double *dz, NewtonState *st,
                              hipStream_t s) {
  GeArgs<L> a{n, ab, scale, x, dz, st};
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

hipError_t launch_ge_dd(int n, int B, double *ab, double *scale, double *x, double *dz, NewtonState *st,
                        hipStream_t s) {
  return launch_ge_L<2>(n, B, ab, scale, x, dz, st, s);
}

}  // namespace qdp
