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
  if (fit) {
    const size_t lds = ge_lds_bytes(L, n, true);
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_ge<L, NT, true>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_ge<L, NT, true>), dim3(B), dim3(NT), lds, s, a);
  } else {
    const size_t lds = ge_lds_bytes(L, n, false);
    hipLaunchKernelGGL((k_ge<L, NT, false>), dim3(B), dim3(NT), lds, s, a);
  }
  return hipGetLastError();
}

hipError_t launch_ge_f64(int n, int B, double *ab, double *scale, double *x, double *dz, NewtonState *st,
                        hipStream_t s) {
  return launch_ge_L<1>(n, B, ab, scale, x, dz, st, s);
}

}  // namespace qdp
