// Evaluation launchers for one precision each (split so that the three
// precisions compile in parallel).
#include "eval_kernel.hpp"

namespace qdp {

static int next_pow2(int v) {
  int p = 1;
  while (p < v) p <<= 1;
  return p;
}

template <int L, int CH, int NT>
static hipError_t launch_lm(int LM, const EvalArgs<L> &a, size_t lds, hipStream_t st) {
  dim3 grid(a.s.n), block(NT);
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

size_t eval_lds_bytes(int L, const DevSystem &s);

hipError_t launch_eval_dd(const DevSystem &s, const double *x, const HomArgs &h, const EvalOut &o,
                          const NewtonState *gate, hipStream_t st) {
  EvalArgs<2> a{s, x, h, o, gate};
  const size_t lds = eval_lds_bytes(2, s);
  constexpr int CH = 4;
  const int LM = next_pow2((s.n + CH - 1) / CH);
  if (LM > 64) return hipErrorInvalidValue;
  return launch_lm<2, CH, 512>(LM, a, lds, st);
}

}  // namespace qdp
