// Evaluation launcher for one precision (the three precisions compile in
// parallel, one file each).
#include "eval_kernel.hpp"

namespace qdp {

// Past 64 variables, eight per lane (fewer lanes per monomial, so fewer
// butterfly levels; measured faster at n = 128, slower at n = 64: 701 against
// 608 us at 256 points, where 232 registers leave two workgroups per CU).
hipError_t launch_eval_dd(const DevSystem &s, const double *x, long bx, int B, const HomArgs &h, const EvalOut &o,
                         const NewtonState *gate, const EvalSplit &sp, hipStream_t st) {
  if (s.supp > 0)
    return s.n > 64 ? launch_supp_T<2, 8>(s, x, bx, B, h, o, gate, sp.supp_v, st)
                    : launch_supp_T<2, 4>(s, x, bx, B, h, o, gate, sp.supp_v, st);
  if (s.n > 64) return launch_eval_T<2, 8>(s, x, bx, B, h, o, gate, sp, st);
  return launch_eval_T<2, 4>(s, x, bx, B, h, o, gate, sp, st);
}

}  // namespace qdp
