// Evaluation launcher for one precision (the three precisions compile in
// parallel, one file each).
#include "eval_kernel.hpp"

namespace qdp {

hipError_t launch_eval_qd(const DevSystem &s, const double *x, long bx, int B, const HomArgs &h, const EvalOut &o,
                         const NewtonState *gate, const EvalSplit &sp, hipStream_t st) {
  if (s.supp > 0) return launch_supp_T<4, 2>(s, x, bx, B, h, o, gate, sp.supp_v, st);
  return launch_eval_T<4, 2>(s, x, bx, B, h, o, gate, sp, st);
}

}  // namespace qdp
