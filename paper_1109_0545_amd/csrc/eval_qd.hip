// Evaluation launcher for one precision (the three precisions compile in
// parallel, one file each).
#include "eval_kernel.hpp"

namespace qdp {

hipError_t launch_eval_qd(const DevSystem &s, const double *x, long bx, int B, const HomArgs &h, const EvalOut &o,
                         const NewtonState *gate, const EvalSplit &sp, hipStream_t st) {
  if (s.supp > 0) return launch_supp_T<4, 2>(s, x, bx, B, h, o, gate, sp.supp_v, st);
  // four variables per lane when the launch is not split (enough points for
  // 512 workgroups): 16 lanes per monomial at n = 64, 352 complex products per
  // monomial instead of 512 with two per lane, despite spilling 76 registers
  // (n = 64 at 64 points: 2,448 -> 1,985 us per evaluation); a split
  // evaluation (few points) keeps two per lane (one point: 86.5 against 96.6 us)
  if (s.n <= 64 && (long)s.n * B >= 512) return launch_eval_T<4, 4>(s, x, bx, B, h, o, gate, sp, st);
  return launch_eval_T<4, 2>(s, x, bx, B, h, o, gate, sp, st);
}

}  // namespace qdp
