// Evaluation dispatch by precision.
#include "common.hpp"

namespace qdp {

hipError_t launch_eval_f64(const DevSystem &, const double *, long, int, const HomArgs &, const EvalOut &,
                           const NewtonState *, const EvalSplit &, hipStream_t);
hipError_t launch_eval_dd(const DevSystem &, const double *, long, int, const HomArgs &, const EvalOut &,
                          const NewtonState *, const EvalSplit &, hipStream_t);
hipError_t launch_eval_qd(const DevSystem &, const double *, long, int, const HomArgs &, const EvalOut &,
                          const NewtonState *, const EvalSplit &, hipStream_t);

// The launcher splits polynomials only while fewer than 512 workgroups would
// run, i.e. for batches of B < 512 / n points: scratch for at most that many.
size_t eval_part_doubles(int L, int n, int B) {
  const int bs = B < 511 / n ? B : 511 / n;
  // records of (n+1) complex partial sums and a scale sum, then the start-system powers
  return (size_t)bs * n * (kMaxEvalParts * ((size_t)(n + 1) * 2 * L + 1) + 4 * (size_t)L);
}


size_t eval_supp_doubles(int L, int n, int supp) { return supp_v_doubles(supp, n, L); }

hipError_t launch_eval(int L, const DevSystem &s, const double *x, long bx, int B, const HomArgs &h,
                       const EvalOut &o, const NewtonState *gate, const EvalSplit &split, hipStream_t st) {
  // a common-support system is evaluated through its monomial partials: the
  // caller must bring the scratch for them
  if (s.supp > 0 && (!split.supp_v || B > split.supp_cap)) return hipErrorInvalidValue;
  switch (L) {
    case 1: return launch_eval_f64(s, x, bx, B, h, o, gate, split, st);
    case 2: return launch_eval_dd(s, x, bx, B, h, o, gate, split, st);
    case 4: return launch_eval_qd(s, x, bx, B, h, o, gate, split, st);
  }
  return hipErrorInvalidValue;
}

}  // namespace qdp
