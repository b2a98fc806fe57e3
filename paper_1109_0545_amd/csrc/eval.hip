// Evaluation dispatch by precision.
#include "common.hpp"

namespace qdp {

hipError_t launch_eval_f64(const DevSystem &, const double *, const HomArgs &, const EvalOut &, const NewtonState *,
                           hipStream_t);
hipError_t launch_eval_dd(const DevSystem &, const double *, const HomArgs &, const EvalOut &, const NewtonState *,
                          hipStream_t);
hipError_t launch_eval_qd(const DevSystem &, const double *, const HomArgs &, const EvalOut &, const NewtonState *,
                          hipStream_t);

// LDS of the evaluation kernel (512 threads = 8 wavefronts): two power
// tables of 2L limb planes [emax+1][n rounded up to 32], or the cross-wave
// reduction buffer of 2L planes [8][n+1] plus 8 scale sums, whichever is larger
size_t eval_lds_bytes(int L, const DevSystem &s) {
  const size_t nv = ((size_t)s.n + 31) & ~(size_t)31;
  const size_t tables = 2 * 2 * (size_t)L * (s.emax + 1) * nv;
  const size_t red = 2 * (size_t)L * 8 * (s.n + 1) + 8;
  return (tables > red ? tables : red) * sizeof(double);
}

hipError_t launch_eval(int L, const DevSystem &s, const double *x, const HomArgs &h, const EvalOut &o,
                       const NewtonState *gate, hipStream_t st) {
  switch (L) {
    case 1: return launch_eval_f64(s, x, h, o, gate, st);
    case 2: return launch_eval_dd(s, x, h, o, gate, st);
    case 4: return launch_eval_qd(s, x, h, o, gate, st);
  }
  return hipErrorInvalidValue;
}

}  // namespace qdp
