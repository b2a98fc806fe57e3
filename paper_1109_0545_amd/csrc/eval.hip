// Evaluation dispatch by precision.
#include "common.hpp"

namespace qdp {

hipError_t launch_eval_f64(const DevSystem &, const double *, const HomArgs &, const EvalOut &, const NewtonState *,
                           hipStream_t);
hipError_t launch_eval_dd(const DevSystem &, const double *, const HomArgs &, const EvalOut &, const NewtonState *,
                          hipStream_t);
hipError_t launch_eval_qd(const DevSystem &, const double *, const HomArgs &, const EvalOut &, const NewtonState *,
                          hipStream_t);

size_t eval_lds_bytes(int L, const DevSystem &s) {
  const size_t el = 16 * (size_t)L;
  size_t tables = 2 * (size_t)s.n * (s.emax + 1) * el;
  size_t red = 16 * (size_t)(s.n + 1) * el + 16 * sizeof(double);
  return tables > red ? tables : red;
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
