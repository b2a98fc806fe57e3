// Elimination dispatch by precision.
#include "common.hpp"

namespace qdp {

hipError_t launch_ge_f64(int, int, double *, double *, double *, double *, NewtonState *, hipStream_t);
hipError_t launch_ge_dd(int, int, double *, double *, double *, double *, NewtonState *, hipStream_t);
hipError_t launch_ge_qd(int, int, double *, double *, double *, double *, NewtonState *, hipStream_t);

size_t ge_lds_bytes(int L, int n, bool in_lds) {
  size_t d = (size_t)2 * n * 2 * L + 16;  // inverses + rhs + reduction
  if (in_lds) d += (size_t)n * (n + 1) * 2 * L;
  return d * sizeof(double) + 4 * (size_t)n * sizeof(int) + 64;
}

// B points, one workgroup each (see GeArgs for the batch layout)
hipError_t launch_ge_scaled(int L, int n, int B, double *ab, double *scale, double *x, double *dz, NewtonState *st,
                            hipStream_t s) {
  if (B < 1) return hipErrorInvalidValue;
  switch (L) {
    case 1: return launch_ge_f64(n, B, ab, scale, x, dz, st, s);
    case 2: return launch_ge_dd(n, B, ab, scale, x, dz, st, s);
    case 4: return launch_ge_qd(n, B, ab, scale, x, dz, st, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace qdp
