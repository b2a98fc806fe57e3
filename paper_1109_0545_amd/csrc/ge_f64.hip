// Elimination launcher for L = 1 limbs (one precision per translation unit).
#include "ge_launch.hpp"

namespace qdp {

hipError_t launch_ge_f64(int n, int B, double *ab, double *scale, double *x, double *dz, NewtonState *st,
                        const GeMc &mc, hipStream_t s) {
  return launch_ge_L<1>(n, B, ab, scale, x, dz, st, mc, s);
}

}  // namespace qdp
