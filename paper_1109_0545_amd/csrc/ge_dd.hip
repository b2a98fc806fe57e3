// Elimination launcher for L = 2 limbs (one precision per translation unit).
#include "ge_launch.hpp"

namespace qdp {

hipError_t launch_ge_dd(int n, int B, double *ab, double *scale, double *x, double *dz, NewtonState *st,
                        const GeMc &mc, hipStream_t s) {
  return launch_ge_L<2>(n, B, ab, scale, x, dz, st, mc, s);
}

}  // namespace qdp
