// Inputs of the learned step-size controller (a growth direction of the
// tracker of Algorithm 3.1, not in the paper): 16 features of the state after
// an accepted corrector stage.  The same function serves the host (probe
// records, training data) and the device (the network runs right after each
// corrector stage, before the tracker reads the stage back).
#pragma once
#include <hip/hip_runtime.h>

namespace qdp {

struct CtlFeatIn {
  double lam[3];  // last accepted step sizes, newest first
  int iters;      // Newton iterations of the last accepted stage
  double rho_first, rho_last, cond, dz_first, znorm, pred_dist;
  double t;       // the accepted t
  int run;        // consecutive successes
  int rejected;   // rejections among the last 8 attempts
  long long accepted;
};

__host__ __device__ inline double ctl_lg(double v, double lo) { return log10(v > lo ? v : lo); }

__host__ __device__ inline void ctl_features(const CtlFeatIn &h, float *f) {
  const double zn = h.znorm > 1.0 ? h.znorm : 1.0;
  const double acc = h.accepted < 1000 ? (double)h.accepted : 1000.0;
  const double v[16] = {
      log2(h.lam[0] / 0.01),
      log2(h.lam[1] / 0.01),
      log2(h.lam[2] / 0.01),
      (double)h.iters,
      ctl_lg(h.rho_first, 1e-40) / 10.0,
      ctl_lg(h.rho_last, 1e-40) / 10.0,
      ctl_lg(h.cond, 1.0) / 5.0,
      h.t,
      ctl_lg(1.0 - h.t, 1e-16),
      ctl_lg(h.znorm, 1e-300),
      ctl_lg(h.pred_dist / zn, 1e-40) / 10.0,
      ctl_lg(h.dz_first / zn, 1e-40) / 10.0,
      (h.run < 10 ? h.run : 10) / 10.0,
      h.rejected / 8.0,
      (ctl_lg(h.dz_first, 1e-300) - ctl_lg(h.pred_dist, 1e-300)) / 10.0,
      acc / 1000.0,
  };
  for (int k = 0; k < 16; ++k) f[k] = (float)v[k];
}

}  // namespace qdp
