// Shared host/device declarations of the HIP path: device-resident system
// layout, kernel argument blocks and launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mw.hpp"

namespace qdp {

// Device copy of a sparse system (the paper's normalized monomials stored as
// dense exponent rows, Section 6).
struct DevSystem {
  int n;               // equations = variables
  int terms;           // total monomials
  int LS;              // limbs stored per real component
  int npad;            // exponent row stride in bytes (>= next_pow2(n), >= 8)
  int emax;            // largest exponent
  int maxm;            // most monomials in one polynomial
  const int32_t *offsets;  // [n+1]
  const uint8_t *exps;     // [terms][npad], zero padded
  const double *coefs;     // [terms][2][LS]
  const int32_t *deg;      // [n] total degree d_i of f_i
};

// Where evaluation results go.  All strides count doubles.  Limb c of the
// complex element J(i,v) (c < L real limbs, then L imaginary limbs) sits at
// J[c*psJ + i*rsJ + v*csJ]; limb c of value i at y[c*psy + i*sy] (times
// ysign); scale_i -> scale[i] (nullable).
struct EvalOut {
  double *J;
  long psJ, rsJ, csJ;
  double *y;
  long psy, sy;
  double ysign;
  double *scale;
};

// Homotopy h = t f + (1-t) gamma (x^d - 1); homotopy = 0 evaluates f alone.
struct HomArgs {
  int homotopy;
  double t;
  double gamma[8];  // [re limbs][im limbs] at the compute L (first 2L used)
};

// Per-call Newton state kept on the device.
struct NewtonState {
  int active;       // loop still running
  int iterations;   // i of Algorithm 4.1
  int success;      // residual < eps at exit
  int singular;     // zero pivot met
  int nonfinite;    // NaN/Inf met
  int max_it;
  double eps;
  double rho;        // last residual
  double rho_first;  // residual at the first iteration
  double cond_est;   // max |u_jj| / min |u_jj| of the last elimination
  double dz_norm;    // ||dz||_inf (leading limbs) of the last update
  double refine_err; // mixed precision: last ||correction||_inf / ||dz||_inf
  int refine_steps;  // mixed precision: refinements done in the last solve
  int pad;
  double dz_first;   // ||dz||_inf of the first iteration
  double xnorm;      // ||x||_inf after the last update
};

// launchers (defined per translation unit; return hipError_t)
hipError_t launch_eval(int L, const DevSystem &s, const double *x, const HomArgs &h, const EvalOut &o,
                       const NewtonState *gate, hipStream_t st);
size_t eval_lds_bytes(int L, const DevSystem &s);

hipError_t launch_ge(int L, int n, double *ab, double *x, double *dz, NewtonState *state, int update,
                     hipStream_t st);
hipError_t launch_mixed(int n, double *ab_dd, double *x, double *work, NewtonState *state, int max_refine,
                        hipStream_t st);

}  // namespace qdp
