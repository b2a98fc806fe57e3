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
  int supp;                // common support: every polynomial has the same M = supp exponent
                           // rows (those of f_0); 0 otherwise
};

// Where evaluation results go.  All strides count doubles.  Limb c of the
// complex element J(i,v) of point b (c < L real limbs, then L imaginary
// limbs) sits at J[b*bJ + c*psJ + i*rsJ + v*csJ]; limb c of value i at
// y[b*by + c*psy + i*sy] (times ysign); scale_i -> scale[b*bS + i] (nullable).
struct EvalOut {
  double *J;
  long psJ, rsJ, csJ;
  double *y;
  long psy, sy;
  double ysign;
  double *scale;
  long bJ, by, bS;
};

// Monomial split of the evaluation: with part != nullptr the monomials of a
// polynomial may be spread over up to max_parts workgroups, whose partial
// rows ([B][n][parts] records of (n+1) complex values and one scale sum) a
// second kernel adds in part order.  part == nullptr: one workgroup per
// polynomial.
struct EvalSplit {
  double *part;
  int max_parts;
  double *supp_v;  // common-support systems: scratch for the monomial partials of
  int supp_cap;    // up to supp_cap points (eval_supp_doubles each); required there
};
constexpr int kMaxEvalParts = 8;

// Column-parallel elimination (one workgroup per column of each point): ws
// holds B per-point workspaces of ge_mc_doubles(L, n), epoch tags this
// launch's flags.  ws == nullptr: one workgroup per point.
struct GeMc {
  double *ws;
  unsigned epoch;
  int blocks;  // 1: blocks of columns per workgroup (double double, n <= 64)
};

// Per-point workspace of the column-parallel elimination, in doubles
// (RMAX = 64 rows per lane slot, 128 past n = 64):
//   mult [n][2L][RMAX]  multipliers of each column
//   tri  [2L][TT]       scaled U packed by columns (column c: pivot-order
//                       rows 0..c-1 at c(c-1)/2), TT = n(n-1)/2 + 1
//   invp [2L][RMAX]     pivot inverses by column
//   pmag [RMAX]         |Re|+|Im| of each pivot's leading limb
//   ctl  [RMAX]         int2: pivot row, zero-pivot flag
//   pub  [RMAX]         u64 flag: column published
//   fin  [RMAX]         u64 flag: column's triangle stored (or failed)
__host__ __device__ inline int mc_rows(int n) { return n <= 64 ? 64 : 128; }
__host__ __device__ inline size_t mc_tri_doubles(int n) { return (size_t)n * (n - 1) / 2 + 1; }
__host__ __device__ inline size_t ge_mc_doubles(int L, int n) {
  const size_t R = (size_t)mc_rows(n), E2 = 2 * (size_t)L;
  const size_t d = (size_t)n * E2 * R + E2 * mc_tri_doubles(n) + E2 * R + 4 * R;
  return (d + 31) & ~(size_t)31;
}

// Homotopy h = t f + (1-t) gamma (x^d - 1); homotopy = 0 evaluates f alone.
struct HomArgs {
  int homotopy;
  double t;
  double gamma[8];     // [re limbs][im limbs] at the compute L (first 2L used)
  const double *tb;    // [B] t of each point (device), or nullptr: t for every point
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

// What the tracker reads back after a corrector stage, gathered on the device
// into one record so that one copy brings it to (pinned) host memory.
struct StageReadback {
  NewtonState st;
  double aux[4];   // predictor distance, blend-label sums
  float pout[8];   // the step-size network's outputs (learned control)
};

// Launchers (defined per translation unit; return hipError_t).  A launch
// covers B independent points: x holds B points bx doubles apart, gate B
// Newton states (nullable).
hipError_t launch_eval(int L, const DevSystem &s, const double *x, long bx, int B, const HomArgs &h,
                       const EvalOut &o, const NewtonState *gate, const EvalSplit &split, hipStream_t st);
// Doubles of partial-row scratch a split evaluation of B points needs.
size_t eval_part_doubles(int L, int n, int B);
// Doubles of monomial-partial scratch per point of a common-support system:
// V [M][2L limb planes][n+1] (the partials and value of every support
// monomial), then the start-system powers x_i^(d_i - 1), x_i^(d_i) of every
// row ([n][2][2L]).
__host__ __device__ inline size_t supp_pow_offset(int M, int n, int L) { return (size_t)M * 2 * L * (n + 1); }
__host__ __device__ inline size_t supp_v_doubles(int M, int n, int L) {
  return supp_pow_offset(M, n, L) + (size_t)n * 4 * L;
}
size_t eval_supp_doubles(int L, int n, int supp);

}  // namespace qdp
