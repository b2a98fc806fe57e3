/* qdpath: Newton corrector and path tracker for polynomial homotopies in
 * double-double and quad-double complex arithmetic on AMD Instinct MI355X
 * (gfx950).
 *
 * The operations follow Verschelde & Yoffe, "Quality Up in Polynomial
 * Homotopy Continuation by Multithreaded Path Tracking" (2011):
 *   - path tracking (Algorithm 3.1): given h(x,t) = 0 and a start solution z
 *     at t = 0, return z with h(z,1) = 0, or fail;
 *   - Newton's method (Algorithm 4.1): given h, z, epsilon and Max_It,
 *     return z with ||h(z,t)|| < epsilon, or fail;
 *   - evaluation (Section 4, array Y; Section 6): every polynomial value and
 *     every partial derivative at a point.
 *
 * Conventions for every call:
 *   - A complex multiword number is stored as [2][L] doubles: the L limbs of
 *     the real part, largest first, then the L limbs of the imaginary part;
 *     its value is the exact sum of the limbs.  L = 1 (double), 2 (double
 *     double), 4 (quad double): the qdp_prec value IS L.
 *   - Arrays are row-major with the complex number innermost.
 *   - Functions without the _dev suffix take host pointers and return after
 *     the GPU work finished.  _dev functions take device pointers (HIP device
 *     memory, e.g. torch.Tensor.data_ptr() of a CUDA/HIP tensor) and only
 *     enqueue work on hip_stream (NULL = the default stream).
 *   - The caller owns every buffer passed in; handles own their device data.
 *   - Every function returns a qdp_status; no exception crosses the ABI.
 *     qdp_last_error() returns the message of the last failure on the calling
 *     thread.  Numerical failure (Newton not converging, a zero pivot, a path
 *     that stops before t = 1) is NOT an error status: it is reported in the
 *     info / stats structs with QDP_OK, as the paper's "or fail" outputs.
 *   - A handle's device workspace is shared by all calls on that handle:
 *     calls on one handle from different streams must be ordered by the
 *     caller; different handles are independent.
 */
#ifndef QDPATH_H
#define QDPATH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum { QDP_F64 = 1, QDP_DD = 2, QDP_QD = 4 } qdp_prec;

typedef enum {
  QDP_OK = 0,
  QDP_EINVAL = 1,      /* bad argument: size, pointer, precision, exponent range */
  QDP_ENOMEM = 2,      /* device allocation failed */
  QDP_EDEVICE = 3,     /* a HIP runtime error */
  QDP_ENONFINITE = 4,  /* NaN or Inf in an input */
  QDP_EUNSUPPORTED = 5 /* a valid request this build does not implement */
} qdp_status;

typedef enum { QDP_SOLVE_FULL = 0, QDP_SOLVE_MIXED_IR = 1 } qdp_solve;
typedef enum { QDP_PRED_SECANT = 0, QDP_PRED_LEARNED = 1, QDP_PRED_QUADRATIC = 2 } qdp_pred;
typedef enum { QDP_ELIM_AUTO = 0, QDP_ELIM_POINT = 1, QDP_ELIM_COLUMNS = 2, QDP_ELIM_BLOCKS = 3 } qdp_elim;

typedef struct qdp_system qdp_system;
typedef struct qdp_homotopy qdp_homotopy;

/* Upload a sparse system f of n polynomials in n variables (Section 6: each
 * polynomial is a sum of normalized monomials c x^a).
 *   n            : 1 <= n <= 256 (quad double: n <= 128)
 *   poly_offsets : [n+1] int32, poly_offsets[0] = 0, nondecreasing; the terms of
 *                  polynomial i are poly_offsets[i] .. poly_offsets[i+1]-1
 *   exps         : [terms][n] uint8 exponents (0 = variable absent)
 *   coefs        : [terms][2][prec] doubles
 *   prec         : limbs stored; the system can later be evaluated at this or
 *                  any lower precision (limbs are truncated), never higher
 * Common support (the workload of Table 1): when n >= 2, every polynomial
 * has exactly f_0's exponent rows in the same order and the M monomials'
 * partials of one point take at most 8 MiB (M (n+1) 2 prec doubles), every evaluation of the
 * system forms the partials and values of those M monomials once per point and
 * multiplies by the n x M coefficient matrix (a dense complex product); the
 * results are those of the sparse evaluation up to rounding order.  The
 * system then holds a scratch for one point: evaluation calls on one such
 * system (qdp_eval_jacobian*, qdp_eval_homotopy*) must not overlap.
 * Errors: QDP_EINVAL (sizes, offsets, a polynomial without terms, the power
 * table n*(max exponent+1) beyond the LDS budget), QDP_ENONFINITE (a
 * coefficient limb), QDP_ENOMEM / QDP_EDEVICE. */
qdp_status qdp_system_create(int32_t n, const int32_t *poly_offsets, const uint8_t *exps,
                             const double *coefs, qdp_prec prec, qdp_system **out);
void qdp_system_destroy(qdp_system *f);

/* The total-degree homotopy h(x,t) = t f(x) + (1-t) gamma g(x) with
 * g_i = x_i^(d_i) - 1, d_i the total degree of f_i (the paper writes only
 * h(x,t); this is the homotopy of the path-tracking workloads).
 *   gamma : [2][prec of f] doubles; the homotopy keeps a reference to f. */
qdp_status qdp_homotopy_create(const qdp_system *f, const double *gamma, qdp_homotopy **out);
void qdp_homotopy_destroy(qdp_homotopy *h);

/* Evaluate f and its Jacobian at x (Section 4, array Y).
 *   x   : [n][2][prec]
 *   y   : [n][2][prec] out, y[i] = f_i(x)
 *   jac : [n][n][2][prec] out, jac[i][v] = d f_i / d x_v
 * prec must not exceed the system's stored precision. */
qdp_status qdp_eval_jacobian(const qdp_system *f, const double *x, qdp_prec prec, double *y, double *jac,
                             void *hip_stream);
qdp_status qdp_eval_jacobian_dev(const qdp_system *f, const double *x, qdp_prec prec, double *y, double *jac,
                                 void *hip_stream);

/* Evaluate h(x,t), its Jacobian in x, and the componentwise scale
 *   scale[i] = |t| sum_j |c_ij x^a_ij| + |(1-t) gamma| (|x_i|^(d_i) + 1)   (FP64, nullable). */
qdp_status qdp_eval_homotopy(const qdp_homotopy *h, double t, const double *x, qdp_prec prec, double *y,
                             double *jac, double *scale, void *hip_stream);
qdp_status qdp_eval_homotopy_dev(const qdp_homotopy *h, double t, const double *x, qdp_prec prec, double *y,
                                 double *jac, double *scale, void *hip_stream);
/* The same at B points in one launch (device memory, asynchronous): x [B][n][2][L],
 * y [B][n][2][L], jac [B][n][n][2][L], scale [B][n] (nullable), point b's block
 * following point b-1's.  The monomials of a polynomial may be split over several
 * workgroups whose partial sums are added in a fixed order: results are
 * reproducible for a given (system, B) but may differ in the last bits from
 * qdp_eval_homotopy_dev, which uses one workgroup per polynomial.  Uses scratch
 * memory of h (allocated on first use or growth of B, which synchronises the
 * device): calls on one h must not overlap.  1 <= B <= 65536. */
qdp_status qdp_eval_homotopy_batch_dev(const qdp_homotopy *h, double t, const double *x, int32_t B,
                                       qdp_prec prec, double *y, double *jac, double *scale, void *hip_stream);

typedef struct {
  int32_t iterations;   /* Newton iterations run */
  int32_t success;      /* residual < eps at exit (Algorithm 4.1: fail := residual >= eps) */
  int32_t singular;     /* a zero pivot stopped the elimination */
  int32_t nonfinite;    /* NaN/Inf met in the residual */
  double residual_first;/* residual at the input point */
  double residual_last; /* residual at the last evaluated point (before its update) */
  double cond_est;      /* max/min pivot magnitude of the last elimination */
  double dz_norm;       /* ||dz||_inf (leading limbs) of the last correction */
  double refine_err;    /* MIXED_IR: relative size of the last refinement correction */
  int32_t refine_steps; /* MIXED_IR: refinements in the last solve */
  int32_t pad;
} qdp_newton_info;

/* Newton's method at fixed t (Algorithm 4.1): residual initialised to 1;
 * while residual > eps and iterations < max_it: evaluate h and J at x,
 * residual := max_i |h_i|_1 / max_i scale_i, solve J dx = -h by Gaussian
 * elimination with partial pivoting, x := x + dx.  The residual uses
 * |Re| + |Im| of the leading limbs.
 *   x    : [n][2][prec] in/out
 *   mode : QDP_SOLVE_FULL eliminates in working precision; QDP_SOLVE_MIXED_IR
 *          factors an FP64 copy of J and refines the correction against the
 *          working-precision residual (double or quad double, n <= 128;
 *          QDP_EUNSUPPORTED otherwise).
 * info may be NULL.  max_it >= 0; eps >= 0. */
qdp_status qdp_newton_step(const qdp_homotopy *h, double t, double *x, qdp_prec prec, qdp_solve mode,
                           double eps, int32_t max_it, qdp_newton_info *info, void *hip_stream);
/* Same with x in device memory; asynchronous; read info with qdp_homotopy_last_info. */
qdp_status qdp_newton_step_dev(const qdp_homotopy *h, double t, double *x, qdp_prec prec, qdp_solve mode,
                               double eps, int32_t max_it, void *hip_stream);
/* For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid allocation): qdp_newton_step_dev
 * with its whole workspace ([A | -h], scales, state, split-evaluation partial
 * rows, common-support partials, FP64 factors or the column-parallel
 * elimination's multipliers and flags, of one point) in a static device
 * array of 8 MiB per GPU instead of the homotopy's allocated workspace; it calls
 * no allocating routine.  Results are bit for bit those of qdp_newton_step_dev.
 *   x        : [n][2][prec] device memory, in/out
 *   info_dev : nullable; device memory receiving one qdp_newton_info when the
 *              call's kernels have run (read it after synchronising the stream)
 * QDP_EINVAL (before any launch) when the system needs more than the 8 MiB (for
 * example double double at n > 128); the message states the sizes.  Every call on
 * one GPU shares its array: calls that overlap on a GPU (several streams or
 * threads) race.  Timing (qdp_set_timing) is not recorded for this entry point.
 * The array's address is taken on the first call on each device, which must be
 * current then. */
qdp_status qdp_newton_step_noalloc_dev(const qdp_homotopy *h, double t, double *x, qdp_prec prec, qdp_solve mode,
                                       double eps, int32_t max_it, qdp_newton_info *info_dev, void *hip_stream);
/* Synchronise hip_stream and return the info of the last Newton call on h at precision prec
 * (of its first point for a batch call). */
qdp_status qdp_homotopy_last_info(const qdp_homotopy *h, qdp_prec prec, qdp_newton_info *info, void *hip_stream);
/* Algorithm 4.1 at B independent points of the same homotopy and t (B paths at
 * one value of the parameter), x [B][n][2][L] in device memory, updated in place;
 * each point runs its own loop (own residual test and iteration count).  One
 * launch per kernel covers all points; asynchronous.  Calls on one h must not
 * overlap.  1 <= B <= 65536. */
qdp_status qdp_newton_batch_dev(const qdp_homotopy *h, double t, double *x, int32_t B, qdp_prec prec,
                                qdp_solve mode, double eps, int32_t max_it, void *hip_stream);
/* Synchronise and return info[0..B-1] of the last Newton call on h at precision prec. */
qdp_status qdp_homotopy_last_info_batch(const qdp_homotopy *h, qdp_prec prec, int32_t B, qdp_newton_info *info,
                                        void *hip_stream);

/* ---- learned step control (a growth direction of the tracker, not in the paper) ----
 * A step-size network: widths w_0 (features) .. w_last (outputs), ReLU hidden
 * layers; parameters are FP32, flat: for each layer its weights [out][in]
 * (row-major) then its bias [out].  Outputs 0 .. w_last-2 are logits of
 * "a step of lambda * 2^(k-1) would be accepted" (k = 0..w_last-2); the last
 * output is the weight of the quadratic predictor against the secant.  Training loss,
 * over a batch of B rows with targets Y and a 0/1 mask M (both [B][w_last]):
 *   (1/B) sum_b [ sum_{k<last} M_bk BCE(o_bk, Y_bk) + M_b,last (o_b,last - Y_b,last)^2 ]. */
typedef struct qdp_policy qdp_policy;

/* n_widths in [2, 9], widths in [1, 256], at least two outputs; params (host) FP32 in the flat
 * layout; feat_mean / feat_std [w_0] (host) normalise raw features as (x - mean) / std (std > 0).
 * Adam moments start at zero. */
qdp_status qdp_policy_create(int32_t n_widths, const int32_t *widths, const float *params,
                             const float *feat_mean, const float *feat_std, qdp_policy **out);
void qdp_policy_destroy(qdp_policy *p);
/* Synchronises the device and copies the FP32 parameters to host memory. */
qdp_status qdp_policy_get_params(const qdp_policy *p, float *params);
/* Write the network to a file: widths, FP32 parameters and the feature
 * normalisation (not the Adam moments); little-endian binary with an 8-byte
 * tag.  QDP_EINVAL if the file cannot be written. */
qdp_status qdp_policy_save(const qdp_policy *p, const char *path);
/* Create a network from a file written by qdp_policy_save (as qdp_policy_create;
 * Adam moments start at zero).  QDP_EINVAL for a missing or malformed file. */
qdp_status qdp_policy_load(const char *path, qdp_policy **out);
/* Loss and gradient of a batch (device pointers X [B][w_0] raw features, Y, M [B][w_last]).
 * grad_out: device [n_params] or NULL (kept internally for qdp_policy_adam_step); loss_out: host
 * or NULL (non-NULL synchronises the stream).  1 <= B <= 65536. */
qdp_status qdp_policy_gradient(qdp_policy *p, const float *X, const float *Y, const float *M, int32_t B,
                               float *grad_out, float *loss_out, void *hip_stream);
/* One Adam step with bias correction: m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
 * p -= lr (m/(1-b1^t)) / (sqrt(v/(1-b2^t)) + eps); grad NULL uses the last internal gradient. */
qdp_status qdp_policy_adam_step(qdp_policy *p, const float *grad, float lr, float b1, float b2, float eps,
                                void *hip_stream);
/* qdp_policy_gradient followed by qdp_policy_adam_step. */
qdp_status qdp_policy_train_step(qdp_policy *p, const float *X, const float *Y, const float *M, int32_t B,
                                 float lr, float b1, float b2, float eps, float *loss_out, void *hip_stream);
/* Inference of B rows (device X raw features, Y outputs): use_bf16 != 0 uses the parameters
 * rounded to BF16 (round to nearest even), else FP32; accumulation in FP32. */
qdp_status qdp_policy_forward(const qdp_policy *p, const float *X, int32_t B, int32_t use_bf16, float *Y,
                              void *hip_stream);
/* One row from host features to host outputs with BF16 weights (synchronous). */
qdp_status qdp_policy_infer_host(const qdp_policy *p, const float *x, float *y, void *hip_stream);

typedef struct {
  double lambda0;       /* initial step size */
  double lambda_min;    /* stop when the step size falls below this */
  double lambda_max;    /* largest step size */
  double shrink;        /* step factor after a failed correction (step back) */
  double expand;        /* step factor after expand_after consecutive successes */
  int32_t expand_after;
  int32_t max_it_path;  /* Newton iterations per correction along the path */
  double eps_path;      /* Newton residual tolerance along the path */
  double eps_end;       /* residual tolerance of the end refinement at t = 1 (0: 64 * 2^(-53 L)) */
  int32_t max_it_end;   /* Newton iterations of the end refinement */
  int32_t predictor;    /* qdp_pred */
  int64_t max_steps;    /* stop after this many corrections */
  int32_t mode;         /* qdp_solve */
  int32_t probe;        /* data collection: at every accepted state, also try the step multipliers
                           2^-1..2^3 (quadratic predictor) and log a probe record (kind 1) per
                           state; the path itself follows the plain rule */
  const qdp_policy *policy; /* learned step control (QDP_PRED_LEARNED), else NULL */
  double lambda_max_learned; /* cap of the learned step size (0: 4 * lambda_max) */
  double accept_threshold;   /* smallest acceptance probability a proposed multiplier may have (0: 0.3) */
  int32_t policy_rule;       /* 0: the multiplier of largest expected progress p_k 2^(k-1) among those
                                with p_k >= accept_threshold; 1: the largest multiplier with
                                p_k >= accept_threshold */
  int32_t pad2;
} qdp_track_params;

typedef struct {
  int32_t fail;              /* stopped with t < 1 */
  int32_t end_success;       /* the end refinement met eps_end */
  double t_final;
  int64_t succ_corrections;  /* accepted corrector stages */
  int64_t corrections;       /* all corrector stages */
  int64_t newton_iterations;
  double avg_step;           /* mean accepted step size */
  double min_step;           /* smallest accepted step size */
  double seconds;            /* wall time of the call */
  double end_residual;       /* residual of the last end-refinement iteration */
  int64_t policy_used;       /* steps whose size came from the learned policy */
  int64_t policy_rejected;   /* learned proposals the Newton test rejected */
  int64_t log_count;         /* records written to step_log */
  int64_t probe_corrections; /* corrector stages spent on probes (probe mode) */
} qdp_track_stats;

/* Fill p with the default step-size control (lambda0 0.01, halving on failure,
 * doubling after 3 successes up to 0.08, lambda_min 0.01*2^-30, eps_path 1e-10,
 * 4 Newton iterations per correction, 10 at the end, secant predictor, full
 * working-precision solve, no probing; learned cap 0.32, expected-progress rule with
 * probability floor 0.3). */
qdp_status qdp_track_params_default(qdp_track_params *p);

/* Number of features of the learned step controller (the network's w_0). */
#define QDP_POLICY_FEATURES 16
/* Number of step multipliers it scores: 2^-1, 2^0, 2^1, 2^2, 2^3. */
#define QDP_POLICY_MULTIPLIERS 5

/* One record written by qdp_track_path when step_log is not NULL. */
typedef struct {
  double t;          /* t before the step */
  double lambda;     /* kind 0: step size tried; kind 1: the base step size of the multipliers */
  double rho_first;  /* Newton residual at the predicted point */
  double rho_last;   /* last Newton residual */
  double dz_first;   /* ||dz||_inf of the first Newton iteration (the predictor's error) */
  double cond_est;
  double znorm;      /* ||z||_inf before the step */
  double pred_dist;  /* ||z_pred - z||_inf */
  double blend_label;/* kind 1: least-squares weight of the quadratic predictor against the secant for
                        the 2^0 step (NaN when that step failed or fewer than 3 points exist) */
  float features[QDP_POLICY_FEATURES]; /* the learned controller's inputs in this state */
  int32_t iterations;
  int32_t accepted;
  int32_t kind;      /* 0: a corrector stage of the path; 1: a probe record (no step taken) */
  int32_t probe_ok;  /* kind 1: bit k set when the step lambda * 2^(k-1) converged, k = 0..4 */
} qdp_step_record;

/* Track one path from t = 0 to t = 1 (Algorithm 3.1): predict (secant
 * predictor: linear extrapolation through the last two accepted points;
 * quadratic predictor (Section 5): per coordinate, the parabola through the
 * last three accepted points evaluated at the new t; before enough points,
 * the lower-order one, and constant before the second point), correct with Newton at the new t, control
 * the step size (step back and shrink on failure, expand after successes),
 * stop when the step is below lambda_min or after max_steps corrections; at
 * t = 1 refine the endpoint.  fail = (t < 1 at exit).
 * With predictor = QDP_PRED_LEARNED and a policy, after every accepted step the
 * network scores the multipliers 2^-1..2^3 of the last accepted step size (acceptance
 * probabilities p_k); the multiplier chosen by policy_rule is tried (capped by
 * lambda_max_learned and 1 - t; 2^-1 when no multiplier qualifies) with the predictor
 * (1 - w) secant + w quadratic, w the network's last output clamped to [-0.5, 1.5].
 * The Newton test judges: a failed correction steps back and falls back to the
 * plain rule (shrink, quadratic predictor) until the next success.
 *   x        : [n][2][prec] in: start solution at t = 0; out: end point
 *   step_log : NULL, or room for log_cap records; records are written in order
 *              (corrector stages, plus probe records in probe mode) until full */
qdp_status qdp_track_path(const qdp_homotopy *h, double *x, qdp_prec prec, const qdp_track_params *p,
                          qdp_track_stats *st, qdp_step_record *step_log, int64_t log_cap, void *hip_stream);

/* Track B paths of one homotopy together (Algorithm 3.1 for each): x [B][n][2][prec]
 * host memory, in: start solutions, out: end points; stats [B].  Every round
 * predicts and corrects all unfinished paths with one launch per kernel, each
 * path at its own t with its own step size, predictor history and Newton loop;
 * step-size control, stop criterion and end refinement are those of
 * qdp_track_path, path by path.  Plain control only: predictor SECANT or
 * QUADRATIC (else QDP_EUNSUPPORTED), no probe mode.  stats[b].seconds is the
 * time of the whole call.  Calls on one h must not overlap.  1 <= B <= 65536. */
qdp_status qdp_track_paths(const qdp_homotopy *h, double *x, int32_t B, qdp_prec prec, const qdp_track_params *p,
                           qdp_track_stats *stats, void *hip_stream);

/* Multiword arithmetic test entry: out[i] = op(a[i], b[i], c[i]) for
 * count elements on the GPU (device pointers, asynchronous).  Real ops take
 * [L] doubles per element, complex ops [2][L].
 * op: 0 add, 1 sub, 2 mul, 3 div (real); 10 cadd, 11 csub, 12 cmul, 13 cdiv,
 *     14 cfms (a - b*c), 15 cinv (1/a);
 *     16 the elimination's pivot search: a complex, count a multiple of 64; for
 *        each group of 64, out[i][0] = index in the group of the largest
 *        |Re| + |Im| of the leading limbs (keys equal in their leading 32 bits
 *        tie, the lowest index wins; -1 when every key is zero or NaN). */
qdp_status qdp_arith_batch(int32_t op, qdp_prec prec, int64_t count, const double *a, const double *b,
                           const double *c, double *out, void *hip_stream);

/* How the working-precision elimination of Section 4 (GE with partial
 * pivoting and Back_Subs) is laid out on the GPU, process-wide, for
 * QDP_SOLVE_FULL Newton calls made after this one:
 *   QDP_ELIM_POINT   one workgroup per point (the matrix in that workgroup's
 *                    registers, LDS or global memory);
 *   QDP_ELIM_COLUMNS one single-wavefront workgroup per column of [A | -h],
 *                    the pivot columns' multipliers passed through device
 *                    memory, for double and quad double, n <= 128 and
 *                    points x (n+1) <= 1024 (other calls: one per point);
 *   QDP_ELIM_BLOCKS  double double up to n = 128, quad double up to n = 64:
 *                    blocks of 16 columns per workgroup (the register
 *                    elimination inside a block, device memory between
 *                    blocks), points x blocks <= 128; other calls as
 *                    QDP_ELIM_COLUMNS;
 *   QDP_ELIM_AUTO    (default) blocks for double double at 48 < n <= 128 and
 *                    for quad double up to n = 64; columns for quad double
 *                    past n = 64; one per point elsewhere (and wherever the
 *                    chosen layout's limits are exceeded).
 * Blocks and columns give bit for bit the same results, and so does one per
 * point where it is the register kernel (double double, n <= 64); elsewhere
 * one per point compares pivot magnitudes in full and may order near ties
 * differently.
 * QDP_EINVAL for another value. */
qdp_status qdp_set_elimination(int32_t policy);

/* Kernel timing with HIP events on the call's stream.  After
 * qdp_set_timing(1) (process-wide), every Newton iteration enqueued by
 * qdp_newton_step / _dev records an event before the evaluation kernel,
 * between it and the elimination kernel, and after the elimination.
 * qdp_homotopy_last_timing synchronises hip_stream and returns, for the last
 * Newton call on h at precision prec, the summed milliseconds of all
 * evaluation launches and of all elimination launches, and the number of
 * iterations timed (launches of each). */
qdp_status qdp_set_timing(int32_t on);
qdp_status qdp_homotopy_last_timing(const qdp_homotopy *h, qdp_prec prec, double *eval_ms, double *solve_ms,
                                    int32_t *launches, void *hip_stream);

const char *qdp_last_error(void);
const char *qdp_version(void);

#ifdef __cplusplus
}
#endif

#endif /* QDPATH_H */
