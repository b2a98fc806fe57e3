// C-ABI of the HIP path: handles, validation, device workspace, the Newton
// loop of Algorithm 4.1 as a fixed sequence of gated kernels, and the path
// tracker of Algorithm 3.1.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/qdpath.h"
#include "common.hpp"
#include "ctl_features.hpp"

namespace qdp {
hipError_t launch_ge_scaled(int L, int n, int B, double *ab, double *scale, double *x, double *dz, NewtonState *st,
                            double *mc_ws, hipStream_t s);
void set_ge_policy(int p);
bool ge_mc_possible(int L, int n, int B);
hipError_t launch_arith(int op, int L, int64_t count, const double *a, const double *b, const double *c,
                        double *out, hipStream_t s);
hipError_t launch_init_state(NewtonState *st, int B, double eps, int max_it, const int *mask, hipStream_t s);
hipError_t launch_predict_batch(int L, int n, int B, const double *x, const double *xp, const double *xpp,
                                const double *cf, const int *mask, double *xw, hipStream_t s);
hipError_t launch_accept_batch(int L, int n, int B, const int *acc, double *x, double *xp, double *xpp,
                               const double *xw, hipStream_t s);
hipError_t launch_predict(int L, int n, const double *x, const double *xprev, const double *xprev2, double c1,
                          double c2, double *xpred, double *aux, hipStream_t s);
hipError_t launch_blend_label(int L, int n, const double *x, const double *xprev, const double *xprev2,
                              const double *xcorr, double s1, double q1, double q2, double *aux, hipStream_t s);
hipError_t launch_copy(double *dst, const double *src, size_t count, hipStream_t s);
hipError_t launch_ctl_features(const CtlFeatIn &h, const NewtonState *st, const double *aux, float *f,
                               hipStream_t s);
hipError_t launch_stage_readback(const NewtonState *st, const double *aux, const float *pout, StageReadback *rb,
                                 hipStream_t s);
hipError_t launch_mixed_solve(int L, int n, int B, const double *ab, const double *scale, double *x,
                              NewtonState *st, double *lu, int refinements, hipStream_t s);
size_t mixed_ws_doubles(int n);
}  // namespace qdp

using qdp::DevSystem;
using qdp::NewtonState;

// ------------------------------------------------------------------ errors

static thread_local std::string g_err;
// mixed precision (FP64 factorization + refinement): double and quad double
// working precision, n up to the register kernel's 128 rows
static bool mixed_supported(int L, int n) { return (L == 2 || L == 4) && n >= 1 && n <= 128; }
// refinements per correction: each gains about 16 - log10(kappa) digits
static int mixed_refinements(int L) { return L == 4 ? 6 : 3; }
static int g_timing = 0;

static qdp_status fail(qdp_status s, const std::string &msg) {
  g_err = msg;
  return s;
}
#define HIPCHK(expr)                                                                     \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess)                                                                \
      return fail(QDP_EDEVICE, std::string(#expr ": ") + hipGetErrorString(e_));          \
  } while (0)

extern "C" const char *qdp_last_error(void) { return g_err.c_str(); }

namespace qdp {
qdp_status set_error(qdp_status s, const std::string &msg) { return fail(s, msg); }
}  // namespace qdp
extern "C" const char *qdp_version(void) { return "qdpath 0.1 (gfx950)"; }

static bool valid_prec(int p) { return p == 1 || p == 2 || p == 4; }

// ------------------------------------------------------------------ handles

struct qdp_system {
  int n = 0, L = 0, terms = 0, emax = 0, maxm = 0, npad = 0;
  std::vector<int32_t> deg;
  int supp = 0;  // common support: M monomials shared by every polynomial (0: not common)
  int32_t *d_offsets = nullptr, *d_deg = nullptr;
  uint8_t *d_exps = nullptr;
  double *d_coefs = nullptr;
  double *d_suppv = nullptr;  // common support: monomial partials of one point (eval entry points)
  DevSystem dev() const {
    return DevSystem{n, terms, L, npad, emax, maxm, d_offsets, d_exps, d_coefs, d_deg, supp};
  }
};

struct Workspace {
  int L = 0;
  int bcap = 0;             // points the batch-sized buffers hold
  double *ab = nullptr;     // [bcap] (n+1) x n column-major [A | -h]
  double *scale = nullptr;  // [bcap][n]
  double *part = nullptr;   // split-evaluation partial rows (EvalSplit)
  double *suppv = nullptr;  // [bcap] common-support monomial partials (EvalSplit)
  double *x = nullptr;      // [n] point (compute precision)
  double *xprev = nullptr;  // [n] previous accepted point
  double *xprev2 = nullptr; // [n] the accepted point before that
  double *xw = nullptr;     // [n] working point (predicted / corrected)
  double *y = nullptr;      // [n] values (eval entry points)
  double *jac = nullptr;    // [n][n] Jacobian (eval entry points)
  double *lu = nullptr;     // [bcap] mixed precision: FP64 factors
  double *mc = nullptr;     // [mc_cap] column-parallel elimination workspaces
  int mc_cap = 0;
  NewtonState *st = nullptr;  // [bcap]
  double *aux = nullptr;       // [4] predictor distance, blend-label sums
  float *pfeat = nullptr;      // [16] controller features, then [8] network outputs
  qdp::StageReadback *rb_dev = nullptr;   // a corrector stage's results, gathered
  qdp::StageReadback *rb_host = nullptr;  // pinned host copy of rb_dev
  std::vector<hipEvent_t> ev;  // timing: 3 events per iteration (before eval, between, after solve)
  int timed_its = 0;
};

struct qdp_homotopy {
  const qdp_system *f = nullptr;
  double gamma[8] = {0};  // [2][L of f]
  Workspace ws[3];        // by compute precision: L = 1, 2, 4
  std::mutex mu;
};

static int ws_index(int L) { return L == 1 ? 0 : (L == 2 ? 1 : 2); }

static void free_batch(Workspace &w) {
  hipFree(w.ab);
  hipFree(w.scale);
  hipFree(w.part);
  hipFree(w.suppv);
  hipFree(w.lu);
  hipFree(w.mc);
  hipFree(w.st);
  w.ab = w.scale = w.part = w.suppv = w.lu = w.mc = nullptr;
  w.st = nullptr;
  w.bcap = w.mc_cap = 0;
}

// Workspace of (h, L) able to hold B points; growing it waits for the device
// (earlier asynchronous work may still use the old buffers).
static qdp_status ensure_ws(qdp_homotopy *h, int L, int B, Workspace **out) {
  Workspace &w = h->ws[ws_index(L)];
  const int n = h->f->n;
  const size_t e = 2 * (size_t)L;
  if (!w.x) {
    HIPCHK(hipMalloc(&w.x, (size_t)n * e * sizeof(double)));
    HIPCHK(hipMalloc(&w.xprev, (size_t)n * e * sizeof(double)));
    HIPCHK(hipMalloc(&w.xprev2, (size_t)n * e * sizeof(double)));
    HIPCHK(hipMalloc(&w.xw, (size_t)n * e * sizeof(double)));
    HIPCHK(hipMalloc(&w.y, (size_t)n * e * sizeof(double)));
    HIPCHK(hipMalloc(&w.jac, (size_t)n * n * e * sizeof(double)));
    HIPCHK(hipMalloc(&w.aux, 4 * sizeof(double)));
    HIPCHK(hipMalloc(&w.pfeat, 24 * sizeof(float)));
    HIPCHK(hipMalloc(&w.rb_dev, sizeof(qdp::StageReadback)));
    HIPCHK(hipHostMalloc(&w.rb_host, sizeof(qdp::StageReadback), hipHostMallocDefault));
    w.L = L;
  }
  if (B > w.bcap) {
    if (w.bcap > 0) {
      HIPCHK(hipDeviceSynchronize());
      free_batch(w);
    }
    const size_t Bs = (size_t)B;
    HIPCHK(hipMalloc(&w.ab, Bs * n * (n + 1) * e * sizeof(double)));
    HIPCHK(hipMalloc(&w.scale, Bs * n * sizeof(double)));
    HIPCHK(hipMalloc(&w.st, Bs * sizeof(NewtonState)));
    const size_t pd = qdp::eval_part_doubles(L, n, B);
    if (pd > 0) HIPCHK(hipMalloc(&w.part, pd * sizeof(double)));
    if (h->f->supp > 0) HIPCHK(hipMalloc(&w.suppv, Bs * qdp::eval_supp_doubles(L, n, h->f->supp) * sizeof(double)));
    if (mixed_supported(L, n) && qdp::mixed_ws_doubles(n) > 0)
      HIPCHK(hipMalloc(&w.lu, Bs * qdp::mixed_ws_doubles(n) * sizeof(double)));
    if (qdp::ge_mc_possible(L, n, 1)) {
      int cap = B;
      while (cap > 1 && !qdp::ge_mc_possible(L, n, cap)) --cap;
      const size_t bytes = (size_t)cap * qdp::ge_mc_doubles(L, n) * sizeof(double);
      HIPCHK(hipMalloc(&w.mc, bytes));
      HIPCHK(hipMemset(w.mc, 0, bytes));
      w.mc_cap = cap;
    }
    w.bcap = B;
  }
  *out = &w;
  return QDP_OK;
}

static void free_ws(Workspace &w) {
  free_batch(w);
  hipFree(w.x);
  hipFree(w.xprev);
  hipFree(w.xprev2);
  hipFree(w.xw);
  hipFree(w.y);
  hipFree(w.jac);
  hipFree(w.aux);
  hipFree(w.pfeat);
  hipFree(w.rb_dev);
  hipHostFree(w.rb_host);
  for (auto &e : w.ev) hipEventDestroy(e);
  w = Workspace();
}

// LDS bytes of the evaluation kernel's two power tables (2L limb planes of
// [emax+1][n rounded up to 32] doubles each)
static size_t table_bytes(int n, int emax, int L) {
  return 2 * 2 * (size_t)L * (emax + 1) * (((size_t)n + 31) & ~(size_t)31) * sizeof(double);
}

extern "C" qdp_status qdp_system_create(int32_t n, const int32_t *off, const uint8_t *exps, const double *coefs,
                                        qdp_prec prec, qdp_system **out) {
  if (!out) return fail(QDP_EINVAL, "out is NULL");
  *out = nullptr;
  const int L = (int)prec;
  if (!valid_prec(L)) return fail(QDP_EINVAL, "prec must be 1, 2 or 4");
  if (n < 1 || n > 256) return fail(QDP_EINVAL, "n must be in [1, 256]");
  if (L == 4 && n > 128) return fail(QDP_EINVAL, "quad double supports n <= 128");
  if (!off || !exps || !coefs) return fail(QDP_EINVAL, "NULL input array");
  if (off[0] != 0) return fail(QDP_EINVAL, "poly_offsets[0] must be 0");
  int maxm = 0;
  for (int i = 0; i < n; ++i) {
    if (off[i + 1] <= off[i]) return fail(QDP_EINVAL, "every polynomial needs at least one term");
    maxm = std::max(maxm, off[i + 1] - off[i]);
  }
  const int terms = off[n];
  if (terms > (1 << 26)) return fail(QDP_EINVAL, "too many terms");
  for (size_t q = 0; q < (size_t)terms * 2 * L; ++q)
    if (!std::isfinite(coefs[q])) return fail(QDP_ENONFINITE, "non-finite coefficient limb");
  auto *s = new qdp_system();
  s->n = n;
  s->L = L;
  s->terms = terms;
  s->maxm = maxm;
  int np = 8;
  while (np < n) np <<= 1;
  s->npad = np;
  std::vector<uint8_t> padded((size_t)terms * np, 0);
  int emax = 0;
  s->deg.assign(n, 0);
  for (int i = 0; i < n; ++i)
    for (int j = off[i]; j < off[i + 1]; ++j) {
      int tot = 0;
      for (int v = 0; v < n; ++v) {
        const uint8_t e = exps[(size_t)j * n + v];
        padded[(size_t)j * np + v] = e;
        emax = std::max(emax, (int)e);
        tot += e;
      }
      s->deg[i] = std::max(s->deg[i], tot);
    }
  s->emax = emax;
  // common support (n >= 2): every polynomial has f_0's exponent rows, in
  // the same order; then the monomial partials are formed once per point
  {
    const int M = off[1];
    bool common = n >= 2;
    for (int i = 1; i < n && common; ++i) {
      if (off[i + 1] - off[i] != M) {
        common = false;
        break;
      }
      common = std::memcmp(exps + (size_t)off[i] * n, exps, (size_t)M * n) == 0;
    }
    // and only while the partials of one point stay modest (the scratch is
    // per point: a batch of B points holds B of them)
    if (common && qdp::supp_v_doubles(M, n, L) * sizeof(double) > (size_t(8) << 20)) common = false;
    s->supp = common ? M : 0;
  }
  // the power tables of the evaluation kernel live in LDS; the reduction
  // area reuses the same space
  if (table_bytes(n, emax, L) > 150 * 1024) {
    delete s;
    return fail(QDP_EINVAL, "n * (max exponent + 1) too large for the LDS power table");
  }
  hipError_t e = hipSuccess;
  e = hipMalloc(&s->d_offsets, (n + 1) * sizeof(int32_t));
  if (e == hipSuccess) e = hipMalloc(&s->d_deg, n * sizeof(int32_t));
  if (e == hipSuccess) e = hipMalloc(&s->d_exps, padded.size());
  if (e == hipSuccess) e = hipMalloc(&s->d_coefs, (size_t)terms * 2 * L * sizeof(double));
  if (e == hipSuccess && s->supp > 0)
    e = hipMalloc(&s->d_suppv, qdp::eval_supp_doubles(L, n, s->supp) * sizeof(double));
  if (e == hipSuccess) e = hipMemcpy(s->d_offsets, off, (n + 1) * sizeof(int32_t), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(s->d_deg, s->deg.data(), n * sizeof(int32_t), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(s->d_exps, padded.data(), padded.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(s->d_coefs, coefs, (size_t)terms * 2 * L * sizeof(double), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    qdp_system_destroy(s);
    return fail(e == hipErrorOutOfMemory ? QDP_ENOMEM : QDP_EDEVICE, hipGetErrorString(e));
  }
  *out = s;
  return QDP_OK;
}

extern "C" void qdp_system_destroy(qdp_system *s) {
  if (!s) return;
  hipFree(s->d_offsets);
  hipFree(s->d_deg);
  hipFree(s->d_exps);
  hipFree(s->d_coefs);
  hipFree(s->d_suppv);
  delete s;
}

extern "C" qdp_status qdp_homotopy_create(const qdp_system *f, const double *gamma, qdp_homotopy **out) {
  if (!out || !f || !gamma) return fail(QDP_EINVAL, "NULL argument");
  for (int k = 0; k < 2 * f->L; ++k)
    if (!std::isfinite(gamma[k])) return fail(QDP_ENONFINITE, "non-finite gamma");
  auto *h = new qdp_homotopy();
  h->f = f;
  for (int k = 0; k < 2 * f->L; ++k) h->gamma[k] = gamma[k];
  *out = h;
  return QDP_OK;
}

extern "C" void qdp_homotopy_destroy(qdp_homotopy *h) {
  if (!h) return;
  for (auto &w : h->ws) free_ws(w);
  delete h;
}

// gamma truncated to L limbs: [re L][im L]
static qdp::HomArgs hom_args(const qdp_homotopy *h, int L, double t, int on) {
  qdp::HomArgs a{};
  a.homotopy = on;
  a.t = t;
  const int LS = h ? h->f->L : L;
  if (h)
    for (int k = 0; k < L; ++k) {
      a.gamma[k] = h->gamma[k];
      a.gamma[L + k] = h->gamma[LS + k];
    }
  return a;
}

// ------------------------------------------------------------------ evaluation

static qdp_status check_point(int n, int L, const double *x) {
  for (size_t q = 0; q < (size_t)n * 2 * L; ++q)
    if (!std::isfinite(x[q])) return fail(QDP_ENONFINITE, "non-finite point limb");
  return QDP_OK;
}

static qdp_status eval_common(const qdp_system *f, const qdp_homotopy *h, double t, const double *x_dev, int L,
                              double *y_dev, double *jac_dev, double *scale_dev, hipStream_t st) {
  if (!f) return fail(QDP_EINVAL, "NULL system");
  if (!valid_prec(L) || L > f->L) return fail(QDP_EINVAL, "prec must be 1, 2 or 4 and not above the system's");
  if (!x_dev || !y_dev || !jac_dev) return fail(QDP_EINVAL, "NULL buffer");
  // row-major [i][v][2][L] and [i][2][L]: limb c at offset c
  const long e = 2 * L;
  qdp::EvalOut o{jac_dev, 1, (long)f->n * e, e, y_dev, 1, e, 1.0, scale_dev, 0, 0, 0};
  // one workgroup per polynomial: no split scratch; a common-support system uses its own scratch
  const qdp::EvalSplit whole{nullptr, 1, f->d_suppv, 1};
  HIPCHK(qdp::launch_eval(L, f->dev(), x_dev, 0, 1, hom_args(h, L, t, h != nullptr), o, nullptr, whole, st));
  return QDP_OK;
}

extern "C" qdp_status qdp_eval_jacobian_dev(const qdp_system *f, const double *x, qdp_prec prec, double *y,
                                            double *jac, void *stream) {
  return eval_common(f, nullptr, 1.0, x, (int)prec, y, jac, nullptr, (hipStream_t)stream);
}

extern "C" qdp_status qdp_eval_homotopy_dev(const qdp_homotopy *h, double t, const double *x, qdp_prec prec,
                                            double *y, double *jac, double *scale, void *stream) {
  if (!h) return fail(QDP_EINVAL, "NULL homotopy");
  if (!std::isfinite(t)) return fail(QDP_ENONFINITE, "non-finite t");
  return eval_common(h->f, h, t, x, (int)prec, y, jac, scale, (hipStream_t)stream);
}

static qdp_status eval_host(const qdp_system *f, const qdp_homotopy *h, double t, const double *x, int L,
                            double *y, double *jac, double *scale, hipStream_t st) {
  if (!f || !x || !y || !jac) return fail(QDP_EINVAL, "NULL argument");
  if (!valid_prec(L) || L > f->L) return fail(QDP_EINVAL, "prec must be 1, 2 or 4 and not above the system's");
  qdp_status s = check_point(f->n, L, x);
  if (s != QDP_OK) return s;
  const int n = f->n;
  const size_t e = 2 * (size_t)L;
  double *dx = nullptr, *dy = nullptr, *dj = nullptr, *ds = nullptr;
  auto cleanup = [&]() {
    hipFree(dx);
    hipFree(dy);
    hipFree(dj);
    hipFree(ds);
  };
  hipError_t err = hipMalloc(&dx, n * e * sizeof(double));
  if (err == hipSuccess) err = hipMalloc(&dy, n * e * sizeof(double));
  if (err == hipSuccess) err = hipMalloc(&dj, (size_t)n * n * e * sizeof(double));
  if (err == hipSuccess && scale) err = hipMalloc(&ds, n * sizeof(double));
  if (err == hipSuccess) err = hipMemcpyAsync(dx, x, n * e * sizeof(double), hipMemcpyHostToDevice, st);
  if (err != hipSuccess) {
    cleanup();
    return fail(QDP_ENOMEM, hipGetErrorString(err));
  }
  s = eval_common(f, h, t, dx, L, dy, dj, ds, st);
  if (s == QDP_OK) {
    err = hipMemcpyAsync(y, dy, n * e * sizeof(double), hipMemcpyDeviceToHost, st);
    if (err == hipSuccess) err = hipMemcpyAsync(jac, dj, (size_t)n * n * e * sizeof(double), hipMemcpyDeviceToHost, st);
    if (err == hipSuccess && scale) err = hipMemcpyAsync(scale, ds, n * sizeof(double), hipMemcpyDeviceToHost, st);
    if (err == hipSuccess) err = hipStreamSynchronize(st);
    if (err != hipSuccess) s = fail(QDP_EDEVICE, hipGetErrorString(err));
  }
  cleanup();
  return s;
}

extern "C" qdp_status qdp_eval_jacobian(const qdp_system *f, const double *x, qdp_prec prec, double *y,
                                        double *jac, void *stream) {
  return eval_host(f, nullptr, 1.0, x, (int)prec, y, jac, nullptr, (hipStream_t)stream);
}

extern "C" qdp_status qdp_eval_homotopy(const qdp_homotopy *h, double t, const double *x, qdp_prec prec,
                                        double *y, double *jac, double *scale, void *stream) {
  if (!h) return fail(QDP_EINVAL, "NULL homotopy");
  if (!std::isfinite(t)) return fail(QDP_ENONFINITE, "non-finite t");
  return eval_host(h->f, h, t, x, (int)prec, y, jac, scale, (hipStream_t)stream);
}

// ------------------------------------------------------------------ Newton

// Enqueue max_it iterations of (evaluate h and J into [A | -h], eliminate and
// update).  Every kernel reads the device flag `active` first and returns at
// once when the loop of Algorithm 4.1 has ended, so the host never waits
// between iterations.
// tb (device, nullable): t of each point instead of t; mask (device, nullable):
// only points with mask[b] != 0 run.
static qdp_status enqueue_newton(qdp_homotopy *h, Workspace *w, int L, double t, double *x_dev, int B, int mode,
                                 double eps, int max_it, hipStream_t st, const double *tb = nullptr,
                                 const int *mask = nullptr, bool allow_timing = true) {
  const qdp_system *f = h->f;
  const int n = f->n;
  HIPCHK(qdp::launch_init_state(w->st, B, eps, max_it, mask, st));
  // [A | -h] column-major in limb planes: limb c of (r,k) at c*n(n+1) + k*n + r,
  // one such block per point
  const long ps = (long)n * (n + 1);
  const long pb = ps * 2 * L;
  qdp::EvalOut o{w->ab, ps, 1, n, w->ab + (size_t)n * n, ps, 1, -1.0, w->scale, pb, pb, n};
  const qdp::EvalSplit split{w->part, qdp::kMaxEvalParts, w->suppv, w->bcap};
  qdp::HomArgs ha = hom_args(h, L, t, 1);
  ha.tb = tb;
  const bool timing = g_timing != 0 && allow_timing;
  if (timing) {
    while (w->ev.size() < 3 * (size_t)max_it) {
      hipEvent_t e;
      HIPCHK(hipEventCreate(&e));
      w->ev.push_back(e);
    }
  }
  w->timed_its = timing ? max_it : 0;
  for (int it = 0; it < max_it; ++it) {
    if (timing) HIPCHK(hipEventRecord(w->ev[3 * it], st));
    HIPCHK(qdp::launch_eval(L, f->dev(), x_dev, (long)n * 2 * L, B, ha, o, w->st, split, st));
    if (timing) HIPCHK(hipEventRecord(w->ev[3 * it + 1], st));
    if (mode == QDP_SOLVE_MIXED_IR)
      HIPCHK(qdp::launch_mixed_solve(L, n, B, w->ab, w->scale, x_dev, w->st, w->lu, mixed_refinements(L), st));
    else
      HIPCHK(qdp::launch_ge_scaled(L, n, B, w->ab, w->scale, x_dev, nullptr, w->st, B <= w->mc_cap ? w->mc : nullptr,
                                   st));
    if (timing) HIPCHK(hipEventRecord(w->ev[3 * it + 2], st));
  }
  return QDP_OK;
}

static void info_from_state(const NewtonState &s, qdp_newton_info *info) {
  info->iterations = s.iterations;
  info->success = s.success;
  info->singular = s.singular;
  info->nonfinite = s.nonfinite;
  info->residual_first = s.rho_first;
  info->residual_last = s.rho;
  info->cond_est = s.cond_est;
  info->dz_norm = s.dz_norm;
  info->refine_err = s.refine_err;
  info->refine_steps = s.refine_steps;
  info->pad = 0;
}

static qdp_status newton_checks(const qdp_homotopy *h, double t, const double *x, int L, int mode, double eps,
                                int max_it) {
  if (!h || !x) return fail(QDP_EINVAL, "NULL argument");
  if (!valid_prec(L) || L > h->f->L) return fail(QDP_EINVAL, "prec must be 1, 2 or 4 and not above the system's");
  if (!std::isfinite(t)) return fail(QDP_ENONFINITE, "non-finite t");
  if (!(eps >= 0) || max_it < 0) return fail(QDP_EINVAL, "eps must be >= 0 and max_it >= 0");
  if (mode != QDP_SOLVE_FULL && mode != QDP_SOLVE_MIXED_IR) return fail(QDP_EINVAL, "bad solve mode");
  if (mode == QDP_SOLVE_MIXED_IR && !mixed_supported(L, h->f->n))
    return fail(QDP_EUNSUPPORTED, "mixed-precision refinement is implemented for double and quad double, n <= 128");
  return QDP_OK;
}

extern "C" qdp_status qdp_newton_step_dev(const qdp_homotopy *hc, double t, double *x, qdp_prec prec,
                                          qdp_solve mode, double eps, int32_t max_it, void *stream) {
  qdp_status s = newton_checks(hc, t, x, (int)prec, mode, eps, max_it);
  if (s != QDP_OK) return s;
  auto *h = const_cast<qdp_homotopy *>(hc);
  std::lock_guard<std::mutex> g(h->mu);
  Workspace *w = nullptr;
  if ((s = ensure_ws(h, (int)prec, 1, &w)) != QDP_OK) return s;
  return enqueue_newton(h, w, (int)prec, t, x, 1, mode, eps, max_it, (hipStream_t)stream);
}

// ---- Newton's method with no device allocation ---------------------------
//
// For callers that cannot allocate device memory (code under stream capture,
// tight serving loops): the Newton workspace of one point ([A | -h], scales,
// state, split-evaluation partial rows, common-support partials, FP64
// factors) lives in one static device array per GPU.  The array's address is
// taken once per device (with that device current) and kept; host code uses
// that address, never the array's name.  Every call on a GPU shares its array:
// calls that overlap on one GPU (other streams, other threads) race.
constexpr size_t kScratchDoubles = (size_t)1 << 20;  // 8 MiB
static __device__ __align__(256) double scratch[kScratchDoubles];
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static double *g_scratch_ptr[kMaxDevices] = {nullptr};

static qdp_status scratch_base(double **out) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(QDP_EDEVICE, "device index out of range");
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(QDP_EDEVICE, "no device address for the scratch array");
    g_scratch_ptr[dev] = static_cast<double *>(p);
  }
  *out = g_scratch_ptr[dev];
  return QDP_OK;
}

__global__ void k_info_from_state(const NewtonState *s, qdp_newton_info *info) {
  info->iterations = s->iterations;
  info->success = s->success;
  info->singular = s->singular;
  info->nonfinite = s->nonfinite;
  info->residual_first = s->rho_first;
  info->residual_last = s->rho;
  info->cond_est = s->cond_est;
  info->dz_norm = s->dz_norm;
  info->refine_err = s->refine_err;
  info->refine_steps = s->refine_steps;
  info->pad = 0;
}

// doubles of scratch one point of (h, L, mode) takes, each part rounded up to 32 doubles
static size_t scratch_need(const qdp_homotopy *h, int L, int mode, size_t *ab, size_t *scale, size_t *part,
                           size_t *suppv, size_t *lu, size_t *mc, size_t *st) {
  const int n = h->f->n;
  auto up = [](size_t d) { return (d + 31) & ~(size_t)31; };
  *ab = up((size_t)n * (n + 1) * 2 * L);
  *scale = up((size_t)n);
  *part = up(qdp::eval_part_doubles(L, n, 1));
  *suppv = h->f->supp > 0 ? up(qdp::eval_supp_doubles(L, n, h->f->supp)) : 0;
  *lu = mode == QDP_SOLVE_MIXED_IR ? up(qdp::mixed_ws_doubles(n)) : 0;
  *mc = mode == QDP_SOLVE_FULL && qdp::ge_mc_possible(L, n, 1) ? up(qdp::ge_mc_doubles(L, n)) : 0;
  *st = up((sizeof(NewtonState) + sizeof(double) - 1) / sizeof(double));
  return *ab + *scale + *part + *suppv + *lu + *mc + *st;
}

extern "C" qdp_status qdp_newton_step_noalloc_dev(const qdp_homotopy *hc, double t, double *x, qdp_prec prec,
                                                  qdp_solve mode, double eps, int32_t max_it,
                                                  qdp_newton_info *info_dev, void *stream) {
  qdp_status s = newton_checks(hc, t, x, (int)prec, mode, eps, max_it);
  if (s != QDP_OK) return s;
  const int L = (int)prec;
  size_t nab, nsc, npt, nsv, nlu, nmc, nst;
  const size_t need = scratch_need(hc, L, mode, &nab, &nsc, &npt, &nsv, &nlu, &nmc, &nst);
  if (need > kScratchDoubles)
    return fail(QDP_EINVAL, "this system needs " + std::to_string(need * sizeof(double)) +
                                " bytes of Newton workspace; the no-allocation entry point has " +
                                std::to_string(kScratchDoubles * sizeof(double)));
  double *base = nullptr;
  if ((s = scratch_base(&base)) != QDP_OK) return s;
  Workspace w;  // views into the scratch array; nothing here is freed or allocated
  w.L = L;
  w.bcap = 1;
  w.ab = base;
  w.scale = w.ab + nab;
  w.part = npt > 0 ? w.scale + nsc : nullptr;
  w.suppv = nsv > 0 ? w.scale + nsc + npt : nullptr;
  w.lu = nlu > 0 ? w.scale + nsc + npt + nsv : nullptr;
  w.mc = nmc > 0 ? w.scale + nsc + npt + nsv + nlu : nullptr;
  w.mc_cap = nmc > 0 ? 1 : 0;
  w.st = reinterpret_cast<NewtonState *>(w.scale + nsc + npt + nsv + nlu + nmc);
  auto *h = const_cast<qdp_homotopy *>(hc);
  hipStream_t st = (hipStream_t)stream;
  if ((s = enqueue_newton(h, &w, L, t, x, 1, mode, eps, max_it, st, nullptr, nullptr, false)) != QDP_OK) return s;
  if (info_dev) {
    hipLaunchKernelGGL(k_info_from_state, dim3(1), dim3(1), 0, st, w.st, info_dev);
    HIPCHK(hipGetLastError());
  }
  return QDP_OK;
}

extern "C" qdp_status qdp_newton_batch_dev(const qdp_homotopy *hc, double t, double *x, int32_t B, qdp_prec prec,
                                           qdp_solve mode, double eps, int32_t max_it, void *stream) {
  qdp_status s = newton_checks(hc, t, x, (int)prec, mode, eps, max_it);
  if (s != QDP_OK) return s;
  if (B < 1 || B > (1 << 16)) return fail(QDP_EINVAL, "B must be in [1, 65536]");
  auto *h = const_cast<qdp_homotopy *>(hc);
  std::lock_guard<std::mutex> g(h->mu);
  Workspace *w = nullptr;
  if ((s = ensure_ws(h, (int)prec, B, &w)) != QDP_OK) return s;
  return enqueue_newton(h, w, (int)prec, t, x, B, mode, eps, max_it, (hipStream_t)stream);
}

extern "C" qdp_status qdp_eval_homotopy_batch_dev(const qdp_homotopy *hc, double t, const double *x, int32_t B,
                                                  qdp_prec prec, double *y, double *jac, double *scale,
                                                  void *stream) {
  if (!hc) return fail(QDP_EINVAL, "NULL homotopy");
  if (!std::isfinite(t)) return fail(QDP_ENONFINITE, "non-finite t");
  const int L = (int)prec;
  if (!valid_prec(L) || L > hc->f->L) return fail(QDP_EINVAL, "prec must be 1, 2 or 4 and not above the system's");
  if (!x || !y || !jac) return fail(QDP_EINVAL, "NULL buffer");
  if (B < 1 || B > (1 << 16)) return fail(QDP_EINVAL, "B must be in [1, 65536]");
  auto *h = const_cast<qdp_homotopy *>(hc);
  std::lock_guard<std::mutex> g(h->mu);
  Workspace *w = nullptr;
  qdp_status s = ensure_ws(h, L, B, &w);
  if (s != QDP_OK) return s;
  const int n = h->f->n;
  const long e = 2 * L;
  qdp::EvalOut o{jac, 1, (long)n * e, e, y, 1, e, 1.0, scale, (long)n * n * e, (long)n * e, n};
  const qdp::EvalSplit split{w->part, qdp::kMaxEvalParts, w->suppv, w->bcap};
  HIPCHK(qdp::launch_eval(L, h->f->dev(), x, (long)n * e, B, hom_args(h, L, t, 1), o, nullptr, split,
                          (hipStream_t)stream));
  return QDP_OK;
}

extern "C" qdp_status qdp_homotopy_last_info_batch(const qdp_homotopy *hc, qdp_prec prec, int32_t B,
                                                   qdp_newton_info *info, void *stream) {
  if (!hc || !info) return fail(QDP_EINVAL, "NULL argument");
  if (!valid_prec((int)prec)) return fail(QDP_EINVAL, "prec must be 1, 2 or 4");
  auto *h = const_cast<qdp_homotopy *>(hc);
  std::lock_guard<std::mutex> g(h->mu);
  HIPCHK(hipStreamSynchronize((hipStream_t)stream));
  Workspace &w = h->ws[ws_index((int)prec)];
  if (!w.st) return fail(QDP_EINVAL, "no Newton call on this homotopy at this precision yet");
  if (B < 1 || B > w.bcap) return fail(QDP_EINVAL, "B must be in [1, points of the workspace]");
  std::vector<NewtonState> ns(B);
  HIPCHK(hipMemcpy(ns.data(), w.st, B * sizeof(NewtonState), hipMemcpyDeviceToHost));
  for (int b = 0; b < B; ++b) info_from_state(ns[b], info + b);
  return QDP_OK;
}

extern "C" qdp_status qdp_homotopy_last_info(const qdp_homotopy *hc, qdp_prec prec, qdp_newton_info *info,
                                             void *stream) {
  return qdp_homotopy_last_info_batch(hc, prec, 1, info, stream);
}

extern "C" qdp_status qdp_newton_step(const qdp_homotopy *hc, double t, double *x, qdp_prec prec,
                                      qdp_solve mode, double eps, int32_t max_it, qdp_newton_info *info,
                                      void *stream) {
  const int L = (int)prec;
  qdp_status s = newton_checks(hc, t, x, L, mode, eps, max_it);
  if (s != QDP_OK) return s;
  auto *h = const_cast<qdp_homotopy *>(hc);
  if ((s = check_point(h->f->n, L, x)) != QDP_OK) return s;
  std::lock_guard<std::mutex> g(h->mu);
  Workspace *w = nullptr;
  if ((s = ensure_ws(h, L, 1, &w)) != QDP_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  const size_t bytes = (size_t)h->f->n * 2 * L * sizeof(double);
  HIPCHK(hipMemcpyAsync(w->xw, x, bytes, hipMemcpyHostToDevice, st));
  if ((s = enqueue_newton(h, w, L, t, w->xw, 1, mode, eps, max_it, st)) != QDP_OK) return s;
  NewtonState ns;
  HIPCHK(hipMemcpyAsync(x, w->xw, bytes, hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(&ns, w->st, sizeof(ns), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (info) info_from_state(ns, info);
  return QDP_OK;
}

extern "C" qdp_status qdp_set_elimination(int32_t policy) {
  if (policy < QDP_ELIM_AUTO || policy > QDP_ELIM_BLOCKS) return fail(QDP_EINVAL, "policy must be 0, 1, 2 or 3");
  qdp::set_ge_policy(policy);
  return QDP_OK;
}

extern "C" qdp_status qdp_set_timing(int32_t on) {
  g_timing = on ? 1 : 0;
  return QDP_OK;
}

extern "C" qdp_status qdp_homotopy_last_timing(const qdp_homotopy *hc, qdp_prec prec, double *eval_ms,
                                               double *solve_ms, int32_t *launches, void *stream) {
  if (!hc || !eval_ms || !solve_ms || !launches) return fail(QDP_EINVAL, "NULL argument");
  if (!valid_prec((int)prec)) return fail(QDP_EINVAL, "prec must be 1, 2 or 4");
  auto *h = const_cast<qdp_homotopy *>(hc);
  std::lock_guard<std::mutex> g(h->mu);
  HIPCHK(hipStreamSynchronize((hipStream_t)stream));
  Workspace &w = h->ws[ws_index((int)prec)];
  double a = 0, b = 0;
  int k = 0;
  // iterations that ran gated-off still count as launches; their kernels
  // return at once, which the caller sees as a shorter average
  for (int it = 0; it < w.timed_its; ++it) {
    float ea = 0, eb = 0;
    HIPCHK(hipEventElapsedTime(&ea, w.ev[3 * it], w.ev[3 * it + 1]));
    HIPCHK(hipEventElapsedTime(&eb, w.ev[3 * it + 1], w.ev[3 * it + 2]));
    a += ea;
    b += eb;
    ++k;
  }
  *eval_ms = a;
  *solve_ms = b;
  *launches = k;
  return QDP_OK;
}

// ------------------------------------------------------------------ tracker

extern "C" qdp_status qdp_track_params_default(qdp_track_params *p) {
  if (!p) return fail(QDP_EINVAL, "NULL params");
  std::memset(p, 0, sizeof(*p));
  p->lambda0 = 0.01;
  p->lambda_min = 0.01 * std::ldexp(1.0, -30);
  p->lambda_max = 0.08;
  p->shrink = 0.5;
  p->expand = 2.0;
  p->expand_after = 3;
  p->max_it_path = 4;
  p->eps_path = 1e-10;
  p->eps_end = 0.0;
  p->max_it_end = 10;
  p->predictor = QDP_PRED_SECANT;
  p->max_steps = 2000000;
  p->mode = QDP_SOLVE_FULL;
  p->probe = 0;
  p->policy = nullptr;
  p->lambda_max_learned = 0.32;
  p->accept_threshold = 0.3;
  p->policy_rule = 0;
  return QDP_OK;
}

extern "C" qdp_status qdp_policy_infer_host(const qdp_policy *p, const float *x, float *y, void *hip_stream);

namespace {

// Host-side history the learned controller reads (all FP64, features are FP32).
struct CtlHistory {
  double lam_acc[3] = {0.01, 0.01, 0.01};  // last accepted step sizes, newest first
  int run = 0;                              // consecutive successes
  unsigned recent = 0;                      // accept bits of the last 8 attempts (bit 0 newest)
  int attempts = 0;
  int64_t accepted = 0;
  // outcome of the last accepted correction
  int iters = 0;
  double rho_first = 1.0, rho_last = 1.0, cond = 1.0, dz_first = 0.0, znorm = 1.0, pred_dist = 0.0;
};

// the controller's state after the last accepted step, for the shared feature function
static qdp::CtlFeatIn feat_in(const CtlHistory &h, double t) {
  qdp::CtlFeatIn f;
  f.lam[0] = h.lam_acc[0];
  f.lam[1] = h.lam_acc[1];
  f.lam[2] = h.lam_acc[2];
  f.iters = h.iters;
  f.rho_first = h.rho_first;
  f.rho_last = h.rho_last;
  f.cond = h.cond;
  f.dz_first = h.dz_first;
  f.znorm = h.znorm;
  f.pred_dist = h.pred_dist;
  f.t = t;
  f.run = h.run;
  int rej = 0;
  for (int k = 0; k < 8 && k < h.attempts; ++k) rej += ((h.recent >> k) & 1u) ? 0 : 1;
  f.rejected = rej;
  f.accepted = h.accepted;
  return f;
}

// The 16 inputs of the step-size network in the state after an accepted step.
static void features(const CtlHistory &h, double t, float *f) { qdp::ctl_features(feat_in(h, t), f); }

}  // namespace

extern "C" qdp_status qdp_track_path(const qdp_homotopy *hc, double *x, qdp_prec prec, const qdp_track_params *pp,
                                     qdp_track_stats *stats, qdp_step_record *log, int64_t log_cap, void *stream) {
  const int L = (int)prec;
  if (!hc || !x || !stats) return fail(QDP_EINVAL, "NULL argument");
  if (!valid_prec(L) || L > hc->f->L) return fail(QDP_EINVAL, "prec must be 1, 2 or 4 and not above the system's");
  qdp_track_params p;
  if (pp)
    p = *pp;
  else
    qdp_track_params_default(&p);
  if (!(p.lambda0 > 0) || !(p.shrink > 0 && p.shrink < 1) || !(p.expand >= 1) || p.max_it_path < 1 ||
      p.max_it_end < 0 || !(p.lambda_max >= p.lambda0))
    return fail(QDP_EINVAL, "bad step-size control parameters");
  if (p.mode != QDP_SOLVE_FULL && p.mode != QDP_SOLVE_MIXED_IR) return fail(QDP_EINVAL, "bad solve mode");
  if (p.mode == QDP_SOLVE_MIXED_IR && !mixed_supported(L, hc->f->n))
    return fail(QDP_EUNSUPPORTED, "mixed-precision refinement is implemented for double and quad double, n <= 128");
  const bool learned = p.predictor == QDP_PRED_LEARNED;
  if (learned && !p.policy) return fail(QDP_EINVAL, "learned predictor needs a policy");
  if (p.predictor != QDP_PRED_SECANT && p.predictor != QDP_PRED_QUADRATIC && !learned)
    return fail(QDP_EINVAL, "unknown predictor");
  // quadratic weight of the plain predictor; the learned controller falls back to the quadratic one
  const double plain_wq = p.predictor == QDP_PRED_SECANT ? 0.0 : 1.0;
  const double lam_cap = learned ? (p.lambda_max_learned > 0 ? p.lambda_max_learned : 4 * p.lambda_max) : p.lambda_max;
  const double thr = p.accept_threshold > 0 ? p.accept_threshold : 0.3;
  if (thr >= 1.0) return fail(QDP_EINVAL, "accept_threshold must be below 1");
  if (p.policy_rule != 0 && p.policy_rule != 1) return fail(QDP_EINVAL, "policy_rule must be 0 or 1");
  auto *h = const_cast<qdp_homotopy *>(hc);
  const int n = h->f->n;
  qdp_status s = check_point(n, L, x);
  if (s != QDP_OK) return s;
  std::lock_guard<std::mutex> g(h->mu);
  Workspace *w = nullptr;
  if ((s = ensure_ws(h, L, 1, &w)) != QDP_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  const size_t bytes = (size_t)n * 2 * L * sizeof(double);
  const auto t_start = std::chrono::steady_clock::now();
  HIPCHK(hipMemcpyAsync(w->x, x, bytes, hipMemcpyHostToDevice, st));

  std::memset(stats, 0, sizeof(*stats));
  double t = 0.0, tprev = 0.0, tprev2 = 0.0, lam = p.lambda0;
  int npts = 1;  // accepted points available to the predictor (1, 2, 3 = three or more)
  bool stop = false, from_policy = false;
  int run = 0;
  int64_t succ = 0, corr = 0, nit = 0, nlog = 0, used = 0, rejected = 0, probes = 0;
  double sum_step = 0.0, min_step = INFINITY;
  NewtonState ns;
  double aux[4] = {0, 0, 0, 0};
  CtlHistory hist;
  float pout[8] = {0, 0, 0, 0, 0, 0, 0, 0};  // network outputs for the state the last main stage led to
  auto push = [&](const qdp_step_record &r) {
    if (log && nlog < log_cap) log[nlog++] = r;
  };
  // predictor coefficients at tn: secant s1, quadratic (q1, q2) (see k_predict)
  auto coefs = [&](double tn, double &s1, double &q1, double &q2) {
    s1 = npts >= 2 ? -(tn - t) / (t - tprev) : 0.0;
    q1 = q2 = 0.0;
    if (npts >= 3) {
      q1 = ((tn - t) * (tn - tprev2)) / ((tprev - t) * (tprev - tprev2));
      q2 = ((tn - t) * (tn - tprev)) / ((tprev2 - t) * (tprev2 - tprev));
    }
  };
  // one corrector stage from the current accepted point with step `step`;
  // wq weights the quadratic predictor against the secant (0 = secant).
  // infer: run the network, on the device and before the stage is read back,
  // on the state this stage leads to if the Newton test accepts it (the only
  // case in which the next step asks the network)
  auto correct = [&](double step, double wq, double &tn_out, bool infer) -> qdp_status {
    const double tn = (t + step >= 1.0) ? 1.0 : t + step;
    tn_out = tn;
    double s1, q1, q2;
    coefs(tn, s1, q1, q2);
    double c1 = s1, c2 = 0.0;
    if (npts >= 3) {
      c1 = (1.0 - wq) * s1 + wq * q1;
      c2 = wq * q2;
    }
    HIPCHK(qdp::launch_predict(L, n, w->x, w->xprev, w->xprev2, c1, c2, w->xw, w->aux, st));
    qdp_status e = enqueue_newton(h, w, L, tn, w->xw, 1, p.mode, p.eps_path, p.max_it_path, st);
    if (e != QDP_OK) return e;
    if (infer) {
      CtlHistory next = hist;  // the history after accepting this stage
      next.lam_acc[2] = hist.lam_acc[1];
      next.lam_acc[1] = hist.lam_acc[0];
      next.lam_acc[0] = step;
      next.recent = (hist.recent << 1) | 1u;
      next.attempts = hist.attempts + 1;
      next.accepted = succ + 1;
      next.run = run + 1;
      HIPCHK(qdp::launch_ctl_features(feat_in(next, tn), w->st, w->aux, w->pfeat, st));
      if ((e = qdp_policy_forward(p.policy, w->pfeat, 1, 1, w->pfeat + 16, st)) != QDP_OK) return e;
    }
    // one gathered record, one copy into pinned memory, one synchronisation
    HIPCHK(qdp::launch_stage_readback(w->st, w->aux, infer ? w->pfeat + 16 : nullptr, w->rb_dev, st));
    HIPCHK(hipMemcpyAsync(w->rb_host, w->rb_dev, sizeof(qdp::StageReadback), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    ns = w->rb_host->st;
    std::memcpy(aux, w->rb_host->aux, sizeof(aux));
    if (infer) std::memcpy(pout, w->rb_host->pout, sizeof(pout));
    return QDP_OK;
  };

  while (t < 1.0 && !stop) {
    // ---- probes (data collection): all multipliers from this accepted state
    if (p.probe && npts >= 2) {
      qdp_step_record rec;
      std::memset(&rec, 0, sizeof(rec));
      rec.kind = 1;
      rec.t = t;
      rec.lambda = hist.lam_acc[0];
      rec.blend_label = NAN;
      features(hist, t, rec.features);
      for (int k = 0; k < 5; ++k) {
        const double step = std::min(hist.lam_acc[0] * std::ldexp(1.0, k - 1), 1.0 - t);
        double tn;
        if ((s = correct(step, 1.0, tn, false)) != QDP_OK) return s;
        ++probes;
        if (ns.success) {
          rec.probe_ok |= 1 << k;
          if (k == 1 && npts >= 3) {
            double s1, q1, q2;
            coefs(tn, s1, q1, q2);
            HIPCHK(qdp::launch_blend_label(L, n, w->x, w->xprev, w->xprev2, w->xw, s1, q1, q2, w->aux, st));
            HIPCHK(hipMemcpyAsync(aux, w->aux, sizeof(aux), hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            if (aux[2] > 0) rec.blend_label = aux[1] / aux[2];
          }
        }
      }
      push(rec);
    }
    // ---- choose the step
    double step = std::min(lam, 1.0 - t);
    double wgt = plain_wq;
    from_policy = false;
    if (learned && npts >= 2 && run > 0) {
      // after a success: the network proposes the multiplier and the secant
      // weight; it ran on this state right after the stage that reached it
      const float *out = pout;
      int best = -1;
      double best_score = -1.0;
      for (int k = 0; k < 5; ++k) {
        const double pk = 1.0 / (1.0 + std::exp(-(double)out[k]));
        if (pk < thr) continue;
        const double score = p.policy_rule == 0 ? pk * std::ldexp(1.0, k - 1) : (double)k;
        if (score > best_score) {
          best_score = score;
          best = k;
        }
      }
      const double mult = best >= 0 ? std::ldexp(1.0, best - 1) : 0.5;
      step = std::min(std::min(hist.lam_acc[0] * mult, lam_cap), 1.0 - t);
      step = std::max(step, std::min(p.lambda_min, 1.0 - t));
      wgt = std::min(std::max((double)out[5], -0.5), 1.5);
      from_policy = true;
    }
    double tn;
    if ((s = correct(step, wgt, tn, learned)) != QDP_OK) return s;
    ++corr;
    nit += ns.iterations;
    const bool ok = ns.success != 0;
    {
      qdp_step_record rec;
      std::memset(&rec, 0, sizeof(rec));
      rec.kind = 0;
      rec.t = t;
      rec.lambda = step;
      rec.rho_first = ns.rho_first;
      rec.rho_last = ns.rho;
      rec.dz_first = ns.dz_first;
      rec.cond_est = ns.cond_est;
      rec.znorm = hist.znorm;
      rec.pred_dist = aux[0];
      rec.blend_label = NAN;
      features(hist, t, rec.features);
      rec.iterations = ns.iterations;
      rec.accepted = ok ? 1 : 0;
      push(rec);
    }
    hist.recent = (hist.recent << 1) | (ok ? 1u : 0u);
    hist.attempts += 1;
    if (from_policy) {
      ++used;
      if (!ok) ++rejected;
    }
    if (ok) {
      // accept: (x_prev2, x_prev, x) <- (x_prev, x, corrected), same for t
      std::swap(w->xprev2, w->xprev);
      std::swap(w->xprev, w->x);
      std::swap(w->x, w->xw);
      tprev2 = tprev;
      tprev = t;
      t = tn;
      npts = std::min(npts + 1, 3);
      ++succ;
      sum_step += step;
      min_step = std::min(min_step, step);
      hist.lam_acc[2] = hist.lam_acc[1];
      hist.lam_acc[1] = hist.lam_acc[0];
      hist.lam_acc[0] = step;
      hist.accepted = succ;
      hist.iters = ns.iterations;
      hist.rho_first = ns.rho_first;
      hist.rho_last = ns.rho;
      hist.cond = ns.cond_est;
      hist.dz_first = ns.dz_first;
      hist.znorm = ns.xnorm;
      hist.pred_dist = aux[0];
      hist.run = ++run;
      if (from_policy) {
        lam = step;  // the plain rule continues from the learned step after a fallback
      } else if (run >= p.expand_after) {
        lam = std::min(lam * p.expand, p.lambda_max);
        run = 0;
        hist.run = 0;
      }
    } else {
      lam = (from_policy ? step : lam) * p.shrink;  // step back: keep (x, t)
      run = 0;
      hist.run = 0;
    }
    stop = lam < p.lambda_min || corr >= p.max_steps;
  }
  stats->end_success = 0;
  if (t >= 1.0) {
    // end refinement at t = 1: Newton until eps_end, max_it_end, or the
    // residual stops decreasing
    const double eps_end = p.eps_end > 0 ? p.eps_end : 64.0 * std::ldexp(1.0, -53 * L);
    double prev = INFINITY;
    double rho = 1.0;
    int it = 0;
    while (rho > eps_end && it < p.max_it_end) {
      if ((s = enqueue_newton(h, w, L, 1.0, w->x, 1, p.mode, 0.0, 1, st)) != QDP_OK) return s;
      HIPCHK(hipMemcpyAsync(&ns, w->st, sizeof(ns), hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      rho = ns.rho;
      ++it;
      if (ns.singular || !(rho == rho)) break;
      if (rho >= prev) break;
      prev = rho;
    }
    nit += it;
    stats->end_success = rho < eps_end ? 1 : 0;
    stats->end_residual = rho;
  }
  HIPCHK(hipMemcpyAsync(x, w->x, bytes, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  stats->fail = t < 1.0 ? 1 : 0;
  stats->t_final = t;
  stats->succ_corrections = succ;
  stats->corrections = corr;
  stats->newton_iterations = nit;
  stats->avg_step = succ ? sum_step / (double)succ : 0.0;
  stats->min_step = succ ? min_step : 0.0;
  stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
  stats->policy_used = used;
  stats->policy_rejected = rejected;
  stats->log_count = nlog;
  stats->probe_corrections = probes;
  return QDP_OK;
}

// ------------------------------------------------------------------ arithmetic test entry

// ------------------------------------------------------------------ batched tracker

// Algorithm 3.1 for B paths of one homotopy at once: every round predicts and
// corrects all unfinished paths with one launch per kernel (each path at its
// own t with its own step size, predictor history and Newton loop), then
// applies the plain step-size control path by path on the host.  The end
// refinement at t = 1 runs the same way.  Plain control only (secant or
// quadratic predictor).
extern "C" qdp_status qdp_track_paths(const qdp_homotopy *hc, double *x, int32_t B, qdp_prec prec,
                                      const qdp_track_params *pp, qdp_track_stats *stats, void *stream) {
  const int L = (int)prec;
  if (!hc || !x || !stats) return fail(QDP_EINVAL, "NULL argument");
  if (B < 1 || B > (1 << 16)) return fail(QDP_EINVAL, "B must be in [1, 65536]");
  if (!valid_prec(L) || L > hc->f->L) return fail(QDP_EINVAL, "prec must be 1, 2 or 4 and not above the system's");
  qdp_track_params p;
  if (pp)
    p = *pp;
  else
    qdp_track_params_default(&p);
  if (!(p.lambda0 > 0) || !(p.shrink > 0 && p.shrink < 1) || !(p.expand >= 1) || p.max_it_path < 1 ||
      p.max_it_end < 0 || !(p.lambda_max >= p.lambda0))
    return fail(QDP_EINVAL, "bad step-size control parameters");
  if (p.mode != QDP_SOLVE_FULL && p.mode != QDP_SOLVE_MIXED_IR) return fail(QDP_EINVAL, "bad solve mode");
  if (p.mode == QDP_SOLVE_MIXED_IR && !mixed_supported(L, hc->f->n))
    return fail(QDP_EUNSUPPORTED, "mixed-precision refinement is implemented for double and quad double, n <= 128");
  if (p.predictor != QDP_PRED_SECANT && p.predictor != QDP_PRED_QUADRATIC)
    return fail(QDP_EUNSUPPORTED, "batched tracking uses the secant or the quadratic predictor");
  if (p.probe) return fail(QDP_EUNSUPPORTED, "probe mode tracks one path");
  auto *h = const_cast<qdp_homotopy *>(hc);
  const int n = h->f->n;
  const size_t per = (size_t)n * 2 * L;
  qdp_status s = check_point(n * B, L, x);
  if (s != QDP_OK) return s;
  std::lock_guard<std::mutex> g(h->mu);
  Workspace *w = nullptr;
  if ((s = ensure_ws(h, L, B, &w)) != QDP_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  const auto t_start = std::chrono::steady_clock::now();

  // device: points x, x_prev, x_prev2, working point; coefficients [2][B] and
  // t [B] in one array; mask and acceptance flags [2][B]
  double *dx = nullptr, *dxp = nullptr, *dxpp = nullptr, *dxw = nullptr, *dcf = nullptr;
  int *dflags = nullptr;
  auto cleanup = [&]() {
    hipFree(dx);
    hipFree(dxp);
    hipFree(dxpp);
    hipFree(dxw);
    hipFree(dcf);
    hipFree(dflags);
  };
  hipError_t err = hipMalloc(&dx, per * B * sizeof(double));
  if (err == hipSuccess) err = hipMalloc(&dxp, per * B * sizeof(double));
  if (err == hipSuccess) err = hipMalloc(&dxpp, per * B * sizeof(double));
  if (err == hipSuccess) err = hipMalloc(&dxw, per * B * sizeof(double));
  if (err == hipSuccess) err = hipMalloc(&dcf, 3 * (size_t)B * sizeof(double));
  if (err == hipSuccess) err = hipMalloc(&dflags, 2 * (size_t)B * sizeof(int));
  if (err == hipSuccess) err = hipMemcpyAsync(dx, x, per * B * sizeof(double), hipMemcpyHostToDevice, st);
  if (err != hipSuccess) {
    cleanup();
    return fail(err == hipErrorOutOfMemory ? QDP_ENOMEM : QDP_EDEVICE, hipGetErrorString(err));
  }
  int *dmask = dflags, *dacc = dflags + B;
  double *dtn = dcf + 2 * (size_t)B;

  struct PathState {
    double t = 0.0, tprev = 0.0, tprev2 = 0.0, lam = 0.0, sum_step = 0.0, min_step = INFINITY, rho = 1.0,
           prev = INFINITY;
    int npts = 1, run = 0, end_it = 0;
    bool done = false, refining = false, end_stop = false;
    int64_t succ = 0, corr = 0, nit = 0;
  };
  std::vector<PathState> ps(B);
  for (auto &q : ps) q.lam = p.lambda0;
  std::vector<double> hcf(3 * (size_t)B, 0.0);
  std::vector<int> hflags(2 * (size_t)B, 0);
  std::vector<NewtonState> ns(B);
  const double wq = p.predictor == QDP_PRED_QUADRATIC ? 1.0 : 0.0;
  const double eps_end = p.eps_end > 0 ? p.eps_end : 64.0 * std::ldexp(1.0, -53 * L);
  auto run_round = [&](int mode_end) -> qdp_status {
    // flags and coefficients to the device, predict (path rounds), Newton, states back
    HIPCHK(hipMemcpyAsync(dcf, hcf.data(), hcf.size() * sizeof(double), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(dflags, hflags.data(), hflags.size() * sizeof(int), hipMemcpyHostToDevice, st));
    qdp_status e;
    if (!mode_end) {
      HIPCHK(qdp::launch_predict_batch(L, n, B, dx, dxp, dxpp, dcf, dmask, dxw, st));
      e = enqueue_newton(h, w, L, 0.0, dxw, B, p.mode, p.eps_path, p.max_it_path, st, dtn, dmask);
    } else {
      e = enqueue_newton(h, w, L, 1.0, dx, B, p.mode, 0.0, 1, st, nullptr, dmask);
    }
    if (e != QDP_OK) return e;
    HIPCHK(hipMemcpyAsync(ns.data(), w->st, B * sizeof(NewtonState), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    return QDP_OK;
  };
  qdp_status rs = QDP_OK;
  for (;;) {
    // ---- path rounds
    int active = 0;
    for (int b = 0; b < B; ++b) {
      PathState &q = ps[b];
      hflags[b] = 0;
      hflags[B + b] = 0;
      if (q.done || q.refining) continue;
      const double step = std::min(q.lam, 1.0 - q.t);
      const double tn = (q.t + step >= 1.0) ? 1.0 : q.t + step;
      double c1 = 0.0, c2 = 0.0;
      if (q.npts >= 2) c1 = -(tn - q.t) / (q.t - q.tprev);
      if (q.npts >= 3 && wq > 0) {
        c1 = ((tn - q.t) * (tn - q.tprev2)) / ((q.tprev - q.t) * (q.tprev - q.tprev2));
        c2 = ((tn - q.t) * (tn - q.tprev)) / ((q.tprev2 - q.t) * (q.tprev2 - q.tprev));
      }
      hcf[b] = c1;
      hcf[B + b] = c2;
      hcf[2 * (size_t)B + b] = tn;
      hflags[b] = 1;
      ++active;
    }
    if (active == 0) break;
    if ((rs = run_round(0)) != QDP_OK) break;
    for (int b = 0; b < B; ++b) {
      if (!hflags[b]) continue;
      PathState &q = ps[b];
      const double step = std::min(q.lam, 1.0 - q.t);
      const double tn = hcf[2 * (size_t)B + b];
      ++q.corr;
      q.nit += ns[b].iterations;
      if (ns[b].success) {
        hflags[B + b] = 1;
        q.tprev2 = q.tprev;
        q.tprev = q.t;
        q.t = tn;
        q.npts = std::min(q.npts + 1, 3);
        ++q.succ;
        q.sum_step += step;
        q.min_step = std::min(q.min_step, step);
        if (++q.run >= p.expand_after) {
          q.lam = std::min(q.lam * p.expand, p.lambda_max);
          q.run = 0;
        }
      } else {
        q.lam *= p.shrink;
        q.run = 0;
      }
      if (q.t >= 1.0) q.refining = true;
      else if (q.lam < p.lambda_min || q.corr >= p.max_steps) q.done = true;
    }
    HIPCHK(hipMemcpyAsync(dacc, hflags.data() + B, B * sizeof(int), hipMemcpyHostToDevice, st));
    HIPCHK(qdp::launch_accept_batch(L, n, B, dacc, dx, dxp, dxpp, dxw, st));
  }
  // ---- end refinement at t = 1: Newton until eps_end, max_it_end, or the
  // residual stops decreasing, path by path
  while (rs == QDP_OK) {
    int active = 0;
    for (int b = 0; b < B; ++b) {
      PathState &q = ps[b];
      hflags[b] = (q.refining && !q.end_stop && q.rho > eps_end && q.end_it < p.max_it_end) ? 1 : 0;
      active += hflags[b];
    }
    if (active == 0) break;
    if ((rs = run_round(1)) != QDP_OK) break;
    for (int b = 0; b < B; ++b) {
      if (!hflags[b]) continue;
      PathState &q = ps[b];
      q.rho = ns[b].rho;
      ++q.end_it;
      if (ns[b].singular || !(q.rho == q.rho) || q.rho >= q.prev) q.end_stop = true;
      q.prev = q.rho;
    }
  }
  if (rs == QDP_OK) {
    err = hipMemcpyAsync(x, dx, per * B * sizeof(double), hipMemcpyDeviceToHost, st);
    if (err == hipSuccess) err = hipStreamSynchronize(st);
    if (err != hipSuccess) rs = fail(QDP_EDEVICE, hipGetErrorString(err));
  }
  cleanup();
  if (rs != QDP_OK) return rs;
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
  for (int b = 0; b < B; ++b) {
    const PathState &q = ps[b];
    qdp_track_stats &o = stats[b];
    std::memset(&o, 0, sizeof(o));
    o.fail = q.t < 1.0 ? 1 : 0;
    o.end_success = (q.refining && q.rho < eps_end) ? 1 : 0;
    o.t_final = q.t;
    o.succ_corrections = q.succ;
    o.corrections = q.corr;
    o.newton_iterations = q.nit + q.end_it;
    o.avg_step = q.succ ? q.sum_step / (double)q.succ : 0.0;
    o.min_step = q.succ ? q.min_step : 0.0;
    o.seconds = secs;
    o.end_residual = q.refining ? q.rho : 0.0;
  }
  return QDP_OK;
}

extern "C" qdp_status qdp_arith_batch(int32_t op, qdp_prec prec, int64_t count, const double *a, const double *b,
                                      const double *c, double *out, void *stream) {
  const int L = (int)prec;
  if (!valid_prec(L)) return fail(QDP_EINVAL, "prec must be 1, 2 or 4");
  if (count < 0 || !a || !out) return fail(QDP_EINVAL, "bad arguments");
  const bool binary = !(op == 15 || op == 16);
  if (binary && !b) return fail(QDP_EINVAL, "b is NULL");
  if (op == 14 && !c) return fail(QDP_EINVAL, "c is NULL");
  if (!((op >= 0 && op <= 3) || (op >= 10 && op <= 16))) return fail(QDP_EINVAL, "unknown op");
  if (op == 16 && count % 64 != 0) return fail(QDP_EINVAL, "the pivot search works on groups of 64");
  if (count == 0) return QDP_OK;
  HIPCHK(qdp::launch_arith(op, L, count, a, b, c, out, (hipStream_t)stream));
  return QDP_OK;
}
