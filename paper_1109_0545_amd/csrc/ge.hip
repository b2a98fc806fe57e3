// Elimination dispatch by precision, and the choice between one workgroup
// per point and one workgroup per column.
#include <atomic>

#include "common.hpp"

namespace qdp {

hipError_t launch_ge_f64(int, int, double *, double *, double *, double *, NewtonState *, const GeMc &, hipStream_t);
hipError_t launch_ge_dd(int, int, double *, double *, double *, double *, NewtonState *, const GeMc &, hipStream_t);
hipError_t launch_ge_qd(int, int, double *, double *, double *, double *, NewtonState *, const GeMc &, hipStream_t);

// All (n+1) x B workgroups of a column-parallel elimination wait on one
// another, so they must all be resident at once: one wavefront each, at most
// this many per launch (four per compute unit).
constexpr long kMcMaxGroups = 1024;
static std::atomic<int> g_ge_policy{0};
static std::atomic<unsigned> g_mc_epoch{0};

void set_ge_policy(int p) { g_ge_policy.store(p); }
int ge_policy() { return g_ge_policy.load(); }

// whether a column-parallel workspace can serve (L, n, B) at all
bool ge_mc_possible(int L, int n, int B) {
  return (L == 2 || L == 4) && n >= 1 && n <= 128 && B >= 1 && (long)B * (n + 1) <= kMcMaxGroups;
}
// blocks of 16 columns per workgroup (double double up to n = 128, quad
// double up to n = 64): one workgroup per compute unit (its LDS), at most this
// many per launch
constexpr long kMcbMaxGroups = 128;
static bool ge_mcb_possible(int L, int n, int B) {
  return (L == 2 || L == 4) && n >= 1 && n <= (L == 2 ? 128 : 64) && B >= 1 &&
         (long)B * ((n + 16) / 16) <= kMcbMaxGroups;
}
// policy 0 (default): blocks of columns for double double past n = 48 (four
// blocks or more: n = 64 measured 97 us per solve against 127 us for the
// register kernel, n = 128 294 us against 437 us with one workgroup per
// column and 1,176 us on one CU; at n = 32 and below the register kernel is
// faster) and for quad double up to n = 64 (n = 64: 522 us against 613 us
// with one workgroup per column, 953 us on one CU); one workgroup per column
// for quad double past n = 64; else one workgroup per point; 1: one per
// point; 2: columns wherever possible; 3: blocks where possible, else as 2
static GeMc ge_mc_choice(int L, int n, int B, double *ws) {
  const int p = g_ge_policy.load();
  if (!ws || p == 1 || !ge_mc_possible(L, n, B)) return GeMc{nullptr, 0u, 0};
  if ((p == 3 || (p == 0 && (L == 4 || n > 48))) && ge_mcb_possible(L, n, B))
    return GeMc{ws, g_mc_epoch.fetch_add(1u) + 1u, 1};
  if (p == 2 || p == 3 || L == 4 || n > 64) return GeMc{ws, g_mc_epoch.fetch_add(1u) + 1u, 0};
  return GeMc{nullptr, 0u, 0};
}

size_t ge_lds_bytes(int L, int n, bool in_lds) {
  size_t d = (size_t)2 * n * 2 * L + 16;  // inverses + rhs + reduction
  if (in_lds) d += (size_t)n * (n + 1) * 2 * L;
  return d * sizeof(double) + 4 * (size_t)n * sizeof(int) + 64;
}

// B points, one workgroup each (see GeArgs for the batch layout)
// (mc_ws: B column-parallel workspaces, or nullptr)
hipError_t launch_ge_scaled(int L, int n, int B, double *ab, double *scale, double *x, double *dz, NewtonState *st,
                            double *mc_ws, hipStream_t s) {
  if (B < 1) return hipErrorInvalidValue;
  const GeMc mc = ge_mc_choice(L, n, B, mc_ws);
  switch (L) {
    case 1: return launch_ge_f64(n, B, ab, scale, x, dz, st, mc, s);
    case 2: return launch_ge_dd(n, B, ab, scale, x, dz, st, mc, s);
    case 4: return launch_ge_qd(n, B, ab, scale, x, dz, st, mc, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace qdp
