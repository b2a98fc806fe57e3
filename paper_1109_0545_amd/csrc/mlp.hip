// Step-size network for learned step control: FP32 training (forward,
// loss, backward, Adam) and BF16-weight inference, written as plain HIP
// kernels (not in the paper: a growth direction of the tracker).
//
// Network: widths w_0 (features) .. w_L (outputs); hidden layers ReLU.
// Flat FP32 parameters: for each layer its weights [out][in] (row-major)
// then its bias [out].  Outputs 0..w_L-2 are logits trained with binary
// cross-entropy; the last output is a real value trained with squared error;
// a 0/1 mask per target selects the terms:
//   loss = (1/B) sum_b [ sum_{k<w_L-1} M_bk BCE(o_bk, Y_bk) + M_b,last (o_b,last - Y_b,last)^2 ].
// Every sum runs in a fixed order (no atomics), so results are reproducible.

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/qdpath.h"

namespace qdp {

// C[m][n] = sum_k A[m,k] B[k,n] (+ bias[n]) (ReLU), arbitrary strides
// (counted in elements).  64x64 output tile per 256-thread block, 4x4 per
// thread, K staged through LDS 16 at a time.
template <bool RELU>
__global__ __launch_bounds__(256) void k_gemm(int M, int N, int K, const float *A, long sam, long sak,
                                              const float *B, long sbk, long sbn, const float *bias, float *C,
                                              long scm, long scn) {
  __shared__ float As[16][65];
  __shared__ float Bs[16][65];
  const int tm = blockIdx.y * 64, tn = blockIdx.x * 64;
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
  float acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = 0.0f;
  for (int k0 = 0; k0 < K; k0 += 16) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int idx = threadIdx.x + 256 * e;
      const int r = idx / 16, kk = idx % 16;
      As[kk][r] = (tm + r < M && k0 + kk < K) ? A[(long)(tm + r) * sam + (long)(k0 + kk) * sak] : 0.0f;
      const int kb = idx / 64, c = idx % 64;
      Bs[kb][c] = (k0 + kb < K && tn + c < N) ? B[(long)(k0 + kb) * sbk + (long)(tn + c) * sbn] : 0.0f;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      float a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[kk][ty * 4 + i];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Bs[kk][tx * 4 + j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_fmaf(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int m = tm + ty * 4 + i;
    if (m >= M) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int n = tn + tx * 4 + j;
      if (n >= N) continue;
      float v = acc[i][j] + (bias ? bias[n] : 0.0f);
      if (RELU) v = fmaxf(v, 0.0f);
      C[(long)m * scm + (long)n * scn] = v;
    }
  }
}

static hipError_t gemm(bool relu, int M, int N, int K, const float *A, long sam, long sak, const float *B, long sbk,
                       long sbn, const float *bias, float *C, long scm, long scn, hipStream_t s) {
  dim3 g((N + 63) / 64, (M + 63) / 64), b(256);
  if (relu)
    hipLaunchKernelGGL(k_gemm<true>, g, b, 0, s, M, N, K, A, sam, sak, B, sbk, sbn, bias, C, scm, scn);
  else
    hipLaunchKernelGGL(k_gemm<false>, g, b, 0, s, M, N, K, A, sam, sak, B, sbk, sbn, bias, C, scm, scn);
  return hipGetLastError();
}

// (x - mean) / std per feature
__global__ void k_normalize(int B, int F, const float *X, const float *mean, const float *sd, float *out) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= B * F) return;
  const int f = q % F;
  out[q] = (X[q] - mean[f]) / sd[f];
}

// dO = d loss / d o and the per-row loss
__global__ void k_loss_grad(int B, int O, const float *out, const float *Y, const float *Mk, float *g, float *rowloss) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  float l = 0.0f;
  for (int k = 0; k < O; ++k) {
    const int q = b * O + k;
    const float o = out[q], y = Y[q], m = Mk[q];
    if (k < O - 1) {
      l += m * (fmaxf(o, 0.0f) - o * y + log1pf(expf(-fabsf(o))));
      g[q] = m * (1.0f / (1.0f + expf(-o)) - y) / (float)B;
    } else {
      const float d = o - y;
      l += m * d * d;
      g[q] = m * 2.0f * d / (float)B;
    }
  }
  rowloss[b] = l;
}

// one block: loss = sum of row losses / B, fixed order
__global__ __launch_bounds__(256) void k_sum_loss(int B, const float *rowloss, float *loss) {
  __shared__ float part[256];
  float s = 0.0f;
  for (int b = threadIdx.x; b < B; b += 256) s += rowloss[b];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = part[0] / (float)B;
}

// db[n] = sum_m dz[m][n]
__global__ void k_colsum(int M, int N, const float *dz, float *db) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  float s = 0.0f;
  for (int m = 0; m < M; ++m) s += dz[(long)m * N + n];
  db[n] = s;
}

// dz *= (h > 0)
__global__ void k_relu_back(long count, float *dz, const float *h) {
  const long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < count && !(h[q] > 0.0f)) dz[q] = 0.0f;
}

__global__ void k_adam(long count, float *p, const float *g, float *m, float *v, float lr, float b1, float b2,
                       float eps, float c1, float c2) {
  const long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= count) return;
  const float gq = g[q];
  const float mq = b1 * m[q] + (1.0f - b1) * gq;
  const float vq = b2 * v[q] + (1.0f - b2) * gq * gq;
  m[q] = mq;
  v[q] = vq;
  p[q] -= lr * (mq / c1) / (sqrtf(vq / c2) + eps);
}

// FP32 -> BF16, round to nearest even (NaN stays a quiet NaN)
__device__ inline unsigned short to_bf16(float x) {
  unsigned int u = __float_as_uint(x);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (unsigned short)((u >> 16) | 0x40);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ inline float from_bf16(unsigned short h) { return __uint_as_float(((unsigned int)h) << 16); }

// BF16 copy for inference with each layer's weights transposed to [in][out]
// (the bias [out] follows as in the FP32 layout), so that at a fixed input k
// the threads of a workgroup, one per output, read consecutive weights.
__global__ void k_to_bf16_t(int nl, const int *widths, const float *p, unsigned short *out) {
  long off = 0;
  for (int l = 0; l < nl; ++l) {
    const int in = widths[l], o = widths[l + 1];
    const long nw = (long)in * o;
    for (long q = blockIdx.x * (long)blockDim.x + threadIdx.x; q < nw + o; q += (long)gridDim.x * blockDim.x) {
      if (q < nw) {
        const long j = q / in, k = q - j * in;  // source [j][k]
        out[off + k * o + j] = to_bf16(p[off + q]);
      } else {
        out[off + q] = to_bf16(p[off + q]);
      }
    }
    off += nw + o;
  }
}

// Inference of one input row per block: weights in BF16 (or FP32), activations
// and accumulation in FP32; normalisation of the raw features fused.
template <bool BF16>
__global__ __launch_bounds__(256) void k_infer(int B, int nl, const int *widths, const float *X, const float *mean,
                                               const float *sd, const void *params, float *Y) {
  __shared__ float xa[256];
  __shared__ float xb[256];
  const int b = blockIdx.x;
  if (b >= B) return;
  const int F = widths[0];
  for (int f = threadIdx.x; f < F; f += blockDim.x) xa[f] = (X[(long)b * F + f] - mean[f]) / sd[f];
  __syncthreads();
  long off = 0;
  float *cur = xa, *nxt = xb;
  for (int l = 0; l < nl; ++l) {
    const int in = widths[l], out = widths[l + 1];
    for (int j = threadIdx.x; j < out; j += blockDim.x) {
      // BF16 weights are stored [in][out] (k_to_bf16_t), FP32 ones [out][in];
      // weights are loaded KC at a time ahead of their products so that the
      // loads overlap instead of each waiting for the previous product
      auto wt = [&](int k) {
        return BF16 ? from_bf16(static_cast<const unsigned short *>(params)[off + (long)k * out + j])
                    : static_cast<const float *>(params)[off + (long)j * in + k];
      };
      constexpr int KC = 16;
      float s = 0.0f;
      int k = 0;
      for (; k + KC <= in; k += KC) {
        float wv[KC];
#pragma unroll
        for (int u = 0; u < KC; ++u) wv[u] = wt(k + u);
#pragma unroll
        for (int u = 0; u < KC; ++u) s = __builtin_fmaf(wv[u], cur[k + u], s);
      }
      for (; k < in; ++k) s = __builtin_fmaf(wt(k), cur[k], s);
      const long qb = off + (long)out * in + j;
      s += BF16 ? from_bf16(static_cast<const unsigned short *>(params)[qb]) : static_cast<const float *>(params)[qb];
      nxt[j] = (l < nl - 1) ? fmaxf(s, 0.0f) : s;
    }
    off += (long)out * in + out;
    __syncthreads();
    float *t = cur;
    cur = nxt;
    nxt = t;
  }
  const int O = widths[nl];
  for (int j = threadIdx.x; j < O; j += blockDim.x) Y[(long)b * O + j] = cur[j];
}

}  // namespace qdp

// ------------------------------------------------------------------ C-ABI

struct qdp_policy {
  std::vector<int> w;  // widths
  long np = 0;
  int *d_w = nullptr;
  float *d_p = nullptr, *d_m = nullptr, *d_v = nullptr, *d_g = nullptr;
  unsigned short *d_pbf = nullptr;
  float *d_mean = nullptr, *d_sd = nullptr;
  float mean[256], sd[256];
  int step = 0;
  bool bf16_stale = true;
  // training workspace
  int cap = 0;
  float *d_act = nullptr;   // layer inputs/outputs [B][sum widths]
  float *d_dz0 = nullptr, *d_dz1 = nullptr;  // [B][max width]
  float *d_rowloss = nullptr, *d_loss = nullptr;
  // inference workspace (one row)
  float *d_x1 = nullptr, *d_y1 = nullptr;
  std::mutex mu;
};

namespace qdp {
// records the message returned by qdp_last_error (defined with the rest of the ABI)
qdp_status set_error(qdp_status s, const std::string &msg);
}  // namespace qdp
#define qdp_policy_fail qdp::set_error

#define PCHK(expr)                                                                 \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess) return qdp_policy_fail(QDP_EDEVICE, std::string(#expr ": ") + hipGetErrorString(e_)); \
  } while (0)

static long offset_of(const std::vector<int> &w, int l) {
  long off = 0;
  for (int i = 0; i < l; ++i) off += (long)w[i + 1] * w[i] + w[i + 1];
  return off;
}

static qdp_status ensure_train_ws(qdp_policy *p, int B) {
  if (B <= p->cap) return QDP_OK;
  hipFree(p->d_act);
  hipFree(p->d_dz0);
  hipFree(p->d_dz1);
  hipFree(p->d_rowloss);
  long sumw = 0, maxw = 0;
  for (int x : p->w) {
    sumw += x;
    maxw = std::max<long>(maxw, x);
  }
  PCHK(hipMalloc(&p->d_act, (size_t)B * sumw * sizeof(float)));
  PCHK(hipMalloc(&p->d_dz0, (size_t)B * maxw * sizeof(float)));
  PCHK(hipMalloc(&p->d_dz1, (size_t)B * maxw * sizeof(float)));
  PCHK(hipMalloc(&p->d_rowloss, (size_t)B * sizeof(float)));
  p->cap = B;
  return QDP_OK;
}

extern "C" qdp_status qdp_policy_create(int32_t n_widths, const int32_t *widths, const float *params,
                                        const float *feat_mean, const float *feat_std, qdp_policy **out) {
  if (!out || !widths || !params || !feat_mean || !feat_std) return qdp_policy_fail(QDP_EINVAL, "NULL argument");
  *out = nullptr;
  if (n_widths < 2 || n_widths > 9) return qdp_policy_fail(QDP_EINVAL, "between 1 and 8 layers");
  for (int i = 0; i < n_widths; ++i)
    if (widths[i] < 1 || widths[i] > 256) return qdp_policy_fail(QDP_EINVAL, "layer widths must be in [1, 256]");
  if (widths[n_widths - 1] < 2) return qdp_policy_fail(QDP_EINVAL, "at least two outputs");
  auto *p = new qdp_policy();
  p->w.assign(widths, widths + n_widths);
  p->np = offset_of(p->w, n_widths - 1);
  for (long q = 0; q < p->np; ++q)
    if (!std::isfinite(params[q])) {
      delete p;
      return qdp_policy_fail(QDP_ENONFINITE, "non-finite parameter");
    }
  for (int f = 0; f < widths[0]; ++f) {
    if (!(feat_std[f] > 0.0f) || !std::isfinite(feat_mean[f])) {
      delete p;
      return qdp_policy_fail(QDP_EINVAL, "feature std must be > 0 and mean finite");
    }
    p->mean[f] = feat_mean[f];
    p->sd[f] = feat_std[f];
  }
  hipError_t e = hipMalloc(&p->d_w, n_widths * sizeof(int));
  if (e == hipSuccess) e = hipMalloc(&p->d_p, p->np * sizeof(float));
  if (e == hipSuccess) e = hipMalloc(&p->d_m, p->np * sizeof(float));
  if (e == hipSuccess) e = hipMalloc(&p->d_v, p->np * sizeof(float));
  if (e == hipSuccess) e = hipMalloc(&p->d_g, p->np * sizeof(float));
  if (e == hipSuccess) e = hipMalloc(&p->d_pbf, p->np * sizeof(unsigned short));
  if (e == hipSuccess) e = hipMalloc(&p->d_mean, widths[0] * sizeof(float));
  if (e == hipSuccess) e = hipMalloc(&p->d_sd, widths[0] * sizeof(float));
  if (e == hipSuccess) e = hipMalloc(&p->d_loss, sizeof(float));
  if (e == hipSuccess) e = hipMalloc(&p->d_x1, widths[0] * sizeof(float));
  if (e == hipSuccess) e = hipMalloc(&p->d_y1, widths[n_widths - 1] * sizeof(float));
  if (e == hipSuccess) e = hipMemcpy(p->d_w, widths, n_widths * sizeof(int), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(p->d_p, params, p->np * sizeof(float), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(p->d_m, 0, p->np * sizeof(float));
  if (e == hipSuccess) e = hipMemset(p->d_v, 0, p->np * sizeof(float));
  if (e == hipSuccess) e = hipMemcpy(p->d_mean, feat_mean, widths[0] * sizeof(float), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(p->d_sd, feat_std, widths[0] * sizeof(float), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    qdp_policy_destroy(p);
    return qdp_policy_fail(QDP_ENOMEM, hipGetErrorString(e));
  }
  *out = p;
  return QDP_OK;
}

extern "C" void qdp_policy_destroy(qdp_policy *p) {
  if (!p) return;
  for (void *q : {(void *)p->d_w, (void *)p->d_p, (void *)p->d_m, (void *)p->d_v, (void *)p->d_g, (void *)p->d_pbf,
                  (void *)p->d_mean, (void *)p->d_sd, (void *)p->d_act, (void *)p->d_dz0, (void *)p->d_dz1,
                  (void *)p->d_rowloss, (void *)p->d_loss, (void *)p->d_x1, (void *)p->d_y1})
    hipFree(q);
  delete p;
}

extern "C" qdp_status qdp_policy_get_params(const qdp_policy *pc, float *params) {
  if (!pc || !params) return qdp_policy_fail(QDP_EINVAL, "NULL argument");
  auto *p = const_cast<qdp_policy *>(pc);
  std::lock_guard<std::mutex> g(p->mu);
  PCHK(hipDeviceSynchronize());
  PCHK(hipMemcpy(params, p->d_p, p->np * sizeof(float), hipMemcpyDeviceToHost));
  return QDP_OK;
}

// forward of a training batch: keeps every layer's output in d_act
static qdp_status train_forward(qdp_policy *p, const float *X, int B, hipStream_t s) {
  const int nl = (int)p->w.size() - 1;
  float *act = p->d_act;
  const int F = p->w[0];
  hipLaunchKernelGGL(qdp::k_normalize, dim3((B * F + 255) / 256), dim3(256), 0, s, B, F, X, p->d_mean, p->d_sd, act);
  PCHK(hipGetLastError());
  long aoff = 0;
  for (int l = 0; l < nl; ++l) {
    const int in = p->w[l], out = p->w[l + 1];
    const float *W = p->d_p + offset_of(p->w, l);
    const float *bias = W + (long)out * in;
    float *H = act + aoff;
    float *Z = act + aoff + (long)B * in;
    // Z[m][n] = sum_k H[m][k] W[n][k]
    PCHK(qdp::gemm(l < nl - 1, B, out, in, H, in, 1, W, 1, in, bias, Z, out, 1, s));
    aoff += (long)B * in;
  }
  return QDP_OK;
}

// Policy file: the 8 bytes "QDPPOL1\0", int32 n_widths, int32 widths[n_widths],
// float params (flat layout), float feature mean[w_0], float feature std[w_0];
// little-endian, as the host writes them.  Adam moments are not stored.
static const char kPolicyMagic[8] = {'Q', 'D', 'P', 'P', 'O', 'L', '1', '\0'};

extern "C" qdp_status qdp_policy_save(const qdp_policy *pc, const char *path) {
  if (!pc || !path) return qdp_policy_fail(QDP_EINVAL, "NULL argument");
  std::vector<float> params((size_t)pc->np);
  qdp_status s = qdp_policy_get_params(pc, params.data());
  if (s != QDP_OK) return s;
  FILE *f = std::fopen(path, "wb");
  if (!f) return qdp_policy_fail(QDP_EINVAL, std::string("cannot open ") + path + " for writing");
  const int32_t nw = (int32_t)pc->w.size();
  std::vector<int32_t> w(pc->w.begin(), pc->w.end());
  bool ok = std::fwrite(kPolicyMagic, 1, 8, f) == 8 && std::fwrite(&nw, sizeof nw, 1, f) == 1 &&
            std::fwrite(w.data(), sizeof(int32_t), w.size(), f) == w.size() &&
            std::fwrite(params.data(), sizeof(float), params.size(), f) == params.size() &&
            std::fwrite(pc->mean, sizeof(float), (size_t)w[0], f) == (size_t)w[0] &&
            std::fwrite(pc->sd, sizeof(float), (size_t)w[0], f) == (size_t)w[0];
  ok = (std::fclose(f) == 0) && ok;
  return ok ? QDP_OK : qdp_policy_fail(QDP_EINVAL, std::string("write to ") + path + " failed");
}

extern "C" qdp_status qdp_policy_load(const char *path, qdp_policy **out) {
  if (!path || !out) return qdp_policy_fail(QDP_EINVAL, "NULL argument");
  *out = nullptr;
  FILE *f = std::fopen(path, "rb");
  if (!f) return qdp_policy_fail(QDP_EINVAL, std::string("cannot open ") + path);
  char magic[8];
  int32_t nw = 0;
  bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, kPolicyMagic, 8) == 0 &&
            std::fread(&nw, sizeof nw, 1, f) == 1 && nw >= 2 && nw <= 9;
  std::vector<int32_t> w(ok ? (size_t)nw : 0);
  if (ok) ok = std::fread(w.data(), sizeof(int32_t), w.size(), f) == w.size();
  if (ok)
    for (int32_t x : w) ok = ok && x >= 1 && x <= 256;
  std::vector<float> params, mean, sd;
  if (ok) {
    std::vector<int> wi(w.begin(), w.end());
    params.resize((size_t)offset_of(wi, nw - 1));
    mean.resize((size_t)w[0]);
    sd.resize((size_t)w[0]);
    ok = std::fread(params.data(), sizeof(float), params.size(), f) == params.size() &&
         std::fread(mean.data(), sizeof(float), mean.size(), f) == mean.size() &&
         std::fread(sd.data(), sizeof(float), sd.size(), f) == sd.size();
  }
  std::fclose(f);
  if (!ok) return qdp_policy_fail(QDP_EINVAL, std::string(path) + " is not a policy file of this library");
  return qdp_policy_create(nw, w.data(), params.data(), mean.data(), sd.data(), out);
}

extern "C" qdp_status qdp_policy_gradient(qdp_policy *p, const float *X, const float *Y, const float *Mk,
                                          int32_t B, float *grad_out, float *loss_out, void *stream) {
  if (!p || !X || !Y || !Mk) return qdp_policy_fail(QDP_EINVAL, "NULL argument");
  if (B < 1 || B > 65536) return qdp_policy_fail(QDP_EINVAL, "batch must be in [1, 65536]");
  std::lock_guard<std::mutex> g(p->mu);
  hipStream_t s = (hipStream_t)stream;
  qdp_status st = ensure_train_ws(p, B);
  if (st != QDP_OK) return st;
  if ((st = train_forward(p, X, B, s)) != QDP_OK) return st;
  const int nl = (int)p->w.size() - 1;
  const int O = p->w[nl];
  long aoff_last = 0;
  for (int l = 0; l < nl; ++l) aoff_last += (long)B * p->w[l];
  const float *out = p->d_act + aoff_last;
  float *dz = p->d_dz0, *dh = p->d_dz1;
  hipLaunchKernelGGL(qdp::k_loss_grad, dim3((B + 255) / 256), dim3(256), 0, s, B, O, out, Y, Mk, dz, p->d_rowloss);
  PCHK(hipGetLastError());
  hipLaunchKernelGGL(qdp::k_sum_loss, dim3(1), dim3(256), 0, s, B, p->d_rowloss, p->d_loss);
  PCHK(hipGetLastError());
  float *G = grad_out ? grad_out : p->d_g;
  long aoff = aoff_last;
  for (int l = nl - 1; l >= 0; --l) {
    const int in = p->w[l], outw = p->w[l + 1];
    aoff -= (long)B * in;
    const float *H = p->d_act + aoff;  // [B][in]
    const long woff = offset_of(p->w, l);
    const float *W = p->d_p + woff;
    float *dW = G + woff;
    float *db = dW + (long)outw * in;
    // dW[n][k] = sum_m dz[m][n] H[m][k]
    PCHK(qdp::gemm(false, outw, in, B, dz, 1, outw, H, in, 1, nullptr, dW, in, 1, s));
    hipLaunchKernelGGL(qdp::k_colsum, dim3((outw + 255) / 256), dim3(256), 0, s, B, outw, dz, db);
    PCHK(hipGetLastError());
    if (l > 0) {
      // dh[m][k] = sum_n dz[m][n] W[n][k]; dz_prev = dh * (H > 0)
      PCHK(qdp::gemm(false, B, in, outw, dz, outw, 1, W, in, 1, nullptr, dh, in, 1, s));
      const long cnt = (long)B * in;
      hipLaunchKernelGGL(qdp::k_relu_back, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s, cnt, dh, H);
      PCHK(hipGetLastError());
      float *t = dz;
      dz = dh;
      dh = t;
    }
  }
  if (loss_out) {
    PCHK(hipMemcpyAsync(loss_out, p->d_loss, sizeof(float), hipMemcpyDeviceToHost, s));
    PCHK(hipStreamSynchronize(s));
  }
  return QDP_OK;
}

extern "C" qdp_status qdp_policy_adam_step(qdp_policy *p, const float *grad, float lr, float b1, float b2, float eps,
                                           void *stream) {
  if (!p) return qdp_policy_fail(QDP_EINVAL, "NULL policy");
  if (!(lr > 0) || !(b1 >= 0 && b1 < 1) || !(b2 >= 0 && b2 < 1) || !(eps > 0))
    return qdp_policy_fail(QDP_EINVAL, "bad Adam hyper-parameters");
  std::lock_guard<std::mutex> g(p->mu);
  p->step += 1;
  const float c1 = 1.0f - std::pow(b1, (float)p->step), c2 = 1.0f - std::pow(b2, (float)p->step);
  hipLaunchKernelGGL(qdp::k_adam, dim3((unsigned)((p->np + 255) / 256)), dim3(256), 0, (hipStream_t)stream, p->np,
                     p->d_p, grad ? grad : p->d_g, p->d_m, p->d_v, lr, b1, b2, eps, c1, c2);
  PCHK(hipGetLastError());
  p->bf16_stale = true;
  return QDP_OK;
}

extern "C" qdp_status qdp_policy_train_step(qdp_policy *p, const float *X, const float *Y, const float *Mk, int32_t B,
                                            float lr, float b1, float b2, float eps, float *loss_out, void *stream) {
  qdp_status s = qdp_policy_gradient(p, X, Y, Mk, B, nullptr, loss_out, stream);
  if (s != QDP_OK) return s;
  return qdp_policy_adam_step(p, nullptr, lr, b1, b2, eps, stream);
}

static qdp_status refresh_bf16(qdp_policy *p, hipStream_t s) {
  if (!p->bf16_stale) return QDP_OK;
  hipLaunchKernelGGL(qdp::k_to_bf16_t, dim3(64), dim3(256), 0, s, (int)p->w.size() - 1, p->d_w, p->d_p, p->d_pbf);
  PCHK(hipGetLastError());
  p->bf16_stale = false;
  return QDP_OK;
}

extern "C" qdp_status qdp_policy_forward(const qdp_policy *pc, const float *X, int32_t B, int32_t use_bf16, float *Y,
                                         void *stream) {
  if (!pc || !X || !Y) return qdp_policy_fail(QDP_EINVAL, "NULL argument");
  if (B < 1 || B > 65536) return qdp_policy_fail(QDP_EINVAL, "batch must be in [1, 65536]");
  auto *p = const_cast<qdp_policy *>(pc);
  std::lock_guard<std::mutex> g(p->mu);
  hipStream_t s = (hipStream_t)stream;
  const int nl = (int)p->w.size() - 1;
  if (use_bf16) {
    qdp_status st = refresh_bf16(p, s);
    if (st != QDP_OK) return st;
    hipLaunchKernelGGL(qdp::k_infer<true>, dim3(B), dim3(256), 0, s, B, nl, p->d_w, X, p->d_mean, p->d_sd,
                       (const void *)p->d_pbf, Y);
  } else {
    hipLaunchKernelGGL(qdp::k_infer<false>, dim3(B), dim3(256), 0, s, B, nl, p->d_w, X, p->d_mean, p->d_sd,
                       (const void *)p->d_p, Y);
  }
  PCHK(hipGetLastError());
  return QDP_OK;
}

// one-row inference from host features, used by the tracker (synchronous)
extern "C" qdp_status qdp_policy_infer_host(const qdp_policy *pc, const float *x, float *y, void *stream) {
  if (!pc || !x || !y) return qdp_policy_fail(QDP_EINVAL, "NULL argument");
  auto *p = const_cast<qdp_policy *>(pc);
  hipStream_t s = (hipStream_t)stream;
  {
    std::lock_guard<std::mutex> g(p->mu);
    PCHK(hipMemcpyAsync(p->d_x1, x, p->w[0] * sizeof(float), hipMemcpyHostToDevice, s));
  }
  qdp_status st = qdp_policy_forward(pc, p->d_x1, 1, 1, p->d_y1, stream);
  if (st != QDP_OK) return st;
  std::lock_guard<std::mutex> g(p->mu);
  PCHK(hipMemcpyAsync(y, p->d_y1, p->w.back() * sizeof(float), hipMemcpyDeviceToHost, s));
  PCHK(hipStreamSynchronize(s));
  return QDP_OK;
}
