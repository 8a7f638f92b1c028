// Learned PP switch: a perceptron D -> H -> H -> 1 (tanh hidden units,
// sigmoid output) trained with binary cross-entropy and Adam, on the GPU.
// Not part of the paper, which decides with the hand threshold of Alg. 2;
// the network replaces that threshold (declarations in include/cpals.h).
//
// Parameter vector theta (FP32): W1 (D x H, input index slowest), b1 (H),
// W2 (H x H), b2 (H), w3 (H), b3 (1).
// Every reduction over samples runs in sample order in one thread, so
// gradients are bitwise reproducible.
#include <hip/hip_runtime.h>
#include <math.h>

#include <atomic>
#include <cmath>

#include "../../include/cpals.h"

namespace {

constexpr int kMaxHidden = 128;
constexpr int kMaxInput = 16;

struct Offsets {
  int W1, b1, W2, b2, w3, b3, n;
};

__host__ __device__ inline Offsets offsets(int D, int H) {
  Offsets o;
  o.W1 = 0;
  o.b1 = D * H;
  o.W2 = o.b1 + H;
  o.b2 = o.W2 + H * H;
  o.w3 = o.b2 + H;
  o.b3 = o.w3 + H;
  o.n = o.b3 + 1;
  return o;
}

// One thread per sample: hidden layers (kept for the backward pass when H1 /
// H2 are given), probability p = sigmoid(z), and z.
__global__ __launch_bounds__(256) void k_mlp_forward(const float* __restrict__ X, const float* __restrict__ th,
                                                     int B, int D, int H, float* __restrict__ H1,
                                                     float* __restrict__ H2, float* __restrict__ p,
                                                     float* __restrict__ zout) {
  extern __shared__ float sp[];
  const Offsets o = offsets(D, H);
  for (int i = threadIdx.x; i < o.n; i += 256) sp[i] = th[i];
  __syncthreads();
  const int b = blockIdx.x * 256 + threadIdx.x;
  if (b >= B) return;
  float x[kMaxInput];
  for (int d = 0; d < D; ++d) x[d] = X[(int64_t)b * D + d];
  float h1[kMaxHidden];
  for (int j = 0; j < H; ++j) {
    float s = sp[o.b1 + j];
    for (int d = 0; d < D; ++d) s += x[d] * sp[o.W1 + d * H + j];
    h1[j] = tanhf(s);
    if (H1) H1[(int64_t)b * H + j] = h1[j];
  }
  float z = sp[o.b3];
  for (int j = 0; j < H; ++j) {
    float s = sp[o.b2 + j];
    for (int i = 0; i < H; ++i) s += h1[i] * sp[o.W2 + i * H + j];
    const float h2 = tanhf(s);
    if (H2) H2[(int64_t)b * H + j] = h2;
    z += h2 * sp[o.w3 + j];
  }
  p[b] = 1.0f / (1.0f + expf(-z));
  if (zout) zout[b] = z;
}

// One thread per sample: dz = (p - y) / B, dH2 = dz w3 (1 - H2^2),
// dH1 = (dH2 W2^T) (1 - H1^2); also the per-sample loss softplus(z) - y z.
__global__ __launch_bounds__(256) void k_mlp_back_rows(const float* __restrict__ th, const float* __restrict__ y,
                                                       int B, int D, int H, const float* __restrict__ H1,
                                                       const float* __restrict__ H2, const float* __restrict__ p,
                                                       const float* __restrict__ z, float* __restrict__ dz,
                                                       float* __restrict__ dH2, float* __restrict__ dH1,
                                                       float* __restrict__ lrow) {
  extern __shared__ float sp[];
  const Offsets o = offsets(D, H);
  for (int i = threadIdx.x; i < o.n; i += 256) sp[i] = th[i];
  __syncthreads();
  const int b = blockIdx.x * 256 + threadIdx.x;
  if (b >= B) return;
  const float d = (p[b] - y[b]) / (float)B;
  dz[b] = d;
  const float zb = z[b];
  lrow[b] = (zb > 0.f ? zb + log1pf(expf(-zb)) : log1pf(expf(zb))) - y[b] * zb;
  float g2[kMaxHidden];
  for (int j = 0; j < H; ++j) {
    const float h = H2[(int64_t)b * H + j];
    g2[j] = d * sp[o.w3 + j] * (1.f - h * h);
    dH2[(int64_t)b * H + j] = g2[j];
  }
  for (int i = 0; i < H; ++i) {
    float s = 0.f;
    for (int j = 0; j < H; ++j) s += g2[j] * sp[o.W2 + i * H + j];
    const float h = H1[(int64_t)b * H + i];
    dH1[(int64_t)b * H + i] = s * (1.f - h * h);
  }
}

// One thread per parameter: the gradient as a sum over samples in order.
// Thread 0 of block 0 also writes the mean loss to g[n].
__global__ __launch_bounds__(256) void k_mlp_wgrad(const float* __restrict__ X, int B, int D, int H,
                                                   const float* __restrict__ H1, const float* __restrict__ H2,
                                                   const float* __restrict__ dz, const float* __restrict__ dH2,
                                                   const float* __restrict__ dH1, const float* __restrict__ lrow,
                                                   float* __restrict__ g) {
  const Offsets o = offsets(D, H);
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e < o.n) {
    float s = 0.f;
    if (e < o.b1) {
      const int d = e / H, j = e % H;
      for (int b = 0; b < B; ++b) s += X[(int64_t)b * D + d] * dH1[(int64_t)b * H + j];
    } else if (e < o.W2) {
      const int j = e - o.b1;
      for (int b = 0; b < B; ++b) s += dH1[(int64_t)b * H + j];
    } else if (e < o.b2) {
      const int i = (e - o.W2) / H, j = (e - o.W2) % H;
      for (int b = 0; b < B; ++b) s += H1[(int64_t)b * H + i] * dH2[(int64_t)b * H + j];
    } else if (e < o.w3) {
      const int j = e - o.b2;
      for (int b = 0; b < B; ++b) s += dH2[(int64_t)b * H + j];
    } else if (e < o.b3) {
      const int j = e - o.w3;
      for (int b = 0; b < B; ++b) s += H2[(int64_t)b * H + j] * dz[b];
    } else {
      for (int b = 0; b < B; ++b) s += dz[b];
    }
    g[e] = s;
  }
  if (e == 0) {
    float l = 0.f;
    for (int b = 0; b < B; ++b) l += lrow[b];
    g[o.n] = l / (float)B;
  }
}

// Adam (Kingma & Ba, Alg. 1), one thread per parameter; t counts from 1.
__global__ __launch_bounds__(256) void k_adam(float* __restrict__ th, const float* __restrict__ g,
                                              float* __restrict__ m, float* __restrict__ v, int n, float c1,
                                              float c2, float lr, float b1, float b2, float eps) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= n) return;
  const float gi = g[e];
  const float mi = b1 * m[e] + (1.f - b1) * gi;
  const float vi = b2 * v[e] + (1.f - b2) * gi * gi;
  m[e] = mi;
  v[e] = vi;
  th[e] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

inline cp_status hip_status(hipError_t e) { return e == hipSuccess ? CP_OK : CP_ERR_HIP; }

bool dims_ok(int B, int D, int H) {
  return B >= 1 && D >= 1 && D <= kMaxInput && H >= 1 && H <= kMaxHidden;
}

// The largest parameter vector (D = 16, H = 128) takes 75 KB of LDS, above
// the default dynamic limit of 64 KB.
// The attribute belongs to the device: set once per device index (one bit
// each below 64; two first calls at once both set it, harmlessly).
hipError_t allow_large_lds() {
  static std::atomic<uint64_t> done{0};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  const uint64_t bit = (dev >= 0 && dev < 64) ? (1ull << dev) : 0;
  if (bit && (done.load(std::memory_order_acquire) & bit)) return hipSuccess;
  const int bytes = (int)(offsets(kMaxInput, kMaxHidden).n * sizeof(float));
  e = hipFuncSetAttribute((const void*)k_mlp_forward, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)k_mlp_back_rows, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (e == hipSuccess && bit) done.fetch_or(bit, std::memory_order_release);
  return e;
}

}  // namespace

extern "C" {

size_t cp_mlp_param_count(int D, int H) { return (size_t)offsets(D, H).n; }

size_t cp_mlp_scratch_floats(int B, int H) { return (size_t)B * (4 * (size_t)H + 4); }

cp_status cp_mlp_forward(const float* X, int B, int D, int H, const float* theta, float* p, void* stream) {
  if (!X || !theta || !p) return CP_ERR_ARG;
  if (!dims_ok(B, D, H)) return CP_ERR_UNSUPPORTED;
  const size_t lds = (size_t)offsets(D, H).n * sizeof(float);
  if (allow_large_lds() != hipSuccess) return CP_ERR_HIP;
  hipLaunchKernelGGL(k_mlp_forward, dim3((B + 255) / 256), dim3(256), lds, (hipStream_t)stream, X, theta, B, D, H,
                     (float*)nullptr, (float*)nullptr, p, (float*)nullptr);
  return hip_status(hipGetLastError());
}

cp_status cp_mlp_grad(const float* X, const float* y, int B, int D, int H, const float* theta, float* grad,
                      float* scratch, void* stream) {
  if (!X || !y || !theta || !grad || !scratch) return CP_ERR_ARG;
  if (!dims_ok(B, D, H)) return CP_ERR_UNSUPPORTED;
  hipStream_t st = (hipStream_t)stream;
  const Offsets o = offsets(D, H);
  const size_t lds = (size_t)o.n * sizeof(float);
  if (allow_large_lds() != hipSuccess) return CP_ERR_HIP;
  float* H1 = scratch;
  float* H2 = H1 + (size_t)B * H;
  float* dH2 = H2 + (size_t)B * H;
  float* dH1 = dH2 + (size_t)B * H;
  float* p = dH1 + (size_t)B * H;
  float* z = p + B;
  float* dz = z + B;
  float* lrow = dz + B;
  const unsigned nb = (unsigned)((B + 255) / 256);
  hipLaunchKernelGGL(k_mlp_forward, dim3(nb), dim3(256), lds, st, X, theta, B, D, H, H1, H2, p, z);
  hipLaunchKernelGGL(k_mlp_back_rows, dim3(nb), dim3(256), lds, st, theta, y, B, D, H, H1, H2, p, z, dz, dH2, dH1,
                     lrow);
  hipLaunchKernelGGL(k_mlp_wgrad, dim3((o.n + 255) / 256), dim3(256), 0, st, X, B, D, H, H1, H2, dz, dH2, dH1,
                     lrow, grad);
  return hip_status(hipGetLastError());
}

cp_status cp_mlp_adam(float* theta, const float* grad, float* m, float* v, int n, int t, float lr, float beta1,
                      float beta2, float eps, void* stream) {
  if (!theta || !grad || !m || !v || n < 1 || t < 1) return CP_ERR_ARG;
  // bias corrections in FP64: 1 - beta2^t cancels heavily for small t
  const float c1 = (float)(1.0 - std::pow((double)beta1, (double)t));
  const float c2 = (float)(1.0 - std::pow((double)beta2, (double)t));
  hipLaunchKernelGGL(k_adam, dim3((n + 255) / 256), dim3(256), 0, (hipStream_t)stream, theta, grad, m, v, n, c1, c2,
                     lr, beta1, beta2, eps);
  return hip_status(hipGetLastError());
}

}  // extern "C"
