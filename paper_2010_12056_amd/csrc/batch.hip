// Batched CP-ALS on many small independent order-3 tensors in one persistent
// launch (not from the paper; the paper decomposes one large tensor).
//
// Work queue: a device counter hands whole tensors, largest first (the host
// orders them by s0 s1 s2 R), to whichever workgroup is free; the workgroup
// runs all requested sweeps of that tensor and takes the next.  Tensors are
// independent, so no workgroup ever waits for another, and every workgroup
// leaves the loop once the counter passes the last tensor.
//
// One sweep per tensor is the standard dimension tree for N = 3 (Sec. II-C,
// Alg. 1): Y = T x_2 A2 (first-level contraction over the last mode) serves
// modes 0 and 1, Z = T x_0 A0 (over the first mode) serves mode 2:
//   M0[i][r] = sum_j Y[i][j][r] A1[j][r]      A0 <- M0 Gamma0^-1   (Eq. (1))
//   M1[j][r] = sum_i Y[i][j][r] A0[i][r]      A1 <- M1 Gamma1^-1
//   M2[k][r] = sum_j Z[j][k][r] A1[j][r]      A2 <- M2 Gamma2^-1
// then the residual by Eq. (3).  Contractions with the tensor run on the
// FP32 matrix cores (16x16x4), Y and Z are FP32 in a per-slot scratch, the
// second level, the Gram matrices, Gamma, its inverse (Gauss-Jordan without
// pivoting, SPD) and the update run in FP64 on factors held in LDS for all the
// tensor's sweeps.  Every reduction has a fixed
// order: results do not depend on which workgroup took which tensor.
#include "kernels.h"
#include "blocked_inverse.h"

#include "../../include/cpals.h"

#include <algorithm>
#include <string>
#include <vector>

namespace cpals {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kMaxS = 96;    // largest mode size
constexpr int kMaxR = 32;    // largest rank
constexpr int kKP = kMaxS + 4;  // staged factor pitch (floats): 16 lanes' rows fall in different banks

struct BatchTensor {
  int64_t t_off;     // first element of the tensor in the packed tensor array
  int idx;           // position in the caller's list (results are stored there)
  int64_t a_off[3];  // first element of each factor in the packed factor array
  int s[3];
  int R;
};

struct BatchArgs {
  const float* T;
  double* A;
  const BatchTensor* items;  // in queue order
  int count;
  int sweeps;
  double* fitness;   // [count][sweeps], by the tensor's position in the caller's list
  int* status;       // [count]: 0 ok, 1 Gamma not positive definite
  long long* ticks;  // [count][2] wall-clock start / end, or null
  int* counter;
  float* scratch;    // gridDim.x slots of slot_floats
  int64_t slot_floats;
};

// Shared state of one workgroup: the three factors of the tensor in work
// (FP64, resident for all its sweeps), their Gram matrices, Gamma and its
// inverse, the MTTKRP of the mode being updated, the FP32 factor staged for
// the contraction with the tensor.  About 145 KB: one workgroup per CU.
struct Lds {
  double F[3][kMaxS * kMaxR];
  double S[3][kMaxR * kMaxR];
  double G[kMaxR * (kMaxR + 1)];   // Gamma, then its inverse in place (RP x RP, pitch RP + 1)
  double M[kMaxS * kMaxR];
  float Bt[kMaxR * kKP];            // FP32 factor transposed for the contraction, zero padded
  double red[512];
  int item;
  int fail;
};

template <int NT>
__device__ inline double block_sum(Lds& L, double v) {
  const int t = threadIdx.x;
  L.red[t] = v;
  __syncthreads();
  for (int h = NT / 2; h > 0; h >>= 1) {
    if (t < h) L.red[t] += L.red[t + h];
    __syncthreads();
  }
  const double s = L.red[0];
  __syncthreads();
  return s;
}

// Stage factor m (s x R, FP64 in LDS) as Bt[c][k] (FP32), zero for k >= s or c >= R.
template <int NT, int RP>
__device__ __forceinline__ void stage_factor(Lds& L, int m, int s, int R) {
  const int KP = (s + 15) & ~15;
  for (int e = threadIdx.x; e < RP * KP; e += NT) {
    const int c = e / KP, k = e - c * KP;
    L.Bt[c * kKP + k] = (k < s && c < R) ? (float)L.F[m][k * R + c] : 0.f;
  }
}

// C[p][r] = sum_k X[p][k] B[k][r] (X is P x K row-major): 16-row tiles per wave.
// NB = ceil(K / 16) is a template parameter so that every loop over the
// contraction is unrolled (the staged factor is zero up to 16 NB).  Lane
// (i, g) feeds k = 16 t + 4 g + u at MFMA step (t, u) (one 16-byte load when
// the row is 16-byte aligned, VEC: K % 4 == 0); its factor operands are the
// same for every tile and stay in registers.  Every load is unconditional:
// rows past P read row P - 1 (never stored) and indices past K read index
// K - 1 (or K - 4), which the factor's zero padding cancels.  The next tile's
// rows are in flight while a tile is multiplied (past the last tile it
// reloads the last, unused), and a scheduling barrier keeps those loads
// ahead of the products.
template <int NT, int RP, int NB, bool VEC>
__device__ __forceinline__ void ttm_rows(Lds& L, const float* X, int64_t P, int K, int R, float* C) {
  constexpr int NCB = RP / 16;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, l16 = lane & 15;
  const int64_t ntiles = (P + 15) / 16;
  auto load_tile = [&](int64_t tile, f32x4 (&a)[NB]) {
    const int64_t p0 = tile * 16;
    const int64_t row = (p0 + l16 < P) ? p0 + l16 : P - 1;
    const float* xr = X + row * K;
#pragma unroll
    for (int t = 0; t < NB; ++t) {
      const int k0 = 16 * t + 4 * g;
      if (VEC) {
        a[t] = *(const f32x4*)(xr + (k0 + 4 <= K ? k0 : K - 4));
      } else {
#pragma unroll
        for (int u = 0; u < 4; ++u) a[t][u] = xr[k0 + u < K ? k0 + u : K - 1];
      }
    }
  };
  constexpr int NW = NT / 64;
  if (wave >= ntiles) return;
  f32x4 b[NB][NCB];
#pragma unroll
  for (int t = 0; t < NB; ++t)
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) b[t][cb] = *(const f32x4*)&L.Bt[(cb * 16 + l16) * kKP + 16 * t + 4 * g];
  f32x4 an[NB];
  load_tile(wave, an);
  for (int64_t tile = wave; tile < ntiles; tile += NW) {
    f32x4 a[NB];
#pragma unroll
    for (int t = 0; t < NB; ++t) a[t] = an[t];
    load_tile(tile + NW < ntiles ? tile + NW : tile, an);
    __builtin_amdgcn_sched_barrier(0);
    const int64_t p0 = tile * 16;
    f32x4 acc[NCB];
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) acc[cb] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int t = 0; t < NB; ++t)
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb)
          acc[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[t][u], b[t][cb][u], acc[cb], 0, 0, 0);
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t p = p0 + 4 * g + v;
        const int c = cb * 16 + l16;
        if (p < P && c < R) C[p * R + c] = acc[cb][v];
      }
  }
}

// C[q][r] = sum_k X[k][q] B[k][r] (X is K x Q, q contiguous): 16-row tiles of
// q per wave; lane (i, g) feeds X[4 t + g][q0 + i] (16 lanes read 64
// contiguous bytes), NB = ceil(K / 16) as in ttm_rows, the factor operands
// read from LDS at each step, unconditional clamped loads (q past Q read column Q - 1, never
// stored; k past K read row K - 1, cancelled by the factor's zero padding),
// the next tile in flight while a tile is multiplied.
template <int NT, int RP, int NB>
__device__ __forceinline__ void ttm_cols(Lds& L, const float* X, int K, int64_t Q, int R, float* C) {
  constexpr int NCB = RP / 16;
  constexpr int NKS = 4 * NB;  // 4-index steps
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, l16 = lane & 15;
  const int64_t ntiles = (Q + 15) / 16;
  auto load_tile = [&](int64_t tile, float (&a)[NKS]) {
    const int64_t q = tile * 16 + l16 < Q ? tile * 16 + l16 : Q - 1;
    const float* xq = X + q;
#pragma unroll
    for (int t = 0; t < NKS; ++t) {
      const int k = 4 * t + g;
      a[t] = xq[(int64_t)(k < K ? k : K - 1) * Q];
    }
  };
  constexpr int NW = NT / 64;
  if (wave >= ntiles) return;
  float an[NKS];
  load_tile(wave, an);
  for (int64_t tile = wave; tile < ntiles; tile += NW) {
    float a[NKS];
#pragma unroll
    for (int t = 0; t < NKS; ++t) a[t] = an[t];
    load_tile(tile + NW < ntiles ? tile + NW : tile, an);
    __builtin_amdgcn_sched_barrier(0);
    const int64_t q0 = tile * 16;
    f32x4 acc[NCB];
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) acc[cb] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int t = 0; t < NKS; ++t)
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb)
        acc[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[t], L.Bt[(cb * 16 + l16) * kKP + 4 * t + g], acc[cb], 0, 0, 0);
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t q = q0 + 4 * g + v;
        const int c = cb * 16 + l16;
        if (q < Q && c < R) C[q * R + c] = acc[cb][v];
      }
  }
}

// The contractions for K <= kMaxS, with the block count as a compile-time constant.
template <int NT, int RP, bool VEC>
__device__ __forceinline__ void ttm_rows_kv(Lds& L, const float* X, int64_t P, int K, int R, float* C) {
  switch ((K + 15) / 16) {
    case 1: ttm_rows<NT, RP, 1, VEC>(L, X, P, K, R, C); break;
    case 2: ttm_rows<NT, RP, 2, VEC>(L, X, P, K, R, C); break;
    case 3: ttm_rows<NT, RP, 3, VEC>(L, X, P, K, R, C); break;
    case 4: ttm_rows<NT, RP, 4, VEC>(L, X, P, K, R, C); break;
    case 5: ttm_rows<NT, RP, 5, VEC>(L, X, P, K, R, C); break;
    default: ttm_rows<NT, RP, 6, VEC>(L, X, P, K, R, C); break;
  }
}
template <int NT, int RP>
__device__ __forceinline__ void ttm_rows_k(Lds& L, const float* X, int64_t P, int K, int R, float* C) {
  if (K % 4 == 0 && ((uintptr_t)X & 15) == 0)
    ttm_rows_kv<NT, RP, true>(L, X, P, K, R, C);
  else
    ttm_rows_kv<NT, RP, false>(L, X, P, K, R, C);
}
template <int NT, int RP>
__device__ __forceinline__ void ttm_cols_k(Lds& L, const float* X, int K, int64_t Q, int R, float* C) {
  switch ((K + 15) / 16) {
    case 1: ttm_cols<NT, RP, 1>(L, X, K, Q, R, C); break;
    case 2: ttm_cols<NT, RP, 2>(L, X, K, Q, R, C); break;
    case 3: ttm_cols<NT, RP, 3>(L, X, K, Q, R, C); break;
    case 4: ttm_cols<NT, RP, 4>(L, X, K, Q, R, C); break;
    case 5: ttm_cols<NT, RP, 5>(L, X, K, Q, R, C); break;
    default: ttm_cols<NT, RP, 6>(L, X, K, Q, R, C); break;
  }
}
static_assert(kMaxS <= 6 * 16, "contraction block dispatch covers kMaxS");

// Gamma = S[a] * S[b] (Hadamard), padded to RP x RP with the identity and
// inverted in place by the blocked Gauss-Jordan elimination without pivoting
// (SPD: every pivot is a positive Schur-complement diagonal); a pivot at or
// below R eps max(diag) flags L.fail.
template <int NT, int RP>
__device__ __forceinline__ void gamma_inverse(Lds& L, int a, int b, int R) {
  constexpr int P = RP + 1;
  double dm = 0.0;
  for (int e = threadIdx.x; e < RP * RP; e += NT) {
    const int i = e / RP, j = e - i * RP;
    double v;
    if (i < R && j < R) {
      v = L.S[a][i * R + j] * L.S[b][i * R + j];
      if (i == j) dm = fmax(dm, v);
    } else {
      v = (i == j) ? 1.0 : 0.0;
    }
    L.G[i * P + j] = v;
  }
  // largest diagonal entry (fixed tree, every thread gets it)
  L.red[threadIdx.x] = dm;
  __syncthreads();
  for (int h = NT / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) L.red[threadIdx.x] = fmax(L.red[threadIdx.x], L.red[threadIdx.x + h]);
    __syncthreads();
  }
  const double tol = L.red[0] * (double)R * 2.220446049250313e-16;
  __syncthreads();
  if (!gj_inverse_lds<RP, NT / 64, false>(L.G, tol, &L.fail, L.red)) {
    if (threadIdx.x == 0) L.fail = 1;
    __syncthreads();
  }
}

// F[m] <- M Ginv (FP64, s x R, in LDS; Ginv with pitch RP + 1) and S[m] <- F[m]^T F[m].
template <int NT, int RP>
__device__ __forceinline__ void update_factor(Lds& L, int s, int R, int m) {
  constexpr int P = RP + 1;
  for (int e = threadIdx.x; e < s * R; e += NT) {
    const int i = e / R, r = e - i * R;
    double acc = 0.0;
    for (int c = 0; c < R; ++c) acc += L.M[i * R + c] * L.G[c * P + r];
    L.F[m][e] = acc;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < R * R; e += NT) {
    const int a = e / R, b = e - a * R;
    double acc = 0.0;
    for (int i = 0; i < s; ++i) acc += L.F[m][i * R + a] * L.F[m][i * R + b];
    L.S[m][e] = acc;
  }
  __syncthreads();
}

// M[o][r] = sum_x Y[(o * so + x * sx) * R + r] * F[f][x][r] for o < n, x < nx
// (the second level).  Thread t owns the outputs t, t + NT, ... and takes
// them three at a time: eight x of the three are loaded at once (clamped
// indices, masked terms), 24 loads in flight; each sum runs in x order.
template <int NT>
__device__ __forceinline__ void second_level(Lds& L, const float* Y, int n, int nx, int64_t so, int64_t sx, int f, int R) {
  constexpr int J = 3;
  const int nout = n * R;
  const int64_t step = sx * R;
  for (int e0 = threadIdx.x; e0 < nout; e0 += NT * J) {
    const float* yp[J];
    int rr[J];
    double acc[J];
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int e = e0 + NT * j;
      const int ee = e < nout ? e : e0;
      const int o = ee / R;
      rr[j] = ee - o * R;
      yp[j] = Y + (int64_t)o * so * R + rr[j];
      acc[j] = 0.0;
    }
#pragma unroll 1
    for (int x0 = 0; x0 < nx; x0 += 8) {
      float yv[J][8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int64_t off = (int64_t)(x0 + u < nx ? x0 + u : nx - 1) * step;
#pragma unroll
        for (int j = 0; j < J; ++j) yv[j][u] = yp[j][off];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        if (x0 + u < nx) {
#pragma unroll
          for (int j = 0; j < J; ++j) acc[j] += (double)yv[j][u] * L.F[f][(x0 + u) * R + rr[j]];
        }
      }
    }
#pragma unroll
    for (int j = 0; j < J; ++j)
      if (e0 + NT * j < nout) L.M[e0 + NT * j] = acc[j];
  }
}

template <int NT, int RP>
__device__ __forceinline__ void run_tensor(Lds& L, const BatchArgs& a, const BatchTensor& t, int idx, float* scratch) {
  const int s0 = t.s[0], s1 = t.s[1], s2 = t.s[2], R = t.R;
  const int sz[3] = {s0, s1, s2};
  const float* T = a.T + t.t_off;
  const int64_t numel = (int64_t)s0 * s1 * s2;
  // the factors into LDS, ||T||^2, the Gram matrices of the initial factors
  for (int m = 0; m < 3; ++m)
    for (int e = threadIdx.x; e < sz[m] * R; e += NT) L.F[m][e] = a.A[t.a_off[m] + e];
  // ||T||^2: thread t takes the 16-byte pieces t, t + NT, ... (the packed
  // tensors start 16-byte aligned), eight pieces in flight, then the tail
  double nt = 0.0;
  {
    const int64_t nv = (((uintptr_t)T & 15) == 0) ? numel / 4 : 0;  // else element by element
    const f32x4* T4 = (const f32x4*)T;
    for (int64_t v0 = threadIdx.x; v0 < nv; v0 += 8 * (int64_t)NT) {
      f32x4 x[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int64_t v = v0 + (int64_t)u * NT;
        x[u] = T4[v < nv ? v : 0];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (v0 + (int64_t)u * NT < nv)
#pragma unroll
          for (int c = 0; c < 4; ++c) nt += (double)x[u][c] * (double)x[u][c];
    }
    for (int64_t e = nv * 4 + threadIdx.x; e < numel; e += NT) nt += (double)T[e] * (double)T[e];
  }
  const double normT2 = block_sum<NT>(L, nt);  // (its barriers also publish F)
  for (int m = 0; m < 3; ++m)
    for (int e = threadIdx.x; e < R * R; e += NT) {
      const int p = e / R, q = e - p * R;
      double acc = 0.0;
      for (int i = 0; i < sz[m]; ++i) acc += L.F[m][i * R + p] * L.F[m][i * R + q];
      L.S[m][e] = acc;
    }
  if (threadIdx.x == 0) L.fail = 0;
  __syncthreads();
  float* Y = scratch;
  for (int sw = 0; sw < a.sweeps; ++sw) {
    // Y = T x_2 A2 over rows (i, j)
    stage_factor<NT, RP>(L, 2, s2, R);
    __syncthreads();
    ttm_rows_k<NT, RP>(L, T, (int64_t)s0 * s1, s2, R, Y);
    __syncthreads();
    // mode 0: M0[i] = sum_j Y[i][j] * A1[j]
    second_level<NT>(L, Y, s0, s1, s1, 1, 1, R);
    gamma_inverse<NT, RP>(L, 1, 2, R);
    if (L.fail) break;
    update_factor<NT, RP>(L, s0, R, 0);
    // mode 1: M1[j] = sum_i Y[i][j] * A0[i]
    second_level<NT>(L, Y, s1, s0, 1, s1, 0, R);
    gamma_inverse<NT, RP>(L, 0, 2, R);
    if (L.fail) break;
    update_factor<NT, RP>(L, s1, R, 1);
    // Z = T x_0 A0 over columns (j, k)
    stage_factor<NT, RP>(L, 0, s0, R);
    __syncthreads();
    ttm_cols_k<NT, RP>(L, T, s0, (int64_t)s1 * s2, R, Y);
    __syncthreads();
    // mode 2: M2[k] = sum_j Z[j][k] * A1[j]
    second_level<NT>(L, Y, s2, s1, 1, s2, 1, R);
    gamma_inverse<NT, RP>(L, 0, 1, R);
    if (L.fail) break;
    update_factor<NT, RP>(L, s2, R, 2);
    // residual, Eq. (3): ||T||^2 + <Gamma2, S2> - 2 <M2, A2>, Gamma2 = S0 * S1
    double part = 0.0;
    for (int e = threadIdx.x; e < R * R; e += NT) part += L.S[0][e] * L.S[1][e] * L.S[2][e];
    for (int e = threadIdx.x; e < s2 * R; e += NT) part -= 2.0 * L.M[e] * L.F[2][e];
    const double num = normT2 + block_sum<NT>(L, part);
    if (threadIdx.x == 0) a.fitness[(int64_t)idx * a.sweeps + sw] = 1.0 - sqrt((num > 0.0 ? num : 0.0) / normT2);
  }
  // factors back to the caller's array
  for (int m = 0; m < 3; ++m)
    for (int e = threadIdx.x; e < sz[m] * R; e += NT) a.A[t.a_off[m] + e] = L.F[m][e];
  if (threadIdx.x == 0) a.status[idx] = L.fail ? 1 : 0;
  __syncthreads();
}

template <int NT>
__global__ __launch_bounds__(NT) void k_batch(BatchArgs a) {
  __shared__ Lds L;
  float* scratch = a.scratch + (int64_t)blockIdx.x * a.slot_floats;
  for (;;) {
    if (threadIdx.x == 0) L.item = atomicAdd(a.counter, 1);
    __syncthreads();
    const int q = L.item;
    __syncthreads();
    if (q >= a.count) break;  // uniform: every workgroup leaves once the queue is empty
    const BatchTensor t = a.items[q];
    const int idx = t.idx;
    long long t0 = 0;
    if (threadIdx.x == 0 && a.ticks) t0 = wall_clock64();
    if (t.R <= 16)
      run_tensor<NT, 16>(L, a, t, idx, scratch);
    else
      run_tensor<NT, 32>(L, a, t, idx, scratch);
    if (threadIdx.x == 0 && a.ticks) {
      a.ticks[2 * idx] = t0;
      a.ticks[2 * idx + 1] = wall_clock64();
    }
  }
}

__global__ void k_reset_counter(int* c) {
  if (threadIdx.x == 0) *c = 0;
}

}  // namespace
}  // namespace cpals

using namespace cpals;

struct cp_batch_s {
  int count = 0;
  hipStream_t st = nullptr;
  std::vector<BatchTensor> items;  // queue order
  std::vector<int> order;          // queue position -> creation index
  int64_t t_total = 0, a_total = 0;
  int64_t slot_floats = 0;
  int waves = 4, groups_per_cu = 2, cus = 256;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  std::string err;
};

namespace {
constexpr size_t kAlign = 256;
size_t up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }
int grid_of(const cp_batch_s* b) { return b->cus * b->groups_per_cu; }
size_t ws_need(const cp_batch_s* b) {
  const size_t items = up(sizeof(BatchTensor) * (size_t)b->count);
  const size_t counter = up(sizeof(int));
  const size_t scratch = up((size_t)grid_of(b) * (size_t)b->slot_floats * sizeof(float));
  return items + counter + scratch;
}
}  // namespace

extern "C" {

cp_status cp_batch_create(cp_batch* out, int count, const int64_t* dims, const int* ranks, void* hip_stream) {
  if (!out || !dims || !ranks || count < 1) return CP_ERR_ARG;
  *out = nullptr;
  cp_batch_s* b = new cp_batch_s();
  b->count = count;
  b->st = (hipStream_t)hip_stream;
  std::vector<BatchTensor> byidx(count);
  int64_t toff = 0, aoff = 0;
  for (int i = 0; i < count; ++i) {
    BatchTensor t{};
    t.R = ranks[i];
    if (t.R < 1 || t.R > kMaxR) {
      delete b;
      return CP_ERR_UNSUPPORTED;
    }
    for (int m = 0; m < 3; ++m) {
      const int64_t s = dims[3 * i + m];
      if (s < 1 || s > kMaxS) {
        delete b;
        return CP_ERR_UNSUPPORTED;
      }
      t.s[m] = (int)s;
    }
    t.idx = i;
    t.t_off = toff;
    toff += ((int64_t)t.s[0] * t.s[1] * t.s[2] + 3) / 4 * 4;  // 16-byte aligned tensors
    for (int m = 0; m < 3; ++m) {
      t.a_off[m] = aoff;
      aoff += (int64_t)t.s[m] * t.R;
    }
    const int64_t need = std::max((int64_t)t.s[0] * t.s[1], (int64_t)t.s[1] * t.s[2]) * t.R;
    b->slot_floats = std::max(b->slot_floats, (need + 63) / 64 * 64);
    byidx[i] = t;
  }
  b->t_total = toff;
  b->a_total = aoff;
  // queue: largest work first (longest-processing-time order)
  b->order.resize(count);
  for (int i = 0; i < count; ++i) b->order[i] = i;
  std::stable_sort(b->order.begin(), b->order.end(), [&](int x, int y) {
    const BatchTensor &u = byidx[x], &v = byidx[y];
    return (double)u.s[0] * u.s[1] * u.s[2] * u.R > (double)v.s[0] * v.s[1] * v.s[2] * v.R;
  });
  for (int q = 0; q < count; ++q) b->items.push_back(byidx[b->order[q]]);
  int dev = 0;
  if (hipGetDevice(&dev) == hipSuccess) {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0) b->cus = cus;
  }
  *out = b;
  return CP_OK;
}

cp_status cp_batch_layout(cp_batch b, int64_t* t_offsets, int64_t* a_offsets, int64_t* t_total, int64_t* a_total) {
  if (!b) return CP_ERR_ARG;
  for (int q = 0; q < b->count; ++q) {
    const int i = b->order[q];
    const BatchTensor& t = b->items[q];
    if (t_offsets) t_offsets[i] = t.t_off;
    if (a_offsets)
      for (int m = 0; m < 3; ++m) a_offsets[3 * i + m] = t.a_off[m];
  }
  if (t_total) *t_total = b->t_total;
  if (a_total) *a_total = b->a_total;
  return CP_OK;
}

cp_status cp_batch_set_launch(cp_batch b, int waves_per_group, int groups_per_cu) {
  if (!b) return CP_ERR_ARG;
  if ((waves_per_group != 4 && waves_per_group != 8) || groups_per_cu < 1 || groups_per_cu > 4) return CP_ERR_UNSUPPORTED;
  if (b->ws) return CP_ERR_STATE;  // the workspace size depends on the grid
  b->waves = waves_per_group;
  b->groups_per_cu = groups_per_cu;
  return CP_OK;
}

cp_status cp_batch_workspace_size(cp_batch b, size_t* bytes) {
  if (!b || !bytes) return CP_ERR_ARG;
  *bytes = ws_need(b);
  return CP_OK;
}

cp_status cp_batch_set_workspace(cp_batch b, void* dptr, size_t bytes) {
  if (!b || !dptr) return CP_ERR_ARG;
  if (((uintptr_t)dptr) % kAlign) return CP_ERR_ARG;
  if (bytes < ws_need(b)) return CP_ERR_ARG;
  b->ws = (char*)dptr;
  b->ws_bytes = bytes;
  // the queue order and offsets are static: upload them once
  hipError_t e = hipMemcpyAsync(b->ws, b->items.data(), sizeof(BatchTensor) * b->items.size(), hipMemcpyHostToDevice,
                                b->st);
  if (e == hipSuccess) e = hipStreamSynchronize(b->st);
  return e == hipSuccess ? CP_OK : CP_ERR_HIP;
}

cp_status cp_batch_sweeps(cp_batch b, const float* T, double* A, int sweeps, double* fitness, int* status,
                          long long* ticks) {
  if (!b || !T || !A || !fitness || !status || sweeps < 1) return CP_ERR_ARG;
  if (!b->ws) return CP_ERR_STATE;
  BatchArgs a{};
  a.T = T;
  a.A = A;
  a.items = (const BatchTensor*)b->ws;
  a.count = b->count;
  a.sweeps = sweeps;
  a.fitness = fitness;
  a.status = status;
  a.ticks = ticks;
  a.counter = (int*)(b->ws + up(sizeof(BatchTensor) * (size_t)b->count));
  a.scratch = (float*)((char*)a.counter + up(sizeof(int)));
  a.slot_floats = b->slot_floats;
  hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(64), 0, b->st, a.counter);
  const unsigned grid = (unsigned)grid_of(b);
  if (b->waves == 8)
    hipLaunchKernelGGL(k_batch<512>, dim3(grid), dim3(512), 0, b->st, a);
  else
    hipLaunchKernelGGL(k_batch<256>, dim3(grid), dim3(256), 0, b->st, a);
  return hipGetLastError() == hipSuccess ? CP_OK : CP_ERR_HIP;
}

cp_status cp_batch_tick_rate(cp_batch b, double* hz) {
  if (!b || !hz) return CP_ERR_ARG;
  int dev = 0, khz = 0;
  if (hipGetDevice(&dev) != hipSuccess) return CP_ERR_HIP;
  if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess) return CP_ERR_HIP;
  *hz = (double)khz * 1e3;
  return CP_OK;
}

void cp_batch_destroy(cp_batch b) { delete b; }

}  // extern "C"
