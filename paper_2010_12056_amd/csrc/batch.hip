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
// BF16 matrix cores as three-part products to about FP32 accuracy (below),
// Y and Z are FP32 in a per-slot scratch, the
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
constexpr int kKP = kMaxS + 8;  // staged factor pitch (BF16 elements): 16 lanes' 16-byte reads fall in different banks

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
  uint16_t Bt[3][kMaxR * kKP];      // the factor's three BF16 parts, transposed, zero padded
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

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__device__ inline bf16x8 as_bf16x8(u32x4 v) { return __builtin_bit_cast(bf16x8, v); }

// x rounded to BF16 (nearest, ties to even), as the FP32 bit pattern.
__device__ __forceinline__ uint32_t rne16(float x) {
  const uint32_t u = __float_as_uint(x);
  return (u + 0x7fffu + ((u >> 16) & 1u)) & 0xffff0000u;
}

// The three BF16 parts (bit patterns) of x: x == x1 + x2 + x3 exactly, each
// rounded to nearest (x2 = bf16(x - x1), x3 = x - x1 - x2; both differences
// exact, the last one has at most 8 significant bits).
__device__ __forceinline__ void split3(float x, uint32_t& h1, uint32_t& h2, uint32_t& h3) {
  const uint32_t u1 = rne16(x);
  const float r1 = x - __uint_as_float(u1);
  const uint32_t u2 = rne16(r1);
  const float r2 = r1 - __uint_as_float(u2);
  h1 = u1 >> 16;
  h2 = u2 >> 16;
  h3 = __float_as_uint(r2) >> 16;
}

// Eight values as the three BF16 part vectors of one MFMA operand.
__device__ __forceinline__ void split8(const float (&x)[8], u32x4& a1, u32x4& a2, u32x4& a3) {
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    uint32_t h1a, h2a, h3a, h1b, h2b, h3b;
    split3(x[2 * w], h1a, h2a, h3a);
    split3(x[2 * w + 1], h1b, h2b, h3b);
    a1[w] = h1a | (h1b << 16);
    a2[w] = h2a | (h2b << 16);
    a3[w] = h3a | (h3b << 16);
  }
}

// acc += (a1 + a2 + a3) (b1 + b2 + b3) without the three products below
// 2^-23 of it (a2 b3, a3 b2, a3 b3); small products first.
__device__ __forceinline__ f32x4 mfma_x3(const u32x4& a1, const u32x4& a2, const u32x4& a3, const uint16_t* bp,
                                         f32x4 acc) {
  const bf16x8 b1 = as_bf16x8(*(const u32x4*)bp);
  const bf16x8 b2 = as_bf16x8(*(const u32x4*)(bp + kMaxR * kKP));
  const bf16x8 b3 = as_bf16x8(*(const u32x4*)(bp + 2 * kMaxR * kKP));
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(a2), b2, acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(a3), b1, acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(a1), b3, acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(a2), b1, acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(a1), b2, acc, 0, 0, 0);
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(a1), b1, acc, 0, 0, 0);
}

// Stage factor m (s x R, FP64 in LDS) as Bt[part][c][k]: the three BF16
// parts of its FP32 rounding, zero for k >= s or c >= R, up to the next
// multiple of 32 in k.
template <int NT, int RP>
__device__ __forceinline__ void stage_factor(Lds& L, int m, int s, int R) {
  const int KP = (s + 31) & ~31;
  for (int e = threadIdx.x; e < RP * KP; e += NT) {
    const int c = e / KP, k = e - c * KP;
    uint32_t h1 = 0, h2 = 0, h3 = 0;
    if (k < s && c < R) split3((float)L.F[m][k * R + c], h1, h2, h3);
    L.Bt[0][c * kKP + k] = (uint16_t)h1;
    L.Bt[1][c * kKP + k] = (uint16_t)h2;
    L.Bt[2][c * kKP + k] = (uint16_t)h3;
  }
}

// The contractions with the tensor run on the BF16 matrix cores
// (v_mfma_f32_16x16x32_bf16): tensor values and factor entries split into
// three BF16 parts each (split3), six part products per pair accumulated in
// FP32 (mfma_x3), an FP32 contraction to about one FP32 rounding per
// product.  Operand layout: lane (i = lane % 16, g = lane / 16) supplies row
// i of A and column i of B with the eight indices 32 t + 8 g .. + 7 of step
// t; register v of lane (i, g) holds C[4 g + v][i].

// C[p][r] = sum_k X[p][k] B[k][r] (X is P x K row-major): 16-row tiles per
// wave.  nb = ceil(K / 32) <= 3 steps: every loop over them is unrolled to
// three with uniform guards (one instance for every K, so that the
// instances do not add up in the register allocation of the persistent
// kernel; the staged factor is zero up to 32 nb).  Lane
// (i, g) loads row i of the tile, indices 32 t + 8 g .. + 7 (two 16-byte
// loads when VEC: K % 4 == 0 and 16-byte aligned rows; a half past K reads
// a clamped, whole in-row half, cancelled by the zero padding; otherwise
// element by element, indices past K clamped).  Every load is
// unconditional: rows past P read row P - 1 (never stored).  The next tile's
// rows are in flight while a tile is multiplied (past the last tile it
// reloads the last, unused), and a scheduling barrier keeps those loads
// ahead of the products.
template <int NT, int RP, bool VEC>
__device__ __forceinline__ void ttm_rows(Lds& L, const float* X, int64_t P, int K, int R, float* C) {
  constexpr int NCB = RP / 16;
  constexpr int NB = 3;
  const int nb = (K + 31) / 32;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);  // uniform (not inferred from tid / 64)
  const int g = lane >> 4, l16 = lane & 15;
  const int64_t ntiles = (P + 15) / 16;
  // 32-bit byte offsets from X (a tensor here is at most 96^3 values)
  auto load_tile = [&](int64_t tile, float (&a)[NB][8]) {
    const int64_t p0 = tile * 16;
    const uint32_t row = (uint32_t)((p0 + l16 < P) ? p0 + l16 : P - 1);
    const uint32_t rb = row * (uint32_t)K * 4u;
    const char* xb = (const char*)X;
#pragma unroll
    for (int t = 0; t < NB; ++t) {
      if (t >= nb) break;
      const int k0 = 32 * t + 8 * g;
      if (VEC) {
        const f32x4 v0 = *(const f32x4*)(xb + (rb + 4u * (uint32_t)(k0 + 4 <= K ? k0 : K - 4)));
        const f32x4 v1 = *(const f32x4*)(xb + (rb + 4u * (uint32_t)(k0 + 8 <= K ? k0 + 4 : K - 4)));
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          a[t][u] = v0[u];
          a[t][4 + u] = v1[u];
        }
      } else {
#pragma unroll
        for (int u = 0; u < 8; ++u)
          a[t][u] = *(const float*)(xb + (rb + 4u * (uint32_t)(k0 + u < K ? k0 + u : K - 1)));
      }
    }
  };
  constexpr int NW = NT / 64;
  if (wave >= ntiles) return;
  float an[NB][8];
  load_tile(wave, an);
  for (int64_t tile = wave; tile < ntiles; tile += NW) {
    asm volatile("" ::: "memory");  // the factor's LDS reads stay in the loop (not hoisted into registers)
    u32x4 a1[NB], a2[NB], a3[NB];
#pragma unroll
    for (int t = 0; t < NB; ++t)
      if (t < nb) split8(an[t], a1[t], a2[t], a3[t]);
    load_tile(tile + NW < ntiles ? tile + NW : tile, an);
    __builtin_amdgcn_sched_barrier(0);
    const int64_t p0 = tile * 16;
    f32x4 acc[NCB];
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) acc[cb] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int t = 0; t < NB; ++t) {
      if (t >= nb) break;
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb)
        acc[cb] = mfma_x3(a1[t], a2[t], a3[t], &L.Bt[0][(cb * 16 + l16) * kKP + 32 * t + 8 * g], acc[cb]);
    }
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
// q per wave; lane (i, g) loads X[32 t + 8 g + j][q0 + i] for its eight j
// (16 lanes on 64 contiguous bytes; q past Q reads column Q - 1, never
// stored; k past K reads row K - 1, cancelled by the zero padding), nb as in
// ttm_rows, the next tile in flight while a tile is multiplied.
template <int NT, int RP>
__device__ __forceinline__ void ttm_cols(Lds& L, const float* X, int K, int64_t Q, int R, float* C) {
  constexpr int NCB = RP / 16;
  constexpr int NB = 3;
  const int nb = (K + 31) / 32;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);  // uniform (not inferred from tid / 64)
  const int g = lane >> 4, l16 = lane & 15;
  const int64_t ntiles = (Q + 15) / 16;
  // 32-bit byte offsets from X (a tensor here is at most 96^3 values)
  auto load_tile = [&](int64_t tile, float (&a)[NB][8]) {
    const uint32_t qb = 4u * (uint32_t)(tile * 16 + l16 < Q ? tile * 16 + l16 : Q - 1);
    const uint32_t Qb = 4u * (uint32_t)Q;
    const char* xb = (const char*)X;
#pragma unroll
    for (int t = 0; t < NB; ++t) {
      if (t >= nb) break;
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int k = 32 * t + 8 * g + u;
        a[t][u] = *(const float*)(xb + (qb + (uint32_t)(k < K ? k : K - 1) * Qb));
      }
    }
  };
  constexpr int NW = NT / 64;
  if (wave >= ntiles) return;
  float an[NB][8];
  load_tile(wave, an);
  for (int64_t tile = wave; tile < ntiles; tile += NW) {
    asm volatile("" ::: "memory");  // the factor's LDS reads stay in the loop (not hoisted into registers)
    u32x4 a1[NB], a2[NB], a3[NB];
#pragma unroll
    for (int t = 0; t < NB; ++t)
      if (t < nb) split8(an[t], a1[t], a2[t], a3[t]);
    load_tile(tile + NW < ntiles ? tile + NW : tile, an);
    __builtin_amdgcn_sched_barrier(0);
    const int64_t q0 = tile * 16;
    f32x4 acc[NCB];
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) acc[cb] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int t = 0; t < NB; ++t) {
      if (t >= nb) break;
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb)
        acc[cb] = mfma_x3(a1[t], a2[t], a3[t], &L.Bt[0][(cb * 16 + l16) * kKP + 32 * t + 8 * g], acc[cb]);
    }
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

template <int NT, int RP>
__device__ __forceinline__ void ttm_rows_k(Lds& L, const float* X, int64_t P, int K, int R, float* C) {
  if (K % 4 == 0 && ((uintptr_t)X & 15) == 0)
    ttm_rows<NT, RP, true>(L, X, P, K, R, C);
  else
    ttm_rows<NT, RP, false>(L, X, P, K, R, C);
}
template <int NT, int RP>
__device__ __forceinline__ void ttm_cols_k(Lds& L, const float* X, int K, int64_t Q, int R, float* C) {
  ttm_cols<NT, RP>(L, X, K, Q, R, C);
}
static_assert(kMaxS <= 3 * 32, "three 32-index steps cover kMaxS");

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
  if (!gj_inverse_lds<RP, NT / 64>(L.G, tol, &L.fail, L.red)) {
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
  const int s0c = t.s[0], s1c = t.s[1], s2c = t.s[2], Rc = t.R;
  const int s0 = s0c, s1 = s1c, s2 = s2c, R = Rc;
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
    // the sizes pass through an empty asm statement each sweep, so that the
    // phases' per-thread index arithmetic is not hoisted out of the sweep
    // loop (it would stay live, in registers, across every other phase)
    int s0 = s0c, s1 = s1c, s2 = s2c, R = Rc;
    asm volatile("" : "+s"(s0), "+s"(s1), "+s"(s2), "+s"(R));
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
    const int q = __builtin_amdgcn_readfirstlane(L.item);  // uniform: the tensor record loads into scalar registers
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
