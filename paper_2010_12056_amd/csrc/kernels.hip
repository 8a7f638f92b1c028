// gfx950 kernels of the CP-ALS hot path.
//
//  k_ttm        first-level contraction of the tensor with one factor (a
//               dense GEMM / batched GEMM) on the matrix cores (MFMA f32 or
//               f64 16x16x4), tiles staged through LDS.      Sec. II-C, Sec. III
//  k_mttv       batched tensor-times-vector down the tree, HBM streaming,
//               lanes over the contiguous (q, r) block.       Sec. II-C
//  k_prep       Gamma^(n) (Eq. (1)), its inverse, and the bracket of Eq. (7)
//  k_update     A^(n) <- M Gamma^-1 (plus V^(n) in PP), Gram, dS, norms, the
//               residual by Eq. (3), Gamma of the next mode and its inverse
//  k_pp_mttkrp  first-order PP correction, Eqs. (5)-(6)
//
// Every floating-point reduction runs in a fixed order (no atomics), so two
// runs give bitwise-identical results.
#include <math.h>

#include <algorithm>
#include <atomic>

#include "kernels.h"
#include "blocked_inverse.h"

namespace cpals {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// Matrix-core wrappers.  Operand layout of the 16x16x4 instructions (checked
// on gfx950 with a one-wave probe): lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16].  Accumulator register v of lane l holds
//   f32: C[4 * (l / 16) + v][l % 16]
//   f64: C[(l / 16) + 4 * v][l % 16]
// ---------------------------------------------------------------------------
template <typename T>
struct Mma;
template <>
struct Mma<float> {
  typedef f32x4 acc_t;
  __device__ static inline acc_t zero() { return acc_t{0.f, 0.f, 0.f, 0.f}; }
  __device__ static inline acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static inline int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};
template <>
struct Mma<double> {
  typedef f64x4 acc_t;
  __device__ static inline acc_t zero() { return acc_t{0.0, 0.0, 0.0, 0.0}; }
  __device__ static inline acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static inline int row(int lane, int v) { return (lane >> 4) + 4 * v; }
};

constexpr int kTtmWaves = 8;  // waves per workgroup of the resident-factor kernels
constexpr int kTtmThreads = kTtmWaves * 64;
constexpr int TBM = 128;  // output rows per workgroup (4 waves x 32)
constexpr int TBN = 64;   // output columns (rank entries) per workgroup
constexpr int TBK = 32;   // contraction depth per LDS stage

// C[p][q][r] = sum_k X[p][k][q] * B[k][r].
// KC (contraction index contiguous, Q == 1): rows of the tile are p.
// otherwise: rows of the tile are q inside batch p (X[p] is K x Q, Q contiguous).
template <typename T, bool KC>
__global__ __launch_bounds__(256) void k_ttm(const T* __restrict__ X, const T* __restrict__ B,
                                             T* __restrict__ C, int64_t P, int64_t K, int64_t Q,
                                             int R, int64_t tilesQ) {
  constexpr int XS = KC ? TBM * (TBK + 1) : TBK * (TBM + 1);
  __shared__ T Xs[XS];
  __shared__ T Bs[TBK * (TBN + 1)];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform (not inferred from tid / 64)
  int64_t rowbase, nrows;
  const T* Xb;
  T* Cb;
  if (KC) {
    rowbase = (int64_t)blockIdx.x * TBM;
    nrows = P;
    Xb = X;
    Cb = C;
  } else {
    const int64_t p = blockIdx.x / tilesQ, qt = blockIdx.x % tilesQ;
    rowbase = qt * TBM;
    nrows = Q;
    Xb = X + p * K * Q;
    Cb = C + p * Q * R;
  }
  const int c0 = blockIdx.y * TBN;
  typename Mma<T>::acc_t acc[2][4];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = Mma<T>::zero();

  for (int64_t k0 = 0; k0 < K; k0 += TBK) {
#pragma unroll 4
    for (int it = 0; it < TBM * TBK / 256; ++it) {
      const int idx = tid + 256 * it;
      if (KC) {
        const int r = idx / TBK, kk = idx % TBK;
        const int64_t gr = rowbase + r, gk = k0 + kk;
        Xs[r * (TBK + 1) + kk] = (gr < nrows && gk < K) ? Xb[gr * K + gk] : T(0);
      } else {
        const int kk = idx / TBM, q = idx % TBM;
        const int64_t gq = rowbase + q, gk = k0 + kk;
        Xs[kk * (TBM + 1) + q] = (gq < nrows && gk < K) ? Xb[gk * Q + gq] : T(0);
      }
    }
#pragma unroll 4
    for (int it = 0; it < TBK * TBN / 256; ++it) {
      const int idx = tid + 256 * it;
      const int kk = idx / TBN, c = idx % TBN;
      const int64_t gk = k0 + kk;
      const int gc = c0 + c;
      Bs[kk * (TBN + 1) + c] = (gk < K && gc < R) ? B[gk * R + gc] : T(0);
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < TBK / 4; ++ks) {
      const int kk = ks * 4 + (lane >> 4);
      T a[2], b[4];
#pragma unroll
      for (int rb = 0; rb < 2; ++rb) {
        const int r = wave * 32 + rb * 16 + (lane & 15);
        a[rb] = KC ? Xs[r * (TBK + 1) + kk] : Xs[kk * (TBM + 1) + r];
      }
#pragma unroll
      for (int cb = 0; cb < 4; ++cb) b[cb] = Bs[kk * (TBN + 1) + cb * 16 + (lane & 15)];
#pragma unroll
      for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) acc[rb][cb] = Mma<T>::mma(a[rb], b[cb], acc[rb][cb]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int rb = 0; rb < 2; ++rb)
#pragma unroll
    for (int cb = 0; cb < 4; ++cb)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = wave * 32 + rb * 16 + Mma<T>::row(lane, v);
        const int c = c0 + cb * 16 + (lane & 15);
        const int64_t gr = rowbase + r;
        if (gr < nrows && c < R) Cb[gr * R + c] = acc[rb][cb][v];
      }
}

template <typename T>
struct Vec16;
template <>
struct Vec16<float> {
  typedef f32x4 type;
};
template <>
struct Vec16<double> {
  typedef double __attribute__((ext_vector_type(2))) type;
};

// First-level contraction with the factor resident in LDS (K <= 256).
//   C[p][q][r] = sum_k X[p][k][q] * B[k][r]
// The factor sits transposed (Bt[c][k], row pitch Kp + V) for the whole
// workgroup.  Each wave owns 32-row x 16*NCB-column output tiles and walks
// them grid-stride.  The contraction index is permuted so that a lane feeds
// V = 16 / sizeof(T) consecutive k values to V consecutive MFMA steps: lane
// (row, g = lane / 16) supplies k = kc + t*4V + g*V + u at step (t, u), which
// turns the row-contiguous case (KC) into one 16-byte load per lane and the
// factor side into one 16-byte LDS read per lane.
template <typename T, bool KC, int NCB>
__global__ __launch_bounds__(512) void k_ttm_rb(const T* __restrict__ X, const T* __restrict__ B,
                                                T* __restrict__ C, int64_t P, int64_t K, int64_t Q,
                                                int R, int64_t tilesQ, int64_t ntiles, int Kp, int vec) {
  constexpr int V = 16 / sizeof(T);
  constexpr int KT = 4 * V;
  constexpr int NTS = KC ? 8 : 4;  // t steps per register chunk (NTS * KT k values)
  typedef typename Vec16<T>::type VT;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  T* Bt = (T*)lds_raw;
  const int pitch = Kp + V;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform (not inferred from tid / 64)
  const int g = lane >> 4, l16 = lane & 15;
  const int c0 = blockIdx.y * NCB * 16;
  constexpr int NC = NCB * 16;
  for (int idx = tid; idx < Kp * NC; idx += kTtmThreads) {
    const int k = idx / NC, col = idx - k * NC;
    Bt[col * pitch + k] = (k < K && c0 + col < R) ? B[(int64_t)k * R + c0 + col] : T(0);
  }
  __syncthreads();
  for (int64_t tile = (int64_t)blockIdx.x * kTtmWaves + wave; tile < ntiles;
       tile += (int64_t)gridDim.x * kTtmWaves) {
    // keep the factor reads inside the loop (re-read from LDS per tile rather
    // than hoisted into registers), which keeps occupancy high
    asm volatile("" ::: "memory");
    int64_t rowbase, nrows;
    const T* Xb;
    T* Cb;
    if (KC) {
      rowbase = tile * 32;
      nrows = P;
      Xb = X;
      Cb = C;
    } else {
      const int64_t p = tile / tilesQ;
      rowbase = (tile - p * tilesQ) * 32;
      nrows = Q;
      Xb = X + p * K * Q;
      Cb = C + p * Q * R;
    }
    typename Mma<T>::acc_t acc[2][NCB];
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) acc[rb][cb] = Mma<T>::zero();
    for (int kc = 0; kc < Kp; kc += NTS * KT) {
      VT a[2][NTS];
#pragma unroll
      for (int rb = 0; rb < 2; ++rb) {
        const int64_t row = rowbase + rb * 16 + l16;
        const bool rin = row < nrows;
        if (KC) {
          const T* xr = Xb + row * K;
#pragma unroll
          for (int t = 0; t < NTS; ++t) {
            const int64_t k = kc + t * KT + g * V;
            if (vec && rin && k + V <= K) {
              a[rb][t] = *(const VT*)(xr + k);
            } else {
#pragma unroll
              for (int u = 0; u < V; ++u) a[rb][t][u] = (rin && k + u < K) ? xr[k + u] : T(0);
            }
          }
        } else {
          // lane pointer at (k = kc + g*V, q = row); steps add uniform multiples of Q
          const int kl = kc + g * V;
          const T* xl = Xb + (int64_t)kl * Q + row;
#pragma unroll
          for (int t = 0; t < NTS; ++t)
#pragma unroll
            for (int u = 0; u < V; ++u) {
              const int k = kl + t * KT + u;
              a[rb][t][u] = (rin && k < K) ? xl[(int64_t)(t * KT + u) * Q] : T(0);
            }
        }
      }
#pragma unroll
      for (int t = 0; t < NTS; ++t) {
        VT b[NCB];
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb)
          b[cb] = *(const VT*)(Bt + (cb * 16 + l16) * pitch + kc + t * KT + g * V);
#pragma unroll
        for (int u = 0; u < V; ++u)
#pragma unroll
          for (int rb = 0; rb < 2; ++rb)
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) acc[rb][cb] = Mma<T>::mma(a[rb][t][u], b[cb][u], acc[rb][cb]);
      }
    }
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int64_t row = rowbase + rb * 16 + Mma<T>::row(lane, v);
          const int c = c0 + cb * 16 + l16;
          if (row < nrows && c < R) Cb[row * R + c] = acc[rb][cb][v];
        }
  }
}

// First-level contraction over a mode followed by a short run of q
// (1 < Q < 64), K <= 8 * 4V: the output rows (p, q) are numbered
// rho = p Q + q, as C[p][q][r] is stored, and tiled 16 at a time as in
// k_ttm_kc, so no row of a tile is wasted on a short q.  Element k of row
// rho is X[p][k][q] at (rho / Q) K Q + rho % Q + k Q: lane (row, g = lane /
// 16) loads the four elements k = t*4V + g*V + u, u < V, of its row with
// four single loads per t (runs of Q elements; the tensor is still read
// about once, from the caches).  Rows beyond P Q are clamped for loads and
// masked for stores; k beyond K is clamped to K - 1 and meets zero rows of
// the staged factor.
template <typename T, int NCB, int NTS>
__global__ __launch_bounds__(512) void k_ttm_sq(const T* __restrict__ X, const T* __restrict__ B,
                                                T* __restrict__ C, int64_t rows, int64_t K, int64_t Q, int R,
                                                int64_t ntiles) {
  constexpr int V = 16 / sizeof(T);
  constexpr int KT = 4 * V;
  constexpr int KP = NTS * KT;
  constexpr int pitch = KP + V;
  constexpr int NC = NCB * 16;
  typedef typename Vec16<T>::type VT;
  __shared__ __align__(16) T Bt[NC * pitch];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform (not inferred from tid / 64)
  const int g = lane >> 4, l16 = lane & 15;
  const int c0 = blockIdx.y * NC;
  for (int idx = tid; idx < KP * NC; idx += kTtmThreads) {
    const int k = idx / NC, col = idx - k * NC;
    Bt[col * pitch + k] = (k < K && c0 + col < R) ? B[(int64_t)k * R + c0 + col] : T(0);
  }
  __syncthreads();
  auto load_tile = [&](int64_t t, VT (&a)[NTS]) {
    int64_t rho = t * 16 + l16;
    rho = rho < rows ? rho : rows - 1;
    const int64_t p = rho / Q;
    const T* xr = X + p * K * Q + (rho - p * Q);
#pragma unroll
    for (int st = 0; st < NTS; ++st)
#pragma unroll
      for (int u = 0; u < V; ++u) {
        const int64_t k = st * KT + g * V + u;
        a[st][u] = xr[(k < K ? k : K - 1) * Q];
      }
  };
  const int64_t stride = (int64_t)gridDim.x * kTtmWaves;
  int64_t tile = (int64_t)blockIdx.x * kTtmWaves + wave;
  VT an[NTS];
  if (tile < ntiles) load_tile(tile, an);
  for (; tile < ntiles; tile += stride) {
    asm volatile("" ::: "memory");  // factor reads stay in the loop
    VT a[NTS];
#pragma unroll
    for (int st = 0; st < NTS; ++st) a[st] = an[st];
    load_tile(tile + stride < ntiles ? tile + stride : tile, an);
    __builtin_amdgcn_sched_barrier(0);
    typename Mma<T>::acc_t acc[NCB];
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) acc[cb] = Mma<T>::zero();
#pragma unroll
    for (int st = 0; st < NTS; ++st) {
      VT b[NCB];
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) b[cb] = *(const VT*)(Bt + (cb * 16 + l16) * pitch + st * KT + g * V);
#pragma unroll
      for (int u = 0; u < V; ++u)
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) acc[cb] = Mma<T>::mma(a[st][u], b[cb][u], acc[cb]);
    }
    T* ct = C + tile * 16 * R;
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = Mma<T>::row(lane, v);
        const int c = c0 + cb * 16 + l16;
        if (tile * 16 + r < rows && c < R) ct[r * R + c] = acc[cb][v];
      }
  }
}

// First-level contraction over the last mode for K <= 8 * 4V (one register
// chunk): X is P x K row-major.  16-row output tiles per wave, eight waves
// per workgroup, the factor transposed in LDS and re-read per tile; each
// wave loads its next tile while it multiplies the current one.  Lane
// (row, g = lane / 16) feeds k = t*4V + g*V + u at MFMA step (t, u) from one
// 16-byte load per t.  Rows beyond P are clamped for loads and masked for
// stores; k beyond K meets zero rows of the staged factor.
template <typename T, int NCB, int NTS, bool FULLK>
__global__ __launch_bounds__(512) void k_ttm_kc(const T* __restrict__ X, const T* __restrict__ B,
                                                T* __restrict__ C, int64_t P, int64_t K_, int R,
                                                int64_t ntiles, int vec) {
  constexpr int V = 16 / sizeof(T);
  constexpr int KT = 4 * V;
  constexpr int KP = NTS * KT;
  constexpr int pitch = KP + V;
  constexpr int NC = NCB * 16;
  const int64_t K = FULLK ? (int64_t)KP : K_;  // FULLK: K == KP, 16-byte aligned rows
  typedef typename Vec16<T>::type VT;
  __shared__ __align__(16) T Bt[NC * pitch];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform (not inferred from tid / 64)
  const int g = lane >> 4, l16 = lane & 15;
  const int c0 = blockIdx.y * NC;
  for (int idx = tid; idx < KP * NC; idx += kTtmThreads) {
    const int k = idx / NC, col = idx - k * NC;
    Bt[col * pitch + k] = (k < K && c0 + col < R) ? B[(int64_t)k * R + c0 + col] : T(0);
  }
  __syncthreads();
  // the 16 rows of tile t, this lane's NTS 16-byte pieces (rows past P are clamped for the
  // loads and masked at the store; indices past K read zero)
  auto load_tile = [&](int64_t t, VT (&a)[NTS]) {
    int lrow = l16;
    if ((t + 1) * 16 > P) {
      const int64_t last = P - 1 - t * 16;
      lrow = lrow < last ? lrow : (int)last;
    }
    const T* xr = X + t * 16 * K + lrow * (int)K + g * V;
#pragma unroll
    for (int s = 0; s < NTS; ++s) {
      const int k = s * KT + g * V;
      if (FULLK) {
        a[s] = *(const VT*)(xr + s * KT);
      } else if (vec) {
        if (k + V <= K) a[s] = *(const VT*)(xr + s * KT);
        else a[s] = VT{};
      } else {
#pragma unroll
        for (int u = 0; u < V; ++u) a[s][u] = (k + u < K) ? xr[s * KT + u] : T(0);
      }
    }
  };
  const int64_t stride = (int64_t)gridDim.x * kTtmWaves;
  int64_t tile = (int64_t)blockIdx.x * kTtmWaves + wave;
  // the next tile's rows are in flight while this one is multiplied.  The
  // loaded registers are copied at the top of the iteration, before the next
  // loads are issued, so the products read registers with no load pending
  // (the wait falls on the copy, for loads issued a whole tile earlier).
  VT an[NTS];
  if (tile < ntiles) load_tile(tile, an);
  for (; tile < ntiles; tile += stride) {
    asm volatile("" ::: "memory");  // factor reads stay in the loop
    VT a[NTS];
#pragma unroll
    for (int s = 0; s < NTS; ++s) a[s] = an[s];
    // unconditional (past the last tile it reloads this one, unused): no
    // branch around the loads; the scheduling barrier keeps them ahead of
    // the products
    load_tile(tile + stride < ntiles ? tile + stride : tile, an);
    __builtin_amdgcn_sched_barrier(0);
    const bool full_tile = (tile + 1) * 16 <= P;
    T* ct = C + tile * 16 * R;
    typename Mma<T>::acc_t acc[NCB];
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) acc[cb] = Mma<T>::zero();
#pragma unroll
    for (int t = 0; t < NTS; ++t) {
      VT b[NCB];
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) b[cb] = *(const VT*)(Bt + (cb * 16 + l16) * pitch + t * KT + g * V);
#pragma unroll
      for (int u = 0; u < V; ++u)
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) acc[cb] = Mma<T>::mma(a[t][u], b[cb][u], acc[cb]);
    }
    if (full_tile && c0 + NC <= R) {
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
        for (int v = 0; v < 4; ++v) ct[Mma<T>::row(lane, v) * R + c0 + cb * 16 + l16] = acc[cb][v];
    } else {
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = Mma<T>::row(lane, v);
          const int c = c0 + cb * 16 + l16;
          if (tile * 16 + r < P && c < R) ct[r * R + c] = acc[cb][v];
        }
    }
  }
}

// First-level contraction over the last mode for FP32 and K == 128 (16-byte
// aligned rows) on v_mfma_f32_32x32x2f32: 32-row output tiles per wave,
// 32-column blocks.  In step s, lane (i = lane % 32, h = lane / 32) loads
// X[row i][8 s + 4 h .. + 3] with one 16-byte load and feeds element j to
// instruction j, whose contraction slot h then holds index 8 s + 4 h + j; the
// factor lane of the same slot reads the same indices from the transposed
// factor in LDS.  Register v of lane l holds output row 8 (v / 4) + 4 h +
// v % 4, column l % 32.  Otherwise as k_ttm_kc (factor staged once, the next
// tile in flight, prefetched registers copied before the next loads).
template <int NCB>
__global__ __launch_bounds__(512) void k_ttm_kc32(const float* __restrict__ X, const float* __restrict__ B,
                                                  float* __restrict__ C, int64_t P, int R, int64_t ntiles) {
  constexpr int K = 128;
  constexpr int NS = K / 8;
  constexpr int pitch = K + 4;
  constexpr int NC = NCB * 32;
  __shared__ __align__(16) float Bt[NC * pitch];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform (not inferred from tid / 64)
  const int h = lane >> 5, l32 = lane & 31;
  const int c0 = blockIdx.y * NC;
  for (int idx = tid; idx < K * NC; idx += kTtmThreads) {
    const int k = idx / NC, col = idx - k * NC;
    Bt[col * pitch + k] = (c0 + col < R) ? B[(int64_t)k * R + c0 + col] : 0.f;
  }
  __syncthreads();
  // whole tiles: the tile's base (uniform) plus the lane's byte offset (row l32, index 4 h)
  const uint32_t xlo = ((uint32_t)l32 * (uint32_t)K + 4u * (uint32_t)h) * 4u;
  auto load_tile = [&](int64_t t, f32x4 (&a)[NS]) {
    if (t * 32 + 32 <= P) {
      const char* xb = (const char*)(X + t * 32 * K) + xlo;
#pragma unroll
      for (int st = 0; st < NS; ++st) a[st] = *(const f32x4*)(xb + 32 * st);
      return;
    }
    int64_t row = t * 32 + l32;
    row = row < P ? row : P - 1;
    const float* xr = X + row * K + 4 * h;
#pragma unroll
    for (int st = 0; st < NS; ++st) a[st] = *(const f32x4*)(xr + 8 * st);
  };
  const int64_t stride = (int64_t)gridDim.x * kTtmWaves;
  int64_t tile = (int64_t)blockIdx.x * kTtmWaves + wave;
  f32x4 an[NS];
  if (tile < ntiles) load_tile(tile, an);
  for (; tile < ntiles; tile += stride) {
    asm volatile("" ::: "memory");  // factor reads stay in the loop
    f32x4 a[NS];
#pragma unroll
    for (int st = 0; st < NS; ++st) a[st] = an[st];
    load_tile(tile + stride < ntiles ? tile + stride : tile, an);
    __builtin_amdgcn_sched_barrier(0);
    f32x16 acc[NCB];
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[cb][v] = 0.f;
#pragma unroll
    for (int st = 0; st < NS; ++st) {
      f32x4 b[NCB];
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) b[cb] = *(const f32x4*)(Bt + (cb * 32 + l32) * pitch + 8 * st + 4 * h);
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb)
          acc[cb] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[st][j], b[cb][j], acc[cb], 0, 0, 0);
    }
    const int64_t r0 = tile * 32;
    if (r0 + 32 <= P && c0 + NC <= R) {
      // row bases uniform, the lane's offset (row 4 h, column l32) in 32 bits
      const uint32_t so = ((uint32_t)(4 * h) * (uint32_t)R + (uint32_t)l32) * 4u;
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
        for (int v = 0; v < 16; ++v)
          *(float*)((char*)(C + (r0 + 8 * (v >> 2) + (v & 3)) * R + c0 + cb * 32) + so) = acc[cb][v];
    } else {
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const int64_t row = r0 + 8 * (v >> 2) + 4 * h + (v & 3);
          const int c = c0 + cb * 32 + l32;
          if (row < P && c < R) C[row * R + c] = acc[cb][v];
        }
    }
  }
}

// The leading half's first two levels in one pass (standard dimension tree,
// Sec. II-C: a first-level node there feeds exactly one second-level node):
// the contraction over the last mode as in k_ttm_kc32 (K == 128), and in its
// epilogue the one over the mode before it, of size S (a multiple of 32,
// at most kFusedMaxS), so the first-level node is never stored:
//   C[o][r] = sum_i A2[i][r] Y[o S + i][r],  Y[p][r] = sum_k X[p][k] B[k][r].
// A wave takes the S / 32 consecutive row tiles of one output row o; lane
// (l32, h) weights its 16 product rows of a tile (rows 8 m + 4 h + e) by A2,
// staged transposed in LDS, and sums them in FP32 over the row's tiles; the
// two lane halves are added at the end.  The first level's sums are those of
// k_ttm_kc32; the second level's are taken in another order than k_mttv's.
// STORE: the first-level node is written too, as k_ttm_kc32 writes it (for
// a tree that keeps it for a later child, MSDT).
constexpr int kFusedMaxS = 256;
template <int NCB, bool STORE>
__global__ __launch_bounds__(512) void k_ttm_kc32f(const float* __restrict__ X, const float* __restrict__ B,
                                                   const float* __restrict__ A2, float* __restrict__ C,
                                                   float* __restrict__ Y, int R, int S, int64_t ngroups) {
  constexpr int K = 128;
  constexpr int NS = K / 8;
  constexpr int pitch = K + 4;
  constexpr int NC = NCB * 32;
  __shared__ __align__(16) float Bt[NC * pitch];
  extern __shared__ __align__(16) float Wt[];  // NC x (S + 4): A2 transposed
  const int wp = S + 4;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform (not inferred from tid / 64)
  const int h = lane >> 5, l32 = lane & 31;
  const int c0 = blockIdx.y * NC;
  for (int idx = tid; idx < K * NC; idx += kTtmThreads) {
    const int k = idx / NC, col = idx - k * NC;
    Bt[col * pitch + k] = (c0 + col < R) ? B[(int64_t)k * R + c0 + col] : 0.f;
  }
  for (int idx = tid; idx < S * NC; idx += kTtmThreads) {
    const int i = idx / NC, col = idx - i * NC;
    Wt[col * wp + i] = (c0 + col < R) ? A2[(int64_t)i * R + c0 + col] : 0.f;
  }
  __syncthreads();
  const int G = S / 32;  // tiles per output row
  const uint32_t xlo = ((uint32_t)l32 * (uint32_t)K + 4u * (uint32_t)h) * 4u;
  auto load_tile = [&](int64_t t, f32x4 (&a)[NS]) {  // whole tiles: P = ngroups S rows
    const char* xb = (const char*)(X + t * 32 * K) + xlo;
#pragma unroll
    for (int st = 0; st < NS; ++st) a[st] = *(const f32x4*)(xb + 32 * st);
  };
  const int64_t stride = (int64_t)gridDim.x * kTtmWaves;
  int64_t grp = (int64_t)blockIdx.x * kTtmWaves + wave;
  f32x4 an[NS];
  if (grp < ngroups) load_tile(grp * G, an);
  for (; grp < ngroups; grp += stride) {
    float part[NCB];
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) part[cb] = 0.f;
    for (int q = 0; q < G; ++q) {
      asm volatile("" ::: "memory");  // factor reads stay in the loop
      const int64_t tile = grp * G + q;
      f32x4 a[NS];
#pragma unroll
      for (int st = 0; st < NS; ++st) a[st] = an[st];
      const int64_t tn = q + 1 < G ? tile + 1 : (grp + stride < ngroups ? (grp + stride) * G : tile);
      load_tile(tn, an);
      __builtin_amdgcn_sched_barrier(0);
      f32x16 acc[NCB];
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[cb][v] = 0.f;
#pragma unroll
      for (int st = 0; st < NS; ++st) {
        f32x4 b[NCB];
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) b[cb] = *(const f32x4*)(Bt + (cb * 32 + l32) * pitch + 8 * st + 4 * h);
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
          for (int cb = 0; cb < NCB; ++cb)
            acc[cb] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[st][j], b[cb][j], acc[cb], 0, 0, 0);
      }
      // register v of the lane is product row 8 (v / 4) + 4 h + v % 4 of the tile.
      // The stored node is read back from HBM by the subtree's second child
      // (it outgrows the caches): non-temporal stores leave no dirty lines to
      // be written back during that read, which then runs ~12 % faster, for
      // ~2 % more time here.
      if constexpr (STORE) {
        const int64_t r0 = tile * 32;
        if (c0 + NC <= R) {
          const uint32_t so = ((uint32_t)(4 * h) * (uint32_t)R + (uint32_t)l32) * 4u;
#pragma unroll
          for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
            for (int v = 0; v < 16; ++v)
              __builtin_nontemporal_store(acc[cb][v], (float*)((char*)(Y + (r0 + 8 * (v >> 2) + (v & 3)) * R + c0 + cb * 32) + so));
        } else {
#pragma unroll
          for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
              const int c = c0 + cb * 32 + l32;
              if (c < R) Y[(r0 + 8 * (v >> 2) + 4 * h + (v & 3)) * R + c] = acc[cb][v];
            }
        }
      }
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          // 16-byte pieces (wp is a multiple of 4): single 16-byte LDS reads
          const f32x4 w = ((const f32x4*)Wt)[(cb * 32 + l32) * (wp / 4) + 8 * q + 2 * m + h];
#pragma unroll
          for (int e = 0; e < 4; ++e) part[cb] = fmaf(acc[cb][4 * m + e], w[e], part[cb]);
        }
    }
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
      const float tot = part[cb] + __shfl_xor(part[cb], 32);
      const int c = c0 + cb * 32 + l32;
      if (h == 0 && c < R) C[grp * R + c] = tot;
    }
  }
}

// First-level contraction over the last mode (Q == 1) when K is larger than
// one register tile: the k_ttm_kc layout (a wave owns 16 rows, lane (i, g)
// loads 16 bytes of row i per 4V-index step) with K in chunks of KP = 8 * 4V
// indices.  The factor chunk sits transposed in LDS, double-buffered: while
// chunk c is multiplied out of one buffer, chunk c + 1 is loaded (before the
// rows' prefetch, so the wait for it does not wait on the rows) and written
// into the other; one barrier per chunk.  The waves of a workgroup step
// through the same (tile, chunk) sequence, a wave past the last tile
// recomputing the last one without storing it.  The rows of the next chunk
// (or of the next tile's first) are in flight while a chunk is multiplied.
//
// Split K (gridDim.z > 1): workgroup z takes chunks [z cps, (z + 1) cps) of
// every tile and writes its partial product to C + z P R; k_sum_parts adds
// the partials in z order.
template <typename T, int NCB>
__global__ __launch_bounds__(512) void k_ttm_kcx(const T* __restrict__ X, const T* __restrict__ B,
                                                 T* __restrict__ C, int64_t P, int64_t K, int R,
                                                 int64_t ntiles, int vec, int cps) {
  constexpr int V = 16 / sizeof(T);
  constexpr int KT = 4 * V;
  constexpr int NTS = 8;
  constexpr int KP = NTS * KT;
  constexpr int pitch = KP + V;
  constexpr int NC = NCB * 16;
  constexpr int BPER = KP * NC / kTtmThreads;  // factor elements per thread and chunk
  typedef typename Vec16<T>::type VT;
  __shared__ __align__(16) T Bt[2][NC * pitch];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform (not inferred from tid / 64)
  const int g = lane >> 4, l16 = lane & 15;
  const int c0 = blockIdx.y * NC;
  const int nall = (int)((K + KP - 1) / KP);
  const int cbeg = (int)blockIdx.z * cps;
  const int cend = cbeg + cps < nall ? cbeg + cps : nall;
  const int nch = cend - cbeg;
  C += (int64_t)blockIdx.z * P * R;
  auto load_b = [&](int c, T (&bv)[BPER]) {
#pragma unroll
    for (int q = 0; q < BPER; ++q) {
      const int idx = tid + kTtmThreads * q, k = idx / NC, col = idx - k * NC;
      const int64_t gk = (int64_t)c * KP + k;
      bv[q] = (gk < K && c0 + col < R) ? B[gk * R + c0 + col] : T(0);
    }
  };
  auto store_b = [&](int buf, const T (&bv)[BPER]) {
#pragma unroll
    for (int q = 0; q < BPER; ++q) {
      const int idx = tid + kTtmThreads * q, k = idx / NC, col = idx - k * NC;
      Bt[buf][col * pitch + k] = bv[q];
    }
  };
  // rows of tile t, chunk c: this lane's NTS 16-byte pieces (rows past P
  // clamped, indices past K read as zero)
  auto load_rows = [&](int64_t t, int c, VT (&a)[NTS]) {
    int lrow = l16;
    if ((t + 1) * 16 > P) {
      const int64_t last = P - 1 - t * 16;
      lrow = lrow < last ? lrow : (int)last;
    }
    const T* xr = X + (t * 16 + lrow) * K + (int64_t)c * KP + g * V;
#pragma unroll
    for (int s2 = 0; s2 < NTS; ++s2) {
      const int64_t k = (int64_t)c * KP + s2 * KT + g * V;
      if (vec && k + V <= K) {
        a[s2] = *(const VT*)(xr + s2 * KT);
      } else {
#pragma unroll
        for (int u = 0; u < V; ++u) a[s2][u] = (k + u < K) ? xr[s2 * KT + u] : T(0);
      }
    }
  };
  const int64_t stride = (int64_t)gridDim.x * kTtmWaves;
  int64_t tb = (int64_t)blockIdx.x * kTtmWaves;
  if (tb >= ntiles || nch < 1) return;  // uniform: the whole workgroup
  {
    T bv[BPER];
    load_b(cbeg, bv);
    store_b(0, bv);
  }
  VT an[NTS];
  load_rows(tb + wave < ntiles ? tb + wave : ntiles - 1, cbeg, an);
  __syncthreads();
  int buf = 0;
  for (; tb < ntiles; tb += stride) {
    asm volatile("" ::: "memory");
    const int64_t tile = tb + wave < ntiles ? tb + wave : ntiles - 1;
    const bool own = tb + wave < ntiles;
    const int64_t tnext = tb + stride + wave < ntiles ? tb + stride + wave : (tb + stride < ntiles ? ntiles - 1 : tile);
    typename Mma<T>::acc_t acc[NCB];
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) acc[cb] = Mma<T>::zero();
    for (int c = cbeg; c < cend; ++c) {
      VT a[NTS];
#pragma unroll
      for (int s2 = 0; s2 < NTS; ++s2) a[s2] = an[s2];
      // the factor's next chunk first, then the next rows
      const bool more = c + 1 < cend;
      const int cn = more ? c + 1 : cbeg;
      T bv[BPER];
      load_b(cn, bv);
      load_rows(more ? tile : tnext, cn, an);
      __builtin_amdgcn_sched_barrier(0);
      const T* bb = Bt[buf];
#pragma unroll
      for (int t = 0; t < NTS; ++t) {
        VT b[NCB];
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) b[cb] = *(const VT*)(bb + (cb * 16 + l16) * pitch + t * KT + g * V);
#pragma unroll
        for (int u = 0; u < V; ++u)
#pragma unroll
          for (int cb = 0; cb < NCB; ++cb) acc[cb] = Mma<T>::mma(a[t][u], b[cb][u], acc[cb]);
      }
      if (nch > 1 || tb + stride < ntiles) {
        store_b(buf ^ 1, bv);
        buf ^= 1;
      }
      __syncthreads();
    }
    if (own) {
      T* ct = C + tile * 16 * R;
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = Mma<T>::row(lane, v);
          const int col = c0 + cb * 16 + l16;
          if (tile * 16 + r < P && col < R) ct[r * R + col] = acc[cb][v];
        }
    }
  }
}

// C[i] = sum over z of parts[z][i] in z order (the split-K partials of
// k_ttm_kcx), 16-byte pieces; n is a multiple of the piece.
template <typename T>
__global__ __launch_bounds__(256) void k_sum_parts(const T* __restrict__ parts, T* __restrict__ C, int64_t n,
                                                   int Z) {
  typedef typename Vec16<T>::type VT;
  constexpr int V = 16 / sizeof(T);
  const int64_t nv = n / V;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < nv; i += (int64_t)gridDim.x * 256) {
    VT acc = ((const VT*)parts)[i];
    for (int z = 1; z < Z; ++z) {
      const VT v = ((const VT*)(parts + (int64_t)z * n))[i];
#pragma unroll
      for (int u = 0; u < V; ++u) acc[u] += v[u];
    }
    ((VT*)C)[i] = acc;
  }
}

// First-level contraction over the last mode for FP32 when K is longer than
// 128, on v_mfma_f32_32x32x2f32: the k_ttm_kc32 layout (a wave owns 32 rows;
// lane (i = lane % 32, h = lane / 32) loads X[row i][8 s + 4 h .. + 3] of
// each 8-index step s and feeds element j to instruction j) with K in chunks
// of 128 indices, as in k_ttm_kcx: the factor chunk transposed in LDS,
// double-buffered, the waves of a workgroup in lockstep over (tile, chunk),
// one barrier per chunk, a wave past the last tile recomputing the last one
// without storing.  The next chunk's factor is staged a quarter per four
// steps (written into the other buffer after their products), and the
// rows of the next chunk (or of the next tile's first) are in flight while a
// chunk is multiplied.  Loads are unconditional: rows past P read row P - 1;
// indices past K read within the row (clamped) and meet zero factor rows.
template <int NCB, bool VEC>
__global__ __launch_bounds__(512) void k_ttm_kcx32(const float* __restrict__ X, const float* __restrict__ B,
                                                   float* __restrict__ C, int64_t P, int64_t K, int R,
                                                   int64_t ntiles) {
  constexpr int KP = 128;
  constexpr int NS = KP / 8;
  constexpr int pitch = KP + 4;
  constexpr int NC = NCB * 32;
  constexpr int BPER = KP * NC / kTtmThreads;
  constexpr int BQ = BPER / 4;
  __shared__ __align__(16) float Bt[2][NC * pitch];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform (not inferred from tid / 64)
  const int h = lane >> 5, l32 = lane & 31;
  const int c0 = blockIdx.y * NC;
  const int nch = (int)((K + KP - 1) / KP);
  // factor loads are unconditional (index and column clamped); indices past
  // K are zeroed when written to LDS, columns past R are never stored
  auto load_b = [&](int c, int j, float (&bv)[BQ]) {
#pragma unroll
    for (int i = 0; i < BQ; ++i) {
      const int idx = tid + kTtmThreads * (j * BQ + i), k = idx / NC, col = idx - k * NC;
      const int64_t gk = (int64_t)c * KP + k;
      bv[i] = B[(gk < K ? gk : K - 1) * R + (c0 + col < R ? c0 + col : R - 1)];
    }
  };
  auto store_b = [&](int buf, int c, int j, const float (&bv)[BQ]) {
#pragma unroll
    for (int i = 0; i < BQ; ++i) {
      const int idx = tid + kTtmThreads * (j * BQ + i), k = idx / NC, col = idx - k * NC;
      Bt[buf][col * pitch + k] = (int64_t)c * KP + k < K ? bv[i] : 0.f;
    }
  };
  auto load_rows = [&](int64_t t, int c, f32x4 (&a)[NS]) {
    int64_t row = t * 32 + l32;
    row = row < P ? row : P - 1;
    const float* xr = X + row * K;
#pragma unroll
    for (int st = 0; st < NS; ++st) {
      const int64_t k = (int64_t)c * KP + 8 * st + 4 * h;
      if (VEC) {
        a[st] = *(const f32x4*)(xr + (k + 4 <= K ? k : K - 4));
      } else {
#pragma unroll
        for (int u = 0; u < 4; ++u) a[st][u] = xr[k + u < K ? k + u : K - 1];
      }
    }
  };
  const int64_t stride = (int64_t)gridDim.x * kTtmWaves;
  int64_t tb = (int64_t)blockIdx.x * kTtmWaves;
  if (tb >= ntiles) return;  // uniform: the whole workgroup
  for (int j = 0; j < 4; ++j) {
    float bv[BQ];
    load_b(0, j, bv);
    store_b(0, 0, j, bv);
  }
  f32x4 an[NS];
  load_rows(tb + wave < ntiles ? tb + wave : ntiles - 1, 0, an);
  __syncthreads();
  int buf = 0;
  for (; tb < ntiles; tb += stride) {
    asm volatile("" ::: "memory");
    const int64_t tile = tb + wave < ntiles ? tb + wave : ntiles - 1;
    const bool own = tb + wave < ntiles;
    const int64_t tnext = tb + stride + wave < ntiles ? tb + stride + wave : (tb + stride < ntiles ? ntiles - 1 : tile);
    f32x16 acc[NCB];
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[cb][v] = 0.f;
    for (int c = 0; c < nch; ++c) {
      f32x4 a[NS];
#pragma unroll
      for (int st = 0; st < NS; ++st) a[st] = an[st];
      const bool more = c + 1 < nch;
      const int cn = more ? c + 1 : 0;
      float bv[BQ];
      load_b(cn, 0, bv);
      load_rows(more ? tile : tnext, cn, an);
      __builtin_amdgcn_sched_barrier(0);
      const float* bb = Bt[buf];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
#pragma unroll
        for (int st = 4 * j; st < 4 * j + 4; ++st) {
          f32x4 b[NCB];
#pragma unroll
          for (int cb = 0; cb < NCB; ++cb) b[cb] = *(const f32x4*)(bb + (cb * 32 + l32) * pitch + 8 * st + 4 * h);
#pragma unroll
          for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb)
              acc[cb] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[st][q], b[cb][q], acc[cb], 0, 0, 0);
        }
        __builtin_amdgcn_sched_barrier(0);
        store_b(buf ^ 1, cn, j, bv);
        if (j < 3) load_b(cn, j + 1, bv);
      }
      buf ^= 1;
      __syncthreads();
    }
    if (own) {
      const int64_t r0 = tile * 32;
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const int64_t row = r0 + 8 * (v >> 2) + 4 * h + (v & 3);
          const int col = c0 + cb * 32 + l32;
          if (row < P && col < R) C[row * R + col] = acc[cb][v];
        }
    }
  }
}

// First-level contraction when the contracted mode is not the last one
// (X[p] is K x Q with q contiguous), FP32, factor resident in LDS (K <= 256).
// A wave owns 64 consecutive q and 16*NCB rank columns.  Lane (i = lane % 16,
// g = lane / 16) loads X[k][q0 + 4i .. 4i + 3] as one 16-byte load for
// k = kc + 4t + g, and feeds its four values to four MFMAs u = 0..3 in which
// it plays row i; MFMA u therefore produces output rows q0 + 4i + u.  A
// 16-lane group reads 256 contiguous bytes per load.  The factor is stored
// transposed with k permuted inside each 32-wide chunk (k = kc + 4t + g at
// position kc + 8g + t) so a lane reads its eight t-values with two 16-byte
// LDS reads.  The next 32-index chunk (across tiles too) is loaded while the
// current one is multiplied.  FULL (whole 64-q tiles and 32-index chunks,
// 16-byte aligned, Q < 2^28): loads and stores take a wave-uniform base in
// scalar registers plus the lane's 32-bit byte offset.
template <int NCB, bool FULL>
__global__ __launch_bounds__(512) void k_ttm_q(const float* __restrict__ X, const float* __restrict__ B,
                                               float* __restrict__ C, int64_t P, int64_t K, int64_t Q,
                                               int R, int64_t tilesQ, int64_t ntiles, int Kp, int vec) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  float* Bt = (float*)lds_raw;
  const int pitch = Kp + 4;
  const int tid = threadIdx.x, lane = tid & 63;
  // wave-uniform, which the compiler cannot infer from tid / 64: without it
  // the tile's slice and offset (a 64-bit division) were computed per lane,
  // in every chunk, behind divergent branches
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int g = lane >> 4, l16 = lane & 15;
  const int c0 = blockIdx.y * NCB * 16;
  constexpr int NC = NCB * 16;
  for (int idx = tid; idx < Kp * NC; idx += kTtmThreads) {
    const int k = idx / NC, col = idx - k * NC;
    const int kc = k & ~31, kr = k & 31;            // k = kc + 4t + g
    const int pos = kc + 8 * (kr & 3) + (kr >> 2);  // -> kc + 8g + t
    Bt[col * pitch + pos] = (k < K && c0 + col < R) ? B[(int64_t)k * R + c0 + col] : 0.f;
  }
  __syncthreads();
  // this lane's eight 16-byte pieces of the 32-index chunk kc of tile t
  auto load_chunk = [&](int64_t t, int kc, f32x4 (&a)[8]) {
    const int64_t p = t / tilesQ;
    const int64_t qa = (t - p * tilesQ) * 64 + 4 * l16;
    const bool full = vec && qa + 4 <= Q;
    const float* Xb = X + p * K * Q;
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      const int64_t k = kc + 4 * s + g;
      const float* src = Xb + k * Q + qa;
      if (FULL || (k < K && full)) {  // FULL: whole 64-q tiles and 32-index chunks, aligned
        a[s] = *(const f32x4*)src;
      } else {
#pragma unroll
        for (int u = 0; u < 4; ++u) a[s][u] = (k < K && qa + u < Q) ? src[u] : 0.f;
      }
    }
  };
  // FULL: the tile's base (uniform) and the lane's byte offset (index g, q 4 l16)
  const uint32_t lofs = ((uint32_t)g * (uint32_t)Q + 4u * (uint32_t)l16) * 4u;
  auto tile_base = [&](int64_t t) {
    const int64_t p = t / tilesQ;
    return X + p * K * Q + (t - p * tilesQ) * 64;
  };
  auto load_full = [&](const float* xb, int kc, f32x4 (&a)[8]) {
#pragma unroll
    for (int s = 0; s < 8; ++s) a[s] = *(const f32x4*)((const char*)(xb + (int64_t)(kc + 4 * s) * Q) + lofs);
  };
  // prefetching needs 32 more registers: kept for up to 64 factor columns per wave
  constexpr bool PF = NCB <= 4;
  const int64_t stride = (int64_t)gridDim.x * kTtmWaves;
  int64_t tile = (int64_t)blockIdx.x * kTtmWaves + wave;
  // as in k_ttm_kc, the prefetched registers are copied before the next
  // chunk's loads are issued, so the products wait on nothing in flight
  f32x4 an[8];
  const float* xcur = FULL && tile < ntiles ? tile_base(tile) : X;
  if (PF && tile < ntiles) {
    if (FULL) load_full(xcur, 0, an);
    else load_chunk(tile, 0, an);
  }
  for (; tile < ntiles; tile += stride) {
    asm volatile("" ::: "memory");  // factor reads stay in the loop (see k_ttm_rb)
    const int64_t p = tile / tilesQ;
    const int64_t q0 = (tile - p * tilesQ) * 64;
    float* Cb = C + p * Q * R;
    const bool has_next = tile + stride < ntiles;
    const float* xnext = FULL && has_next ? tile_base(tile + stride) : xcur;
    f32x4 acc[4][NCB];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) acc[u][cb] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int kc = 0; kc < Kp; kc += 32) {
      // the next chunk (or the next tile's first) is in flight while this one is multiplied
      f32x4 a[8];
      if (PF) {
#pragma unroll
        for (int s = 0; s < 8; ++s) a[s] = an[s];
      }
      if (!PF) {
        if (FULL) load_full(xcur, kc, a);
        else load_chunk(tile, kc, a);
      } else {
        // unconditional (after the last chunk of the last tile it reloads
        // this tile's first, unused): no branch around the loads, and the
        // scheduling barrier keeps them ahead of the products
        const bool more = kc + 32 < Kp;
        if (FULL) {
          load_full(more ? xcur : xnext, more ? kc + 32 : 0, an);
        } else {
          const int64_t tn = more ? tile : (has_next ? tile + stride : tile);
          load_chunk(tn, more ? kc + 32 : 0, an);
        }
        __builtin_amdgcn_sched_barrier(0);
      }
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) {
        const float* bp = Bt + (cb * 16 + l16) * pitch + kc + 8 * g;
        const f32x4 b0 = *(const f32x4*)bp;
        const f32x4 b1 = *(const f32x4*)(bp + 4);
#pragma unroll
        for (int t = 0; t < 8; ++t) {
          const float bv = t < 4 ? b0[t & 3] : b1[t & 3];
#pragma unroll
          for (int u = 0; u < 4; ++u)
            acc[u][cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[t][u], bv, acc[u][cb], 0, 0, 0);
        }
      }
    }
    if (FULL && c0 + NC <= R) {
      // whole tile: row bases uniform, the lane's offset (row 16 g, column l16) in 32 bits
      const uint32_t so = ((uint32_t)(16 * g) * (uint32_t)R + (uint32_t)l16) * 4u;
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
          for (int v = 0; v < 4; ++v)
            *(float*)((char*)(Cb + (q0 + 4 * v + u) * R + c0 + cb * 16) + so) = acc[u][cb][v];
    } else {
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int64_t q = q0 + 16 * g + 4 * v + u;
            const int c = c0 + cb * 16 + l16;
            if (q < Q && c < R) Cb[q * R + c] = acc[u][cb][v];
          }
    }
    xcur = xnext;
  }
}

// A first-level contraction in the k_ttm_q layout with the contraction over
// one more index i in its epilogue (a dimension-tree node's first child
// formed in the same pass).  Element (p', i, k, q) of X sits at
// p' pstride + i sstride + k kstride + q (q contiguous, Q a multiple of 64;
// K a multiple of 32, 16-byte aligned); B (K x R) is contracted over k and
// W (S x R) over i:
//   out[z][p'][q][r] = sum_{i in range z} W[i][r] sum_k X[p', i, k, q] B[k][r],
// and with STORE the first-level node itself, Y[p' S + i][q][r], is written
// too (when the tree keeps it for a later child).  A wave keeps one pair
// (p', block of 64 q) and walks the indices i of its range z = blockIdx.z in
// order; after each index's product tile (summed over k as in k_ttm_q) it
// adds the tile times W[i][r] to registers.  The launcher adds the ranges'
// partials in range order.  The standard tree's trailing half is the case
// p' = (), i = mode 1 (sstride Qp, kstride S Qp); MSDT's root at a middle
// mode m the case p' = modes before m - 1, i = mode m - 1.
template <int NCB, bool STORE>
__global__ __launch_bounds__(512) void k_ttm_qg(const float* __restrict__ X, const float* __restrict__ B,
                                                const float* __restrict__ W, float* __restrict__ out,
                                                float* __restrict__ Y, QgShape sh, int R, int L) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  float* Bt = (float*)lds_raw;
  const int Kp = (int)sh.K;  // a multiple of 32
  const int pitch = Kp + 4;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform (not inferred from tid / 64)
  const int g = lane >> 4, l16 = lane & 15;
  const int c0 = blockIdx.y * NCB * 16;
  constexpr int NC = NCB * 16;
  for (int idx = tid; idx < Kp * NC; idx += kTtmThreads) {
    const int k = idx / NC, col = idx - k * NC;
    const int kc = k & ~31, kr = k & 31;            // k = kc + 4t + g
    const int pos = kc + 8 * (kr & 3) + (kr >> 2);  // -> kc + 8g + t
    Bt[col * pitch + pos] = (c0 + col < R) ? B[(int64_t)k * R + c0 + col] : 0.f;
  }
  __syncthreads();
  const int64_t nqb = sh.Q / 64;
  const int64_t pair = (int64_t)blockIdx.x * kTtmWaves + wave;
  if (pair >= sh.nP * nqb) return;  // uniform in the wave; no barrier follows
  const int64_t pp = pair / nqb, qb = pair - pp * nqb;
  const int ia = (int)blockIdx.z * L;
  const int ib = ia + L < sh.S ? ia + L : (int)sh.S;
  const uint32_t lofs = ((uint32_t)g * (uint32_t)sh.kstride + 4u * (uint32_t)l16) * 4u;
  auto load_full = [&](const float* xb, int kc, f32x4 (&a)[8]) {
#pragma unroll
    for (int s = 0; s < 8; ++s)
      a[s] = *(const f32x4*)((const char*)(xb + (int64_t)(kc + 4 * s) * sh.kstride) + lofs);
  };
  const float* xp = X + pp * sh.pstride + qb * 64;
  f32x4 part[4][NCB];
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) part[u][cb] = f32x4{0.f, 0.f, 0.f, 0.f};
  f32x4 an[8];
  load_full(xp + (int64_t)ia * sh.sstride, 0, an);
  for (int i = ia; i < ib; ++i) {
    asm volatile("" ::: "memory");  // factor reads stay in the loop
    const float* xcur = xp + (int64_t)i * sh.sstride;
    const float* xnext = i + 1 < ib ? xcur + sh.sstride : xcur;
    float w[NCB];
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
      const int c = c0 + cb * 16 + l16;
      w[cb] = c < R ? W[(int64_t)i * R + c] : 0.f;
    }
    f32x4 acc[4][NCB];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) acc[u][cb] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int kc = 0; kc < Kp; kc += 32) {
      f32x4 a[8];
#pragma unroll
      for (int st = 0; st < 8; ++st) a[st] = an[st];
      const bool more = kc + 32 < Kp;
      load_full(more ? xcur : xnext, more ? kc + 32 : 0, an);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) {
        const float* bp = Bt + (cb * 16 + l16) * pitch + kc + 8 * g;
        const f32x4 b0 = *(const f32x4*)bp;
        const f32x4 b1 = *(const f32x4*)(bp + 4);
#pragma unroll
        for (int t = 0; t < 8; ++t) {
          const float bv = t < 4 ? b0[t & 3] : b1[t & 3];
#pragma unroll
          for (int u = 0; u < 4; ++u)
            acc[u][cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[t][u], bv, acc[u][cb], 0, 0, 0);
        }
      }
    }
    if constexpr (STORE) {
      // the first-level node, row p' S + i: register v of block u is q = 16 g + 4 v + u of the block
      // (non-temporal stores, as in k_ttm_kc32f)
      float* Yr = Y + ((pp * sh.S + i) * sh.Q + qb * 64) * R;
      if (c0 + NC <= R) {
        const uint32_t so = ((uint32_t)(16 * g) * (uint32_t)R + (uint32_t)l16) * 4u;
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
            for (int v = 0; v < 4; ++v)
              __builtin_nontemporal_store(acc[u][cb][v], (float*)((char*)(Yr + (int64_t)(4 * v + u) * R + c0 + cb * 16) + so));
      } else {
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const int c = c0 + cb * 16 + l16;
              if (c < R) Yr[(int64_t)(16 * g + 4 * v + u) * R + c] = acc[u][cb][v];
            }
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
        for (int v = 0; v < 4; ++v) part[u][cb][v] = fmaf(acc[u][cb][v], w[cb], part[u][cb][v]);
  }
  float* Pz = out + ((int64_t)blockIdx.z * sh.nP + pp) * sh.Q * R;
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t q = qb * 64 + 16 * g + 4 * v + u;
        const int c = c0 + cb * 16 + l16;
        if (c < R) Pz[q * R + c] = part[u][cb][v];
      }
}

// A first-level contraction over a mode a in the k_ttm_q layout (X[p][k][q],
// P slices, whole 64-q tiles, K a multiple of 32 up to 256) with the
// contraction over the last mode (the fastest part of q, of size S = 64 G
// with G = 1, 2 or 4) in the epilogue:
//   C[p Q/S + o][r] = sum_i W[i][r] Y[p][o S + i][r],  Y[p][q][r] = sum_k X[p][k][q] B[k][r],
// and with STORE the first-level node Y too.  MSDT's root at mode 0 (P = 1,
// the node kept for the subtree's later children) and a PP initialization
// node whose single pair child contracts the last mode.  The workgroup's eight waves take
// eight consecutive tiles per step (G waves per output row, wave j of a row
// its tile j), so the tensor is read as k_ttm_q reads it; lane (g, l16)
// weights its 16 product rows of the tile (q = 16 g + 4 v + u) by W (staged
// transposed in LDS), the lane groups are added by shuffles, and the G waves'
// sums of a row through LDS in tile order.  The waves step together (two
// barriers a step); a wave past the last row recomputes it without storing.
template <int NCB, bool STORE>
__global__ __launch_bounds__(512) void k_ttm_qr(const float* __restrict__ X, const float* __restrict__ B,
                                                const float* __restrict__ W, float* __restrict__ C,
                                                float* __restrict__ Y, int64_t P, int64_t K, int64_t Q, int R,
                                                int S) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  const int Kp = (int)K;
  const int pitch = Kp + 4, wp = S + 4;
  constexpr int NC = NCB * 16;
  float* Bt = (float*)lds_raw;    // NC x pitch
  float* Wt = Bt + NC * pitch;    // NC x wp: W transposed
  float* red = Wt + NC * wp;      // kTtmWaves x NC: the waves' sums of a step
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform (not inferred from tid / 64)
  const int g = lane >> 4, l16 = lane & 15;
  const int c0 = blockIdx.y * NC;
  for (int idx = tid; idx < Kp * NC; idx += kTtmThreads) {
    const int k = idx / NC, col = idx - k * NC;
    const int kc = k & ~31, kr = k & 31;            // k = kc + 4t + g
    const int pos = kc + 8 * (kr & 3) + (kr >> 2);  // -> kc + 8g + t
    Bt[col * pitch + pos] = (c0 + col < R) ? B[(int64_t)k * R + c0 + col] : 0.f;
  }
  for (int idx = tid; idx < S * NC; idx += kTtmThreads) {
    const int i = idx / NC, col = idx - i * NC;
    Wt[col * wp + i] = (c0 + col < R) ? W[(int64_t)i * R + c0 + col] : 0.f;
  }
  __syncthreads();
  const int G = S / 64;                 // waves (tiles) per output row
  const int RPS = kTtmWaves / G;        // output rows per step
  const int j = wave % G, orow = wave / G;
  const int64_t nrows = P * (Q / S);  // output rows; an output row never straddles two slices
  const int64_t QT = Q / 64;           // tiles per slice
  const int64_t stride = (int64_t)gridDim.x * RPS;
  const uint32_t lofs = ((uint32_t)g * (uint32_t)Q + 4u * (uint32_t)l16) * 4u;
  // tile t: slice t / QT, q = 64 (t % QT) ..; node and output rows follow the tile index
  auto tile_base = [&](int64_t t) {
    const int64_t p = t / QT;
    return X + p * K * Q + (t - p * QT) * 64;
  };
  auto load_full = [&](const float* xb, int kc, f32x4 (&a)[8]) {
#pragma unroll
    for (int s = 0; s < 8; ++s) a[s] = *(const f32x4*)((const char*)(xb + (int64_t)(kc + 4 * s) * Q) + lofs);
  };
  int64_t o0 = (int64_t)blockIdx.x * RPS;
  if (o0 >= nrows) return;  // uniform: the whole workgroup
  f32x4 an[8];
  {
    const int64_t o = o0 + orow < nrows ? o0 + orow : nrows - 1;
    load_full(tile_base(o * G + j), 0, an);
  }
  for (; o0 < nrows; o0 += stride) {
    asm volatile("" ::: "memory");  // factor reads stay in the loop
    const bool own = o0 + orow < nrows;
    const int64_t o = own ? o0 + orow : nrows - 1;
    const int64_t tile = o * G + j;
    const int64_t on = o0 + stride + orow < nrows ? o0 + stride + orow : (o0 + stride < nrows ? nrows - 1 : o);
    const int64_t tn = on * G + j;
    const float* xcur = tile_base(tile);
    const float* xnext = tile_base(tn);
    f32x4 acc[4][NCB];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) acc[u][cb] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int kc = 0; kc < Kp; kc += 32) {
      f32x4 a[8];
#pragma unroll
      for (int st = 0; st < 8; ++st) a[st] = an[st];
      const bool more = kc + 32 < Kp;
      load_full(more ? xcur : xnext, more ? kc + 32 : 0, an);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) {
        const float* bp = Bt + (cb * 16 + l16) * pitch + kc + 8 * g;
        const f32x4 b0 = *(const f32x4*)bp;
        const f32x4 b1 = *(const f32x4*)(bp + 4);
#pragma unroll
        for (int t = 0; t < 8; ++t) {
          const float bv = t < 4 ? b0[t & 3] : b1[t & 3];
#pragma unroll
          for (int u = 0; u < 4; ++u)
            acc[u][cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[t][u], bv, acc[u][cb], 0, 0, 0);
        }
      }
    }
    if (STORE && own) {
      // the first-level node (non-temporal stores, as in k_ttm_kc32f)
      float* Yr = Y + tile * 64 * R;
      if (c0 + NC <= R) {
        const uint32_t so = ((uint32_t)(16 * g) * (uint32_t)R + (uint32_t)l16) * 4u;
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
            for (int v = 0; v < 4; ++v)
              __builtin_nontemporal_store(acc[u][cb][v], (float*)((char*)(Yr + (int64_t)(4 * v + u) * R + c0 + cb * 16) + so));
      } else {
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const int c = c0 + cb * 16 + l16;
              if (c < R) Yr[(int64_t)(16 * g + 4 * v + u) * R + c] = acc[u][cb][v];
            }
      }
    }
    // register v of block u is product row q = 16 g + 4 v + u of the tile, index 64 j + q of the row
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
      float part = 0.f;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const f32x4 w = ((const f32x4*)Wt)[(cb * 16 + l16) * (wp / 4) + 16 * j + 4 * g + v];
#pragma unroll
        for (int u = 0; u < 4; ++u) part = fmaf(acc[u][cb][v], w[u], part);
      }
      part += __shfl_xor(part, 16);
      part += __shfl_xor(part, 32);
      if (g == 0) red[wave * NC + cb * 16 + l16] = part;
    }
    __syncthreads();
    if (j == 0 && own && g == 0) {
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) {
        float tot = red[wave * NC + cb * 16 + l16];
        for (int jj = 1; jj < G; ++jj) tot += red[(wave + jj) * NC + cb * 16 + l16];
        const int c = c0 + cb * 16 + l16;
        if (c < R) C[o * R + c] = tot;
      }
    }
    __syncthreads();
  }
}

// First-level contraction over a mode other than the last (the k_ttm_q
// layout: a wave owns 64 consecutive q, lane (i, g) loads X[k][q0 + 4i ..
// 4i + 3] for k = kc + 4t + g) when K is too long for the whole factor in
// LDS: the factor in chunks of 128 indices, double-buffered in LDS with the
// k_ttm_q permutation inside each 32-index piece; the next chunk is loaded
// at the first piece of the current one (ahead of the rows' prefetch) and
// written into the other buffer after its last piece, one barrier per
// chunk.  Waves of a workgroup step through the same (tile, piece)
// sequence; a wave past the last tile recomputes it without storing.  The
// tile's slice and offset are wave-uniform and computed once per tile.  FQ
// (whole 64-q tiles and 32-index pieces, 16-byte aligned, Q < 2^28): the
// loads and stores take that base plus the lane's 32-bit byte offset.
template <int NCB, bool FQ>
__global__ __launch_bounds__(512) void k_ttm_qx(const float* __restrict__ X, const float* __restrict__ B,
                                                float* __restrict__ C, int64_t P, int64_t K, int64_t Q,
                                                int R, int64_t tilesQ, int64_t ntiles, int vec, int cps) {
  constexpr int KCH = 128;
  constexpr int pitch = KCH + 4;
  constexpr int NC = NCB * 16;
  constexpr int BPER = KCH * NC / kTtmThreads;
  constexpr int BQ = BPER / 4;  // factor elements per thread and quarter chunk
  __shared__ __align__(16) float Bt[2][NC * pitch];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform (not inferred from tid / 64)
  const int g = lane >> 4, l16 = lane & 15;
  const int c0 = blockIdx.y * NC;
  // split K (gridDim.z > 1): this layer takes chunks [cbeg, cend) and writes
  // its partial product to C + z P Q R
  const int nall = (int)((K + KCH - 1) / KCH);
  const int cbeg = (int)blockIdx.z * cps;
  const int cend = cbeg + cps < nall ? cbeg + cps : nall;
  C += (int64_t)blockIdx.z * P * Q * R;
  // quarter j of factor chunk c: the thread's elements q = j BQ .. j BQ + BQ - 1
  auto load_b = [&](int c, int j, float (&bv)[BQ]) {
#pragma unroll
    for (int i = 0; i < BQ; ++i) {
      const int q = j * BQ + i;
      const int idx = tid + kTtmThreads * q, k = idx / NC, col = idx - k * NC;
      const int64_t gk = (int64_t)c * KCH + k;
      bv[i] = (gk < K && c0 + col < R) ? B[gk * R + c0 + col] : 0.f;
    }
  };
  auto store_b = [&](int buf, int j, const float (&bv)[BQ]) {
#pragma unroll
    for (int i = 0; i < BQ; ++i) {
      const int q = j * BQ + i;
      const int idx = tid + kTtmThreads * q, k = idx / NC, col = idx - k * NC;
      const int kc = k & ~31, kr = k & 31;
      Bt[buf][col * pitch + kc + 8 * (kr & 3) + (kr >> 2)] = bv[i];
    }
  };
  // tile t: slice p, first q, and base X[p][0][q0] (all uniform)
  struct TileX {
    const float* xb;
    int64_t p, q0;
  };
  auto tile_at = [&](int64_t t) {
    TileX r;
    r.p = t / tilesQ;
    r.q0 = (t - r.p * tilesQ) * 64;
    r.xb = X + r.p * K * Q + r.q0;
    return r;
  };
  const uint32_t lofs = ((uint32_t)g * (uint32_t)Q + 4u * (uint32_t)l16) * 4u;
  auto load_piece = [&](const TileX& tx, int64_t kc, f32x4 (&a)[8]) {
    if (FQ) {
#pragma unroll
      for (int s2 = 0; s2 < 8; ++s2) a[s2] = *(const f32x4*)((const char*)(tx.xb + (kc + 4 * s2) * Q) + lofs);
      return;
    }
    const bool full = vec && tx.q0 + 4 * l16 + 4 <= Q;
#pragma unroll
    for (int s2 = 0; s2 < 8; ++s2) {
      const int64_t k = kc + 4 * s2 + g;
      const float* src = tx.xb + k * Q + 4 * l16;
      if (k < K && full) {
        a[s2] = *(const f32x4*)src;
      } else {
#pragma unroll
        for (int u = 0; u < 4; ++u) a[s2][u] = (k < K && tx.q0 + 4 * l16 + u < Q) ? src[u] : 0.f;
      }
    }
  };
  const int64_t stride = (int64_t)gridDim.x * kTtmWaves;
  int64_t tb = (int64_t)blockIdx.x * kTtmWaves;
  if (tb >= ntiles || cbeg >= cend) return;  // uniform: the whole workgroup
  for (int j = 0; j < 4; ++j) {
    float bv[BQ];
    load_b(cbeg, j, bv);
    store_b(0, j, bv);
  }
  const int pall = (int)((K + 31) / 32);                  // 32-index pieces of K
  const int npc = cend * 4 < pall ? cend * 4 : pall;      // end of this layer's pieces
  f32x4 an[8];
  TileX tcur = tile_at(tb + wave < ntiles ? tb + wave : ntiles - 1);
  load_piece(tcur, (int64_t)cbeg * KCH, an);
  __syncthreads();
  int buf = 0;
  for (; tb < ntiles; tb += stride) {
    asm volatile("" ::: "memory");
    const int64_t tile = tb + wave < ntiles ? tb + wave : ntiles - 1;
    const bool own = tb + wave < ntiles;
    const int64_t tnext = tb + stride + wave < ntiles ? tb + stride + wave : (tb + stride < ntiles ? ntiles - 1 : tile);
    const TileX txn = tile_at(tnext);
    f32x4 acc[4][NCB];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) acc[u][cb] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int c = cbeg; c < cend; ++c) {
      const int cn = c + 1 < cend ? c + 1 : cbeg;
      const int pend = (c + 1) * 4 < npc ? (c + 1) * 4 : npc;  // pieces of this chunk
      // piece j of the chunk loads quarter j of the next chunk's factor and
      // writes it into the other buffer after its products (that buffer was
      // last read before the previous barrier); a chunk of fewer than four
      // pieces (the last, K % 128 != 0) writes the remaining quarters at its end
      for (int pc = c * 4; pc < pend; ++pc) {
        f32x4 a[8];
#pragma unroll
        for (int s2 = 0; s2 < 8; ++s2) a[s2] = an[s2];
        float bv[BQ];
        load_b(cn, pc - c * 4, bv);
        const bool more = pc + 1 < npc;
        load_piece(more ? tcur : txn, more ? (int64_t)(pc + 1) * 32 : (int64_t)cbeg * KCH, an);
        __builtin_amdgcn_sched_barrier(0);
        const int kl = (pc - c * 4) * 32;
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) {
          const float* bp = Bt[buf] + (cb * 16 + l16) * pitch + kl + 8 * g;
          const f32x4 b0 = *(const f32x4*)bp;
          const f32x4 b1 = *(const f32x4*)(bp + 4);
#pragma unroll
          for (int t = 0; t < 8; ++t) {
            const float bval = t < 4 ? b0[t & 3] : b1[t & 3];
#pragma unroll
            for (int u = 0; u < 4; ++u)
              acc[u][cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[t][u], bval, acc[u][cb], 0, 0, 0);
          }
        }
        __builtin_amdgcn_sched_barrier(0);
        store_b(buf ^ 1, pc - c * 4, bv);
      }
      for (int j = pend - c * 4; j < 4; ++j) {
        float bv[BQ];
        load_b(cn, j, bv);
        store_b(buf ^ 1, j, bv);
      }
      buf ^= 1;
      __syncthreads();
    }
    if (own) {
      const int64_t q0 = tcur.q0;
      float* Cb = C + tcur.p * Q * R;
      if (FQ && c0 + NC <= R) {
        // row bases uniform, the lane's offset (row 16 g, column l16) in 32 bits
        const uint32_t so = ((uint32_t)(16 * g) * (uint32_t)R + (uint32_t)l16) * 4u;
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
            for (int v = 0; v < 4; ++v)
              *(float*)((char*)(Cb + (q0 + 4 * v + u) * R + c0 + cb * 16) + so) = acc[u][cb][v];
      } else {
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const int64_t q = q0 + 16 * g + 4 * v + u;
              const int col = c0 + cb * 16 + l16;
              if (q < Q && col < R) Cb[q * R + col] = acc[u][cb][v];
            }
      }
    }
    tcur = txn;
  }
}

// Y[p][q][r] = sum_i X[p][i][q][r] * A[i][r]; one thread per output element.
template <typename TI, typename TO>
__global__ __launch_bounds__(256) void k_mttv(const TI* __restrict__ X, const TI* __restrict__ A,
                                              TO* __restrict__ Y, int64_t total, int64_t I,
                                              int64_t QR, int R) {
  const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (g >= total) return;
  const int64_t p = g / QR, j = g - p * QR;
  const int r = (int)(j % R);
  const TI* x = X + p * I * QR + j;
  TO acc0 = 0, acc1 = 0, acc2 = 0, acc3 = 0;
  int64_t i = 0;
  for (; i + 4 <= I; i += 4) {
    acc0 += (TO)x[(i + 0) * QR] * (TO)A[(i + 0) * R + r];
    acc1 += (TO)x[(i + 1) * QR] * (TO)A[(i + 1) * R + r];
    acc2 += (TO)x[(i + 2) * QR] * (TO)A[(i + 2) * R + r];
    acc3 += (TO)x[(i + 3) * QR] * (TO)A[(i + 3) * R + r];
  }
  for (; i < I; ++i) acc0 += (TO)x[i * QR] * (TO)A[i * R + r];
  Y[g] = (acc0 + acc1) + (acc2 + acc3);
}

// As k_mttv with four consecutive outputs per thread (R % 4 == 0): 16-byte
// loads of X and of the factor row.
template <typename TO>
__global__ __launch_bounds__(256) void k_mttv4(const float* __restrict__ X, const float* __restrict__ A,
                                               TO* __restrict__ Y, int64_t total4, int64_t I,
                                               int64_t QR, int R) {
  const int64_t g4 = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (g4 >= total4) return;
  const int64_t g = g4 * 4;
  const int64_t p = g / QR, j = g - p * QR;
  const int r = (int)(j % R);
  const float* x = X + p * I * QR + j;
  const float* a = A + r;
  TO s0[4] = {0, 0, 0, 0}, s1[4] = {0, 0, 0, 0};
  int64_t i = 0;
  for (; i + 2 <= I; i += 2) {
    const f32x4 x0 = *(const f32x4*)(x + i * QR);
    const f32x4 x1 = *(const f32x4*)(x + (i + 1) * QR);
    const f32x4 a0 = *(const f32x4*)(a + i * R);
    const f32x4 a1 = *(const f32x4*)(a + (i + 1) * R);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      s0[u] += (TO)x0[u] * (TO)a0[u];
      s1[u] += (TO)x1[u] * (TO)a1[u];
    }
  }
  if (i < I) {
    const f32x4 x0 = *(const f32x4*)(x + i * QR);
    const f32x4 a0 = *(const f32x4*)(a + i * R);
#pragma unroll
    for (int u = 0; u < 4; ++u) s0[u] += (TO)x0[u] * (TO)a0[u];
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) Y[g + u] = s0[u] + s1[u];
}

// Two children of a node that keeps three modes, from one pass over it (the
// last level of the PP initialization, Sec. II-D, Fig. 1b: a node has up to
// three pair children, each contracting a different mode of it).  With z, u,
// v the node's modes in any order (element strides Sz, Su, Sv; the rank
// index contiguous):
//   Ycv[z][u][r] = sum_v X[z][u][v][r] Av[v][r]   (contract v)
//   Ycu[z][v][r] = sum_u X[z][u][v][r] Au[u][r]   (contract u)
// each written with its own strides.  Workgroup (iz, y) takes slice z = iz
// and the u-indices [y uc, (y + 1) uc); thread (g, lr): rank entries
// 4 lr .. 4 lr + 3 (RQ = R / 4 threads per rank vector) of the v-indices g,
// g + NG, ... (at most VMAX); UB values of u at a time are read with every
// load in flight.  Ycu accumulates in registers over the workgroup's u in
// order (with more than one u range, each range's sum goes to its own
// partial, Ycu + y pstride, added in range order afterwards); Ycv's sums
// over v are per thread, then over the groups in order through LDS.  All
// FP32 sums in a fixed order.
template <int RQ>
__global__ __launch_bounds__(256) void k_mttv_pair(const float* __restrict__ X, const float* __restrict__ Au,
                                                   const float* __restrict__ Av, float* __restrict__ Ycv,
                                                   float* __restrict__ Ycu, int64_t su, int64_t sv, int64_t Sz,
                                                   int64_t Su, int64_t Sv, int64_t ozv, int64_t ouv, int64_t ozu,
                                                   int64_t ovu, int64_t uc, int64_t pstride) {
  constexpr int NG = 256 / RQ, VMAX = 8, UB = 4;
  constexpr int R = 4 * RQ;
  __shared__ f32x4 part[NG][UB][RQ];
  const int tid = threadIdx.x, g = tid / RQ, lr = tid - g * RQ;
  const int64_t iz = blockIdx.x;
  const int64_t ub = (int64_t)blockIdx.y * uc;
  const int64_t ue = ub + uc < su ? ub + uc : su;
  Ycu += (int64_t)blockIdx.y * pstride;
  const float* Xz = X + iz * Sz + 4 * lr;
  f32x4 av[VMAX], acc[VMAX];
  bool vin[VMAX];
#pragma unroll
  for (int j = 0; j < VMAX; ++j) {
    const int64_t v = g + (int64_t)NG * j;
    vin[j] = v < sv;
    av[j] = vin[j] ? *(const f32x4*)(Av + v * R + 4 * lr) : f32x4{0.f, 0.f, 0.f, 0.f};
    acc[j] = f32x4{0.f, 0.f, 0.f, 0.f};
  }
  for (int64_t u0 = ub; u0 < ue; u0 += UB) {
    f32x4 x[UB][VMAX], au[UB];
#pragma unroll
    for (int b = 0; b < UB; ++b) {
      const int64_t u = u0 + b < ue ? u0 + b : ue - 1;  // clamped: its products are discarded
      au[b] = *(const f32x4*)(Au + u * R + 4 * lr);
#pragma unroll
      for (int j = 0; j < VMAX; ++j) {
        const int64_t v = vin[j] ? g + (int64_t)NG * j : 0;
        x[b][j] = *(const f32x4*)(Xz + u * Su + v * Sv);
      }
    }
#pragma unroll
    for (int b = 0; b < UB; ++b) {
      const bool uin = u0 + b < ue;
      f32x4 pv = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int j = 0; j < VMAX; ++j) {
        if (!vin[j]) continue;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          pv[e] += x[b][j][e] * av[j][e];
          if (uin) acc[j][e] += x[b][j][e] * au[b][e];
        }
      }
      part[g][b][lr] = pv;
    }
    __syncthreads();
    // Ycv for these u: the group partials summed in group order
    for (int t = tid; t < UB * RQ; t += 256) {
      const int b = t / RQ, l = t - b * RQ;
      if (u0 + b < ue) {
        f32x4 sum = part[0][b][l];
        for (int q = 1; q < NG; ++q) sum += part[q][b][l];
        *(f32x4*)(Ycv + iz * ozv + (u0 + b) * ouv + 4 * l) = sum;
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int j = 0; j < VMAX; ++j) {
    if (!vin[j]) continue;
    const int64_t v = g + (int64_t)NG * j;
    *(f32x4*)(Ycu + iz * ozu + v * ovu + 4 * lr) = acc[j];
  }
}

template <typename T>
__global__ void k_convert(const double* __restrict__ s, T* __restrict__ d, int64_t n) {
  const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (g < n) d[g] = (T)s[g];
}

// Khatri-Rao product of two factors as the contraction operand of two
// adjacent modes a, b (b contiguous): B[i sb + j][r] = Aa[i][r] Ab[j][r]
// (Sec. II-A), the product of the two values rounded once.
template <typename T>
__global__ void k_krp2(const T* __restrict__ Aa, const T* __restrict__ Ab, int64_t sb, int R, int64_t n,
                       T* __restrict__ B) {
  const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (g >= n) return;
  const int64_t k = g / R;
  const int r = (int)(g - k * R);
  const int64_t i = k / sb, j = k - i * sb;
  B[g] = (T)((double)Aa[i * R + r] * (double)Ab[j * R + r]);
}

__global__ void k_copy_f64(const double* __restrict__ s, double* __restrict__ d, int64_t n) {
  const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (g < n) d[g] = s[g];
}

__global__ void k_zero_f64(double* __restrict__ d, int64_t n) {
  const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (g < n) d[g] = 0.0;
}

__global__ void k_zero_u32(uint32_t* __restrict__ d, int64_t n) {
  const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (g < n) d[g] = 0u;
}

// Fixed-order block reduction of one double per thread (256 threads).
__device__ inline double block_sum(double v, double* sh) {
  const int tid = threadIdx.x;
  sh[tid] = v;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) sh[tid] += sh[tid + w];
    __syncthreads();
  }
  const double out = sh[0];
  __syncthreads();
  return out;
}

// Sums of K doubles per thread over 256 threads in a fixed order: an xor
// butterfly inside each wave, then the four wave totals in wave order.  Every
// thread gets the totals (sh: at least 4 K doubles of LDS).
template <int K>
__device__ inline void block_sums(double (&v)[K], double* sh) {
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);  // uniform (not inferred from tid / 64)
#pragma unroll
  for (int k = 0; k < K; ++k)
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_xor(v[k], off);
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) sh[wave * K + k] = v[k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = ((sh[k] + sh[K + k]) + sh[2 * K + k]) + sh[3 * K + k];
  __syncthreads();
}

// Sum of squares of the 16-byte piece v (E elements of type T), in element order.
template <typename T>
__device__ inline double piece_norm2(u32x4 v) {
  double s = 0.0;
  if constexpr (sizeof(T) == 8) {
    const f64x2 d = __builtin_bit_cast(f64x2, v);
    s = d[0] * d[0] + d[1] * d[1];
  } else if constexpr (sizeof(T) == 4) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const double x = (double)__uint_as_float(v[u]);
      s += x * x;
    }
  } else if constexpr (sizeof(T) == 2) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const uint32_t w = v[u >> 1];
      const double x = (double)__uint_as_float((u & 1) ? (w & 0xffff0000u) : (w << 16));
      s += x * x;
    }
  } else {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const auto lo = __builtin_amdgcn_cvt_pk_f32_fp8((int)v[u], false);  // bytes 0, 1
      const auto hi = __builtin_amdgcn_cvt_pk_f32_fp8((int)v[u], true);   // bytes 2, 3
      const double x0 = lo[0], x1 = lo[1], x2 = hi[0], x3 = hi[1];
      s += x0 * x0;
      s += x1 * x1;
      s += x2 * x2;
      s += x3 * x3;
    }
  }
  return s;
}

// Partial sums of squares: thread t of workgroup b takes the 16-byte pieces
// g, g + G, ... (g = 256 b + t, G = 256 gridDim.x), four in flight, each into
// its own FP64 sum; the elements after the last whole piece (or all of them
// when X is not 16-byte aligned) one by one.  Fixed order: deterministic.
template <typename T>
__global__ __launch_bounds__(256) void k_norm2_part(const T* __restrict__ X, int64_t n,
                                                    double* __restrict__ part) {
  __shared__ double sh[256];
  constexpr int E = 16 / (int)sizeof(T);
  const int64_t nv = (((uintptr_t)X & 15) == 0) ? n / E : 0;
  const u32x4* __restrict__ V = (const u32x4*)X;
  const int64_t G = (int64_t)gridDim.x * 256;
  int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  for (; i + 3 * G < nv; i += 4 * G) {
    u32x4 v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = V[i + u * G];
#pragma unroll
    for (int u = 0; u < 4; ++u) s[u] += piece_norm2<T>(v[u]);
  }
  for (; i < nv; i += G) s[0] += piece_norm2<T>(V[i]);
  for (int64_t e = nv * E + (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += G) {
    const double v = (double)X[e];
    s[1] += v * v;
  }
  const double t = block_sum((s[0] + s[1]) + (s[2] + s[3]), sh);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

__global__ __launch_bounds__(256) void k_norm2_final(const double* __restrict__ part, int np,
                                                     DevStats* stats) {
  __shared__ double sh[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < np; i += 256) s += part[i];
  const double t = block_sum(s, sh);
  if (threadIdx.x == 0) stats->normT2 = t;
}

// S[a][b] = sum_r A[r][a] A[r][b]: a workgroup takes 64 entries; thread
// group g (of four) the rows r = g, g + 4, ..., four of them per pass into
// four partial sums (eight loads in flight); the groups' sums are added in a
// fixed order.
__global__ __launch_bounds__(256) void k_gram(const double* __restrict__ A, int64_t s, int R,
                                              double* __restrict__ S) {
  __shared__ double red[4][64];
  const int jj = threadIdx.x & 63, ig = threadIdx.x >> 6;
  const int e = blockIdx.x * 64 + jj;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  if (e < R * R) {
    const int a = e / R, b = e - (e / R) * R;
    int64_t r = ig;
    for (; r + 12 < s; r += 16) {
      double x[4], y[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        x[u] = A[(r + 4 * u) * R + a];
        y[u] = A[(r + 4 * u) * R + b];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) acc[u] += x[u] * y[u];
    }
    for (; r < s; r += 4) acc[0] += A[r * R + a] * A[r * R + b];
  }
  red[ig][jj] = (acc[0] + acc[1]) + (acc[2] + acc[3]);
  __syncthreads();
  if (ig == 0 && e < R * R) S[e] = (red[0][jj] + red[1][jj]) + (red[2][jj] + red[3][jj]);
}

// One launch of independent setup operations; workgroup b runs operation
// i for first[i] <= b < first[i + 1] (256 threads: 256 elements per
// workgroup for conversions and fills; 64 Gram entries, as k_gram).
struct SetupArgs {
  SetupOp op[kMaxSetupOps];
  int first[kMaxSetupOps + 1];
  int nops;
};
__global__ __launch_bounds__(256) void k_setup(SetupArgs a) {
  __shared__ double red[4][64];
  int i = 0;
  while (i + 1 < a.nops && (int)blockIdx.x >= a.first[i + 1]) ++i;  // uniform
  const SetupOp o = a.op[i];
  const int64_t lb = (int64_t)blockIdx.x - a.first[i];
  if (o.kind == kSetupGram) {
    const int R = o.R;
    const int64_t s = o.n;
    const double* A = o.src;
    const int jj = threadIdx.x & 63, ig = threadIdx.x >> 6;
    const int e = (int)lb * 64 + jj;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    if (e < R * R) {
      const int ea = e / R, eb = e - (e / R) * R;
      int64_t r = ig;
      for (; r + 12 < s; r += 16) {
        double x[4], y[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          x[u] = A[(r + 4 * u) * R + ea];
          y[u] = A[(r + 4 * u) * R + eb];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) acc[u] += x[u] * y[u];
      }
      for (; r < s; r += 4) acc[0] += A[r * R + ea] * A[r * R + eb];
    }
    red[ig][jj] = (acc[0] + acc[1]) + (acc[2] + acc[3]);
    __syncthreads();
    if (ig == 0 && e < R * R) ((double*)o.dst)[e] = (red[0][jj] + red[1][jj]) + (red[2][jj] + red[3][jj]);
    return;
  }
  const int64_t g = lb * 256 + threadIdx.x;
  if (g >= o.n) return;
  if (o.kind == kSetupToF32) ((float*)o.dst)[g] = (float)o.src[g];
  else if (o.kind == kSetupToF64) ((double*)o.dst)[g] = o.src[g];
  else ((uint32_t*)o.dst)[g] = 0u;
}

// Entry e of Gamma^(n) and of W^(n): the product over m != n of S[m][e]
// (Eq. (1)) and the coefficient of t^2 in the product over m != n of
// (S[m][e] + t dS[m][e]), which is the bracket of Eq. (7).
__device__ inline void gamma_entry(const double* const* S, const double* const* dS, int N, int n,
                                   int e, bool pp, double* g_out, double* w_out) {
  double sv[kMaxOrder], dv[kMaxOrder];
#pragma unroll
  for (int m = 0; m < kMaxOrder; ++m) {
    const bool in = (m < N) && (m != n);
    sv[m] = in ? S[m][e] : 1.0;
    dv[m] = (in && pp) ? dS[m][e] : 0.0;
  }
  double v = 1.0, f0 = 1.0, f1 = 0.0, f2 = 0.0;
#pragma unroll
  for (int m = 0; m < kMaxOrder; ++m) {
    v *= sv[m];
    f2 = f2 * sv[m] + f1 * dv[m];
    f1 = f1 * sv[m] + f0 * dv[m];
    f0 = f0 * sv[m];
  }
  *g_out = v;
  *w_out = f2;
}

__global__ __launch_bounds__(256) void k_gamma(GammaArgs a) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= a.R * a.R) return;
  double g, w;
  gamma_entry(a.S, a.dS, a.N, a.n, e, a.pp != 0, &g, &w);
  a.Gamma[e] = g;
  if (a.pp) a.W[e] = w;
}

// Largest of one double per thread over 256 threads (red: 256 doubles of LDS).
__device__ inline double block_max(double v, double* red) {
  const int tid = threadIdx.x;
  red[tid] = v;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (tid < h) red[tid] = fmax(red[tid], red[tid + h]);
    __syncthreads();
  }
  const double out = red[0];
  __syncthreads();
  return out;
}

// LDS doubles used by pinv_lds for rank R.
__host__ __device__ inline size_t pinv_lds_doubles(int R) { return (size_t)R * (R + 1) + R + 128 + 64 + 2; }

// Gamma^dagger by the cyclic Jacobi eigenvalue method (Golub and Van Loan,
// Matrix Computations, Sec. 8.5) in parallel round-robin order, NT threads.
// Each round rotates R/2 disjoint index pairs (p, q), chosen by the circle
// method (with a bye for odd R), with the rotation that zeroes A[p][q]; rows,
// then columns of the working matrix A (LDS, pitch R + 1) and the columns of
// V (kept in Gi's memory) are updated.  A pair with
// |A[p][q]| <= eps sqrt(|A[p][p] A[q][q]|) is not rotated (its entry is set
// to zero); the sweeps stop when none rotates.  Then
// Gi = V diag(w+) V^T with w+ = 1 / w for w > R eps max(w), else 0.
// Non-finite entries of Gm zero Gi and set bit 0 of stats->status.
template <int NT>
__device__ void pinv_lds(const double* __restrict__ Gm, double* __restrict__ Gi, int R, DevStats* stats,
                         double* lds) {
  constexpr double eps = 2.220446049250313e-16;
  const int pitch = R + 1;
  double* A = lds;                     // R x pitch
  double* w = A + (size_t)R * pitch;   // R eigenvalues
  double* cs = w + R;                  // 2 x 64 rotation (c, s)
  int* pq = (int*)(cs + 128);          // 2 x 64 pair indices
  int* flags = pq + 128;               // bad, rot
  int& bad = flags[0];
  int& rot = flags[1];
  const int tid = threadIdx.x;
  const int RR = R * R;
  if (tid == 0) bad = 0;
  __syncthreads();
  for (int e = tid; e < RR; e += NT) {
    const int i = e / R, j = e - i * R;
    const double v = Gm[e];
    if (!isfinite(v)) bad = 1;
    A[i * pitch + j] = v;
    Gi[e] = (i == j) ? 1.0 : 0.0;  // V = I
  }
  __syncthreads();
  if (bad) {
    for (int e = tid; e < RR; e += NT) Gi[e] = 0.0;
    if (tid == 0) {
      stats->status |= 1;
      stats->pinv_pending = 0;
    }
    return;
  }
  const int n = R + (R & 1);  // players; index R is the bye when R is odd
  const int npair = n / 2;
  for (int sweep = 0; sweep < 60; ++sweep) {
    if (tid == 0) rot = 0;
    __syncthreads();
    for (int round = 0; round < n - 1; ++round) {
      if (tid < npair) {
        const int k = tid;
        const int a = (round + k) % (n - 1);
        const int b = (k == 0) ? n - 1 : (round - k + n - 1) % (n - 1);
        const int p = a < b ? a : b, q = a < b ? b : a;
        double c = 1.0, sn = 0.0;
        if (q < R) {
          const double apq = A[p * pitch + q], app = A[p * pitch + p], aqq = A[q * pitch + q];
          if (apq != 0.0 && fabs(apq) > eps * sqrt(fabs(app * aqq))) {
            const double tau = (aqq - app) / (2.0 * apq);
            const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + t * t);
            sn = t * c;
            rot = 1;
          }
        }
        pq[2 * k] = p;
        pq[2 * k + 1] = q < R ? q : p;  // the bye pairs p with itself: identity
        cs[2 * k] = c;
        cs[2 * k + 1] = sn;
      }
      __syncthreads();
      // rows p, q of A
      for (int e = tid; e < npair * R; e += NT) {
        const int k = e / R, j = e - k * R;
        const int p = pq[2 * k], q = pq[2 * k + 1];
        if (p == q) continue;
        const double c = cs[2 * k], sn = cs[2 * k + 1];
        const double x = A[p * pitch + j], y = A[q * pitch + j];
        A[p * pitch + j] = c * x - sn * y;
        A[q * pitch + j] = sn * x + c * y;
      }
      __syncthreads();
      // columns p, q of A and of V
      for (int e = tid; e < npair * R; e += NT) {
        const int k = e / R, i = e - k * R;
        const int p = pq[2 * k], q = pq[2 * k + 1];
        if (p == q) continue;
        const double c = cs[2 * k], sn = cs[2 * k + 1];
        const double x = A[i * pitch + p], y = A[i * pitch + q];
        A[i * pitch + p] = c * x - sn * y;
        A[i * pitch + q] = sn * x + c * y;
        const double vx = Gi[i * R + p], vy = Gi[i * R + q];
        Gi[i * R + p] = c * vx - sn * vy;
        Gi[i * R + q] = sn * vx + c * vy;
      }
      __syncthreads();
      if (tid < npair) {
        const int p = pq[2 * tid], q = pq[2 * tid + 1];
        if (p != q) {
          A[p * pitch + q] = 0.0;
          A[q * pitch + p] = 0.0;
        }
      }
      __syncthreads();
    }
    const bool done = (rot == 0);  // read after the round's last barrier
    __syncthreads();
    if (done) break;
  }
  for (int i = tid; i < R; i += NT) w[i] = A[i * pitch + i];
  __syncthreads();
  double wmax = 0.0;
  for (int i = 0; i < R; ++i) wmax = fmax(wmax, w[i]);
  const double cut = (double)R * eps * wmax;
  __syncthreads();
  for (int i = tid; i < R; i += NT) w[i] = (w[i] > cut) ? 1.0 / w[i] : 0.0;
  __syncthreads();
  for (int e = tid; e < RR; e += NT) {
    const int i = e / R, j = e - i * R;
    double acc = 0.0;
    for (int k = 0; k < R; ++k) acc += Gi[i * R + k] * w[k] * Gi[j * R + k];
    A[i * pitch + j] = acc;
  }
  __syncthreads();
  for (int e = tid; e < RR; e += NT) {
    const int i = e / R, j = e - i * R;
    Gi[e] = A[i * pitch + j];
  }
  if (tid == 0) {
    stats->pinv_pending = 0;
    stats->pinv_count += 1;
  }
}

// LDS doubles of gamma_inverse_wg for padded rank RP and rank R.
__host__ __device__ inline size_t gamma_inverse_lds_doubles(int RP, int R) {
  const size_t gj = (size_t)RP * (RP + 1) + 256 + 1;
  const size_t pv = pinv_lds_doubles(R);
  return gj > pv ? gj : pv;
}

// Gi = Gm^dagger by one workgroup of 256 threads: the blocked Gauss-Jordan
// inverse with look-ahead (gj_inverse_la), and when a pivot falls to
// R eps max(diag) or below, the Jacobi pseudo-inverse (pinv_lds) in the same
// workgroup.  Wave 0 takes the largest diagonal entry and inverts the first
// diagonal block straight from global memory while waves 1-3 copy the rest of
// the matrix (padded with the identity) into LDS, every load of a batch in
// flight before its first store.
template <int RP>
__device__ __forceinline__ void gamma_inverse_wg(const double* __restrict__ Gm, double* __restrict__ Gi, int R, DevStats* stats,
                                 double* lds) {
  constexpr int P = RP + 1;
  double* A = lds;
  int* fail = (int*)(A + RP * P);
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  double tol = 0.0;  // wave 0's
  if (wave == 0) {
    double dm = 0.0;
    for (int i = lane; i < R; i += 64) dm = fmax(dm, Gm[(int64_t)i * R + i]);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) dm = fmax(dm, __shfl_xor(dm, o));
    tol = dm * (double)R * 2.220446049250313e-16;
    const int g = lane >> 4, l16 = lane & 15;
    double x[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int j = 4 * g + c;
      x[c] = (l16 < R && j < R) ? Gm[l16 * R + j] : (l16 == j ? 1.0 : 0.0);
    }
    const bool ok = gj_block16(x, tol);
#pragma unroll
    for (int c = 0; c < 4; ++c) A[l16 * P + 4 * g + c] = x[c];
    if (lane == 0) *fail = ok ? 0 : 1;
  } else {
    constexpr int NT = 192;
    constexpr int PER = (RP * RP + NT - 1) / NT;
    constexpr int BAT = PER < 16 ? PER : 16;
    const int t = tid - 64;
#pragma unroll
    for (int q0 = 0; q0 < PER; q0 += BAT) {
      double vals[BAT];
#pragma unroll
      for (int q = 0; q < BAT; ++q) {
        const int e = t + NT * (q0 + q), i = e / RP, j = e - i * RP;
        vals[q] = (q0 + q < PER && e < RP * RP && i < R && j < R) ? Gm[i * R + j] : (i == j ? 1.0 : 0.0);
      }
#pragma unroll
      for (int q = 0; q < BAT; ++q) {
        const int e = t + NT * (q0 + q), i = e / RP, j = e - i * RP;
        if (q0 + q < PER && e < RP * RP && (i >= 16 || j >= 16)) A[i * P + j] = vals[q];
      }
    }
  }
  if (gj_inverse_la<RP>(A, tol, fail)) {
    for (int e = tid; e < R * R; e += 256) {
      const int i = e / R, j = e - i * R;
      Gi[e] = A[i * P + j];
    }
  } else {
    __syncthreads();
    pinv_lds<256>(Gm, Gi, R, stats, lds);
  }
}

// Ginv = Gamma^dagger in one workgroup (gamma_inverse_wg).
template <int RP>
__global__ __launch_bounds__(256) void k_inv_blk(const double* __restrict__ Gm, double* __restrict__ Gi, int R,
                                                 DevStats* stats) {
  extern __shared__ double lds_d[];
  gamma_inverse_wg<RP>(Gm, Gi, R, stats, lds_d);
}

// LDS doubles of k_update's solve phase for padded rank RP: the R x R
// operand chunk(s) (Ginv, and W in PP, whole when RP <= 64) and four 16 x RP
// row buffers (M~, new A, dA, reference A).
__host__ __device__ inline size_t update_solve_lds_doubles(int RP) {
  const int CH = RP < 64 ? RP : 64;
  const int nbuf = (RP <= 64) ? 2 : 1;
  return (size_t)nbuf * RP * (CH + 1) + 4 * 16 * (size_t)(RP + 1);
}

// One mode update in one launch (Alg. 1 inner body; Alg. 2 with Eq. (7) in
// PP).  Workgroup b takes the 16-row blocks b, b + G, ... of mode n:
//   M~ = M (+ A_old W in PP),  A_new = M~ Ginv,
// the shadows, dA (A_new - A_old, or A_new - A_p in PP), ||A||^2, ||dA||^2
// and <M~, A_new> over its rows, and its partial Gram A^T A (and dS = A^T dA)
// accumulated on the f64 matrix cores across its row blocks.  The last
// workgroup to finish (a ticket counter, which it resets) sums the partials
// in workgroup order into S^(n), dS^(n) and the norms, forms the residual
// of Eq. (3) after the last mode (with <Gamma^(n), S^(n)>), writes Gamma and
// W of the next mode nx = (n + 1) mod N, and, when inv_next is set, inverts
// Gamma^(nx) into Ginv in place (gj_inverse_lds; the Jacobi
// pseudo-inverse when a pivot is too small), so that the next mode needs no
// separate inverse.  All workgroups read Ginv, W and Gamma before taking
// their ticket, so the last one may overwrite them.
template <typename T, int RP, bool PP>
__global__ __launch_bounds__(256) void k_update(UpdateArgs<T> a) {
  constexpr int CH = RP < 64 ? RP : 64, NCH = RP / CH;
  constexpr int PG = CH + 1, PM = RP + 1, NB = RP / 16;
  constexpr int NGW = (NB * NB + 3) / 4;  // Gram blocks per wave
  // Gram accumulators live in registers across row blocks, except where
  // they would not fit (RP = 128 with dS)
  constexpr bool kGramInRegs = !(RP == 128 && PP);
  extern __shared__ double lds[];
  __shared__ double sh[256];
  __shared__ int flag;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform (not inferred from tid / 64)
  const int l16 = lane & 15, lg = lane >> 4;
  const int R = a.R;
  constexpr bool pp = PP;
  double* Gi = lds;                                // RP x PG: Ginv (chunk)
  double* Gw = (NCH == 1) ? Gi + RP * PG : Gi;     // RP x PG: W (PP)
  double* Mt = Gi + (NCH == 1 ? 2 : 1) * RP * PG;  // 16 x PM
  double* An = Mt + 16 * PM;
  double* dAn = An + 16 * PM;
  double* Ao = dAn + 16 * PM;
  auto stage = [&](double* dst, const double* src, int c0) {
    constexpr int PER = RP * CH / 256;
    double v[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int e = tid + 256 * q, k = e / CH, c = e - k * CH;
      v[q] = (k < R && c0 + c < R) ? src[k * R + c0 + c] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int e = tid + 256 * q, k = e / CH, c = e - k * CH;
      dst[k * PG + c] = v[q];
    }
  };
  // X (16 x RP, pitch PM) times the staged chunk B -> 16 x 16 block at column block cbl
  auto block_mm = [&](const double* X, const double* B, int cbl) {
    constexpr int KU = RP <= 64 ? RP / 4 : 8;  // k-steps unrolled (register pressure at RP = 128)
    f64x4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 1
    for (int k0 = 0; k0 < RP / 4; k0 += KU) {
#pragma unroll
      for (int ks = k0; ks < k0 + KU; ++ks) {
        const int k = ks * 4 + lg;
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(X[l16 * PM + k], B[k * PG + cbl * 16 + l16], acc, 0, 0, 0);
      }
    }
    return acc;
  };
  if (NCH == 1) {
    stage(Gi, a.Ginv, 0);
    if (pp) stage(Gw, a.W, 0);
  }
  f64x4 accS[kGramInRegs ? NGW : 1], accD[kGramInRegs ? NGW : 1];
#pragma unroll
  for (int t = 0; t < (kGramInRegs ? NGW : 1); ++t) {
    accS[t] = f64x4{0.0, 0.0, 0.0, 0.0};
    accD[t] = f64x4{0.0, 0.0, 0.0, 0.0};
  }
  double nA2 = 0.0, nd2 = 0.0, ma = 0.0;
  for (int rb = blockIdx.x; rb < a.nrb; rb += gridDim.x) {
    const int64_t r0 = (int64_t)rb * 16;
    const int rows = (int)((a.s - r0) < 16 ? (a.s - r0) : 16);
    {
      constexpr int PR = RP / 16;
      double m[PR], an[PR], ao[PR];
#pragma unroll
      for (int q = 0; q < PR; ++q) {
        const int e = tid + 256 * q, r = e / RP, c = e - r * RP;
        const bool in = r < rows && c < R;
        const int64_t gi = (r0 + r) * R + c;
        m[q] = in ? a.M[gi] : 0.0;
        an[q] = in ? a.A[gi] : 0.0;
        ao[q] = (in && pp) ? a.Ap[gi] : an[q];
      }
#pragma unroll
      for (int q = 0; q < PR; ++q) {
        const int e = tid + 256 * q, r = e / RP, c = e - r * RP;
        Mt[r * PM + c] = m[q];
        An[r * PM + c] = an[q];
        Ao[r * PM + c] = ao[q];
      }
    }
    __syncthreads();
    if (pp) {
      // M~ = M + V^(n), V^(n) = A^(n) W with the current (old) A^(n)  (Eq. (7))
      for (int c0 = 0; c0 < RP; c0 += CH) {
        if (NCH > 1) {
          stage(Gw, a.W, c0);
          __syncthreads();
        }
        for (int cbl = wave; cbl < CH / 16; cbl += 4) {
          const f64x4 acc = block_mm(An, Gw, cbl);
#pragma unroll
          for (int v = 0; v < 4; ++v) Mt[(lg + 4 * v) * PM + c0 + cbl * 16 + l16] += acc[v];
        }
        __syncthreads();
      }
    }
    for (int c0 = 0; c0 < RP; c0 += CH) {
      if (NCH > 1) {
        stage(Gi, a.Ginv, c0);
        __syncthreads();
      }
      for (int cbl = wave; cbl < CH / 16; cbl += 4) {
        const f64x4 acc = block_mm(Mt, Gi, cbl);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = lg + 4 * v, c = c0 + cbl * 16 + l16;
          double val = 0.0, d = 0.0;
          if (r < rows && c < R) {
            val = acc[v];
            d = val - Ao[r * PM + c];
            const int64_t gi = (r0 + r) * R + c;
            a.A[gi] = val;
            a.Ash[gi] = (T)val;
            if (pp) a.dAsh[gi] = (T)d;
            nA2 += val * val;
            nd2 += d * d;
            ma += Mt[r * PM + c] * val;
          }
          An[r * PM + c] = val;
          dAn[r * PM + c] = d;
        }
      }
      __syncthreads();
    }
    // partial Gram (and dS) of these rows
    auto gram_block = [&](int ab, int bb, f64x4& sacc, f64x4& dacc) {
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) {
        const int r = ks * 4 + lg;
        const double x = An[r * PM + ab * 16 + l16];
        sacc = __builtin_amdgcn_mfma_f64_16x16x4f64(x, An[r * PM + bb * 16 + l16], sacc, 0, 0, 0);
        if (pp) dacc = __builtin_amdgcn_mfma_f64_16x16x4f64(x, dAn[r * PM + bb * 16 + l16], dacc, 0, 0, 0);
      }
    };
    if constexpr (kGramInRegs) {
#pragma unroll
      for (int t = 0; t < NGW; ++t) {
        const int blk = wave + 4 * t;
        if (blk < NB * NB) gram_block(blk / NB, blk % NB, accS[t], accD[t]);
      }
    } else {
      // too many accumulators to keep: add into this workgroup's partials
      const bool first = rb == (int)blockIdx.x;
#pragma unroll 1
      for (int t = 0; t < NGW; ++t) {
        const int blk = wave + 4 * t;
        if (blk < NB * NB) {
          const int ab = blk / NB, bb = blk - ab * NB;
          f64x4 sacc = {0.0, 0.0, 0.0, 0.0}, dacc = {0.0, 0.0, 0.0, 0.0};
          gram_block(ab, bb, sacc, dacc);
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int ar = ab * 16 + lg + 4 * v, bc = bb * 16 + l16;
            if (ar < R && bc < R) {
              const int64_t idx = (int64_t)blockIdx.x * R * R + ar * R + bc;
              a.partS[idx] = first ? sacc[v] : a.partS[idx] + sacc[v];
              if (pp) a.partdS[idx] = first ? dacc[v] : a.partdS[idx] + dacc[v];
            }
          }
        }
      }
    }
    __syncthreads();
  }
  const int RR = R * R;
  if constexpr (kGramInRegs) {
    double* pS = a.partS + (int64_t)blockIdx.x * RR;
    double* pdS = a.partdS + (int64_t)blockIdx.x * RR;
#pragma unroll
    for (int t = 0; t < NGW; ++t) {
      const int blk = wave + 4 * t;
      if (blk < NB * NB) {
        const int ab = blk / NB, bb = blk - ab * NB;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int ar = ab * 16 + lg + 4 * v, bc = bb * 16 + l16;
          if (ar < R && bc < R) {
            pS[ar * R + bc] = accS[t][v];
            if (pp) pdS[ar * R + bc] = accD[t][v];
          }
        }
      }
    }
  }
  {
    double v3[3] = {nA2, nd2, ma};
    block_sums<3>(v3, sh);
    if (tid == 0) {
      a.partSc[blockIdx.x * 4 + 0] = v3[0];
      a.partSc[blockIdx.x * 4 + 1] = v3[1];
      a.partSc[blockIdx.x * 4 + 2] = v3[2];
    }
  }
  if (!a.fused) return;  // k_update_reduce sums the partials
  // The reductions, spread over the G workgroups.  Each waits until every
  // workgroup has written its partials (arrival count G; all G <= 16
  // workgroups are resident at once, and the wait is bounded), then takes
  // a contiguous slice of the R x R entries: S^(n) (and dS^(n)) = the
  // partials summed in workgroup order, its share of <Gamma^(n), S^(n)>,
  // and the entries of Gamma^(nx) (Eq. (1)) and, in PP, W^(nx) (the bracket
  // of Eq. (7)), with S^(n) and dS^(n) from registers.  Every workgroup read
  // Gamma, W and Ginv before arriving, and each overwrites only its own
  // slice of Gamma and W.  The last to finish its slice (arrival count 2G)
  // adds the norms and shares in workgroup order, forms the residual of
  // Eq. (3) after the last mode, and, when inv_next is set, inverts
  // Gamma^(nx) into Ginv (gamma_inverse_wg).
  const int n = a.n, N = a.N, nx = (n + 1) % N, G = gridDim.x;
  __threadfence();
  __syncthreads();
  if (tid == 0) {
    __hip_atomic_fetch_add(a.ticket, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    int spins = 0;
    while (__hip_atomic_load(a.ticket, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < (unsigned)G) {
      __builtin_amdgcn_s_sleep(2);
      if (++spins == (1 << 22)) {  // never expected: the results are then flagged, not waited for
        atomicOr(&a.stats->status, 4);
        break;
      }
    }
  }
  __syncthreads();
  __threadfence();
  {
    const int per = (RR + G - 1) / G;
    const int e0 = (int)blockIdx.x * per;
    const int e1 = e0 + per < RR ? e0 + per : RR;
    double* const Sn = a.S[n];
    double* const dSn = a.dS[n];
    const double* __restrict__ const pS = a.partS;
    const double* __restrict__ const pdS = a.partdS;
    const double* Sm[kMaxOrder];
    const double* dSm[kMaxOrder];
#pragma unroll
    for (int m = 0; m < kMaxOrder; ++m) {
      const bool use = m < N && m != n && m != nx;
      Sm[m] = use ? a.S[m] : nullptr;
      dSm[m] = (use && pp) ? a.dS[m] : nullptr;
    }
    constexpr int EB = 2;
    double gsum = 0.0;
    for (int j0 = e0 + tid; j0 < e1; j0 += 256 * EB) {
      // every load of the batch in flight before the first use (indices
      // clamped into the slice, out-of-range entries discarded afterwards)
      int ei[EB];
      bool in[EB];
      double gm[EB], sv[EB], dv[EB], sm[kMaxOrder][EB], dm[kMaxOrder][EB];
#pragma unroll
      for (int u = 0; u < EB; ++u) {
        const int e = j0 + 256 * u;
        in[u] = e < e1;
        ei[u] = in[u] ? e : e0;
        gm[u] = a.Gamma[ei[u]];
        sv[u] = 0.0;
        dv[u] = 0.0;
      }
#pragma unroll
      for (int m = 0; m < kMaxOrder; ++m)
#pragma unroll
        for (int u = 0; u < EB; ++u) {
          sm[m][u] = Sm[m] ? Sm[m][ei[u]] : 1.0;
          dm[m][u] = dSm[m] ? dSm[m][ei[u]] : 0.0;
        }
      for (int b0 = 0; b0 < G; b0 += 8) {
        double pv[8][EB], pd[8][EB];
#pragma unroll
        for (int bb = 0; bb < 8; ++bb) {
          const int64_t off = (int64_t)(b0 + bb < G ? b0 + bb : G - 1) * RR;
#pragma unroll
          for (int u = 0; u < EB; ++u) {
            pv[bb][u] = pS[off + ei[u]];
            if (pp) pd[bb][u] = pdS[off + ei[u]];
          }
        }
#pragma unroll
        for (int bb = 0; bb < 8; ++bb) {
          const bool inb = b0 + bb < G;
#pragma unroll
          for (int u = 0; u < EB; ++u) {
            sv[u] += inb ? pv[bb][u] : 0.0;
            if (pp) dv[u] += inb ? pd[bb][u] : 0.0;
          }
        }
      }
#pragma unroll
      for (int u = 0; u < EB; ++u) {
        if (!in[u]) continue;
        const int e = ei[u];
        Sn[e] = sv[u];
        if (pp) dSn[e] = dv[u];
        gsum += gm[u] * sv[u];
        // products over m != nx in increasing m (the coefficient of t^2 of
        // the product of S^(m) + t dS^(m) is the bracket of Eq. (7))
        double v = 1.0, f0 = 1.0, f1 = 0.0, f2 = 0.0;
#pragma unroll
        for (int m = 0; m < kMaxOrder; ++m) {
          const double smv = (m == n) ? sv[u] : sm[m][u];
          const double dmv = (m == n) ? (pp ? dv[u] : 0.0) : dm[m][u];
          v *= smv;
          if (pp) {
            f2 = f2 * smv + f1 * dmv;
            f1 = f1 * smv + f0 * dmv;
            f0 = f0 * smv;
          }
        }
        a.Gamma[e] = v;
        if (pp) a.W[e] = f2;
      }
    }
    double g1[1] = {gsum};
    block_sums<1>(g1, sh);
    if (tid == 0) a.partSc[blockIdx.x * 4 + 3] = g1[0];
  }
  __threadfence();
  __syncthreads();
  if (tid == 0) flag = (atomicAdd(a.ticket, 1u) == 2u * (unsigned)G - 1u) ? 1 : 0;
  __syncthreads();
  if (!flag) return;  // uniform
  __threadfence();
  if (tid == 0) atomicExch(a.ticket, 0u);
  double v4[4] = {0.0, 0.0, 0.0, 0.0};
  for (int b = tid; b < G; b += 256) {
    v4[0] += a.partSc[b * 4 + 0];
    v4[1] += a.partSc[b * 4 + 1];
    v4[2] += a.partSc[b * 4 + 2];
    v4[3] += a.partSc[b * 4 + 3];
  }
  block_sums<4>(v4, sh);
  if (tid == 0) {
    a.stats->normA2[n] = v4[0];
    a.stats->normdA2[n] = v4[1];
    if (a.last) {
      const double tn = a.stats->normT2;
      const double num = tn + v4[3] - 2.0 * v4[2];
      a.stats->fit_num = num;
      const double r = sqrt((num > 0.0 ? num : 0.0) / tn);
      a.stats->r = r;
      a.stats->r_clamped = (num < 0.0) ? 1 : 0;
      if (!isfinite(r)) a.stats->status |= 2;
    }
  }
  if (!a.inv_next) return;  // uniform
  __syncthreads();
  gamma_inverse_wg<RP>(a.Gamma, a.Ginv, R, a.stats, lds);
}

//
// With a.Ginv set, the grid has one more workgroup, which inverts Gamma^(n)
// (formed by the previous update) into a.Ginv meanwhile: the inverse is off
// the update's critical path.
template <typename T, int RP>
__global__ __launch_bounds__(256) void k_pp_mttkrp(PPArgs<T> a) {
  if (a.Ginv && blockIdx.x == gridDim.x - 1) {  // uniform
    extern __shared__ double lds_inv[];
    gamma_inverse_wg<RP>(a.Gamma, a.Ginv, a.R, a.stats, lds_inv);
    return;
  }
  __shared__ double red[256];
  const int tid = threadIdx.x, R = a.R;
  const int G = 256 / R;
  const int r = tid % R, yg = tid / R;
  const int64_t x = blockIdx.x;
  const int64_t sn = a.dims[a.n];
  double u = 0.0;
  if (yg < G) {
    for (int i = 0; i < a.N; ++i) {
      if (i == a.n) continue;
      const int64_t si = a.dims[i];
      const T* d = a.dA[i] + r;
      const T* p;
      int64_t ys;  // stride between consecutive y
      if (a.pair_n_first[i]) {
        p = a.pair[i] + x * si * R + r;  // P[x][y][r]
        ys = R;
      } else {
        p = a.pair[i] + x * R + r;  // P[y][x][r]
        ys = sn * R;
      }
      // y = yg, yg + G, ...: eight per pass into eight partial sums (sixteen
      // loads in flight), then the remainder; fixed order
      int64_t y = yg;
      double up[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
      for (; y + 7 * G < si; y += 8 * G) {
        double pv[8], dv[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          pv[k] = (double)p[(y + k * G) * ys];
          dv[k] = (double)d[(y + k * G) * R];
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) up[k] += pv[k] * dv[k];
      }
      for (; y < si; y += G) up[0] += (double)p[y * ys] * (double)d[y * R];
      u += ((up[0] + up[1]) + (up[2] + up[3])) + ((up[4] + up[5]) + (up[6] + up[7]));
    }
  }
  red[tid] = u;
  __syncthreads();
  if (tid < R) {
    double acc = a.Mp[x * R + tid];
    for (int k = 0; k < G; ++k) acc += red[k * R + tid];
    a.M[x * R + tid] = acc;
  }
}

// Small contractions (few outputs, e.g. the leaves): Y[p][j] =
// sum_i X[p][i][j] A[i][j % R] with the i range split over 4 thread groups
// of one workgroup and added in a fixed order.  Block = (p, 64 outputs).
template <typename TI, typename TO>
__global__ __launch_bounds__(256) void k_mttv_split(const TI* __restrict__ X, const TI* __restrict__ A,
                                                    TO* __restrict__ Y, int64_t I, int64_t QR, int R,
                                                    int64_t jblocks) {
  __shared__ TO red[4][64];
  const int tid = threadIdx.x, jj = tid & 63, ig = tid >> 6;
  const int64_t p = blockIdx.x / jblocks;
  const int64_t j = (blockIdx.x - p * jblocks) * 64 + jj;
  TO s = 0;
  if (j < QR) {
    const int r = (int)(j % R);
    const TI* x = X + p * I * QR + j;
    // group ig takes i = ig, ig + 4, ...: eight of them per pass, each into
    // its own partial sum (eight loads in flight), then the remainder
    TO sp[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int64_t i = ig;
    for (; i + 28 < I; i += 32) {
      TI xv[8], av[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        xv[u] = x[(i + 4 * u) * QR];
        av[u] = A[(i + 4 * u) * R + r];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) sp[u] += (TO)xv[u] * (TO)av[u];
    }
    for (; i < I; i += 4) sp[0] += (TO)x[i * QR] * (TO)A[i * R + r];
    s = ((sp[0] + sp[1]) + (sp[2] + sp[3])) + ((sp[4] + sp[5]) + (sp[6] + sp[7]));
  }
  red[ig][jj] = s;
  __syncthreads();
  if (ig == 0 && j < QR) Y[p * QR + j] = (red[0][jj] + red[1][jj]) + (red[2][jj] + red[3][jj]);
}

// r of Eq. (3) for given factors: <M, A> and <Gamma, S> in one workgroup.
__global__ __launch_bounds__(256) void k_fitness(const double* __restrict__ M, const double* __restrict__ A,
                                                 int64_t n, const double* __restrict__ G, const double* __restrict__ S,
                                                 int RR, DevStats* stats) {
  __shared__ double sh[256];
  double ma = 0.0, gs = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) ma += M[i] * A[i];
  for (int i = threadIdx.x; i < RR; i += 256) gs += G[i] * S[i];
  const double tma = block_sum(ma, sh);
  const double tgs = block_sum(gs, sh);
  if (threadIdx.x == 0) {
    const double t2 = stats->normT2;
    const double num = t2 + tgs - 2.0 * tma;
    stats->fit_num = num;
    stats->r = sqrt((num > 0.0 ? num : 0.0) / t2);
    stats->r_clamped = (num < 0.0) ? 1 : 0;
  }
}

inline unsigned nblocks(int64_t n) { return (unsigned)((n + 255) / 256); }

// Raise a kernel's dynamic LDS limit on the current device, once per device
// (the attribute belongs to the device; two first calls at once both set it,
// harmlessly).  `done` holds one bit per device index below 64.
inline hipError_t lds_limit_once(std::atomic<uint64_t>& done, const void* fn, int bytes) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  const uint64_t bit = (dev >= 0 && dev < 64) ? (1ull << dev) : 0;
  if (bit && (done.load(std::memory_order_acquire) & bit)) return hipSuccess;
  e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (e == hipSuccess && bit) done.fetch_or(bit, std::memory_order_release);
  return e;
}



}  // namespace

template <typename T, bool KC, int NCB>
hipError_t launch_ttm_rb(const T* X, const T* B, T* C, int64_t P, int64_t K, int64_t Q, int R,
                         hipStream_t st) {
  constexpr int V = 16 / sizeof(T);
  constexpr int CH = 8 * 4 * V;
  const int Kp = (int)((K + CH - 1) / CH * CH);
  const size_t lds = (size_t)NCB * 16 * (Kp + V) * sizeof(T);
  static std::atomic<uint64_t> attr{0};
  {
    hipError_t e = lds_limit_once(attr, (const void*)k_ttm_rb<T, KC, NCB>, 160 * 1024);
    if (e != hipSuccess) return e;
  }
  const int64_t tilesQ = KC ? 1 : (Q + 31) / 32;
  const int64_t ntiles = KC ? (P + 31) / 32 : P * tilesQ;
  const int64_t want = (ntiles + kTtmWaves - 1) / kTtmWaves;
  const unsigned nx = (unsigned)(want < 2048 ? want : 2048);
  const unsigned ny = (unsigned)((R + NCB * 16 - 1) / (NCB * 16));
  const int vec = (K % V == 0 && ((uintptr_t)X % 16) == 0) ? 1 : 0;
  hipLaunchKernelGGL((k_ttm_rb<T, KC, NCB>), dim3(nx, ny), dim3(kTtmThreads), lds, st, X, B, C, P, K, Q, R,
                     tilesQ, ntiles, Kp, vec);
  return hipGetLastError();
}

template <typename T, int NCB>
hipError_t launch_ttm_kc(const T* X, const T* B, T* C, int64_t P, int64_t K, int R, hipStream_t st) {
  constexpr int V = 16 / sizeof(T);
  const int64_t ntiles = (P + 15) / 16;
  const int64_t want = (ntiles + kTtmWaves - 1) / kTtmWaves;
  const unsigned nx = (unsigned)(want < 256 ? want : 256);  // one workgroup per CU, each wave two tiles deep
  const unsigned ny = (unsigned)((R + NCB * 16 - 1) / (NCB * 16));
  const int vec = (K % V == 0 && ((uintptr_t)X % 16) == 0) ? 1 : 0;
  // NTS t-steps of 4V contraction indices: the padded depth follows K
  const int64_t KT = 4 * V;
  if (K <= 2 * KT) {
    if (vec && K == 2 * KT)
      hipLaunchKernelGGL((k_ttm_kc<T, NCB, 2, true>), dim3(nx, ny), dim3(kTtmThreads), 0, st, X, B, C, P, K, R, ntiles, vec);
    else
      hipLaunchKernelGGL((k_ttm_kc<T, NCB, 2, false>), dim3(nx, ny), dim3(kTtmThreads), 0, st, X, B, C, P, K, R, ntiles, vec);
  } else if (K <= 4 * KT) {
    if (vec && K == 4 * KT)
      hipLaunchKernelGGL((k_ttm_kc<T, NCB, 4, true>), dim3(nx, ny), dim3(kTtmThreads), 0, st, X, B, C, P, K, R, ntiles, vec);
    else
      hipLaunchKernelGGL((k_ttm_kc<T, NCB, 4, false>), dim3(nx, ny), dim3(kTtmThreads), 0, st, X, B, C, P, K, R, ntiles, vec);
  } else {
    if (vec && K == 8 * KT)
      hipLaunchKernelGGL((k_ttm_kc<T, NCB, 8, true>), dim3(nx, ny), dim3(kTtmThreads), 0, st, X, B, C, P, K, R, ntiles, vec);
    else
      hipLaunchKernelGGL((k_ttm_kc<T, NCB, 8, false>), dim3(nx, ny), dim3(kTtmThreads), 0, st, X, B, C, P, K, R, ntiles, vec);
  }
  return hipGetLastError();
}

template <int NCB>
hipError_t launch_ttm_kc32(const float* X, const float* B, float* C, int64_t P, int R, hipStream_t st) {
  const int64_t ntiles = (P + 31) / 32;
  const int64_t want = (ntiles + kTtmWaves - 1) / kTtmWaves;
  const unsigned nx = (unsigned)(want < 256 ? want : 256);
  const unsigned ny = (unsigned)((R + NCB * 32 - 1) / (NCB * 32));
  hipLaunchKernelGGL((k_ttm_kc32<NCB>), dim3(nx, ny), dim3(kTtmThreads), 0, st, X, B, C, P, R, ntiles);
  return hipGetLastError();
}

// The leading half's first and second levels in one pass (k_ttm_kc32f):
// X is (P2 S) x 128 (last mode contracted with B), A2 is S x R (the mode
// before it), C is P2 x R.
bool ttm_kc_fused_fits(const float* X, int64_t K, int64_t S, int R) {
  return K == 128 && S % 32 == 0 && S >= 32 && S <= kFusedMaxS && R > 16 && R <= 64 && ((uintptr_t)X % 16) == 0;
}

template <bool STORE>
hipError_t launch_kc32f(const float* X, const float* B, const float* A2, float* C, float* Y, int64_t P2, int64_t S,
                        int R, hipStream_t st) {
  const int64_t want = (P2 + kTtmWaves - 1) / kTtmWaves;
  const unsigned nx = (unsigned)(want < 256 ? want : 256);
  const size_t lds = (size_t)64 * (S + 4) * sizeof(float);
  if (R <= 32) {
    hipLaunchKernelGGL((k_ttm_kc32f<1, STORE>), dim3(nx, 1), dim3(kTtmThreads), lds / 2, st, X, B, A2, C, Y, R,
                       (int)S, P2);
  } else {
    static std::atomic<uint64_t> attr{0};
    // dynamic part only (the kernel also holds 33 KB of static LDS): 64 (kFusedMaxS + 4) floats
    const hipError_t e = lds_limit_once(attr, (const void*)k_ttm_kc32f<2, STORE>, 96 * 1024);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_ttm_kc32f<2, STORE>), dim3(nx, 1), dim3(kTtmThreads), lds, st, X, B, A2, C, Y, R, (int)S,
                       P2);
  }
  return hipGetLastError();
}

hipError_t launch_ttm_kc_fused(const float* X, const float* B, const float* A2, float* C, float* Y, int64_t P2,
                               int64_t S, int R, hipStream_t st) {
  if (!ttm_kc_fused_fits(X, 128, S, R) || P2 < 1) return hipErrorInvalidValue;
  return Y ? launch_kc32f<true>(X, B, A2, C, Y, P2, S, R, st) : launch_kc32f<false>(X, B, A2, C, Y, P2, S, R, st);
}

// k_ttm_qg's shape limits: K a multiple of 32 up to 256, Q a multiple of 64,
// 32-bit lane offsets (kstride < 2^28), R <= 64, X 16-byte aligned.
bool ttm_qg_shape(const QgShape& sh, int R) {
  return sh.K % 32 == 0 && sh.K >= 32 && sh.K <= 256 && sh.Q % 64 == 0 && sh.Q >= 64 && sh.S >= 1 && sh.nP >= 1 &&
         sh.kstride >= sh.Q && sh.kstride < ((int64_t)1 << 28) && R >= 1 && R <= 64;
}

bool ttm_qg_fits(const float* X, const QgShape& sh, int R) {
  return ttm_qg_shape(sh, R) && ((uintptr_t)X % 16) == 0;
}

// Ranges of i: enough (p', q block) x range waves for about 2048.
int qg_layers(const QgShape& sh) {
  const int64_t pairs = sh.nP * (sh.Q / 64);
  int64_t nz = (2048 + pairs - 1) / (pairs > 0 ? pairs : 1);
  nz = nz < 1 ? 1 : (nz > sh.S ? sh.S : nz);
  const int64_t L = (sh.S + nz - 1) / nz;
  return (int)((sh.S + L - 1) / L);
}

template <int NCB, bool STORE>
hipError_t launch_ttm_qg_ncb(const float* X, const float* B, const float* W, float* out, float* Y, const QgShape& sh,
                             int R, int L, int nz, hipStream_t st) {
  static std::atomic<uint64_t> attr{0};
  const hipError_t e = lds_limit_once(attr, (const void*)k_ttm_qg<NCB, STORE>, 160 * 1024);
  if (e != hipSuccess) return e;
  const size_t lds = (size_t)NCB * 16 * (sh.K + 4) * sizeof(float);
  const int64_t pairs = sh.nP * (sh.Q / 64);
  const unsigned nx = (unsigned)((pairs + kTtmWaves - 1) / kTtmWaves);
  const unsigned ny = (unsigned)((R + NCB * 16 - 1) / (NCB * 16));
  hipLaunchKernelGGL((k_ttm_qg<NCB, STORE>), dim3(nx, ny, (unsigned)nz), dim3(kTtmThreads), lds, st, X, B, W, out, Y,
                     sh, R, L);
  return hipGetLastError();
}

hipError_t launch_ttm_qg(const float* X, const float* B, const float* W, float* C, float* Y, const QgShape& sh, int R,
                         float* parts, hipStream_t st) {
  if (!ttm_qg_fits(X, sh, R)) return hipErrorInvalidValue;
  const int nz = qg_layers(sh);
  const int L = (int)((sh.S + nz - 1) / nz);
  float* out = nz > 1 ? parts : C;
  if (nz > 1 && !parts) return hipErrorInvalidValue;
  hipError_t e;
#define CPALS_QG(NCB)                                                                                      \
  e = Y ? launch_ttm_qg_ncb<NCB, true>(X, B, W, out, Y, sh, R, L, nz, st)                                 \
        : launch_ttm_qg_ncb<NCB, false>(X, B, W, out, Y, sh, R, L, nz, st)
  if (R <= 16) CPALS_QG(1);
  else if (R <= 32) CPALS_QG(2);
  else CPALS_QG(4);
#undef CPALS_QG
  if (e != hipSuccess || nz == 1) return e;
  const int64_t n = sh.nP * sh.Q * R;
  const int64_t nb = (n / 4 + 255) / 256;
  hipLaunchKernelGGL((k_sum_parts<float>), dim3((unsigned)(nb < 2048 ? nb : 2048)), dim3(256), 0, st, parts, C, n, nz);
  return hipGetLastError();
}

// MSDT's root at mode 0 with its first child in the epilogue (k_ttm_qr):
// X is K x Q, B (K x R), W (S x R, the last mode), C ((Q / S) x R), Y the
// first-level node (Q x R) or null.
bool ttm_qr_fits(const float* X, int64_t P, int64_t K, int64_t Q, int64_t S, int R) {
  return P >= 1 && K % 32 == 0 && K >= 32 && K <= 256 && (S == 64 || S == 128 || S == 256) && Q % S == 0 &&
         Q < ((int64_t)1 << 28) && R >= 1 && R <= 64 && ((uintptr_t)X % 16) == 0;
}

template <int NCB, bool STORE>
hipError_t launch_ttm_qr_ncb(const float* X, const float* B, const float* W, float* C, float* Y, int64_t P, int64_t K,
                             int64_t Q, int64_t S, int R, hipStream_t st) {
  static std::atomic<uint64_t> attr{0};
  const hipError_t e = lds_limit_once(attr, (const void*)k_ttm_qr<NCB, STORE>, 160 * 1024);
  if (e != hipSuccess) return e;
  const size_t lds = (size_t)NCB * 16 * ((K + 4) + (S + 4) + kTtmWaves) * sizeof(float);
  const int64_t rps = kTtmWaves / (S / 64);  // output rows per workgroup step
  const int64_t want = (P * (Q / S) + rps - 1) / rps;
  const unsigned nx = (unsigned)(want < 256 ? want : 256);
  const unsigned ny = (unsigned)((R + NCB * 16 - 1) / (NCB * 16));
  hipLaunchKernelGGL((k_ttm_qr<NCB, STORE>), dim3(nx, ny), dim3(kTtmThreads), lds, st, X, B, W, C, Y, P, K, Q, R,
                     (int)S);
  return hipGetLastError();
}

hipError_t launch_ttm_qr(const float* X, const float* B, const float* W, float* C, float* Y, int64_t P, int64_t K,
                         int64_t Q, int64_t S, int R, hipStream_t st) {
  if (!ttm_qr_fits(X, P, K, Q, S, R)) return hipErrorInvalidValue;
#define CPALS_QR(NCB)                                                             \
  return Y ? launch_ttm_qr_ncb<NCB, true>(X, B, W, C, Y, P, K, Q, S, R, st)       \
           : launch_ttm_qr_ncb<NCB, false>(X, B, W, C, Y, P, K, Q, S, R, st)
  if (R <= 16) CPALS_QR(1);
  if (R <= 32) CPALS_QR(2);
  CPALS_QR(4);
#undef CPALS_QR
}

template <typename T, int NCB>
hipError_t launch_ttm_sq(const T* X, const T* B, T* C, int64_t P, int64_t K, int64_t Q, int R, hipStream_t st) {
  constexpr int KT = 4 * (16 / sizeof(T));
  const int64_t rows = P * Q;
  const int64_t ntiles = (rows + 15) / 16;
  const int64_t want = (ntiles + kTtmWaves - 1) / kTtmWaves;
  const unsigned nx = (unsigned)(want < 256 ? want : 256);
  const unsigned ny = (unsigned)((R + NCB * 16 - 1) / (NCB * 16));
  if (K <= 2 * KT)
    hipLaunchKernelGGL((k_ttm_sq<T, NCB, 2>), dim3(nx, ny), dim3(kTtmThreads), 0, st, X, B, C, rows, K, Q, R, ntiles);
  else if (K <= 4 * KT)
    hipLaunchKernelGGL((k_ttm_sq<T, NCB, 4>), dim3(nx, ny), dim3(kTtmThreads), 0, st, X, B, C, rows, K, Q, R, ntiles);
  else
    hipLaunchKernelGGL((k_ttm_sq<T, NCB, 8>), dim3(nx, ny), dim3(kTtmThreads), 0, st, X, B, C, rows, K, Q, R, ntiles);
  return hipGetLastError();
}

template <typename T, int NCB>
hipError_t launch_ttm_kcx(const T* X, const T* B, T* C, int64_t P, int64_t K, int R, hipStream_t st) {
  constexpr int V = 16 / sizeof(T);
  const int64_t ntiles = (P + 15) / 16;
  const int64_t want = (ntiles + kTtmWaves - 1) / kTtmWaves;
  const unsigned nx = (unsigned)(want < 256 ? want : 256);
  const unsigned ny = (unsigned)((R + NCB * 16 - 1) / (NCB * 16));
  const int vec = (K % V == 0 && ((uintptr_t)X % 16) == 0) ? 1 : 0;
  const int nch = (int)((K + 4 * V * 8 - 1) / (4 * V * 8));
  hipLaunchKernelGGL((k_ttm_kcx<T, NCB>), dim3(nx, ny), dim3(kTtmThreads), 0, st, X, B, C, P, K, R, ntiles, vec,
                     nch);
  return hipGetLastError();
}

// The same contraction with K split over Z workgroup layers (partials in
// `parts`, Z P R elements) and a fixed-order sum into C.
template <typename T, int NCB>
hipError_t launch_ttm_kcx_split(const T* X, const T* B, T* C, int64_t P, int64_t K, int R, T* parts, int Z,
                                hipStream_t st) {
  constexpr int V = 16 / sizeof(T);
  const int64_t ntiles = (P + 15) / 16;
  const int64_t want = (ntiles + kTtmWaves - 1) / kTtmWaves;
  const unsigned nx = (unsigned)(want < 256 ? want : 256);
  const unsigned ny = (unsigned)((R + NCB * 16 - 1) / (NCB * 16));
  const int vec = (K % V == 0 && ((uintptr_t)X % 16) == 0) ? 1 : 0;
  const int nch = (int)((K + 4 * V * 8 - 1) / (4 * V * 8));
  const int cps = (nch + Z - 1) / Z;
  const int z = (nch + cps - 1) / cps;  // layers that have chunks
  hipLaunchKernelGGL((k_ttm_kcx<T, NCB>), dim3(nx, ny, (unsigned)z), dim3(kTtmThreads), 0, st, X, B, parts, P, K,
                     R, ntiles, vec, cps);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t n = P * R;
  const int64_t nb = (n / V + 255) / 256;
  hipLaunchKernelGGL((k_sum_parts<T>), dim3((unsigned)(nb < 2048 ? nb : 2048)), dim3(256), 0, st, parts, C, n, z);
  return hipGetLastError();
}

template <int NCB>
hipError_t launch_ttm_kcx32(const float* X, const float* B, float* C, int64_t P, int64_t K, int R, hipStream_t st) {
  const int64_t ntiles = (P + 31) / 32;
  const int64_t want = (ntiles + kTtmWaves - 1) / kTtmWaves;
  const unsigned nx = (unsigned)(want < 256 ? want : 256);
  const unsigned ny = (unsigned)((R + NCB * 32 - 1) / (NCB * 32));
  if (K % 4 == 0 && ((uintptr_t)X % 16) == 0)
    hipLaunchKernelGGL((k_ttm_kcx32<NCB, true>), dim3(nx, ny), dim3(kTtmThreads), 0, st, X, B, C, P, K, R, ntiles);
  else
    hipLaunchKernelGGL((k_ttm_kcx32<NCB, false>), dim3(nx, ny), dim3(kTtmThreads), 0, st, X, B, C, P, K, R, ntiles);
  return hipGetLastError();
}

// whole 64-q tiles and 32-index pieces, 16-byte aligned rows, 32-bit lane offsets
inline bool qx_whole(int vec, int64_t K, int64_t Q) {
  return vec && Q % 64 == 0 && K % 32 == 0 && Q < ((int64_t)1 << 28);
}

template <int NCB>
hipError_t launch_ttm_qx(const float* X, const float* B, float* C, int64_t P, int64_t K, int64_t Q, int R,
                         hipStream_t st) {
  const int64_t tilesQ = (Q + 63) / 64;
  const int64_t ntiles = P * tilesQ;
  const int64_t want = (ntiles + kTtmWaves - 1) / kTtmWaves;
  const unsigned nx = (unsigned)(want < 256 ? want : 256);
  const unsigned ny = (unsigned)((R + NCB * 16 - 1) / (NCB * 16));
  const int vec = (Q % 4 == 0 && ((uintptr_t)X % 16) == 0) ? 1 : 0;
  const int nch = (int)((K + 127) / 128);
  if (qx_whole(vec, K, Q))
    hipLaunchKernelGGL((k_ttm_qx<NCB, true>), dim3(nx, ny), dim3(kTtmThreads), 0, st, X, B, C, P, K, Q, R, tilesQ,
                       ntiles, vec, nch);
  else
    hipLaunchKernelGGL((k_ttm_qx<NCB, false>), dim3(nx, ny), dim3(kTtmThreads), 0, st, X, B, C, P, K, Q, R, tilesQ,
                       ntiles, vec, nch);
  return hipGetLastError();
}

// The same contraction with K split over Z workgroup layers (partials in
// `parts`, Z P Q R elements) and a fixed-order sum into C.
template <int NCB>
hipError_t launch_ttm_qx_split(const float* X, const float* B, float* C, int64_t P, int64_t K, int64_t Q, int R,
                               float* parts, int Z, hipStream_t st) {
  const int64_t tilesQ = (Q + 63) / 64;
  const int64_t ntiles = P * tilesQ;
  const int64_t want = (ntiles + kTtmWaves - 1) / kTtmWaves;
  const unsigned nx = (unsigned)(want < 256 ? want : 256);
  const unsigned ny = (unsigned)((R + NCB * 16 - 1) / (NCB * 16));
  const int vec = (Q % 4 == 0 && ((uintptr_t)X % 16) == 0) ? 1 : 0;
  const int nch = (int)((K + 127) / 128);
  const int cps = (nch + Z - 1) / Z;
  const int z = (nch + cps - 1) / cps;
  if (qx_whole(vec, K, Q))
    hipLaunchKernelGGL((k_ttm_qx<NCB, true>), dim3(nx, ny, (unsigned)z), dim3(kTtmThreads), 0, st, X, B, parts, P, K,
                       Q, R, tilesQ, ntiles, vec, cps);
  else
    hipLaunchKernelGGL((k_ttm_qx<NCB, false>), dim3(nx, ny, (unsigned)z), dim3(kTtmThreads), 0, st, X, B, parts, P,
                       K, Q, R, tilesQ, ntiles, vec, cps);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t n = P * Q * R;
  const int64_t nb = (n / 4 + 255) / 256;
  hipLaunchKernelGGL((k_sum_parts<float>), dim3((unsigned)(nb < 2048 ? nb : 2048)), dim3(256), 0, st, parts, C, n, z);
  return hipGetLastError();
}

template <int NCB>
hipError_t launch_ttm_q(const float* X, const float* B, float* C, int64_t P, int64_t K, int64_t Q, int R,
                        hipStream_t st) {
  const int Kp = (int)((K + 31) / 32 * 32);
  const size_t lds = (size_t)NCB * 16 * (Kp + 4) * sizeof(float);
  static std::atomic<uint64_t> attr_g{0}, attr_f{0};
  {
    hipError_t e = lds_limit_once(attr_g, (const void*)k_ttm_q<NCB, false>, 160 * 1024);
    if (e == hipSuccess) e = lds_limit_once(attr_f, (const void*)k_ttm_q<NCB, true>, 160 * 1024);
    if (e != hipSuccess) return e;
  }
  const int64_t tilesQ = (Q + 63) / 64;
  const int64_t ntiles = P * tilesQ;
  const int64_t want = (ntiles + kTtmWaves - 1) / kTtmWaves;
  const unsigned nx = (unsigned)(want < 512 ? want : 512);
  const unsigned ny = (unsigned)((R + NCB * 16 - 1) / (NCB * 16));
  const int vec = (Q % 4 == 0 && ((uintptr_t)X % 16) == 0) ? 1 : 0;
  if (vec && Q % 64 == 0 && K % 32 == 0 && Q < ((int64_t)1 << 28))
    hipLaunchKernelGGL((k_ttm_q<NCB, true>), dim3(nx, ny), dim3(kTtmThreads), lds, st, X, B, C, P, K, Q, R, tilesQ,
                       ntiles, Kp, vec);
  else
    hipLaunchKernelGGL((k_ttm_q<NCB, false>), dim3(nx, ny), dim3(kTtmThreads), lds, st, X, B, C, P, K, Q, R, tilesQ,
                       ntiles, Kp, vec);
  return hipGetLastError();
}

template <typename T, bool KC>
hipError_t launch_ttm_rb_ncb(const T* X, const T* B, T* C, int64_t P, int64_t K, int64_t Q, int R,
                             hipStream_t st) {
  if (R <= 16) return launch_ttm_rb<T, KC, 1>(X, B, C, P, K, Q, R, st);
  if (R <= 32) return launch_ttm_rb<T, KC, 2>(X, B, C, P, K, Q, R, st);
  // eight column blocks of an FP64 factor with K > 128 exceed the LDS: two
  // passes of four instead
  if (R <= 64 || (sizeof(T) == 8 && K > 128)) return launch_ttm_rb<T, KC, 4>(X, B, C, P, K, Q, R, st);
  return launch_ttm_rb<T, KC, 8>(X, B, C, P, K, Q, R, st);
}

template <typename T>
hipError_t launch_ttm(const T* X, const T* B, T* C, int64_t P, int64_t K, int64_t Q, int R,
                      hipStream_t st) {
  if (sizeof(T) == 4 && Q == 1 && K == 128 && R > 16 && R <= 64 && ((uintptr_t)X % 16) == 0) {
    const float* Xf = (const float*)X;
    const float* Bf = (const float*)B;
    float* Cf = (float*)C;
    if (R <= 32) return launch_ttm_kc32<1>(Xf, Bf, Cf, P, R, st);
    return launch_ttm_kc32<2>(Xf, Bf, Cf, P, R, st);
  }
  if (Q == 1 && K <= 32 * (int64_t)(16 / sizeof(T)) && R <= 64) {
    if (R <= 16) return launch_ttm_kc<T, 1>(X, B, C, P, K, R, st);
    if (R <= 32) return launch_ttm_kc<T, 2>(X, B, C, P, K, R, st);
    return launch_ttm_kc<T, 4>(X, B, C, P, K, R, st);
  }
  if (Q > 1 && Q < 64 && K <= 32 * (int64_t)(16 / sizeof(T)) && R <= 64) {
    // a short run of q after the contracted mode: rows (p, q) tiled without waste
    if (R <= 16) return launch_ttm_sq<T, 1>(X, B, C, P, K, Q, R, st);
    if (R <= 32) return launch_ttm_sq<T, 2>(X, B, C, P, K, Q, R, st);
    return launch_ttm_sq<T, 4>(X, B, C, P, K, Q, R, st);
  }
  if (sizeof(T) == 4 && Q == 1 && K > 128 && R > 16 && R <= 64 && P >= 131072) {
    // FP32, chunked factor on the 32x32x2 instruction, when there are rows enough for 32-row
    // tiles to keep every wave busy (with fewer, the 16-row tiles of k_ttm_kcx are faster;
    // R > 64 spills here)
    const float* Xf = (const float*)X;
    const float* Bf = (const float*)B;
    float* Cf = (float*)C;
    if (R <= 32) return launch_ttm_kcx32<1>(Xf, Bf, Cf, P, K, R, st);
    return launch_ttm_kcx32<2>(Xf, Bf, Cf, P, K, R, st);
  }
  if (Q == 1 && K > 32 * (int64_t)(16 / sizeof(T))) {
    // chunked factor, any K (f32: chunks of 128, f64: 64)
    if (R <= 16) return launch_ttm_kcx<T, 1>(X, B, C, P, K, R, st);
    if (R <= 32) return launch_ttm_kcx<T, 2>(X, B, C, P, K, R, st);
    if (R <= 64) return launch_ttm_kcx<T, 4>(X, B, C, P, K, R, st);
    return launch_ttm_kcx<T, 8>(X, B, C, P, K, R, st);
  }
  if (sizeof(T) == 4 && Q >= 64 && K > 256) {
    // FP32, a mode other than the last, factor too long for LDS: chunked
    const float* Xf = (const float*)X;
    const float* Bf = (const float*)B;
    float* Cf = (float*)C;
    if (R <= 16) return launch_ttm_qx<1>(Xf, Bf, Cf, P, K, Q, R, st);
    if (R <= 32) return launch_ttm_qx<2>(Xf, Bf, Cf, P, K, Q, R, st);
    if (R <= 64) return launch_ttm_qx<4>(Xf, Bf, Cf, P, K, Q, R, st);
    return launch_ttm_qx<8>(Xf, Bf, Cf, P, K, Q, R, st);
  }
  if (K <= 256) {
    if (Q == 1) return launch_ttm_rb_ncb<T, true>(X, B, C, P, K, Q, R, st);
    if (sizeof(T) == 4 && Q >= 64) {
      const float* Xf = (const float*)X;
      const float* Bf = (const float*)B;
      float* Cf = (float*)C;
      if (R <= 16) return launch_ttm_q<1>(Xf, Bf, Cf, P, K, Q, R, st);
      if (R <= 32) return launch_ttm_q<2>(Xf, Bf, Cf, P, K, Q, R, st);
      if (R <= 64) return launch_ttm_q<4>(Xf, Bf, Cf, P, K, Q, R, st);
      return launch_ttm_q<8>(Xf, Bf, Cf, P, K, Q, R, st);
    }
    return launch_ttm_rb_ncb<T, false>(X, B, C, P, K, Q, R, st);
  }
  const unsigned ny = (unsigned)((R + TBN - 1) / TBN);
  if (Q == 1) {
    const int64_t nx = (P + TBM - 1) / TBM;
    hipLaunchKernelGGL((k_ttm<T, true>), dim3((unsigned)nx, ny), dim3(256), 0, st, X, B, C, P, K,
                       Q, R, (int64_t)1);
  } else {
    const int64_t tq = (Q + TBM - 1) / TBM;
    hipLaunchKernelGGL((k_ttm<T, false>), dim3((unsigned)(P * tq), ny), dim3(256), 0, st, X, B, C,
                       P, K, Q, R, tq);
  }
  return hipGetLastError();
}

int ttm_split_layers(int64_t P, int64_t K, int64_t Q, int R, int esz) {
  const int V = 16 / esz;
  if (R > 128) return 1;
  const int ncb = R <= 16 ? 1 : R <= 32 ? 2 : R <= 64 ? 4 : 8;
  const int64_t ny = (R + ncb * 16 - 1) / (ncb * 16);
  int64_t ntiles, nch;
  if (Q == 1) {  // k_ttm_kcx: 16-row tiles, chunks of 32 V indices
    if (K <= 32 * (int64_t)V || (P * R) % V != 0) return 1;
    if (esz == 4 && P >= 131072 && R > 16 && R <= 64) return 1;  // k_ttm_kcx32 fills the chip by itself
    ntiles = (P + 15) / 16;
    nch = (K + 32 * V - 1) / (32 * V);
  } else {  // k_ttm_qx (FP32): 64-q tiles, chunks of 128 indices
    if (esz != 4 || Q < 64 || K <= 256 || (P * Q * R) % 4 != 0) return 1;
    ntiles = P * ((Q + 63) / 64);
    nch = (K + 127) / 128;
  }
  const int64_t nx = std::min<int64_t>((ntiles + kTtmWaves - 1) / kTtmWaves, 256);
  int64_t z = (512 + nx * ny - 1) / (nx * ny);  // two workgroups per compute unit
  z = std::min<int64_t>(z, nch / 4);           // at least four chunks per layer
  z = std::min<int64_t>(z, kMaxSplitLayers);
  return (int)std::max<int64_t>(z, 1);
}

template <typename T>
hipError_t launch_ttm_split(const T* X, const T* B, T* C, int64_t P, int64_t K, int64_t Q, int R, T* parts, int Z,
                            hipStream_t st) {
  if (Z <= 1 || !parts) return launch_ttm<T>(X, B, C, P, K, Q, R, st);
  if (Q == 1) {
    if (R <= 16) return launch_ttm_kcx_split<T, 1>(X, B, C, P, K, R, parts, Z, st);
    if (R <= 32) return launch_ttm_kcx_split<T, 2>(X, B, C, P, K, R, parts, Z, st);
    if (R <= 64) return launch_ttm_kcx_split<T, 4>(X, B, C, P, K, R, parts, Z, st);
    return launch_ttm_kcx_split<T, 8>(X, B, C, P, K, R, parts, Z, st);
  }
  if constexpr (sizeof(T) == 4) {
    const float* Xf = (const float*)X;
    const float* Bf = (const float*)B;
    float* Cf = (float*)C;
    float* Pf = (float*)parts;
    if (R <= 16) return launch_ttm_qx_split<1>(Xf, Bf, Cf, P, K, Q, R, Pf, Z, st);
    if (R <= 32) return launch_ttm_qx_split<2>(Xf, Bf, Cf, P, K, Q, R, Pf, Z, st);
    if (R <= 64) return launch_ttm_qx_split<4>(Xf, Bf, Cf, P, K, Q, R, Pf, Z, st);
    return launch_ttm_qx_split<8>(Xf, Bf, Cf, P, K, Q, R, Pf, Z, st);
  }
  return hipErrorInvalidValue;
}

template <typename TI, typename TO>
hipError_t launch_mttv(const TI* X, const TI* A, TO* Y, int64_t P, int64_t I, int64_t Q, int R,
                       hipStream_t st) {
  const int64_t total = P * Q * R;
  if (total <= (int64_t)1 << 17) {
    const int64_t jb = (Q * R + 63) / 64;
    hipLaunchKernelGGL((k_mttv_split<TI, TO>), dim3((unsigned)(P * jb)), dim3(256), 0, st, X, A, Y, I,
                       Q * R, R, jb);
    return hipGetLastError();
  }
  if (sizeof(TI) == 4 && R % 4 == 0 && ((uintptr_t)X % 16) == 0 && ((uintptr_t)A % 16) == 0) {
    hipLaunchKernelGGL((k_mttv4<TO>), dim3(nblocks(total / 4)), dim3(256), 0, st, (const float*)X,
                       (const float*)A, Y, total / 4, I, Q * R, R);
    return hipGetLastError();
  }
  hipLaunchKernelGGL((k_mttv<TI, TO>), dim3(nblocks(total)), dim3(256), 0, st, X, A, Y, total, I,
                     Q * R, R);
  return hipGetLastError();
}

bool mttv_pair_fits(int64_t sz, int64_t sv, int R) {
  if (R % 4 != 0 || R < 16 || R > 64 || sz < 1) return false;
  const int rq = R / 4;
  return rq == 4 || rq == 8 || rq == 16 ? sv <= 8 * (256 / rq) : false;
}

int mttv_pair_split(int64_t sz, int64_t su) {
  // about two workgroups per compute unit, at least 8 u-indices per range
  int y = (int)std::min<int64_t>((512 + sz - 1) / sz, kMaxPairSplit);
  while (y > 1 && su / y < 8) --y;
  return y < 1 ? 1 : y;
}

hipError_t launch_mttv_pair(const float* X, const float* Au, const float* Av, float* Ycv, float* Ycu, int64_t sz,
                            int64_t su, int64_t sv, int64_t Sz, int64_t Su, int64_t Sv, int64_t ozv, int64_t ouv,
                            int64_t ozu, int64_t ovu, int R, float* parts, hipStream_t st) {
  if (!mttv_pair_fits(sz, sv, R) || su < 1 || ((uintptr_t)X % 16) || ((uintptr_t)Ycv % 16) || ((uintptr_t)Ycu % 16))
    return hipErrorInvalidValue;
  const int y = parts ? mttv_pair_split(sz, su) : 1;
  const int64_t uc = (su + y - 1) / y;
  const int64_t n = sz * sv * R;  // Ycu's elements
  float* dst = y > 1 ? parts : Ycu;
  const int64_t pstride = y > 1 ? n : 0;
  const dim3 grid((unsigned)sz, (unsigned)((su + uc - 1) / uc));
  if (R == 16)
    hipLaunchKernelGGL(k_mttv_pair<4>, grid, dim3(256), 0, st, X, Au, Av, Ycv, dst, su, sv, Sz, Su, Sv, ozv, ouv,
                       ozu, ovu, uc, pstride);
  else if (R == 32)
    hipLaunchKernelGGL(k_mttv_pair<8>, grid, dim3(256), 0, st, X, Au, Av, Ycv, dst, su, sv, Sz, Su, Sv, ozv, ouv,
                       ozu, ovu, uc, pstride);
  else
    hipLaunchKernelGGL(k_mttv_pair<16>, grid, dim3(256), 0, st, X, Au, Av, Ycv, dst, su, sv, Sz, Su, Sv, ozv, ouv,
                       ozu, ovu, uc, pstride);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || grid.y == 1) return e;
  const int64_t nb = (n / 4 + 255) / 256;
  hipLaunchKernelGGL((k_sum_parts<float>), dim3((unsigned)(nb < 2048 ? nb : 2048)), dim3(256), 0, st, parts, Ycu, n,
                     (int)grid.y);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_krp2(const T* Aa, int64_t sa, const T* Ab, int64_t sb, int R, T* B, hipStream_t st) {
  const int64_t n = sa * sb * R;
  if (n <= 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_krp2<T>), dim3(nblocks(n)), dim3(256), 0, st, Aa, Ab, sb, R, n, B);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_convert(const double* src, T* dst, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL((k_convert<T>), dim3(nblocks(n)), dim3(256), 0, st, src, dst, n);
  return hipGetLastError();
}

hipError_t launch_copy_f64(const double* src, double* dst, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_copy_f64, dim3(nblocks(n)), dim3(256), 0, st, src, dst, n);
  return hipGetLastError();
}

hipError_t launch_zero_f64(double* p, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_f64, dim3(nblocks(n)), dim3(256), 0, st, p, n);
  return hipGetLastError();
}

hipError_t launch_fitness(const double* M, const double* A, int64_t s, int R, const double* Gamma,
                          const double* S, DevStats* stats, hipStream_t st) {
  hipLaunchKernelGGL(k_fitness, dim3(1), dim3(256), 0, st, M, A, s * R, Gamma, S, R * R, stats);
  return hipGetLastError();
}

hipError_t launch_setup(const SetupBatch& b, hipStream_t st) {
  if (b.nops < 1) return hipSuccess;
  if (b.nops > kMaxSetupOps) return hipErrorInvalidValue;
  SetupArgs a;
  int blocks = 0;
  for (int i = 0; i < b.nops; ++i) {
    a.op[i] = b.op[i];
    a.first[i] = blocks;
    const SetupOp& o = b.op[i];
    const int64_t nb = (o.kind == kSetupGram) ? ((int64_t)o.R * o.R + 63) / 64 : (o.n + 255) / 256;
    blocks += (int)(nb > 0 ? nb : 1);  // an empty operation keeps one (idle) workgroup
  }
  a.first[b.nops] = blocks;
  a.nops = b.nops;
  hipLaunchKernelGGL(k_setup, dim3((unsigned)blocks), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_zero_bytes(void* p, size_t bytes, hipStream_t st) {
  const int64_t n = (int64_t)(bytes / 4);
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_u32, dim3(nblocks(n)), dim3(256), 0, st, (uint32_t*)p, n);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_norm2(const T* X, int64_t n, double* partials, int nparts, DevStats* stats,
                        hipStream_t st) {
  hipLaunchKernelGGL((k_norm2_part<T>), dim3(nparts), dim3(256), 0, st, X, n, partials);
  hipLaunchKernelGGL(k_norm2_final, dim3(1), dim3(256), 0, st, partials, nparts, stats);
  return hipGetLastError();
}

hipError_t launch_gram(const double* A, int64_t s, int R, double* S, hipStream_t st) {
  hipLaunchKernelGGL(k_gram, dim3((unsigned)(((int64_t)R * R + 63) / 64)), dim3(256), 0, st, A, s, R, S);
  return hipGetLastError();
}

hipError_t launch_gamma(const GammaArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(k_gamma, dim3(nblocks((int64_t)a.R * a.R)), dim3(256), 0, st, a);
  return hipGetLastError();
}

template <int RP>
hipError_t launch_inv_rp(const double* Gamma, double* Ginv, int R, DevStats* stats, hipStream_t st) {
  static std::atomic<uint64_t> attr{0};
  {
    hipError_t e = lds_limit_once(attr, (const void*)k_inv_blk<RP>, 150 * 1024);
    if (e != hipSuccess) return e;
  }
  const size_t lds = gamma_inverse_lds_doubles(RP, R) * sizeof(double);
  hipLaunchKernelGGL(k_inv_blk<RP>, dim3(1), dim3(256), lds, st, Gamma, Ginv, R, stats);
  return hipGetLastError();
}

hipError_t launch_inverse(const double* Gamma, double* Ginv, int R, DevStats* stats, hipStream_t st) {
  if (R <= 16) return launch_inv_rp<16>(Gamma, Ginv, R, stats, st);
  if (R <= 32) return launch_inv_rp<32>(Gamma, Ginv, R, stats, st);
  if (R <= 64) return launch_inv_rp<64>(Gamma, Ginv, R, stats, st);
  return launch_inv_rp<128>(Gamma, Ginv, R, stats, st);
}

// The reductions of a mode update when the partials are too many for one
// workgroup (the split path of k_update): workgroup w takes the 32 entries
// 32 w .. 32 w + 31 of the R x R matrices; thread (l, i), l = tid / 32, sums
// the partials l, l + 8, l + 16, ... of entry i and the eight sums are added
// in l order.  Each entry then gets S^(n), dS^(n), Gamma^(nx) and (PP)
// W^(nx) as in k_update; the workgroup's share of <Gamma^(n), S^(n)> goes to
// partG, and the last workgroup to finish (ticket) adds the shares and the
// norm partials in order and forms the residual of Eq. (3).
template <typename T, bool PP>
__global__ __launch_bounds__(256) void k_update_reduce(UpdateArgs<T> a, int G) {
  __shared__ double ls[8][33], ld[8][33];
  __shared__ double sh[256];
  __shared__ int flag;
  const int tid = threadIdx.x, es = tid & 31, bl = tid >> 5;
  const int R = a.R, RR = R * R, n = a.n, N = a.N, nx = (n + 1) % N;
  const int e = blockIdx.x * 32 + es;
  const int ei = e < RR ? e : 0;
  double sv = 0.0, dv = 0.0;
  for (int b0 = bl; b0 < G; b0 += 64) {
    double pv[8], pd[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int b = b0 + 8 * k < G ? b0 + 8 * k : b0;
      pv[k] = a.partS[(int64_t)b * RR + ei];
      pd[k] = PP ? a.partdS[(int64_t)b * RR + ei] : 0.0;
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const bool in = b0 + 8 * k < G;
      sv += in ? pv[k] : 0.0;
      if (PP) dv += in ? pd[k] : 0.0;
    }
  }
  ls[bl][es] = sv;
  ld[bl][es] = dv;
  __syncthreads();
  double gpart = 0.0;
  if (bl == 0 && e < RR) {
    double st = ls[0][es], dt = ld[0][es];
#pragma unroll
    for (int q = 1; q < 8; ++q) {
      st += ls[q][es];
      dt += ld[q][es];
    }
    a.S[n][e] = st;
    if (PP) a.dS[n][e] = dt;
    gpart = a.Gamma[e] * st;
    double v = 1.0, f0 = 1.0, f1 = 0.0, f2 = 0.0;
#pragma unroll
    for (int m = 0; m < kMaxOrder; ++m) {
      if (m >= N || m == nx) continue;
      const double smv = (m == n) ? st : a.S[m][e];
      const double dmv = PP ? ((m == n) ? dt : a.dS[m][e]) : 0.0;
      v *= smv;
      if (PP) {
        f2 = f2 * smv + f1 * dmv;
        f1 = f1 * smv + f0 * dmv;
        f0 = f0 * smv;
      }
    }
    a.Gamma[e] = v;
    if (PP) a.W[e] = f2;
  }
  {
    double v1[1] = {gpart};
    block_sums<1>(v1, sh);
    if (tid == 0) a.partG[blockIdx.x] = v1[0];
  }
  __threadfence();
  __syncthreads();
  if (tid == 0) flag = (atomicAdd(a.ticket, 1u) == gridDim.x - 1) ? 1 : 0;
  __syncthreads();
  if (!flag) return;  // uniform
  __threadfence();
  if (tid == 0) atomicExch(a.ticket, 0u);
  double v4[4] = {0.0, 0.0, 0.0, 0.0};
  for (int b = tid; b < G; b += 256) {
    v4[0] += a.partSc[b * 4 + 0];
    v4[1] += a.partSc[b * 4 + 1];
    v4[2] += a.partSc[b * 4 + 2];
  }
  for (int b = tid; b < (int)gridDim.x; b += 256) v4[3] += a.partG[b];
  block_sums<4>(v4, sh);
  if (tid == 0) {
    a.stats->normA2[n] = v4[0];
    a.stats->normdA2[n] = v4[1];
    if (a.last) {
      const double tn = a.stats->normT2;
      const double num = tn + v4[3] - 2.0 * v4[2];
      a.stats->fit_num = num;
      const double r = sqrt((num > 0.0 ? num : 0.0) / tn);
      a.stats->r = r;
      a.stats->r_clamped = (num < 0.0) ? 1 : 0;
      if (!isfinite(r)) a.stats->status |= 2;
    }
  }
}

template <typename T, int RP, bool PP>
hipError_t launch_update_rp(const UpdateArgs<T>& a, int groups, hipStream_t st) {
  static std::atomic<uint64_t> attr{0};
  {
    hipError_t e = lds_limit_once(attr, (const void*)k_update<T, RP, PP>, 150 * 1024);
    if (e != hipSuccess) return e;
  }
  size_t dbl = update_solve_lds_doubles(RP);
  if (a.inv_next && a.fused) dbl = std::max(dbl, gamma_inverse_lds_doubles(RP, a.R));
  hipLaunchKernelGGL((k_update<T, RP, PP>), dim3(groups), dim3(256), dbl * sizeof(double), st, a);
  return hipGetLastError();
}

template <typename T, bool PP>
hipError_t launch_update_pp(const UpdateArgs<T>& a, int groups, hipStream_t st) {
  if (a.R <= 16) return launch_update_rp<T, 16, PP>(a, groups, st);
  if (a.R <= 32) return launch_update_rp<T, 32, PP>(a, groups, st);
  if (a.R <= 64) return launch_update_rp<T, 64, PP>(a, groups, st);
  return launch_update_rp<T, 128, PP>(a, groups, st);
}

// Fused (the last workgroup reduces) while the partials are few and small:
// at most 16 row blocks and about 1 MiB of partials; otherwise up to 64
// workgroups, several row blocks each, and k_update_reduce.
void update_shape(int64_t s, int R, bool pp, int* groups, bool* fused) {
  const int64_t nrb = std::max<int64_t>(1, (s + 15) / 16);
  const int64_t bytes = nrb * (int64_t)R * R * 8 * (pp ? 2 : 1);
  *fused = nrb <= 16 && bytes <= (1 << 20);
  *groups = (int)std::min<int64_t>(nrb, 64);
}

int update_groups_max(int64_t smax, int R) {
  (void)R;
  return (int)std::max<int64_t>(1, std::min<int64_t>((smax + 15) / 16, 64));
}

template <typename T>
hipError_t launch_update(const UpdateArgs<T>& a, int groups, hipStream_t st) {
  if (a.R < 1 || a.R > kMaxRank || groups < 1) return hipErrorInvalidValue;
  hipError_t e = a.pp ? launch_update_pp<T, true>(a, groups, st) : launch_update_pp<T, false>(a, groups, st);
  if (e != hipSuccess || a.fused) return e;
  const unsigned nb = (unsigned)((a.R * a.R + 31) / 32);
  if (a.pp) {
    hipLaunchKernelGGL((k_update_reduce<T, true>), dim3(nb), dim3(256), 0, st, a, groups);
  } else {
    hipLaunchKernelGGL((k_update_reduce<T, false>), dim3(nb), dim3(256), 0, st, a, groups);
  }
  e = hipGetLastError();
  if (e != hipSuccess || !a.inv_next) return e;
  return launch_inverse(a.Gamma, a.Ginv, a.R, a.stats, st);
}

template <typename T, int RP>
hipError_t launch_pp_mttkrp_rp(const PPArgs<T>& a, hipStream_t st) {
  static std::atomic<uint64_t> attr{0};
  {
    hipError_t e = lds_limit_once(attr, (const void*)k_pp_mttkrp<T, RP>, 150 * 1024);
    if (e != hipSuccess) return e;
  }
  const size_t lds = a.Ginv ? gamma_inverse_lds_doubles(RP, a.R) * sizeof(double) : 0;
  const unsigned grid = (unsigned)a.dims[a.n] + (a.Ginv ? 1u : 0u);
  hipLaunchKernelGGL((k_pp_mttkrp<T, RP>), dim3(grid), dim3(256), lds, st, a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_pp_mttkrp(const PPArgs<T>& a, hipStream_t st) {
  if (a.R < 1 || a.R > kMaxRank) return hipErrorInvalidValue;
  if (a.R <= 16) return launch_pp_mttkrp_rp<T, 16>(a, st);
  if (a.R <= 32) return launch_pp_mttkrp_rp<T, 32>(a, st);
  if (a.R <= 64) return launch_pp_mttkrp_rp<T, 64>(a, st);
  return launch_pp_mttkrp_rp<T, 128>(a, st);
}

// explicit instantiations
template hipError_t launch_ttm<float>(const float*, const float*, float*, int64_t, int64_t,
                                      int64_t, int, hipStream_t);
template hipError_t launch_ttm<double>(const double*, const double*, double*, int64_t, int64_t,
                                       int64_t, int, hipStream_t);
template hipError_t launch_ttm_split<float>(const float*, const float*, float*, int64_t, int64_t, int64_t, int,
                                            float*, int, hipStream_t);
template hipError_t launch_ttm_split<double>(const double*, const double*, double*, int64_t, int64_t, int64_t, int,
                                             double*, int, hipStream_t);
template hipError_t launch_mttv<float, float>(const float*, const float*, float*, int64_t, int64_t,
                                              int64_t, int, hipStream_t);
template hipError_t launch_mttv<float, double>(const float*, const float*, double*, int64_t,
                                               int64_t, int64_t, int, hipStream_t);
template hipError_t launch_mttv<double, double>(const double*, const double*, double*, int64_t,
                                                int64_t, int64_t, int, hipStream_t);
template hipError_t launch_krp2<float>(const float*, int64_t, const float*, int64_t, int, float*, hipStream_t);
template hipError_t launch_krp2<double>(const double*, int64_t, const double*, int64_t, int, double*, hipStream_t);
template hipError_t launch_convert<float>(const double*, float*, int64_t, hipStream_t);
template hipError_t launch_convert<double>(const double*, double*, int64_t, hipStream_t);
template hipError_t launch_norm2<float>(const float*, int64_t, double*, int, DevStats*, hipStream_t);
template hipError_t launch_norm2<bf16>(const bf16*, int64_t, double*, int, DevStats*, hipStream_t);
template hipError_t launch_norm2<fp8e4m3>(const fp8e4m3*, int64_t, double*, int, DevStats*, hipStream_t);
template hipError_t launch_norm2<double>(const double*, int64_t, double*, int, DevStats*,
                                         hipStream_t);
template hipError_t launch_update<float>(const UpdateArgs<float>&, int, hipStream_t);
template hipError_t launch_update<double>(const UpdateArgs<double>&, int, hipStream_t);
template hipError_t launch_pp_mttkrp<float>(const PPArgs<float>&, hipStream_t);
template hipError_t launch_pp_mttkrp<double>(const PPArgs<double>&, hipStream_t);

}  // namespace cpals
