// gfx950 kernels of the CP-ALS hot path.
//
//  k_ttm        first-level contraction of the tensor with one factor (a
//               dense GEMM / batched GEMM) on the matrix cores (MFMA f32 or
//               f64 16x16x4), tiles staged through LDS.      Sec. II-C, Sec. III
//  k_mttv       batched tensor-times-vector down the tree, HBM streaming,
//               lanes over the contiguous (q, r) block.       Sec. II-C
//  k_prep       Gamma^(n) (Eq. (1)), its inverse, and the bracket of Eq. (7)
//  k_solve      A^(n) <- M Gamma^-1 (plus V^(n) in PP), partial Gram, dS, norms
//  k_finalize   fixed-order reduction of the partials, residual by Eq. (3)
//  k_pp_mttkrp  first-order PP correction, Eqs. (5)-(6)
//
// Every floating-point reduction runs in a fixed order (no atomics), so two
// runs give bitwise-identical results.
#include <math.h>

#include "kernels.h"

namespace cpals {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
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
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
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
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
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
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
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
  VT a[NTS];
  if (tile < ntiles) load_tile(tile, a);
  for (; tile < ntiles; tile += stride) {
    asm volatile("" ::: "memory");  // factor reads stay in the loop
    // the next tile's rows are in flight while this one is multiplied
    VT an[NTS];
    if (tile + stride < ntiles) {
      load_tile(tile + stride, an);
    } else {
#pragma unroll
      for (int s = 0; s < NTS; ++s) an[s] = VT{};
    }
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
#pragma unroll
    for (int s = 0; s < NTS; ++s) a[s] = an[s];
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
// current one is multiplied.
template <int NCB, bool FULL>
__global__ __launch_bounds__(512) void k_ttm_q(const float* __restrict__ X, const float* __restrict__ B,
                                               float* __restrict__ C, int64_t P, int64_t K, int64_t Q,
                                               int R, int64_t tilesQ, int64_t ntiles, int Kp, int vec) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  float* Bt = (float*)lds_raw;
  const int pitch = Kp + 4;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
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
  // prefetching needs 32 more registers: kept for up to 64 factor columns per wave
  constexpr bool PF = NCB <= 4;
  const int64_t stride = (int64_t)gridDim.x * kTtmWaves;
  int64_t tile = (int64_t)blockIdx.x * kTtmWaves + wave;
  f32x4 a[8];
  if (PF && tile < ntiles) load_chunk(tile, 0, a);
  for (; tile < ntiles; tile += stride) {
    asm volatile("" ::: "memory");  // factor reads stay in the loop (see k_ttm_rb)
    const int64_t p = tile / tilesQ;
    const int64_t q0 = (tile - p * tilesQ) * 64;
    float* Cb = C + p * Q * R;
    f32x4 acc[4][NCB];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) acc[u][cb] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int kc = 0; kc < Kp; kc += 32) {
      // the next chunk (or the next tile's first) is in flight while this one is multiplied
      f32x4 an[8];
      if (!PF) {
        load_chunk(tile, kc, a);
      } else if (kc + 32 < Kp) {
        load_chunk(tile, kc + 32, an);
      } else if (tile + stride < ntiles) {
        load_chunk(tile + stride, 0, an);
      } else {
#pragma unroll
        for (int s = 0; s < 8; ++s) an[s] = f32x4{0.f, 0.f, 0.f, 0.f};
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
      if (PF) {
#pragma unroll
        for (int s = 0; s < 8; ++s) a[s] = an[s];
      }
    }
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

template <typename T>
__global__ void k_convert(const double* __restrict__ s, T* __restrict__ d, int64_t n) {
  const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (g < n) d[g] = (T)s[g];
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

template <typename T>
__global__ __launch_bounds__(256) void k_norm2_part(const T* __restrict__ X, int64_t n,
                                                    double* __restrict__ part) {
  __shared__ double sh[256];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const double v = (double)X[i];
    s += v * v;
  }
  const double t = block_sum(s, sh);
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

// S[a][b] = sum_r A[r][a] A[r][b], one thread per entry, rows in order.
__global__ __launch_bounds__(256) void k_gram(const double* __restrict__ A, int64_t s, int R,
                                              double* __restrict__ S) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= R * R) return;
  const int a = e / R, b = e % R;
  double acc = 0.0;
#pragma unroll 8
  for (int64_t r = 0; r < s; ++r) acc += A[r * R + a] * A[r * R + b];  // eight rows in flight
  S[e] = acc;
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

// Ginv = Gamma^-1 by blocked Gauss-Jordan elimination without pivoting
// (Gamma SPD), 16 x 16 blocks on the f64 matrix cores.  Gamma is padded to
// RP x RP with the identity and kept in LDS.  Block step k, with D the
// diagonal block, row panel A_kj, column panel A_ik, rest A_ij:
//   D <- D^-1 (scalar elimination of the 16 pivots, one wave),
//   A_kj <- D^-1 A_kj,  A_ij <- A_ij - A_ik A_kj (new A_kj),  A_ik <- -A_ik D^-1,
// which is the in-place scalar elimination grouped by 16 pivots: the pivots
// met are the same Schur-complement diagonals.  A pivot at or below
// R eps max(diag) hands over to k_pinv (stats->pinv_pending).  The sequential
// depth is RP / 16 block steps instead of RP pivots.
template <int RP>
__global__ __launch_bounds__(256) void k_inv_blk(const double* __restrict__ Gm, double* __restrict__ Gi, int R,
                                                 DevStats* stats) {
  constexpr int NB = RP / 16;
  constexpr int P = RP + 1;
  __shared__ double A[RP * P];
  __shared__ double red[256];
  __shared__ int fail;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int l16 = lane & 15, g = lane >> 4;
  // every load in flight before the first store (the matrix was just written
  // by another kernel: each load is a trip to the shared cache)
  constexpr int PER = RP * RP / 256;
  double vals[PER];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int e = tid + 256 * q, i = e / RP, j = e - i * RP;
    vals[q] = (i < R && j < R) ? Gm[i * R + j] : (i == j ? 1.0 : 0.0);
  }
  double dm = 0.0;
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int e = tid + 256 * q, i = e / RP, j = e - i * RP;
    A[i * P + j] = vals[q];
    if (i == j && i < R) dm = fmax(dm, vals[q]);
  }
  red[tid] = dm;
  if (tid == 0) fail = 0;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (tid < h) red[tid] = fmax(red[tid], red[tid + h]);
    __syncthreads();
  }
  const double tol = red[0] * (double)R * 2.220446049250313e-16;
  for (int kb = 0; kb < NB; ++kb) {
    const int k0 = 16 * kb;
    // (1) D <- D^-1 by wave 0: lane owns entries e = lane + 64 q of the 16 x 16 block
    if (wave == 0) {
      for (int s = 0; s < 16; ++s) {
        const double piv = A[(k0 + s) * P + k0 + s];
        if (!(piv > tol)) {  // uniform in the wave
          if (lane == 0) fail = 1;
          break;
        }
        const double rinv = 1.0 / piv;
        double nv[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int e = lane + 64 * q, i = e >> 4, j = e & 15;
          const double rk = A[(k0 + s) * P + k0 + j], ck = A[(k0 + i) * P + k0 + s], a = A[(k0 + i) * P + k0 + j];
          if (i == s)
            nv[q] = (j == s) ? rinv : rk * rinv;
          else
            nv[q] = (j == s) ? -ck * rinv : a - ck * rk * rinv;
        }
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int e = lane + 64 * q, i = e >> 4, j = e & 15;
          A[(k0 + i) * P + k0 + j] = nv[q];
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      }
    }
    __syncthreads();
    if (fail) break;  // uniform
    // (2) row panel A_kj <- D^-1 A_kj, one 16 x 16 tile per wave at a time
    for (int jb = wave; jb < NB; jb += 4) {
      if (jb == kb) continue;
      const int j0 = 16 * jb;
      f64x4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int t = 0; t < 4; ++t)
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(A[(k0 + l16) * P + k0 + 4 * t + g],
                                                   A[(k0 + 4 * t + g) * P + j0 + l16], acc, 0, 0, 0);
      __builtin_amdgcn_wave_barrier();
#pragma unroll
      for (int v = 0; v < 4; ++v) A[(k0 + g + 4 * v) * P + j0 + l16] = acc[v];
    }
    __syncthreads();
    // (3) A_ij <- A_ij - A_ik A_kj for every block i, j != k
    for (int tt = wave; tt < NB * NB; tt += 4) {
      const int ib = tt / NB, jb = tt - ib * NB;
      if (ib == kb || jb == kb) continue;
      const int i0 = 16 * ib, j0 = 16 * jb;
      f64x4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int t = 0; t < 4; ++t)
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(A[(i0 + l16) * P + k0 + 4 * t + g],
                                                   A[(k0 + 4 * t + g) * P + j0 + l16], acc, 0, 0, 0);
#pragma unroll
      for (int v = 0; v < 4; ++v) A[(i0 + g + 4 * v) * P + j0 + l16] -= acc[v];
    }
    __syncthreads();
    // (4) column panel A_ik <- -A_ik D^-1
    for (int ib = wave; ib < NB; ib += 4) {
      if (ib == kb) continue;
      const int i0 = 16 * ib;
      f64x4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int t = 0; t < 4; ++t)
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(A[(i0 + l16) * P + k0 + 4 * t + g],
                                                   A[(k0 + 4 * t + g) * P + k0 + l16], acc, 0, 0, 0);
      __builtin_amdgcn_wave_barrier();
#pragma unroll
      for (int v = 0; v < 4; ++v) A[(i0 + g + 4 * v) * P + k0 + l16] = -acc[v];
    }
    __syncthreads();
  }
  const bool failed = fail != 0;
  for (int e = tid; e < R * R; e += 256) {
    const int i = e / R, j = e - i * R;
    Gi[e] = failed ? 0.0 : A[i * P + j];
  }
  if (failed && tid == 0) stats->pinv_pending = 1;
}

// Gamma^dagger when k_inv gave up (stats->pinv_pending): the cyclic Jacobi
// eigenvalue method (Golub and Van Loan, Matrix Computations, Sec. 8.5) in
// parallel round-robin order.  Each round rotates R/2 disjoint index pairs
// (p, q), chosen by the circle method (with a bye for odd R), with the
// rotation that zeroes A[p][q]; rows, then columns of the working matrix A
// (LDS, pitch R + 1) and the columns of V (kept in Ginv's memory) are
// updated.  A pair with |A[p][q]| <= eps sqrt(|A[p][p] A[q][q]|) is not
// rotated (its entry is set to zero); the sweeps stop when none rotates.
// Then Ginv = V diag(w+) V^T with w+ = 1 / w for w > R eps max(w), else 0.
__global__ __launch_bounds__(512) void k_pinv(const double* __restrict__ Gm, double* __restrict__ Gi, int R,
                                              DevStats* stats) {
  if (stats->pinv_pending == 0) return;  // uniform
  constexpr double eps = 2.220446049250313e-16;
  extern __shared__ double lds_d[];
  const int pitch = R + 1;
  double* A = lds_d;                     // R x pitch
  double* w = A + (size_t)R * pitch;     // R eigenvalues
  double* cs = w + R;                    // 2 x 64 rotation (c, s)
  int* pq = (int*)(cs + 128);            // 2 x 64 pair indices
  __shared__ int bad, rot;
  const int tid = threadIdx.x;
  const int RR = R * R;
  if (tid == 0) bad = 0;
  __syncthreads();
  for (int e = tid; e < RR; e += 512) {
    const int i = e / R, j = e - i * R;
    const double v = Gm[e];
    if (!isfinite(v)) bad = 1;
    A[i * pitch + j] = v;
    Gi[e] = (i == j) ? 1.0 : 0.0;  // V = I
  }
  __syncthreads();
  if (bad) {
    for (int e = tid; e < RR; e += 512) Gi[e] = 0.0;
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
      for (int e = tid; e < npair * R; e += 512) {
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
      for (int e = tid; e < npair * R; e += 512) {
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
  for (int i = tid; i < R; i += 512) w[i] = A[i * pitch + i];
  __syncthreads();
  double wmax = 0.0;
  for (int i = 0; i < R; ++i) wmax = fmax(wmax, w[i]);
  const double cut = (double)R * eps * wmax;
  __syncthreads();
  for (int i = tid; i < R; i += 512) w[i] = (w[i] > cut) ? 1.0 / w[i] : 0.0;
  __syncthreads();
  for (int e = tid; e < RR; e += 512) {
    const int i = e / R, j = e - i * R;
    double acc = 0.0;
    for (int k = 0; k < R; ++k) acc += Gi[i * R + k] * w[k] * Gi[j * R + k];
    A[i * pitch + j] = acc;
  }
  __syncthreads();
  for (int e = tid; e < RR; e += 512) {
    const int i = e / R, j = e - i * R;
    Gi[e] = A[i * pitch + j];
  }
  if (tid == 0) {
    stats->pinv_pending = 0;
    stats->pinv_count += 1;
  }
}

// One 16-row block of a mode update on the matrix cores (f64 16x16x4):
//   M~ = M (+ A_old W in PP),  A_new = M~ Ginv,
// then the shadows, dA and this block's partial Gram A^T A, dS = A^T dA,
// ||A||^2, ||dA||^2, <M~, A_new> and <Gamma, S_part>.  R is padded to RP, a
// multiple of 16, with zeros; the R x R operand (W, Ginv, Gamma) is staged in
// LDS in column chunks of at most 64.  Wave w handles column blocks
// w, w + 4, ... of each chunk.
template <typename T>
__global__ __launch_bounds__(256) void k_solve(SolveArgs<T> a) {
  extern __shared__ double lds[];
  __shared__ double sh[256];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int l16 = lane & 15, lg = lane >> 4;
  const int R = a.R, RP = (R + 15) & ~15, CH = RP < 64 ? RP : 64;
  const int PG = CH + 1, PM = RP + 1;
  double* Gs = lds;              // RP x CH chunk of an R x R operand, pitch PG
  double* Mt = Gs + RP * PG;     // 16 x RP, pitch PM
  double* An = Mt + 16 * PM;     // 16 x RP
  double* dAn = An + 16 * PM;    // 16 x RP
  const int64_t r0 = (int64_t)blockIdx.x * 16;
  const int rows = (int)((a.s - r0) < 16 ? (a.s - r0) : 16);
  for (int e = tid; e < 16 * RP; e += 256) {
    const int r = e / RP, c = e - r * RP;
    const bool in = r < rows && c < R;
    Mt[r * PM + c] = in ? a.M[(r0 + r) * R + c] : 0.0;
    An[r * PM + c] = (in && a.pp) ? a.A[(r0 + r) * R + c] : 0.0;
  }
  auto stage = [&](const double* src, int c0) {
    for (int e = tid; e < RP * CH; e += 256) {
      const int k = e / CH, c = e - k * CH;
      Gs[k * PG + c] = (k < R && c0 + c < R) ? src[k * R + c0 + c] : 0.0;
    }
  };
  // X (16 x RP, pitch PM) times the staged chunk -> 16 x 16 block at column cb
  auto block_mm = [&](const double* X, int cbl) {
    Mma<double>::acc_t acc = Mma<double>::zero();
    for (int ks = 0; ks < RP / 4; ++ks) {
      const int k = ks * 4 + lg;
      acc = Mma<double>::mma(X[l16 * PM + k], Gs[k * PG + cbl * 16 + l16], acc);
    }
    return acc;
  };
  if (a.pp) {
    // M~ = M + V^(n), V^(n) = A^(n) W with the current (old) A^(n)  (Eq. (7))
    for (int c0 = 0; c0 < RP; c0 += CH) {
      stage(a.W, c0);
      __syncthreads();
      for (int cbl = wave; cbl < CH / 16; cbl += 4) {
        const Mma<double>::acc_t acc = block_mm(An, cbl);
#pragma unroll
        for (int v = 0; v < 4; ++v) Mt[(lg + 4 * v) * PM + c0 + cbl * 16 + l16] += acc[v];
      }
      __syncthreads();
    }
  }
  double nA2 = 0.0, nd2 = 0.0, ma = 0.0;
  for (int c0 = 0; c0 < RP; c0 += CH) {
    stage(a.Ginv, c0);
    __syncthreads();
    for (int cbl = wave; cbl < CH / 16; cbl += 4) {
      const Mma<double>::acc_t acc = block_mm(Mt, cbl);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = lg + 4 * v, c = c0 + cbl * 16 + l16;
        double val = 0.0, d = 0.0;
        if (r < rows && c < R) {
          val = acc[v];
          const int64_t gi = (r0 + r) * R + c;
          if (a.pp) {
            d = val - a.Ap[gi];
            a.dAsh[gi] = (T)d;
          } else {
            d = val - a.A[gi];
          }
          a.A[gi] = val;
          a.Ash[gi] = (T)val;
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
  // partial Gram (and dS) over this block's rows, with <Gamma, S_part>
  const int ncb = RP / 16;
  double* pS = a.partS + (int64_t)blockIdx.x * R * R;
  double* pdS = a.pp ? a.partdS + (int64_t)blockIdx.x * R * R : nullptr;
  double gs = 0.0;
  for (int c0 = 0; c0 < RP; c0 += CH) {
    stage(a.Gamma, c0);
    __syncthreads();
    const int nbl = CH / 16;
    for (int blk = wave; blk < ncb * nbl; blk += 4) {
      const int ab = blk / nbl, bbl = blk - ab * nbl;
      const int bcol = c0 + bbl * 16 + l16;
      Mma<double>::acc_t s = Mma<double>::zero(), ds = Mma<double>::zero();
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) {
        const int r = ks * 4 + lg;
        const double x = An[r * PM + ab * 16 + l16];
        s = Mma<double>::mma(x, An[r * PM + bcol], s);
        if (a.pp) ds = Mma<double>::mma(x, dAn[r * PM + bcol], ds);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int ar = ab * 16 + lg + 4 * v;
        if (ar < R && bcol < R) {
          pS[ar * R + bcol] = s[v];
          if (a.pp) pdS[ar * R + bcol] = ds[v];
          gs += Gs[ar * PG + bbl * 16 + l16] * s[v];
        }
      }
    }
    __syncthreads();
  }
  const double t0 = block_sum(nA2, sh);
  const double t1 = block_sum(nd2, sh);
  const double t2 = block_sum(ma, sh);
  const double t3 = block_sum(gs, sh);
  if (tid == 0) {
    a.partSc[blockIdx.x * 4 + 0] = t0;
    a.partSc[blockIdx.x * 4 + 1] = t1;
    a.partSc[blockIdx.x * 4 + 2] = t2;
    a.partSc[blockIdx.x * 4 + 3] = t3;
  }
}

// S^(n) (and dS^(n)) = sum of the block partials in block order, one thread
// per entry, which then forms entry e of Gamma and W of the next mode;
// block 0 also sums the scalars and, after the last mode, forms the
// residual of Eq. (3).
__global__ __launch_bounds__(256) void k_finalize(FinalArgs a) {
  const int RR = a.R * a.R;
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e < RR) {
    double sv = 0.0, ds = 0.0;
#pragma unroll 8
    for (int b = 0; b < a.nblk; ++b) sv += a.partS[(int64_t)b * RR + e];
    if (a.pp) {
#pragma unroll 8
      for (int b = 0; b < a.nblk; ++b) ds += a.partdS[(int64_t)b * RR + e];
    }
    a.S[a.n][e] = sv;
    if (a.pp) a.dS[a.n][e] = ds;
    const int nx = (a.n + 1) % a.N;
    double g, w;
    gamma_entry(a.S, a.dS, a.N, nx, e, true, &g, &w);
    a.Gamma[e] = g;
    a.W[e] = w;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    double nA2 = 0.0, nd2 = 0.0, ma = 0.0, gs = 0.0;
    for (int b = 0; b < a.nblk; ++b) {
      nA2 += a.partSc[b * 4 + 0];
      nd2 += a.partSc[b * 4 + 1];
      ma += a.partSc[b * 4 + 2];
      gs += a.partSc[b * 4 + 3];
    }
    a.stats->normA2[a.n] = nA2;
    a.stats->normdA2[a.n] = nd2;
    if (a.last) {
      const double t2 = a.stats->normT2;
      const double num = t2 + gs - 2.0 * ma;
      a.stats->fit_num = num;
      const double r = sqrt((num > 0.0 ? num : 0.0) / t2);
      a.stats->r = r;
      if (!isfinite(r)) a.stats->status |= 2;
    }
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_pp_mttkrp(PPArgs<T> a) {
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
      int64_t y = yg;
      double u0 = 0.0, u1 = 0.0;
      for (; y + G < si; y += 2 * G) {
        u0 += (double)p[y * ys] * (double)d[y * R];
        u1 += (double)p[(y + G) * ys] * (double)d[(y + G) * R];
      }
      if (y < si) u0 += (double)p[y * ys] * (double)d[y * R];
      u += u0 + u1;
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
    TO s0 = 0, s1 = 0;
    int64_t i = ig;
    for (; i + 4 < I; i += 8) {
      s0 += (TO)x[i * QR] * (TO)A[i * R + r];
      s1 += (TO)x[(i + 4) * QR] * (TO)A[(i + 4) * R + r];
    }
    if (i < I) s0 += (TO)x[i * QR] * (TO)A[i * R + r];
    s = s0 + s1;
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
  }
}

inline unsigned nblocks(int64_t n) { return (unsigned)((n + 255) / 256); }



}  // namespace

template <typename T, bool KC, int NCB>
hipError_t launch_ttm_rb(const T* X, const T* B, T* C, int64_t P, int64_t K, int64_t Q, int R,
                         hipStream_t st) {
  constexpr int V = 16 / sizeof(T);
  constexpr int CH = 8 * 4 * V;
  const int Kp = (int)((K + CH - 1) / CH * CH);
  const size_t lds = (size_t)NCB * 16 * (Kp + V) * sizeof(T);
  static bool attr = false;
  if (!attr) {
    hipError_t e = hipFuncSetAttribute((const void*)k_ttm_rb<T, KC, NCB>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
    attr = true;
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
hipError_t launch_ttm_q(const float* X, const float* B, float* C, int64_t P, int64_t K, int64_t Q, int R,
                        hipStream_t st) {
  const int Kp = (int)((K + 31) / 32 * 32);
  const size_t lds = (size_t)NCB * 16 * (Kp + 4) * sizeof(float);
  static bool attr = false;
  if (!attr) {
    hipError_t e = hipFuncSetAttribute((const void*)k_ttm_q<NCB, false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       160 * 1024);
    if (e == hipSuccess)
      e = hipFuncSetAttribute((const void*)k_ttm_q<NCB, true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              160 * 1024);
    if (e != hipSuccess) return e;
    attr = true;
  }
  const int64_t tilesQ = (Q + 63) / 64;
  const int64_t ntiles = P * tilesQ;
  const int64_t want = (ntiles + kTtmWaves - 1) / kTtmWaves;
  const unsigned nx = (unsigned)(want < 512 ? want : 512);
  const unsigned ny = (unsigned)((R + NCB * 16 - 1) / (NCB * 16));
  const int vec = (Q % 4 == 0 && ((uintptr_t)X % 16) == 0) ? 1 : 0;
  if (vec && Q % 64 == 0 && K % 32 == 0)
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
  if (R <= 64) return launch_ttm_rb<T, KC, 4>(X, B, C, P, K, Q, R, st);
  return launch_ttm_rb<T, KC, 8>(X, B, C, P, K, Q, R, st);
}

template <typename T>
hipError_t launch_ttm(const T* X, const T* B, T* C, int64_t P, int64_t K, int64_t Q, int R,
                      hipStream_t st) {
  if (Q == 1 && K <= 32 * (int64_t)(16 / sizeof(T)) && R <= 64) {
    if (R <= 16) return launch_ttm_kc<T, 1>(X, B, C, P, K, R, st);
    if (R <= 32) return launch_ttm_kc<T, 2>(X, B, C, P, K, R, st);
    return launch_ttm_kc<T, 4>(X, B, C, P, K, R, st);
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
  hipLaunchKernelGGL(k_gram, dim3(nblocks((int64_t)R * R)), dim3(256), 0, st, A, s, R, S);
  return hipGetLastError();
}

hipError_t launch_gamma(const GammaArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(k_gamma, dim3(nblocks((int64_t)a.R * a.R)), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_inverse(const double* Gamma, double* Ginv, int R, DevStats* stats, hipStream_t st) {
  if (R <= 16) {
    hipLaunchKernelGGL(k_inv_blk<16>, dim3(1), dim3(256), 0, st, Gamma, Ginv, R, stats);
  } else if (R <= 32) {
    hipLaunchKernelGGL(k_inv_blk<32>, dim3(1), dim3(256), 0, st, Gamma, Ginv, R, stats);
  } else if (R <= 64) {
    hipLaunchKernelGGL(k_inv_blk<64>, dim3(1), dim3(256), 0, st, Gamma, Ginv, R, stats);
  } else {
    hipLaunchKernelGGL(k_inv_blk<128>, dim3(1), dim3(256), 0, st, Gamma, Ginv, R, stats);
  }
  static bool attr = false;
  if (!attr) {
    hipError_t e = hipFuncSetAttribute((const void*)k_pinv, hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024);
    if (e != hipSuccess) return e;
    attr = true;
  }
  const size_t lds = ((size_t)R * (R + 1) + R + 128) * sizeof(double) + 128 * sizeof(int);
  hipLaunchKernelGGL(k_pinv, dim3(1), dim3(512), lds, st, Gamma, Ginv, R, stats);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_solve(const SolveArgs<T>& a, int nblk, hipStream_t st) {
  static bool attr = false;
  if (!attr) {
    hipError_t e = hipFuncSetAttribute((const void*)k_solve<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       150 * 1024);
    if (e != hipSuccess) return e;
    attr = true;
  }
  const int RP = (a.R + 15) & ~15, CH = RP < 64 ? RP : 64;
  const size_t lds = ((size_t)RP * (CH + 1) + 3 * 16 * (size_t)(RP + 1)) * sizeof(double);
  hipLaunchKernelGGL((k_solve<T>), dim3(nblk), dim3(256), lds, st, a);
  return hipGetLastError();
}

hipError_t launch_finalize(const FinalArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(k_finalize, dim3(nblocks((int64_t)a.R * a.R)), dim3(256), 0, st, a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_pp_mttkrp(const PPArgs<T>& a, hipStream_t st) {
  hipLaunchKernelGGL((k_pp_mttkrp<T>), dim3((unsigned)a.dims[a.n]), dim3(256), 0, st, a);
  return hipGetLastError();
}

// explicit instantiations
template hipError_t launch_ttm<float>(const float*, const float*, float*, int64_t, int64_t,
                                      int64_t, int, hipStream_t);
template hipError_t launch_ttm<double>(const double*, const double*, double*, int64_t, int64_t,
                                       int64_t, int, hipStream_t);
template hipError_t launch_mttv<float, float>(const float*, const float*, float*, int64_t, int64_t,
                                              int64_t, int, hipStream_t);
template hipError_t launch_mttv<float, double>(const float*, const float*, double*, int64_t,
                                               int64_t, int64_t, int, hipStream_t);
template hipError_t launch_mttv<double, double>(const double*, const double*, double*, int64_t,
                                                int64_t, int64_t, int, hipStream_t);
template hipError_t launch_convert<float>(const double*, float*, int64_t, hipStream_t);
template hipError_t launch_convert<double>(const double*, double*, int64_t, hipStream_t);
template hipError_t launch_norm2<float>(const float*, int64_t, double*, int, DevStats*, hipStream_t);
template hipError_t launch_norm2<bf16>(const bf16*, int64_t, double*, int, DevStats*, hipStream_t);
template hipError_t launch_norm2<double>(const double*, int64_t, double*, int, DevStats*,
                                         hipStream_t);
template hipError_t launch_solve<float>(const SolveArgs<float>&, int, hipStream_t);
template hipError_t launch_solve<double>(const SolveArgs<double>&, int, hipStream_t);
template hipError_t launch_pp_mttkrp<float>(const PPArgs<float>&, hipStream_t);
template hipError_t launch_pp_mttkrp<double>(const PPArgs<double>&, hipStream_t);

}  // namespace cpals
