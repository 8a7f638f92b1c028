// First-level contraction of a BF16 tensor with one factor on the matrix
// cores (v_mfma_f32_16x16x32_bf16, FP32 accumulation):
//   C[p][q][r] = sum_k X[p][k][q] * B[k][r]
// B is the factor rounded to BF16 (one product) or split into BF16 parts
// B = B_hi + B_lo (two products, B_lo = bf16(B - B_hi)), which carries 16
// significant bits of the factor instead of 8.  The tensor values are used as
// stored.  Not from the paper (it computes in FP64): the precision path of the
// first contraction, which reads the tensor once and dominates the sweep.
//
// Operand layout of the 16x16x32 BF16 instruction: lane l supplies row l % 16
// of A and column l % 16 of B, each with eight contraction indices chosen by
// l / 16; the accumulator layout is that of the 16x16x4 FP32 instruction
// (register v of lane l holds C[4 (l / 16) + v][l % 16]).  The contraction
// order inside an instruction does not matter, so a lane may feed any eight
// indices as long as the factor lane of the same group feeds the same ones.
//
// Workgroup: eight waves, a tile of 512 output rows; each wave owns 64 rows
// (four 16-row MFMA blocks u) by 16 * NCB factor columns.  The factor is kept
// transposed (Bt[c][k], k contiguous) and staged through LDS 256 indices at a
// time; the tensor goes from HBM straight to registers, one contraction step
// (32 indices) ahead of the matrix cores.
//   KC (contraction index contiguous, Q == 1): X is P x K row-major; lane
//      (i = lane % 16, g = lane / 16) of block u loads row 16 u + i, indices
//      8 g .. 8 g + 7 of the step, as one 16-byte load.
//   otherwise: X[p] is K x Q with q contiguous; the lane needs 4 consecutive
//      q for each of its eight indices (two lanes load eight q with one
//      16-byte load per index and swap halves across the pair), then
//      transposes the 8 x 4 block in registers, so that block u gets row
//      q0 + 4 i + u.
#include "kernels.h"

namespace cpals {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

constexpr int kWaves = 8;
constexpr int kThreads = kWaves * 64;
constexpr int kTileRows = kWaves * 64;  // output rows per workgroup tile
constexpr int KB = 256;                 // contraction indices per LDS stage
constexpr int KPITCH = KB + 8;          // staged column pitch (bf16 elements)

// Round to nearest, ties to even (finite inputs).
__device__ inline uint32_t bf16_bits(float f) {
  const uint32_t u = __float_as_uint(f);
  return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
}
__device__ inline float bf16_value(uint32_t h) { return __uint_as_float(h << 16); }

// Bt_hi[c][k] = bf16(A[k][c]) (and Bt_lo[c][k] = bf16(A[k][c] - Bt_hi[c][k]))
// for k < K, zero for K <= k < Kp.
__global__ __launch_bounds__(256) void k_split_factor(const float* __restrict__ A, int64_t K, int R, int Kp,
                                                      uint16_t* __restrict__ hi, uint16_t* __restrict__ lo) {
  const int64_t n = (int64_t)R * Kp;
  for (int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x; idx < n; idx += (int64_t)gridDim.x * 256) {
    const int64_t c = idx / Kp, k = idx - c * Kp;
    const float a = k < K ? A[k * R + c] : 0.f;
    const uint32_t h = bf16_bits(a);
    hi[idx] = (uint16_t)h;
    if (lo) lo[idx] = (uint16_t)bf16_bits(a - bf16_value(h));
  }
}

__device__ inline bf16x8 as_bf16x8(u32x4 v) { return __builtin_bit_cast(bf16x8, v); }

template <bool KC, int NCB, bool SPLIT>
__global__ __launch_bounds__(512) void k_ttm_bf16(const uint16_t* __restrict__ X, const uint16_t* __restrict__ Bhi,
                                                  const uint16_t* __restrict__ Blo, float* __restrict__ C,
                                                  int64_t P, int64_t K, int64_t Q, int R, int Kp, int64_t tilesQ,
                                                  int64_t ntiles, int vec) {
  constexpr int NC = NCB * 16;
  constexpr int NPART = SPLIT ? 2 : 1;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  uint16_t* Bs = (uint16_t*)lds_raw;  // [NPART][NC][KPITCH]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, l16 = lane & 15;
  const int c0 = blockIdx.y * NC;
  const bool one_stage = Kp <= KB;

  // columns c0 .. c0 + NC - 1 of Bt, indices k0 .. k0 + KB - 1 (Kp is a multiple of 32)
  auto stage = [&](int k0) {
    const int per_col = (Kp - k0 < KB ? Kp - k0 : KB) / 8;
    const int items = NPART * NC * per_col;
    for (int idx = tid; idx < items; idx += kThreads) {
      const int part = idx / (NC * per_col);
      const int rem = idx - part * NC * per_col;
      const int c = rem / per_col, j = rem - c * per_col;
      u32x4 v = {0u, 0u, 0u, 0u};
      if (c0 + c < R) v = *(const u32x4*)((part ? Blo : Bhi) + (int64_t)(c0 + c) * Kp + k0 + 8 * j);
      *(u32x4*)(Bs + (part * NC + c) * KPITCH + 8 * j) = v;
    }
  };

  if (one_stage) {
    stage(0);
    __syncthreads();
  }
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    // ---- rows of this lane and the load addressing ----
    int64_t row0;      // KC: first row (p) of the wave's 64; else first q of the wave's 64
    const uint16_t* Xb;  // base of the batch (p) in the non-KC layout
    float* Cb;
    int64_t nrows;     // valid extent of the row index (P or Q)
    if (KC) {
      row0 = tile * kTileRows + wave * 64;
      Xb = X;
      Cb = C;
      nrows = P;
    } else {
      const int64_t p = tile / tilesQ;
      row0 = (tile - p * tilesQ) * kTileRows + wave * 64;
      Xb = X + p * K * Q;
      Cb = C + p * Q * R;
      nrows = Q;
    }
    // KC: lane rows row0 + 16u + l16 (clamped for loads); else rows row0 + 4 l16 + u
    int64_t lrow[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t r = KC ? row0 + 16 * u + l16 : row0 + 4 * l16 + u;
      lrow[u] = r < nrows ? r : nrows - 1;
    }
    const bool qfull = !KC && vec && row0 + 4 * l16 + 4 <= Q;

    auto load_a = [&](int ks, bf16x8 (&a)[4]) {
      const int kb = ks + 8 * g;  // this lane's eight indices kb .. kb + 7
      if (KC) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const uint16_t* src = Xb + lrow[u] * K + kb;
          if (vec && kb + 8 <= K) {
            a[u] = as_bf16x8(*(const u32x4*)src);
          } else {
            u32x4 v = {0u, 0u, 0u, 0u};
#pragma unroll
            for (int j = 0; j < 8; ++j) {
              const uint32_t h = (kb + j < K) ? (uint32_t)src[j] : 0u;
              v[j >> 1] |= (j & 1) ? (h << 16) : h;
            }
            a[u] = as_bf16x8(v);
          }
        }
      } else {
        u32x2 raw[8];
        // 16-byte path: lanes 2m and 2m + 1 share eight consecutive q; lane
        // h = l16 & 1 loads them at k = kb + 4h + j (j < 4) and swaps the half
        // that belongs to its partner, so each lane ends with its own four q
        // at all eight indices.  Uniform within a lane pair.
        const int h = l16 & 1;
        const int64_t qpair = row0 + 8 * (l16 >> 1);
        if (vec == 2 && qpair + 8 <= Q && kb + 8 <= K) {
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const u32x4 v = *(const u32x4*)(Xb + (int64_t)(kb + 4 * h + j) * Q + qpair);
            const uint32_t s0 = h ? v[0] : v[2], s1 = h ? v[1] : v[3];
            const uint32_t r0 = (uint32_t)__builtin_amdgcn_mov_dpp((int)s0, 0xB1, 0xF, 0xF, false);
            const uint32_t r1 = (uint32_t)__builtin_amdgcn_mov_dpp((int)s1, 0xB1, 0xF, 0xF, false);
            const u32x2 own = h ? u32x2{v[2], v[3]} : u32x2{v[0], v[1]};
            const u32x2 got = u32x2{r0, r1};
            raw[j] = h ? got : own;
            raw[4 + j] = h ? own : got;
          }
        } else {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const int64_t k = kb + j;
          const uint16_t* src = Xb + k * Q + (row0 + 4 * l16);
          if (k < K && qfull) {
            raw[j] = *(const u32x2*)src;
          } else {
            uint32_t e[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) e[u] = (k < K && row0 + 4 * l16 + u < Q) ? (uint32_t)src[u] : 0u;
            raw[j] = u32x2{e[0] | (e[1] << 16), e[2] | (e[3] << 16)};
          }
        }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          u32x4 v;
#pragma unroll
          for (int m = 0; m < 4; ++m) {
            const uint32_t x0 = raw[2 * m][u >> 1], x1 = raw[2 * m + 1][u >> 1];
            v[m] = (u & 1) ? ((x0 >> 16) | (x1 & 0xffff0000u)) : ((x0 & 0xffffu) | (x1 << 16));
          }
          a[u] = as_bf16x8(v);
        }
      }
    };

    f32x4 acc[4][NCB];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) acc[u][cb] = f32x4{0.f, 0.f, 0.f, 0.f};

    bf16x8 an[4];
    load_a(0, an);
    for (int ks = 0; ks < Kp; ks += 32) {
      const int kl = ks % KB;
      if (!one_stage && kl == 0) {
        __syncthreads();  // every wave is done with the previous stage
        stage(ks);
        __syncthreads();
      }
      bf16x8 a[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) a[u] = an[u];
      if (ks + 32 < Kp) load_a(ks + 32, an);
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) {
        const uint16_t* bp = Bs + (cb * 16 + l16) * KPITCH + kl + 8 * g;
        const bf16x8 bh = as_bf16x8(*(const u32x4*)bp);
#pragma unroll
        for (int u = 0; u < 4; ++u) acc[u][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[u], bh, acc[u][cb], 0, 0, 0);
        if (SPLIT) {
          const bf16x8 bl = as_bf16x8(*(const u32x4*)(bp + NC * KPITCH));
#pragma unroll
          for (int u = 0; u < 4; ++u)
            acc[u][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[u], bl, acc[u][cb], 0, 0, 0);
        }
      }
    }

    // ---- store: register v of block u is output row 4 g + v of the block ----
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = 4 * g + v;
          const int64_t r = KC ? row0 + 16 * u + i : row0 + 4 * i + u;
          const int c = c0 + cb * 16 + l16;
          if (r < nrows && c < R) Cb[r * R + c] = acc[u][cb][v];
        }
  }
}

template <bool KC, int NCB, bool SPLIT>
hipError_t launch_one(const uint16_t* X, const uint16_t* Bhi, const uint16_t* Blo, float* C, int64_t P, int64_t K,
                      int64_t Q, int R, int Kp, hipStream_t st) {
  constexpr int NC = NCB * 16;
  constexpr size_t lds = (size_t)(SPLIT ? 2 : 1) * NC * KPITCH * sizeof(uint16_t);
  static bool attr = false;
  if (!attr) {
    hipError_t e = hipFuncSetAttribute((const void*)k_ttm_bf16<KC, NCB, SPLIT>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    attr = true;
  }
  const int64_t tilesQ = KC ? 1 : (Q + kTileRows - 1) / kTileRows;
  const int64_t ntiles = KC ? (P + kTileRows - 1) / kTileRows : P * tilesQ;
  const unsigned nx = (unsigned)(ntiles < 256 ? ntiles : 256);  // one resident workgroup per CU
  const unsigned ny = (unsigned)((R + NC - 1) / NC);
  // KC: 16-byte row loads; otherwise 2 = 16-byte loads shared by lane pairs, 1 = 8-byte loads
  const int vec = KC ? (K % 8 == 0 && ((uintptr_t)X % 16) == 0)
                     : ((Q % 8 == 0 && ((uintptr_t)X % 16) == 0) ? 2 : (Q % 4 == 0 && ((uintptr_t)X % 8) == 0));
  hipLaunchKernelGGL((k_ttm_bf16<KC, NCB, SPLIT>), dim3(nx, ny), dim3(kThreads), lds, st, X, Bhi, Blo, C, P, K, Q,
                     R, Kp, tilesQ, ntiles, vec);
  return hipGetLastError();
}

template <bool KC, bool SPLIT>
hipError_t launch_ncb(const uint16_t* X, const uint16_t* Bhi, const uint16_t* Blo, float* C, int64_t P, int64_t K,
                      int64_t Q, int R, int Kp, hipStream_t st) {
  if (R <= 16) return launch_one<KC, 1, SPLIT>(X, Bhi, Blo, C, P, K, Q, R, Kp, st);
  if (R <= 32) return launch_one<KC, 2, SPLIT>(X, Bhi, Blo, C, P, K, Q, R, Kp, st);
  if (R <= 64) return launch_one<KC, 4, SPLIT>(X, Bhi, Blo, C, P, K, Q, R, Kp, st);
  return launch_one<KC, 8, SPLIT>(X, Bhi, Blo, C, P, K, Q, R, Kp, st);
}

}  // namespace

int bf16_factor_pitch(int64_t K) { return (int)((K + 31) / 32 * 32); }

hipError_t launch_split_factor(const float* A, int64_t K, int R, uint16_t* hi, uint16_t* lo, hipStream_t st) {
  const int Kp = bf16_factor_pitch(K);
  const int64_t n = (int64_t)R * Kp;
  const int64_t nb = (n + 255) / 256;
  hipLaunchKernelGGL(k_split_factor, dim3((unsigned)(nb < 4096 ? nb : 4096)), dim3(256), 0, st, A, K, R, Kp, hi, lo);
  return hipGetLastError();
}

hipError_t launch_ttm_bf16(const uint16_t* X, const uint16_t* Bhi, const uint16_t* Blo, float* C, int64_t P,
                           int64_t K, int64_t Q, int R, hipStream_t st) {
  if (R < 1 || R > kMaxRank || K < 1 || P < 1 || Q < 1) return hipErrorInvalidValue;
  const int Kp = bf16_factor_pitch(K);
  if (Q == 1) {
    return Blo ? launch_ncb<true, true>(X, Bhi, Blo, C, P, K, Q, R, Kp, st)
               : launch_ncb<true, false>(X, Bhi, Blo, C, P, K, Q, R, Kp, st);
  }
  return Blo ? launch_ncb<false, true>(X, Bhi, Blo, C, P, K, Q, R, Kp, st)
             : launch_ncb<false, false>(X, Bhi, Blo, C, P, K, Q, R, Kp, st);
}

}  // namespace cpals
