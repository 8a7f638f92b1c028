// First-level contraction of a BF16 or FP8 tensor with one factor on the matrix
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
// transposed (Bt[c][k], k contiguous) and staged through LDS in chunks of 64
// indices, double-buffered (the next chunk is loaded while the current one is
// used; one barrier per chunk).  The tensor goes from HBM straight to
// registers, one contraction step (32 indices) ahead of the matrix cores,
// except in the FP8 q-contiguous layout with Q a multiple of 16 (below).
//   KC (contraction index contiguous, Q == 1): X is P x K row-major; lane
//      (i = lane % 16, g = lane / 16) of block u loads row 16 u + i, indices
//      8 g .. 8 g + 7 of the step, as one 16-byte load.
//   otherwise: X[p] is K x Q with q contiguous; the lane needs 4 consecutive
//      q for each of its eight indices (two lanes load eight q with one
//      16-byte load per index and swap halves across the pair), then
//      transposes the 8 x 4 block in registers, so that block u gets row
//      q0 + 4 i + u.
//
// FP8 tensor (E4M3: 4 exponent bits with bias 7, 3 mantissa bits, no
// infinities): every FP8 value is a BF16 value, so the hardware conversion
// to BF16 is exact and the products are those of the stored tensor with the
// BF16 (or split) factor, on the same matrix cores; the tensor's bytes are
// halved.  Both layouts load a whole chunk (64 indices) per register set:
// lane group g holds indices 16 g .. 16 g + 15, step s of the chunk uses
// 16 g + 8 s .. 16 g + 8 s + 7 (the factor is read at the same offsets).
//   KC: one 16-byte load per row; with DEEP, three register sets (the next
//      two chunks in flight).
//   otherwise, TR (Q a multiple of 16, 16-byte aligned): the workgroup's chunk
//      of the tensor (64 indices x 512 q) goes HBM -> registers -> LDS with
//      16-byte loads, double-buffered in static LDS, and each lane reads its
//      operands back with the transposing 8-bit LDS read (ds_read_tr8_b64),
//      which hands it eight consecutive indices of one q.
//   otherwise (other Q): one 4-byte load (four consecutive q) per index; an
//      in-register 4 x 4 byte transpose puts each q's four consecutive indices
//      in one word.
//
// FP8 x FP8 (FF): the same FP8 tensor operands, unwidened, against a factor
// quantized to E4M3 per column on the FP8 matrix cores
// (v_mfma_f32_16x16x32_fp8_fp8, same lane layout with one byte per index):
// column c is scaled by the power of two 2^e_c that puts its largest
// magnitude in (224, 448] and rounded to nearest E4M3 (ties to even,
// k_quant_factor_fp8); each product of two E4M3 values is exact, but the
// instruction sums each lane's group of eight products in a fixed-point
// window under the group's largest (measured on gfx950: a product 2^12 below
// it kept exactly, one 2^14 below dropped; the groups and the accumulator
// at FP32 precision).  The output column is multiplied by 2^-e_c (exact).
// The factor chunk is staged as bytes (80-byte column pitch).
#include <type_traits>

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
constexpr int KB = 64;                  // contraction indices per LDS chunk (two steps)
constexpr int KPITCH = KB + 8;          // chunk column pitch (bf16 elements)

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

// E4M3 code of v (|v| <= 448, finite), rounded to nearest with ties to even:
// below 2^-6 the subnormal steps of 2^-9; otherwise, with |v| = f 2^E
// (f in [0.5, 1)), exponent field E + 6 and mantissa rint(16 f) - 8, where a
// mantissa of 8 carries into the exponent field.
__device__ inline uint32_t e4m3_code(float v) {
  const uint32_t sign = v < 0.f ? 0x80u : 0u;
  const float a = fabsf(v);
  if (a < 0.015625f) return sign | (uint32_t)rintf(a * 512.f);
  int E;
  const float f = frexpf(a, &E);
  return sign | (uint32_t)(((E + 5) << 3) + (int)rintf(16.f * f));
}

// Bq[c][k] = E4M3 code of A[k][c] 2^e_c for k < K (zero up to Kp) and
// inv[c] = 2^-e_c, with e_c the largest exponent that keeps the column's
// largest magnitude at or below 448 (clamped to [-120, 120]; 0 for a zero
// column).  One workgroup per column.
__global__ __launch_bounds__(256) void k_quant_factor_fp8(const float* __restrict__ A, int64_t K, int R, int Kp,
                                                          uint8_t* __restrict__ Bq, float* __restrict__ inv) {
  __shared__ float red[256];
  const int c = blockIdx.x, tid = threadIdx.x;
  float m = 0.f;
  for (int64_t k = tid; k < K; k += 256) m = fmaxf(m, fabsf(A[k * R + c]));
  red[tid] = m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) red[tid] = fmaxf(red[tid], red[tid + w]);
    __syncthreads();
  }
  const float mx = red[0];
  int e = 0;
  if (mx > 0.f) {
    int E;
    const float f = frexpf(mx, &E);
    e = (f <= 0.875f ? 9 : 8) - E;
    e = e < -120 ? -120 : (e > 120 ? 120 : e);
  }
  for (int64_t k = tid; k < Kp; k += 256) Bq[(int64_t)c * Kp + k] = k < K ? (uint8_t)e4m3_code(ldexpf(A[k * R + c], e)) : 0;
  if (tid == 0) inv[c] = ldexpf(1.f, -e);
}

__device__ inline bf16x8 as_bf16x8(u32x4 v) { return __builtin_bit_cast(bf16x8, v); }

// Lane source of one workgroup tile in the unguarded layout: KC, the four
// row pointers (rows row0 + 16 u + l16, clamped to P - 1) at index 8 g;
// otherwise p[0] points at k = 8 g + 4 h, q = qpair (clamped to Q - 8).
// FP8, KC: rows as above at index 16 g; otherwise p[0] points at k = 16 g,
// q = q0 + 4 (lane % 16) (clamped to Q - 4).
template <typename E>
struct LaneSrc {
  const E* p[4];
  uint32_t o;  // BF16 q-contiguous unguarded: the lane's q offset from the slice base p[0]
};

// Two E4M3 values (word half `hi` of w) as two BF16 values, exactly.
template <bool HI>
__device__ inline uint32_t fp8_pair_bf16(uint32_t w) {
  return __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(w, 1.0f, HI));
}

// Bytes of four words x0..x3 transposed: byte b of result t[j] is byte j of x_b.
__device__ inline void byte_transpose4(uint32_t x0, uint32_t x1, uint32_t x2, uint32_t x3, uint32_t (&t)[4]) {
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int sh = 8 * j;
    t[j] = ((x0 >> sh) & 0xffu) | (((x1 >> sh) & 0xffu) << 8) | (((x2 >> sh) & 0xffu) << 16) | (((x3 >> sh) & 0xffu) << 24);
  }
}

constexpr int TPITCH = 528;  // FP8 chunk stage row pitch (bytes): 512 q plus 16 to spread the banks

typedef int i32x2 __attribute__((ext_vector_type(2)));

template <bool KC, int NCB, bool SPLIT, bool FAST, bool F8, bool DEEP, bool TR, bool FF>
__global__ __launch_bounds__(512) void k_ttm_bf16(const void* __restrict__ Xv, const uint16_t* __restrict__ Bhi,
                                                  const uint16_t* __restrict__ Blo, const float* __restrict__ cs,
                                                  float* __restrict__ C,
                                                  int64_t P, int64_t K, int64_t Q, int R, int Kp, int64_t tilesQ,
                                                  int64_t ntiles, int vec) {
  using E = typename std::conditional<F8, uint8_t, uint16_t>::type;
  using Src = LaneSrc<E>;
  const E* __restrict__ X = (const E*)Xv;
  constexpr int NC = NCB * 16;
  constexpr int NPART = SPLIT ? 2 : 1;
  constexpr int PIECES = FF ? KB / 16 : KB / 8;  // 16-byte pieces of one column's chunk
  constexpr int KPB = KB + 16;                   // FF: byte pitch of a staged factor column
  constexpr int BITEMS = NPART * NC * PIECES;    // 16-byte pieces of one factor chunk
  constexpr int BPER = (BITEMS + kThreads - 1) / kThreads;
  // BF16 q-contiguous unguarded: 32-bit offsets from uniform bases for the
  // tensor and factor loads (the launch checks (K + 80) Q < 2^31 and
  // R Kp < 2^31); 64-bit per-lane addresses cost the 128-column split-factor
  // form its registers.  A factor piece's part is uniform when one part's
  // pieces fill whole multiples of the workgroup.
  constexpr bool O32 = FAST && !KC && !F8;
  constexpr bool BUNI = O32 && (NC * (KB / 8)) % kThreads == 0;
  __shared__ __align__(16) uint16_t Bs[2][NPART * NC * KPITCH];  // [buffer][part][column][index]
  // FP8 q-contiguous with TR: the workgroup's chunk of the tensor, [buffer][index][q]
  __shared__ __align__(16) uint8_t Ts[TR ? 2 * KB * TPITCH : 16];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform (not inferred from tid / 64)
  const int g = lane >> 4, l16 = lane & 15;
  const int c0 = blockIdx.y * NC;
  const int nch = Kp / KB;

  // ---- factor chunks: columns c0 .. c0 + NC - 1 (past R clamped to R - 1;
  // their products are never stored), indices ch KB .. ch KB + KB - 1 (the
  // padding up to Kp holds zeros) ----
  auto b_piece = [&](int q, int& part, int& c, int& j) {
    int idx = tid + kThreads * q;
    if (BITEMS % kThreads != 0) idx = idx < BITEMS ? idx : BITEMS - 1;
    part = idx / (NC * PIECES);
    const int rem = idx - part * NC * PIECES;
    c = rem / PIECES;
    j = rem - c * PIECES;
  };
  auto load_b = [&](int ch, u32x4 (&bv)[BPER]) {
#pragma unroll
    for (int q = 0; q < BPER; ++q) {
      int part, c, j;
      b_piece(q, part, c, j);
      const int col = c0 + c < R ? c0 + c : R - 1;
      if constexpr (FF) {
        bv[q] = *(const u32x4*)((const uint8_t*)Bhi + (int64_t)col * Kp + ch * KB + 16 * j);
      } else if constexpr (BUNI) {
        const char* base = (const char*)((q * kThreads) / (NC * (KB / 8)) ? Blo : Bhi);
        bv[q] = *(const u32x4*)(base + 2u * ((uint32_t)col * (uint32_t)Kp + (uint32_t)(ch * KB + 8 * j)));
      } else {
        bv[q] = *(const u32x4*)((part ? Blo : Bhi) + (int64_t)col * Kp + ch * KB + 8 * j);
      }
    }
  };
  auto store_b = [&](int buf, const u32x4 (&bv)[BPER]) {
#pragma unroll
    for (int q = 0; q < BPER; ++q) {
      int part, c, j;
      b_piece(q, part, c, j);
      if constexpr (FF)
        *(u32x4*)((uint8_t*)Bs[buf] + c * KPB + 16 * j) = bv[q];
      else
        *(u32x4*)(Bs[buf] + (part * NC + c) * KPITCH + 8 * j) = bv[q];
    }
  };

  // ---- tile addressing ----
  auto tile_rows = [&](int64_t tile, int64_t& row0, const E*& Xb, float*& Cb, int64_t& nrows) {
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
  };
  auto lane_src = [&](int64_t tile) {
    Src s{};
    int64_t row0, nrows;
    const E* Xb;
    float* Cb;
    tile_rows(tile, row0, Xb, Cb, nrows);
    if (KC) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int64_t r = row0 + 16 * u + l16;
        s.p[u] = Xb + (r < nrows ? r : nrows - 1) * K + (F8 ? 16 : 8) * g;
      }
    } else if (F8) {
      const int64_t q = row0 + 4 * l16;
      s.p[0] = Xb + (int64_t)(16 * g) * Q + (q < Q - 4 ? q : Q - 4);
      s.p[1] = s.p[2] = s.p[3] = s.p[0];
    } else {
      const int64_t qp = row0 + 8 * (l16 >> 1);
      s.p[0] = s.p[1] = s.p[2] = s.p[3] = Xb;  // uniform: the loads' scalar base
      s.o = (uint32_t)(qp < Q - 8 ? qp : Q - 8);
    }
    return s;
  };

  // ---- tensor step (32 indices from ks) into registers ----
  // Unguarded layout (FAST: 16-byte aligned rows, K a multiple of 8 for KC,
  // Q a multiple of 8 otherwise): plain 16-byte loads, converted to MFMA
  // operands only when used, so the loads of the next step stay in flight
  // meanwhile.
  // Guarded layout: the operands are formed at load time with every index
  // checked (indices past K read as zero).
  auto issue = [&](const Src& s, int64_t tile, int ks, u32x4 (&r)[4]) {
    if constexpr (!F8) {
    if (FAST) {
      // indices past K: KC reads the row's last eight (K % 8 == 0, so a
      // piece is wholly inside or wholly past), otherwise row K - 1; the
      // factor's zero padding cancels either
      if (KC) {
        const int kc = ks < K - 8 - 8 * g ? ks : (int)K - 8 - 8 * g;
#pragma unroll
        for (int u = 0; u < 4; ++u) r[u] = *(const u32x4*)(s.p[u] + kc);
      } else {
        // element offset min(kb + ks + j, K - 1) Q + the lane's q
        const uint32_t qq = (uint32_t)Q, last = (uint32_t)(K - 1) * qq;
        const uint32_t kbq = (uint32_t)(8 * g + 4 * (l16 & 1)) * qq;
        const char* base = (const char*)s.p[0];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const uint32_t kq = kbq + (uint32_t)(ks + j) * qq;
          r[j] = *(const u32x4*)(base + 2u * ((kq < last ? kq : last) + s.o));
        }
      }
      return;
    }
    int64_t row0, nrows;
    const E* Xb;
    float* Cb;
    tile_rows(tile, row0, Xb, Cb, nrows);
    const int kb = ks + 8 * g;  // this lane's eight indices kb .. kb + 7
    if (KC) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        int64_t rr = row0 + 16 * u + l16;
        rr = rr < nrows ? rr : nrows - 1;
        const uint16_t* src = Xb + rr * K + kb;
        if (vec && kb + 8 <= K) {
          r[u] = *(const u32x4*)src;
        } else {
          u32x4 v = {0u, 0u, 0u, 0u};
#pragma unroll
          for (int j = 0; j < 8; ++j) {
            const uint32_t h = (kb + j < K) ? (uint32_t)src[j] : 0u;
            v[j >> 1] |= (j & 1) ? (h << 16) : h;
          }
          r[u] = v;
        }
      }
      return;
    }
    const bool qfull = vec && row0 + 4 * l16 + 4 <= Q;
    u32x2 raw[8];
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
#pragma unroll
    for (int u = 0; u < 4; ++u) {
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const uint32_t x0 = raw[2 * m][u >> 1], x1 = raw[2 * m + 1][u >> 1];
        r[u][m] = (u & 1) ? ((x0 >> 16) | (x1 & 0xffff0000u)) : ((x0 & 0xffffu) | (x1 << 16));
      }
    }
    }
  };

  // ---- FP8: the chunk from ks (64 indices) into registers.  KC: r[u] holds
  // row u's indices 16 g .. 16 g + 15; otherwise word r[i / 4][i % 4] holds
  // the lane's four q at index 16 g + i.  Unguarded (FAST: 16-byte aligned
  // rows with K a multiple of 16 for KC, 4-byte aligned with Q a multiple of
  // 4 otherwise): indices past K read clamped addresses, cancelled by the
  // factor's zero padding.  Guarded: indices past K and q past Q read as
  // zero; vec: 4-byte loads allowed (KC, K a multiple of 4, aligned). ----
  auto issue8 = [&](const Src& s, int64_t tile, int ks, u32x4 (&r)[4]) {
    if constexpr (F8) {
      if (FAST) {
        if (KC) {
          const int kc = ks <= K - 16 - 16 * g ? ks : (int)K - 16 - 16 * g;
#pragma unroll
          for (int u = 0; u < 4; ++u) r[u] = *(const u32x4*)(s.p[u] + kc);
        } else {
#pragma unroll
          for (int i = 0; i < 16; ++i) {
            const int64_t k = ks + 16 * g + i < K ? ks + 16 * g + i : K - 1;
            r[i >> 2][i & 3] = *(const uint32_t*)(s.p[0] + (k - 16 * g) * Q);
          }
        }
        return;
      }
      int64_t row0, nrows;
      const E* Xb;
      float* Cb;
      tile_rows(tile, row0, Xb, Cb, nrows);
      const int64_t kb = ks + 16 * g;
      if (KC) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          int64_t rr = row0 + 16 * u + l16;
          rr = rr < nrows ? rr : nrows - 1;
          const E* src = Xb + rr * K + kb;
#pragma unroll
          for (int w = 0; w < 4; ++w) {
            const int64_t k = kb + 4 * w;
            uint32_t x = 0;
            if (vec && k + 4 <= K) {
              x = *(const uint32_t*)(src + 4 * w);
            } else {
#pragma unroll
              for (int b = 0; b < 4; ++b)
                if (k + b < K) x |= (uint32_t)src[4 * w + b] << (8 * b);
            }
            r[u][w] = x;
          }
        }
      } else {
        const int64_t q = row0 + 4 * l16;
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          const int64_t k = kb + i;
          uint32_t w = 0;
          if (k < K) {
#pragma unroll
            for (int b = 0; b < 4; ++b)
              if (q + b < Q) w |= (uint32_t)Xb[k * Q + q + b] << (8 * b);
          }
          r[i >> 2][i & 3] = w;
        }
      }
    }
  };
  // FP8 operand bytes of step s (0 or 1) of the chunk in r: byte j of w[u]
  // is block u's value at the lane's index j of the step.
  auto bytes8 = [&](const u32x4 (&r)[4], int s, u32x2 (&w)[4]) {
    if (KC) {
#pragma unroll
      for (int u = 0; u < 4; ++u) w[u] = u32x2{r[u][2 * s], r[u][2 * s + 1]};
      return;
    }
    uint32_t ta[4], tb[4];  // indices 8 s + 0..3 and 8 s + 4..7, one word per q
    byte_transpose4(r[2 * s][0], r[2 * s][1], r[2 * s][2], r[2 * s][3], ta);
    byte_transpose4(r[2 * s + 1][0], r[2 * s + 1][1], r[2 * s + 1][2], r[2 * s + 1][3], tb);
#pragma unroll
    for (int u = 0; u < 4; ++u) w[u] = u32x2{ta[u], tb[u]};
  };
  // the eight E4M3 values as BF16 operands (exact)
  auto widen8 = [&](const u32x2 (&w)[4], bf16x8 (&a)[4]) {
#pragma unroll
    for (int u = 0; u < 4; ++u)
      a[u] = as_bf16x8(u32x4{fp8_pair_bf16<false>(w[u][0]), fp8_pair_bf16<true>(w[u][0]),
                             fp8_pair_bf16<false>(w[u][1]), fp8_pair_bf16<true>(w[u][1])});
  };
  // Operands of one step.  Unguarded q-contiguous layout: lanes 2m and 2m + 1
  // loaded the same eight q at k = kb + 4h + j (h = l16 & 1, j < 4); each
  // swaps the half that belongs to its partner, so it holds its own four q
  // at all eight indices, and transposes that 8 x 4 block.
  auto operands = [&](const u32x4 (&r)[4], bf16x8 (&a)[4]) {
    if (!FAST || KC) {
#pragma unroll
      for (int u = 0; u < 4; ++u) a[u] = as_bf16x8(r[u]);
      return;
    }
    const int h = l16 & 1;
    u32x2 raw[8];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const u32x4 v = r[j];
      const uint32_t s0 = h ? v[0] : v[2], s1 = h ? v[1] : v[3];
      const uint32_t r0 = (uint32_t)__builtin_amdgcn_mov_dpp((int)s0, 0xB1, 0xF, 0xF, false);
      const uint32_t r1 = (uint32_t)__builtin_amdgcn_mov_dpp((int)s1, 0xB1, 0xF, 0xF, false);
      const u32x2 own = h ? u32x2{v[2], v[3]} : u32x2{v[0], v[1]};
      const u32x2 got = u32x2{r0, r1};
      raw[j] = h ? got : own;
      raw[4 + j] = h ? own : got;
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
  };

  // ---- FP8, q-contiguous, TR (Q a multiple of 16, 16-byte aligned): the
  // chunk (64 indices x the tile's 512 q) goes HBM -> registers -> LDS with
  // 16-byte loads, thread tid taking pieces tid + 512 m (index piece / 32,
  // q offset 16 (piece % 32)); indices past K read row K - 1 (cancelled by
  // the factor's zero padding), q past Q the last 16 (never stored) ----
  auto load_t = [&](int64_t t, int ch, u32x4 (&tv)[4]) {
    if constexpr (TR) {
      const int64_t p = t / tilesQ;
      const int64_t tq0 = (t - p * tilesQ) * kTileRows;
      const E* Xb = X + p * K * Q;
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const int piece = tid + kThreads * m;
        const int64_t k = (int64_t)ch * KB + (piece >> 5);
        const int64_t q = tq0 + 16 * (piece & 31);
        tv[m] = *(const u32x4*)(Xb + (k < K ? k : K - 1) * Q + (q <= Q - 16 ? q : Q - 16));
      }
    }
  };
  auto store_t = [&](int b, const u32x4 (&tv)[4]) {
    if constexpr (TR) {
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const int piece = tid + kThreads * m;
        *(u32x4*)(Ts + b * KB * TPITCH + (piece >> 5) * TPITCH + 16 * (piece & 31)) = tv[m];
      }
    }
  };
  // Operands of step s from the stage: block u holds the wave's q rows
  // 16 u .. 16 u + 15; the transposing read gives lane (g, i) indices
  // 32 s + 8 g .. + 7 of q row i when lane t of the group points at index
  // 32 s + 8 g + t / 2, q 16 u + 8 (t % 2).
  auto bytes_tr = [&](int b, int s8, u32x2 (&w)[4]) {
    if constexpr (TR) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int off = b * KB * TPITCH + (32 * s8 + 8 * g + (l16 >> 1)) * TPITCH + wave * 64 + 16 * u + 8 * (l16 & 1);
        const i32x2 v = __builtin_amdgcn_ds_read_tr8_b64_v2i32((__attribute__((address_space(3))) i32x2*)(Ts + off));
        w[u] = u32x2{(uint32_t)v[0], (uint32_t)v[1]};
      }
    }
  };

  f32x4 acc[4][NCB];
  // the step's products; the lane's factor indices start at ko of the chunk
  auto mfma_step = [&](const bf16x8 (&a)[4], const uint16_t* bs, int ko) {
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
      const uint16_t* bp = bs + (cb * 16 + l16) * KPITCH + ko;
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
  };
  auto multiply = [&](const u32x4 (&r)[4], const uint16_t* bs, int kl) {
    bf16x8 a[4];
    operands(r, a);
    mfma_step(a, bs, kl + 8 * g);
  };
  // FF: the step's products with the E4M3 factor staged as bytes
  auto mfma_step_ff = [&](const u32x2 (&w)[4], const uint16_t* bs, int ko) {
    if constexpr (FF) {
      const uint8_t* b8 = (const uint8_t*)bs;
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) {
        const long bq = *(const long*)(b8 + (cb * 16 + l16) * KPB + ko);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const long aq = (long)(((uint64_t)w[u][1] << 32) | (uint64_t)w[u][0]);
          acc[u][cb] = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(aq, bq, acc[u][cb], 0, 0, 0);
        }
      }
    }
  };
  // FP8 tensor operands (bytes w) against the staged factor at chunk offset ko
  auto step8 = [&](const u32x2 (&w)[4], const uint16_t* bs, int ko) {
    if constexpr (FF) {
      mfma_step_ff(w, bs, ko);
    } else {
      bf16x8 a[4];
      widen8(w, a);
      mfma_step(a, bs, ko);
    }
  };
  auto multiply8 = [&](const u32x4 (&r)[4], const uint16_t* bs, int s) {
    u32x2 w[4];
    bytes8(r, s, w);
    step8(w, bs, 16 * g + 8 * s);
  };

  // ---- main loop: the workgroup's waves step through the same (tile, chunk)
  // sequence; the factor's next chunk and the tensor's next step are loaded
  // while the current step is multiplied ----
  int64_t tile = blockIdx.x;
  if (tile >= ntiles) return;  // uniform: the whole workgroup
  {
    u32x4 bv[BPER];
    load_b(0, bv);
    store_b(0, bv);
  }
  Src cur = FAST ? lane_src(tile) : Src{};
  u32x4 ra[4], rb[4], rc[4];
  if (TR) {
    u32x4 tv[4];
    load_t(tile, 0, tv);
    store_t(0, tv);
  } else if (F8) {
    issue8(cur, tile, 0, ra);
    if (DEEP) issue8(cur, tile, KB, rb);
  } else {
    issue(cur, tile, 0, ra);
  }
  __syncthreads();
  int buf = 0;
  for (; tile < ntiles; tile += gridDim.x) {
    const int64_t tn = tile + gridDim.x < ntiles ? tile + gridDim.x : tile;
    const Src nxt = FAST ? lane_src(tn) : Src{};
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) acc[u][cb] = f32x4{0.f, 0.f, 0.f, 0.f};
    if (F8 && TR) {
      for (int ch = 0; ch < nch; ++ch) {
        const bool more = ch + 1 < nch;
        u32x4 bv[BPER], tv[4];
        load_b(more ? ch + 1 : 0, bv);
        load_t(more ? tile : tn, more ? ch + 1 : 0, tv);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int s8 = 0; s8 < 2; ++s8) {
          u32x2 w[4];
          bytes_tr(buf, s8, w);
          step8(w, Bs[buf], 32 * s8 + 8 * g);
        }
        store_b(buf ^ 1, bv);
        store_t(buf ^ 1, tv);
        buf ^= 1;
        __syncthreads();
      }
    } else if (F8 && DEEP) {
      // three register sets (at least two chunks per tile): the loads of the
      // next two chunks are in flight during the current one
      for (int ch = 0; ch < nch; ++ch) {
        const bool more = ch + 1 < nch;
        u32x4 bv[BPER];
        load_b(more ? ch + 1 : 0, bv);
        {
          const bool same = ch + 2 < nch;
          Src sn;
#pragma unroll
          for (int u = 0; u < 4; ++u) sn.p[u] = same ? cur.p[u] : nxt.p[u];
          issue8(sn, same ? tile : tn, (same ? ch + 2 : ch + 2 - nch) * KB, rc);
        }
        __builtin_amdgcn_sched_barrier(0);
        multiply8(ra, Bs[buf], 0);
        multiply8(ra, Bs[buf], 1);
        store_b(buf ^ 1, bv);
        buf ^= 1;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          ra[u] = rb[u];
          rb[u] = rc[u];
        }
        __syncthreads();
      }
    } else if (F8) {
      // one register set per chunk: the next chunk's loads are in flight
      // during both steps of the current one
      for (int ch = 0; ch < nch; ++ch) {
        const bool more = ch + 1 < nch;
        u32x4 bv[BPER];
        load_b(more ? ch + 1 : 0, bv);
        {
          Src sn;
#pragma unroll
          for (int u = 0; u < 4; ++u) sn.p[u] = more ? cur.p[u] : nxt.p[u];
          issue8(sn, more ? tile : tn, more ? (ch + 1) * KB : 0, rb);
        }
        __builtin_amdgcn_sched_barrier(0);
        multiply8(ra, Bs[buf], 0);
        multiply8(ra, Bs[buf], 1);
        store_b(buf ^ 1, bv);
        buf ^= 1;
#pragma unroll
        for (int u = 0; u < 4; ++u) ra[u] = rb[u];
        __syncthreads();
      }
    } else
    for (int ch = 0; ch < nch; ++ch) {
      const bool more = ch + 1 < nch;
      u32x4 bv[BPER];
      load_b(more ? ch + 1 : 0, bv);  // before the tensor loads: waiting for it leaves them in flight
      issue(cur, tile, ch * KB + 32, rb);
      __builtin_amdgcn_sched_barrier(0);
      multiply(ra, Bs[buf], 0);
      {
        Src sn;
#pragma unroll
        for (int u = 0; u < 4; ++u) sn.p[u] = more ? cur.p[u] : nxt.p[u];
        sn.o = more ? cur.o : nxt.o;
        issue(sn, more ? tile : tn, more ? (ch + 1) * KB : 0, ra);
      }
      __builtin_amdgcn_sched_barrier(0);
      multiply(rb, Bs[buf], 32);
      store_b(buf ^ 1, bv);
      buf ^= 1;
      __syncthreads();
    }

    // ---- store: register v of block u is output row 4 g + v of the block ----
    int64_t row0, nrows;
    const E* Xb;
    float* Cb;
    tile_rows(tile, row0, Xb, Cb, nrows);
    // FF: the column's power-of-two scale removed (exact)
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
      const int c = c0 + cb * 16 + l16;
      const float sc = FF ? cs[c < R ? c : R - 1] : 1.f;
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = 4 * g + v;
          const int64_t r = (KC || TR) ? row0 + 16 * u + i : row0 + 4 * i + u;
          if (r < nrows && c < R) Cb[r * R + c] = FF ? acc[u][cb][v] * sc : acc[u][cb][v];
        }
    }
    cur = nxt;
  }
}

template <bool KC, int NCB, bool SPLIT, bool FAST, bool F8, bool DEEP = false, bool TR = false, bool FF = false>
hipError_t launch_one(const void* X, const uint16_t* Bhi, const uint16_t* Blo, const float* cs, float* C, int64_t P,
                      int64_t K, int64_t Q, int R, int Kp, int vec, hipStream_t st) {
  constexpr int NC = NCB * 16;
  const int64_t tilesQ = KC ? 1 : (Q + kTileRows - 1) / kTileRows;
  const int64_t ntiles = KC ? (P + kTileRows - 1) / kTileRows : P * tilesQ;
  const unsigned nx = (unsigned)(ntiles < 256 ? ntiles : 256);  // one resident workgroup per CU
  const unsigned ny = (unsigned)((R + NC - 1) / NC);
  hipLaunchKernelGGL((k_ttm_bf16<KC, NCB, SPLIT, FAST, F8, DEEP, TR, FF>), dim3(nx, ny), dim3(kThreads), 0, st, X, Bhi,
                     Blo, cs, C, P, K, Q, R, Kp, tilesQ, ntiles, vec);
  return hipGetLastError();
}

template <bool KC, bool SPLIT, bool F8, bool FF = false>
hipError_t launch_ncb(const void* X, const uint16_t* Bhi, const uint16_t* Blo, const float* cs, float* C, int64_t P,
                      int64_t K, int64_t Q, int R, int Kp, hipStream_t st) {
  const uintptr_t a = (uintptr_t)X;
  int vec;
  bool fast;
  if (F8) {
    // KC: unguarded with 16-byte rows, else 4-byte loads where whole; otherwise
    // unguarded with 4-byte aligned groups of four q
    vec = KC ? (K % 4 == 0 && a % 4 == 0) : 0;
    fast = KC ? (K % 16 == 0 && a % 16 == 0) : (Q % 4 == 0 && a % 4 == 0);
  } else {
    // KC: 16-byte row loads; otherwise 2 = 16-byte loads shared by lane pairs, 1 = 8-byte loads
    // (2 also needs the 32-bit offsets of its tensor and factor loads to fit)
    const bool off32 = (K + 80) * Q < ((int64_t)1 << 31) && (int64_t)R * Kp < ((int64_t)1 << 31);
    vec = KC ? (K % 8 == 0 && a % 16 == 0) : ((Q % 8 == 0 && a % 16 == 0 && off32) ? 2 : (Q % 4 == 0 && a % 8 == 0));
    fast = KC ? vec == 1 : vec == 2;
  }
  // FP8 contiguous rows, one factor part, unguarded, at least two chunks:
  // three register sets (0.44 -> 0.34 ms at 1024^3, R = 128; the
  // q-contiguous layouts, with 16 four-byte loads per chunk, were 7 % slower;
  // not with FP8 x FP8 products over 128 columns, which would spill)
  const bool deep = F8 && KC && fast && Kp >= 2 * KB;
  // FP8 q-contiguous with Q a multiple of 16, 16-byte aligned: the chunk staged through LDS
  const bool tr = F8 && !KC && Q % 16 == 0 && a % 16 == 0;
#define CPALS_BF16_NCB(NCB)                                                                                 \
  do {                                                                                                     \
    if constexpr (F8 && KC && (!SPLIT || NCB <= 4) && !(FF && NCB == 8)) {                                 \
      if (deep) return launch_one<KC, NCB, SPLIT, true, F8, true, false, FF>(X, Bhi, Blo, cs, C, P, K, Q, R, Kp, vec, st); \
    }                                                                                                      \
    if constexpr (F8 && !KC) {                                                                             \
      if (tr) return launch_one<KC, NCB, SPLIT, true, F8, false, true, FF>(X, Bhi, Blo, cs, C, P, K, Q, R, Kp, vec, st); \
    }                                                                                                      \
    return fast ? launch_one<KC, NCB, SPLIT, true, F8, false, false, FF>(X, Bhi, Blo, cs, C, P, K, Q, R, Kp, vec, st) \
                : launch_one<KC, NCB, SPLIT, false, F8, false, false, FF>(X, Bhi, Blo, cs, C, P, K, Q, R, Kp, vec, st); \
  } while (0)
  if (R <= 16) CPALS_BF16_NCB(1);
  if (R <= 32) CPALS_BF16_NCB(2);
  // FP8 rows with the split factor: 128 columns in one pass need more than 256
  // registers (spills); two 64-column passes read the tensor twice instead
  if (R <= 64 || (F8 && KC && SPLIT)) CPALS_BF16_NCB(4);
  if constexpr (!(F8 && KC && SPLIT)) CPALS_BF16_NCB(8);  // not instantiated where never taken
#undef CPALS_BF16_NCB
  return hipErrorInvalidValue;
}

template <bool F8>
hipError_t launch_lowp(const void* X, const uint16_t* Bhi, const uint16_t* Blo, float* C, int64_t P, int64_t K,
                       int64_t Q, int R, hipStream_t st) {
  if (R < 1 || R > kMaxRank || K < 1 || P < 1 || Q < 1) return hipErrorInvalidValue;
  const int Kp = bf16_factor_pitch(K);
  if (Q == 1) {
    return Blo ? launch_ncb<true, true, F8>(X, Bhi, Blo, nullptr, C, P, K, Q, R, Kp, st)
               : launch_ncb<true, false, F8>(X, Bhi, Blo, nullptr, C, P, K, Q, R, Kp, st);
  }
  return Blo ? launch_ncb<false, true, F8>(X, Bhi, Blo, nullptr, C, P, K, Q, R, Kp, st)
             : launch_ncb<false, false, F8>(X, Bhi, Blo, nullptr, C, P, K, Q, R, Kp, st);
}

}  // namespace

int bf16_factor_pitch(int64_t K) { return (int)((K + KB - 1) / KB * KB); }

hipError_t launch_split_factor(const float* A, int64_t K, int R, uint16_t* hi, uint16_t* lo, hipStream_t st) {
  const int Kp = bf16_factor_pitch(K);
  const int64_t n = (int64_t)R * Kp;
  const int64_t nb = (n + 255) / 256;
  hipLaunchKernelGGL(k_split_factor, dim3((unsigned)(nb < 4096 ? nb : 4096)), dim3(256), 0, st, A, K, R, Kp, hi, lo);
  return hipGetLastError();
}

hipError_t launch_ttm_bf16(const uint16_t* X, const uint16_t* Bhi, const uint16_t* Blo, float* C, int64_t P,
                           int64_t K, int64_t Q, int R, hipStream_t st) {
  return launch_lowp<false>(X, Bhi, Blo, C, P, K, Q, R, st);
}

hipError_t launch_ttm_fp8(const uint8_t* X, const uint16_t* Bhi, const uint16_t* Blo, float* C, int64_t P,
                          int64_t K, int64_t Q, int R, hipStream_t st) {
  return launch_lowp<true>(X, Bhi, Blo, C, P, K, Q, R, st);
}

hipError_t launch_quant_factor_fp8(const float* A, int64_t K, int R, uint8_t* Bq, float* inv, hipStream_t st) {
  if (R < 1 || R > kMaxRank || K < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_quant_factor_fp8, dim3(R), dim3(256), 0, st, A, K, R, bf16_factor_pitch(K), Bq, inv);
  return hipGetLastError();
}

hipError_t launch_ttm_fp8f8(const uint8_t* X, const uint8_t* Bq, const float* inv, float* C, int64_t P, int64_t K,
                            int64_t Q, int R, hipStream_t st) {
  if (R < 1 || R > kMaxRank || K < 1 || P < 1 || Q < 1) return hipErrorInvalidValue;
  const int Kp = bf16_factor_pitch(K);
  const uint16_t* B = (const uint16_t*)Bq;
  return Q == 1 ? launch_ncb<true, false, true, true>(X, B, nullptr, inv, C, P, K, Q, R, Kp, st)
                : launch_ncb<false, false, true, true>(X, B, nullptr, inv, C, P, K, Q, R, Kp, st);
}

}  // namespace cpals
