// First-level contraction of an FP32 tensor with one factor on the BF16
// matrix cores (v_mfma_f32_16x16x32_bf16, FP32 accumulation) to about FP32
// accuracy:
//   C[p][q][r] = sum_k X[p][k][q] * B[k][r]
// Not from the paper (it computes in FP64): a precision path of the first
// contraction, which reads the tensor once and dominates the sweep.
//
// Every FP32 value is the exact sum of three BF16 values: x1 = x rounded to
// BF16 (nearest even), x2 = x - x1 rounded the same way, x3 = x - x1 - x2;
// both subtractions are exact (x - x1 keeps the low 16 significand bits of x,
// x - x1 - x2 at most 8, which BF16 holds).  With the factor split the same
// way (|x2| <= 2^-8 |x|, |x3| <= 2^-16 |x|), x b is the sum of nine BF16
// products, each exact in FP32; the six kept here are x1 b1, x1 b2, x2 b1,
// x1 b3, x3 b1 and x2 b2; the three dropped ones (x2 b3, x3 b2, x3 b3) are
// below 2^-23 |x b| together and, since rounding to nearest gives the later
// parts either sign, carry no systematic bias (truncated parts would all
// share the sign of x and bias every sum); the sums are FP32 accumulations
// as on the FP32 matrix cores.
//
// Operand layout of the 16x16x32 BF16 instruction: lane l supplies row l % 16
// of A and column l % 16 of B, each with the eight contraction indices
// 8 (l / 16) .. + 7 of the step; register v of lane l holds C[4 (l / 16) + v]
// [l % 16].
//
// Workgroup: eight waves; a tile of 128 U output rows (KC: rows p of X; else
// rows (p, q) numbered p Q + q, so a short Q does not leave tiles part
// empty), each wave 16 U rows as U 16-row blocks u (four, or two with four
// column blocks), times the
// workgroup's 16 NCB factor columns.  The three factor parts (Bt[part][c][k],
// k contiguous, zero past K) go through LDS in chunks of 64 indices,
// double-buffered (the next chunk is loaded into registers while the current
// one is used and stored into the other buffer after it; one barrier per
// chunk).  A long contraction is split over workgroup layers z (blockIdx.z
// takes a range of chunks and writes its partial product; k_sum_layers adds
// the partials in z order) when there are too few tiles to fill the chip.
// The tensor goes from HBM to registers one step (32 indices) ahead of the
// matrix cores and is split there:
//   KC (Q == 1, X is P x K row-major, K a multiple of 8, rows 16-byte
//      aligned): lane (i, g) of block u loads row 16 u + i, indices
//      8 g .. 8 g + 7 of the step, as two 16-byte loads (indices past K read
//      the row's last eight, cancelled by the factor's zero padding);
//   otherwise (X[p] is K x Q, q contiguous): lane (i, g) of block u loads
//      its row's X[p][k][q] for its eight k, 16 lanes on 64 contiguous bytes
//      when Q is a multiple of 16 (k past K reads index K - 1, rows past the
//      end the last row, never stored).
// The five smaller products of one step are summed from zero and then added
// to the running sum (which takes the large product x1 b1) with an FP32
// add: added to a large running sum one by one, their low bits are dropped
// inside the matrix instruction, a bias that grows with K (-4.8e-8 relative
// at K = 16384 with a single running sum).  Two column blocks are in flight,
// eight independent chains.
#include "kernels.h"

namespace cpals {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int kWaves = 8;
constexpr int kThreads = kWaves * 64;
// 16-row blocks per wave: four, or two with four column blocks (registers)
constexpr int x3_blocks(int ncb) { return ncb >= 4 ? 2 : 4; }
constexpr int kStepK = 32;
constexpr int kChunk = 64;  // factor indices per staged chunk (bf16_factor_pitch pads K to it)

}  // namespace
int ttm_x3_layers(int64_t P, int64_t K, int64_t Q, int R);
namespace {

int ttm_x3_cus() {
  static int cus = 0;
  if (cus == 0) {
    int dev = 0, n = 256;
    if (hipGetDevice(&dev) == hipSuccess && hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && n > 0)
      cus = n;
    else
      cus = 256;
  }
  return cus;
}

__device__ inline bf16x8 as_bf16x8(u32x4 v) { return __builtin_bit_cast(bf16x8, v); }

// x rounded to BF16 (nearest, ties to even), as the FP32 bit pattern.
__device__ __forceinline__ uint32_t rne16(float x) {
  const uint32_t u = __float_as_uint(x);
  return (u + 0x7fffu + ((u >> 16) & 1u)) & 0xffff0000u;
}

// The three BF16 parts (bit patterns) of x: x == x1 + x2 + x3 exactly, each
// part rounded to nearest, so the parts after the first have either sign.
__device__ __forceinline__ void split3(float x, uint32_t& h1, uint32_t& h2, uint32_t& h3) {
  const uint32_t u1 = rne16(x);
  const float r1 = x - __uint_as_float(u1);
  const uint32_t u2 = rne16(r1);
  const float r2 = r1 - __uint_as_float(u2);
  h1 = u1 >> 16;
  h2 = u2 >> 16;
  h3 = __float_as_uint(r2) >> 16;
}

// Bt[part][c][k] = part of A[k][c] for k < K, zero for K <= k < Kp.
__global__ __launch_bounds__(256) void k_split3_factor(const float* __restrict__ A, int64_t K, int R, int Kp,
                                                       uint16_t* __restrict__ Bt) {
  const int64_t n = (int64_t)R * Kp;
  for (int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x; idx < n; idx += (int64_t)gridDim.x * 256) {
    const int64_t c = idx / Kp, k = idx - c * Kp;
    uint32_t h1 = 0, h2 = 0, h3 = 0;
    if (k < K) split3(A[k * R + c], h1, h2, h3);
    Bt[idx] = (uint16_t)h1;
    Bt[n + idx] = (uint16_t)h2;
    Bt[2 * n + idx] = (uint16_t)h3;
  }
}

template <bool KC, int NCB>
__global__ __launch_bounds__(kThreads) void k_ttm_x3(const float* __restrict__ X, const uint16_t* __restrict__ Bt,
                                                     float* __restrict__ C, int64_t P, int K, int64_t Q, int R, int Kp,
                                                     int64_t ntiles, int cps) {
  constexpr int NC = NCB * 16;
  constexpr int U = x3_blocks(NCB);                          // 16-row blocks per wave
  constexpr int TILE = kWaves * 16 * U;                      // rows per workgroup tile
  constexpr int PITCH = kChunk + 8;                          // BF16 elements per staged column
  constexpr int BUF = 3 * NC * PITCH;                        // one staged chunk, three parts
  constexpr int PIECES = 3 * NC * (kChunk / 8);              // 16-byte pieces of a chunk
  constexpr int BPER = (PIECES + kThreads - 1) / kThreads;
  __shared__ __align__(16) uint16_t Bs[2 * BUF];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform (not inferred from tid / 64)
  const int g = lane >> 4, l16 = lane & 15;
  const int c0 = blockIdx.y * NC;
  const int64_t n = (int64_t)R * Kp;
  const int nch = Kp / kChunk;
  const int cbeg = (int)blockIdx.z * cps;
  const int cend = cbeg + cps < nch ? cbeg + cps : nch;
  C += (int64_t)blockIdx.z * P * Q * R;  // split K: this layer's partial product

  // a factor chunk: columns c0 .. c0 + NC - 1 (past R: column R - 1, its
  // products never stored), indices ch kChunk .. + kChunk - 1, three parts
  auto piece = [&](int q, int& part, int& c, int& j) {
    int idx = tid + kThreads * q;
    idx = idx < PIECES ? idx : PIECES - 1;
    part = idx / (NC * (kChunk / 8));
    const int rem = idx - part * NC * (kChunk / 8);
    c = rem / (kChunk / 8);
    j = rem - c * (kChunk / 8);
  };
  auto load_b = [&](int ch, u32x4 (&bv)[BPER]) {
#pragma unroll
    for (int q = 0; q < BPER; ++q) {
      int part, c, j;
      piece(q, part, c, j);
      const int col = c0 + c < R ? c0 + c : R - 1;
      bv[q] = *(const u32x4*)(Bt + part * n + (int64_t)col * Kp + (int64_t)ch * kChunk + 8 * j);
    }
  };
  auto store_b = [&](int buf, const u32x4 (&bv)[BPER]) {
#pragma unroll
    for (int q = 0; q < BPER; ++q) {
      int part, c, j;
      piece(q, part, c, j);
      *(u32x4*)(Bs + buf * BUF + (part * NC + c) * PITCH + 8 * j) = bv[q];
    }
  };

  // the lane's eight values of global step gs (indices 32 gs + 8 g .. + 7)
  auto load = [&](int64_t tile, int gs, float (&x)[U][8]) {
    const int kb = kStepK * gs + 8 * g;
    if (KC) {
      const int64_t r0 = tile * TILE + wave * 16 * U;
      const int kc = kb <= K - 8 ? kb : K - 8;
#pragma unroll
      for (int u = 0; u < U; ++u) {
        int64_t row = r0 + 16 * u + l16;
        row = row < P ? row : P - 1;
        const f32x4 v0 = *(const f32x4*)(X + row * K + kc);
        const f32x4 v1 = *(const f32x4*)(X + row * K + kc + 4);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          x[u][j] = v0[j];
          x[u][4 + j] = v1[j];
        }
      }
    } else {
      // rows (p, q) numbered p Q + q; 32-bit byte offsets from X (the
      // tensor is below 4 GiB, ttm_x3_fits)
      const uint32_t r0 = (uint32_t)tile * TILE + wave * 16 * U;
      const uint32_t Qb = (uint32_t)Q * 4u;
      const uint32_t nrow = (uint32_t)(P * Q);
#pragma unroll
      for (int u = 0; u < U; ++u) {
        uint32_t row = r0 + 16 * u + l16;
        row = row < nrow ? row : nrow - 1;
        const uint32_t p = row / (uint32_t)Q, q = row - p * (uint32_t)Q;
        const uint32_t off = (p * (uint32_t)K * (uint32_t)Q + q) * 4u;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const uint32_t k = (uint32_t)(kb + j < K ? kb + j : K - 1);
          x[u][j] = *(const float*)((const char*)X + (off + k * Qb));
        }
      }
    }
  };

  const int gs0 = cbeg * (kChunk / kStepK), gs1 = cend * (kChunk / kStepK);
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    f32x4 acc[U][NCB];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) acc[u][cb] = f32x4{0.f, 0.f, 0.f, 0.f};
    {
      u32x4 bv[BPER];
      load_b(cbeg, bv);
      store_b(0, bv);
    }
    __syncthreads();
    float xn[U][8];
    load(tile, gs0, xn);
    int buf = 0;
    for (int ch = cbeg; ch < cend; ++ch) {
      const bool more = ch + 1 < cend;
      u32x4 bv[BPER];
      if (more) load_b(ch + 1, bv);
#pragma unroll
      for (int s = 0; s < kChunk / kStepK; ++s) {
        const int gs = ch * (kChunk / kStepK) + s;
        // split this step's values; the next step's loads go out meanwhile
        u32x4 a1[U], a2[U], a3[U];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
          for (int w = 0; w < 4; ++w) {
            uint32_t h1a, h2a, h3a, h1b, h2b, h3b;
            split3(xn[u][2 * w], h1a, h2a, h3a);
            split3(xn[u][2 * w + 1], h1b, h2b, h3b);
            a1[u][w] = h1a | (h1b << 16);
            a2[u][w] = h2a | (h2b << 16);
            a3[u][w] = h3a | (h3b << 16);
          }
        load(tile, gs + 1 < gs1 ? gs + 1 : gs, xn);
        __builtin_amdgcn_sched_barrier(0);
        const int ko = kStepK * s + 8 * g;
        // per column block: the five small products summed from zero (so
        // that they are not added to the large running sums, whose rounding
        // inside the matrix instruction would drop their low bits, a bias
        // that grows with K), then added to the running sum, which takes the
        // large product
        constexpr int CG = NCB == 1 ? 1 : 2;  // column blocks in flight: U CG independent chains
#pragma unroll
        for (int cb0 = 0; cb0 < NCB; cb0 += CG) {
          bf16x8 b1[CG], b2[CG], b3[CG];
#pragma unroll
          for (int i = 0; i < CG; ++i) {
            const uint16_t* bp = Bs + buf * BUF + ((cb0 + i) * 16 + l16) * PITCH + ko;
            b1[i] = as_bf16x8(*(const u32x4*)bp);
            b2[i] = as_bf16x8(*(const u32x4*)(bp + NC * PITCH));
            b3[i] = as_bf16x8(*(const u32x4*)(bp + 2 * NC * PITCH));
          }
          f32x4 t[CG][U];
#pragma unroll
          for (int i = 0; i < CG; ++i)
#pragma unroll
            for (int u = 0; u < U; ++u)
              t[i][u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(a2[u]), b2[i], f32x4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
#pragma unroll
          for (int i = 0; i < CG; ++i)
#pragma unroll
            for (int u = 0; u < U; ++u)
              t[i][u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(a3[u]), b1[i], t[i][u], 0, 0, 0);
#pragma unroll
          for (int i = 0; i < CG; ++i)
#pragma unroll
            for (int u = 0; u < U; ++u)
              t[i][u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(a1[u]), b3[i], t[i][u], 0, 0, 0);
#pragma unroll
          for (int i = 0; i < CG; ++i)
#pragma unroll
            for (int u = 0; u < U; ++u)
              t[i][u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(a2[u]), b1[i], t[i][u], 0, 0, 0);
#pragma unroll
          for (int i = 0; i < CG; ++i)
#pragma unroll
            for (int u = 0; u < U; ++u)
              t[i][u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(a1[u]), b2[i], t[i][u], 0, 0, 0);
#pragma unroll
          for (int i = 0; i < CG; ++i)
#pragma unroll
            for (int u = 0; u < U; ++u)
              acc[u][cb0 + i] =
                  __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(a1[u]), b1[i], acc[u][cb0 + i], 0, 0, 0);
#pragma unroll
          for (int i = 0; i < CG; ++i)
#pragma unroll
            for (int u = 0; u < U; ++u) acc[u][cb0 + i] += t[i][u];
        }
      }
      // the next chunk into the other buffer (nobody reads it since the last
      // barrier); one barrier per chunk
      if (more) store_b(buf ^ 1, bv);
      __syncthreads();
      buf ^= 1;
    }
    // store: register v of block u holds row 16 u + 4 g + v, column l16
    // (C[p][q][r] is row p Q + q of a P Q x R matrix)
    const int64_t row0 = tile * TILE + wave * 16 * U;
    const int64_t nrows = P * Q;
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int64_t row = row0 + 16 * u + 4 * g + v;
          const int c = c0 + cb * 16 + l16;
          if (row < nrows && c < R) C[row * R + c] = acc[u][cb][v];
        }
  }
}

// C[i] = sum over z of parts[z][i] in z order (16-byte pieces; n a multiple of 4).
__global__ __launch_bounds__(256) void k_sum_layers(const float* __restrict__ parts, float* __restrict__ C, int64_t n,
                                                    int Z) {
  const int64_t nv = n / 4;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < nv; i += (int64_t)gridDim.x * 256) {
    f32x4 acc = ((const f32x4*)parts)[i];
    for (int z = 1; z < Z; ++z) acc += ((const f32x4*)(parts + (int64_t)z * n))[i];
    ((f32x4*)C)[i] = acc;
  }
}

template <bool KC, int NCB>
hipError_t launch_x3(const float* X, const uint16_t* Bt, float* C, int64_t P, int64_t K, int64_t Q, int R,
                     float* parts, hipStream_t st) {
  const int Kp = bf16_factor_pitch(K);
  const int64_t tile = kWaves * 16 * x3_blocks(NCB);
  const int64_t ntiles = (P * Q + tile - 1) / tile;
  const unsigned gy = (unsigned)((R + NCB * 16 - 1) / (NCB * 16));
  const int cus = ttm_x3_cus();
  const int64_t want = (int64_t)cus * 2 / gy;
  const unsigned gx = (unsigned)(ntiles < want ? ntiles : (want > 0 ? want : 1));
  const int nch = Kp / kChunk;
  const int Z = parts ? ttm_x3_layers(P, K, Q, R) : 1;
  const int cps = (nch + Z - 1) / Z;
  const int z = (nch + cps - 1) / cps;
  hipLaunchKernelGGL((k_ttm_x3<KC, NCB>), dim3(gx, gy, (unsigned)z), dim3(kThreads), 0, st, X, Bt,
                     z > 1 ? parts : C, P, (int)K, Q, R, Kp, ntiles, cps);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || z == 1) return e;
  const int64_t nn = P * Q * R;
  const int64_t nb = (nn / 4 + 255) / 256;
  hipLaunchKernelGGL(k_sum_layers, dim3((unsigned)(nb < 2048 ? nb : 2048)), dim3(256), 0, st, parts, C, nn, z);
  return hipGetLastError();
}

}  // namespace

bool ttm_x3_fits(int64_t P, int64_t K, int64_t Q, int R, const void* X) {
  if (K < 1 || R < 1 || P < 1 || Q < 1) return false;
  if (Q == 1) return K % 8 == 0 && ((uintptr_t)X % 16) == 0;
  return (double)P * (double)K * (double)Q * 4.0 < 4294967296.0;
}

int ttm_x3_layers(int64_t P, int64_t K, int64_t Q, int R) {
  const int ncb = R <= 16 ? 1 : R <= 32 ? 2 : 4;
  const int64_t tile = kWaves * 16 * x3_blocks(ncb);
  const int64_t ntiles = (P * Q + tile - 1) / tile;
  const int64_t gy = (R + 16 * ncb - 1) / (16 * ncb);
  const int64_t wgs = ntiles * gy;
  const int cus = ttm_x3_cus();
  const int nch = bf16_factor_pitch(K) / kChunk;
  if (wgs >= cus || (P * Q * R) % 4 != 0) return 1;
  int64_t z = (cus + wgs - 1) / wgs;
  if (z > nch / 2) z = nch / 2;  // at least two chunks per layer
  if (z > kMaxSplitLayers) z = kMaxSplitLayers;
  return z < 1 ? 1 : (int)z;
}

hipError_t launch_split3_factor(const float* A, int64_t K, int R, uint16_t* Bt, hipStream_t st) {
  const int Kp = bf16_factor_pitch(K);
  const int64_t n = (int64_t)R * Kp;
  const int64_t nb = (n + 255) / 256;
  hipLaunchKernelGGL(k_split3_factor, dim3((unsigned)(nb < 1024 ? nb : 1024)), dim3(256), 0, st, A, K, R, Kp, Bt);
  return hipGetLastError();
}

hipError_t launch_ttm_x3(const float* X, const uint16_t* Bt, float* C, int64_t P, int64_t K, int64_t Q, int R,
                         float* parts, hipStream_t st) {
  if (!ttm_x3_fits(P, K, Q, R, X)) return hipErrorInvalidValue;
  const bool kc = Q == 1;
  if (R <= 16)
    return kc ? launch_x3<true, 1>(X, Bt, C, P, K, Q, R, parts, st) : launch_x3<false, 1>(X, Bt, C, P, K, Q, R, parts, st);
  if (R <= 32)
    return kc ? launch_x3<true, 2>(X, Bt, C, P, K, Q, R, parts, st) : launch_x3<false, 2>(X, Bt, C, P, K, Q, R, parts, st);
  return kc ? launch_x3<true, 4>(X, Bt, C, P, K, Q, R, parts, st) : launch_x3<false, 4>(X, Bt, C, P, K, Q, R, parts, st);
}

}  // namespace cpals
