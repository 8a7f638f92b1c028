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
  for (int64_t r = 0; r < s; ++r) acc += A[r * R + a] * A[r * R + b];
  S[e] = acc;
}

// Gamma^(n), its inverse and (PP) the bracket of Eq. (7).  One workgroup.
__global__ __launch_bounds__(256) void k_prep(PrepArgs a) {
  extern __shared__ double lds[];
  double* g = lds;              // R x R, inverted in place
  double* col = lds + a.R * a.R;  // R
  __shared__ int fail;
  __shared__ double maxdiag;
  const int tid = threadIdx.x, R = a.R, RR = R * R;
  for (int e = tid; e < RR; e += 256) {
    double v = 1.0;
    for (int m = 0; m < a.N; ++m)
      if (m != a.n) v *= a.S[m][e];
    g[e] = v;
    a.Gamma[e] = v;
    if (a.pp) {
      // coefficient of t^2 in the Hadamard product over m != n of (S + t dS)
      double e0 = 1.0, e1 = 0.0, e2 = 0.0;
      for (int m = 0; m < a.N; ++m) {
        if (m == a.n) continue;
        const double s = a.S[m][e], ds = a.dS[m][e];
        e2 = e2 * s + e1 * ds;
        e1 = e1 * s + e0 * ds;
        e0 = e0 * s;
      }
      a.W[e] = e2;
    }
  }
  if (tid == 0) fail = 0;
  __syncthreads();
  if (tid == 0) {
    double m = 0.0;
    for (int i = 0; i < R; ++i) m = fmax(m, g[i * R + i]);
    maxdiag = m;
  }
  __syncthreads();
  const double tol = maxdiag * (double)R * 2.220446049250313e-16;
  // Gauss-Jordan inversion without pivoting (Gamma is SPD; pivots are the
  // positive Schur-complement diagonals).
  for (int k = 0; k < R; ++k) {
    const double piv = g[k * R + k];
    if (!(piv > tol)) {  // uniform across the block: every thread read the same value
      if (tid == 0) fail = 1;
      break;
    }
    for (int i = tid; i < R; i += 256) col[i] = g[i * R + k];
    __syncthreads();
    for (int j = tid; j < R; j += 256) g[k * R + j] = (j == k ? 1.0 : g[k * R + j]) / piv;
    __syncthreads();
    for (int e = tid; e < RR; e += 256) {
      const int i = e / R, j = e - i * R;
      if (i != k) g[e] = (j == k ? 0.0 : g[e]) - col[i] * g[k * R + j];
    }
    __syncthreads();
  }
  __syncthreads();
  if (fail) {
    for (int e = tid; e < RR; e += 256) a.Ginv[e] = 0.0;
    if (tid == 0) a.stats->status |= 1;
  } else {
    // symmetrize the result (the exact inverse is symmetric)
    for (int e = tid; e < RR; e += 256) {
      const int i = e / R, j = e - i * R;
      a.Ginv[e] = 0.5 * (g[e] + g[j * R + i]);
    }
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_solve(SolveArgs<T> a) {
  __shared__ double Mt[kSolveRows * kMaxRank];
  __shared__ double An[kSolveRows * kMaxRank];
  __shared__ double dAn[kSolveRows * kMaxRank];
  __shared__ double sh[256];
  const int tid = threadIdx.x, R = a.R;
  const int64_t r0 = (int64_t)blockIdx.x * kSolveRows;
  const int rows = (int)((a.s - r0) < kSolveRows ? (a.s - r0) : kSolveRows);
  const int nel = rows * R;
  for (int e = tid; e < nel; e += 256) {
    Mt[e] = a.M[r0 * R + e];
    if (a.pp) An[e] = a.A[r0 * R + e];
  }
  __syncthreads();
  if (a.pp) {
    // M~ = M + V^(n), V^(n) = A^(n) W with the current (old) A^(n)  (Eq. (7))
    for (int e = tid; e < nel; e += 256) {
      const int r = e / R, c = e - r * R;
      double v = 0.0;
      for (int j = 0; j < R; ++j) v += An[r * R + j] * a.W[j * R + c];
      Mt[e] += v;
    }
    __syncthreads();
  }
  double nA2 = 0.0, nd2 = 0.0, ma = 0.0;
  for (int e = tid; e < nel; e += 256) {
    const int r = e / R, c = e - r * R;
    double v = 0.0;
    for (int j = 0; j < R; ++j) v += Mt[r * R + j] * a.Ginv[j * R + c];
    const int64_t gi = r0 * R + e;
    double d;
    if (a.pp) {
      d = v - a.Ap[gi];
      a.dAsh[gi] = (T)d;
    } else {
      d = v - a.A[gi];
    }
    a.A[gi] = v;
    a.Ash[gi] = (T)v;
    An[e] = v;
    dAn[e] = d;
    nA2 += v * v;
    nd2 += d * d;
    ma += Mt[e] * v;
  }
  __syncthreads();
  const int RR = R * R;
  double* pS = a.partS + (int64_t)blockIdx.x * RR;
  double* pdS = a.pp ? a.partdS + (int64_t)blockIdx.x * RR : nullptr;
  for (int e = tid; e < RR; e += 256) {
    const int i = e / R, j = e - i * R;
    double s = 0.0, ds = 0.0;
    for (int r = 0; r < rows; ++r) {
      s += An[r * R + i] * An[r * R + j];
      if (a.pp) ds += An[r * R + i] * dAn[r * R + j];
    }
    pS[e] = s;
    if (a.pp) pdS[e] = ds;
  }
  const double t0 = block_sum(nA2, sh);
  const double t1 = block_sum(nd2, sh);
  const double t2 = block_sum(ma, sh);
  if (tid == 0) {
    a.partSc[blockIdx.x * 4 + 0] = t0;
    a.partSc[blockIdx.x * 4 + 1] = t1;
    a.partSc[blockIdx.x * 4 + 2] = t2;
    a.partSc[blockIdx.x * 4 + 3] = 0.0;
  }
}

__global__ __launch_bounds__(256) void k_finalize(FinalArgs a) {
  __shared__ double sh[256];
  const int tid = threadIdx.x, RR = a.R * a.R;
  double g = 0.0;
  for (int e = tid; e < RR; e += 256) {
    double s = 0.0, ds = 0.0;
    for (int b = 0; b < a.nblk; ++b) {
      s += a.partS[(int64_t)b * RR + e];
      if (a.pp) ds += a.partdS[(int64_t)b * RR + e];
    }
    a.S[e] = s;
    if (a.pp) a.dS[e] = ds;
    if (a.last) g += a.Gamma[e] * s;
  }
  const double gs = block_sum(g, sh);
  if (tid == 0) {
    double nA2 = 0.0, nd2 = 0.0, ma = 0.0;
    for (int b = 0; b < a.nblk; ++b) {
      nA2 += a.partSc[b * 4 + 0];
      nd2 += a.partSc[b * 4 + 1];
      ma += a.partSc[b * 4 + 2];
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
  const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t sn = a.dims[a.n];
  if (g >= sn * a.R) return;
  const int64_t x = g / a.R;
  const int r = (int)(g - x * a.R);
  double acc = a.Mp[g];
  for (int i = 0; i < a.N; ++i) {
    if (i == a.n) continue;
    const int64_t si = a.dims[i];
    const T* P = a.pair[i];
    const T* d = a.dA[i];
    double u = 0.0;
    if (a.pair_n_first[i]) {
      const T* p = P + x * si * a.R + r;  // P[x][y][r]
      for (int64_t y = 0; y < si; ++y) u += (double)p[y * a.R] * (double)d[y * a.R + r];
    } else {
      const T* p = P + x * a.R + r;  // P[y][x][r]
      for (int64_t y = 0; y < si; ++y) u += (double)p[y * sn * a.R] * (double)d[y * a.R + r];
    }
    acc += u;
  }
  a.M[g] = acc;
}

inline unsigned nblocks(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

template <typename T>
hipError_t launch_ttm(const T* X, const T* B, T* C, int64_t P, int64_t K, int64_t Q, int R,
                      hipStream_t st) {
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

hipError_t launch_prep(const PrepArgs& a, hipStream_t st) {
  const size_t lds = ((size_t)a.R * a.R + a.R) * sizeof(double);
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void*)k_prep, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)(((size_t)kMaxRank * kMaxRank + kMaxRank) * sizeof(double)));
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  hipLaunchKernelGGL(k_prep, dim3(1), dim3(256), lds, st, a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_solve(const SolveArgs<T>& a, int nblk, hipStream_t st) {
  hipLaunchKernelGGL((k_solve<T>), dim3(nblk), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_finalize(const FinalArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(256), 0, st, a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_pp_mttkrp(const PPArgs<T>& a, hipStream_t st) {
  const int64_t n = a.dims[a.n] * a.R;
  hipLaunchKernelGGL((k_pp_mttkrp<T>), dim3(nblocks(n)), dim3(256), 0, st, a);
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
template hipError_t launch_norm2<double>(const double*, int64_t, double*, int, DevStats*,
                                         hipStream_t);
template hipError_t launch_solve<float>(const SolveArgs<float>&, int, hipStream_t);
template hipError_t launch_solve<double>(const SolveArgs<double>&, int, hipStream_t);
template hipError_t launch_pp_mttkrp<float>(const PPArgs<float>&, hipStream_t);
template hipError_t launch_pp_mttkrp<double>(const PPArgs<double>&, hipStream_t);

}  // namespace cpals
