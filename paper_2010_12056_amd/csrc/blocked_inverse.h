// Blocked Gauss-Jordan inverse of a small SPD matrix held in LDS, shared by
// the mode-update kernels and the batched path (device code only).
#pragma once
#include <hip/hip_runtime.h>

namespace cpals {

typedef double gj_f64x4 __attribute__((ext_vector_type(4)));

// The double held by lane `src` (the same for every lane) of the wave.
__device__ __forceinline__ double gj_readlane(double v, int src) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)u, src);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), src);
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// The double held by lane `src` (per lane) of the wave; every lane active.
__device__ __forceinline__ double gj_bpermute(double v, int src) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = (unsigned)__builtin_amdgcn_ds_bpermute(src * 4, (int)(unsigned)u);
  const unsigned hi = (unsigned)__builtin_amdgcn_ds_bpermute(src * 4, (int)(unsigned)(u >> 32));
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// In-place inverse of an SPD matrix by blocked Gauss-Jordan elimination
// without pivoting, 16 x 16 blocks, NW waves (64 NW threads).  A is RP x RP in LDS with
// pitch RP + 1 (padded with the identity).  Block step k, with D the
// diagonal block, row panel A_kj, column panel A_ik, rest A_ij:
//   D <- D^-1 (scalar elimination of the 16 pivots by one wave),
//   A_kj <- D^-1 A_kj,  A_ij <- A_ij - A_ik A_kj (new A_kj),  A_ik <- -A_ik D^-1,
// which is the in-place scalar elimination grouped by 16 pivots: the pivots
// met are the same Schur-complement diagonals.  The panels and the trailing
// update run on the f64 matrix cores.  Returns false (uniformly, A then
// undefined) when a pivot is at or below tol.  fail: an LDS flag; xb: 144
// doubles of LDS for the XLANE = false form of the diagonal elimination.
template <int RP, int NW = 4, bool XLANE = true>
__device__ __forceinline__ bool gj_inverse_lds(double* A, double tol, int* fail, double* xb = nullptr) {
  constexpr int NB = RP / 16;
  constexpr int P = RP + 1;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int l16 = lane & 15, g = lane >> 4;
  if (tid == 0) *fail = 0;
  __syncthreads();
  for (int kb = 0; kb < NB; ++kb) {
    const int k0 = 16 * kb;
    // (1) D <- D^-1 by wave 0.  Lane (g, l16) keeps D[g + 4q][l16], q < 4, in
    // registers.  Pivot s: its row entry D[s][l16] comes from
    // lane 16 (s % 4) + l16 and its four column entries D[g + 4q][s] from
    // lane 16 g + s (ds_bpermute, a cross-lane read with no LDS round
    // trip), the pivot D[s][s] from lane 16 (s % 4) + s (readlane).  1 /
    // pivot: the hardware reciprocal refined by two Newton steps
    // y <- y + y (1 - p y) (error a few units in the last place; pivots are
    // positive, far from the exponent limits).
    if constexpr (XLANE) {
      if (wave == 0) {
        double x[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) x[q] = A[(k0 + g + 4 * q) * P + k0 + l16];
        bool ok = true;
#pragma unroll 1
        for (int s = 0; s < 16; ++s) {
          const int qs = s >> 2, gs = s & 3;
          const double xs = qs == 0 ? x[0] : qs == 1 ? x[1] : qs == 2 ? x[2] : x[3];
          const double piv = gj_readlane(xs, 16 * gs + s);
          const double rk = gj_bpermute(xs, 16 * gs + l16);
          double ck[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) ck[q] = gj_bpermute(x[q], 16 * g + s);
          ok = ok && (piv > tol);  // uniform; after a failure the rest is discarded
          double rinv = __builtin_amdgcn_rcp(piv);
          rinv = fma(rinv, fma(-piv, rinv, 1.0), rinv);
          rinv = fma(rinv, fma(-piv, rinv, 1.0), rinv);
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            if (g + 4 * q == s)
              x[q] = (l16 == s) ? rinv : rk * rinv;
            else
              x[q] = (l16 == s) ? -ck[q] * rinv : x[q] - ck[q] * rk * rinv;
          }
        }
        if (ok) {
#pragma unroll
          for (int q = 0; q < 4; ++q) A[(k0 + g + 4 * q) * P + k0 + l16] = x[q];
        } else if (lane == 0) {
          *fail = 1;
        }
      }
    } else {
      // the same elimination with the row and column of each pivot passed
      // through LDS (two alternating buffers, one wave-level fence per pivot;
      // the other lanes write a dummy slot): fewer registers
      if (wave == 0) {
        double x[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) x[q] = A[(k0 + g + 4 * q) * P + k0 + l16];
        bool ok = true;
#pragma unroll 1
        for (int s = 0; s < 16; ++s) {
          double* rowb = xb + 32 * (s & 1);  // [0, 16): row s, [16, 32): column s
          double* colb = rowb + 16;
          double* dummy = xb + 64;           // 80 slots nobody reads
          double* rw = (g == (s & 3)) ? rowb + l16 : dummy + lane;
          double* cw = (l16 == s) ? colb + g : dummy + lane;
          const int qs = s >> 2;
          *rw = qs == 0 ? x[0] : qs == 1 ? x[1] : qs == 2 ? x[2] : x[3];
#pragma unroll
          for (int q = 0; q < 4; ++q) cw[4 * q] = x[q];
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
          __builtin_amdgcn_wave_barrier();
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
          const double piv = rowb[s];
          const double rk = rowb[l16];
          double ck[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) ck[q] = colb[g + 4 * q];
          ok = ok && (piv > tol);  // uniform in the wave; after a failure the rest is discarded
          double rinv = __builtin_amdgcn_rcp(piv);
          rinv = fma(rinv, fma(-piv, rinv, 1.0), rinv);
          rinv = fma(rinv, fma(-piv, rinv, 1.0), rinv);
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            if (g + 4 * q == s)
              x[q] = (l16 == s) ? rinv : rk * rinv;
            else
              x[q] = (l16 == s) ? -ck[q] * rinv : x[q] - ck[q] * rk * rinv;
          }
        }
        if (ok) {
#pragma unroll
          for (int q = 0; q < 4; ++q) A[(k0 + g + 4 * q) * P + k0 + l16] = x[q];
        } else if (lane == 0) {
          *fail = 1;
        }
      }
    }
    __syncthreads();
    if (*fail) return false;  // uniform
    // (2) row panel A_kj <- D^-1 A_kj, one 16 x 16 tile per wave at a time
    for (int jb = wave; jb < NB; jb += NW) {
      if (jb == kb) continue;
      const int j0 = 16 * jb;
      gj_f64x4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int t = 0; t < 4; ++t)
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(A[(k0 + l16) * P + k0 + 4 * t + g],
                                                   A[(k0 + 4 * t + g) * P + j0 + l16], acc, 0, 0, 0);
      __builtin_amdgcn_wave_barrier();
#pragma unroll
      for (int v = 0; v < 4; ++v) A[(k0 + g + 4 * v) * P + j0 + l16] = acc[v];
    }
    __syncthreads();
    // (3) A_ij <- A_ij - A_ik A_kj for every block i, j != k: each wave takes
    // tiles wave, wave + NW, ..., up to four at a time, with every operand loaded
    // before the first product and the four accumulation chains interleaved
    constexpr int TPW = (NB * NB + NW - 1) / NW;
    constexpr int GT = TPW < 4 ? TPW : 4;  // tiles per group
#pragma unroll 1
    for (int t0 = 0; t0 < TPW; t0 += GT) {
      gj_f64x4 acc[GT];
      double av[GT][4], bv[GT][4];
      bool use[GT];
      int ti[GT], tj[GT];
#pragma unroll
      for (int t = 0; t < GT; ++t) {
        const int tt = wave + NW * (t0 + t);
        const int ib = tt / NB, jb = tt - ib * NB;
        use[t] = t0 + t < TPW && tt < NB * NB && ib != kb && jb != kb;
        ti[t] = use[t] ? 16 * ib : 0;
        tj[t] = use[t] ? 16 * jb : 0;
        acc[t] = gj_f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          av[t][u] = A[(ti[t] + l16) * P + k0 + 4 * u + g];
          bv[t][u] = A[(k0 + 4 * u + g) * P + tj[t] + l16];
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int t = 0; t < GT; ++t) acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[t][u], bv[t][u], acc[t], 0, 0, 0);
#pragma unroll
      for (int t = 0; t < GT; ++t)
        if (use[t]) {
#pragma unroll
          for (int v = 0; v < 4; ++v) A[(ti[t] + g + 4 * v) * P + tj[t] + l16] -= acc[t][v];
        }
    }
    __syncthreads();
    // (4) column panel A_ik <- -A_ik D^-1
    for (int ib = wave; ib < NB; ib += NW) {
      if (ib == kb) continue;
      const int i0 = 16 * ib;
      gj_f64x4 acc = {0.0, 0.0, 0.0, 0.0};
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
  return true;
}

}  // namespace cpals
