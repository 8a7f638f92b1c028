// Blocked Gauss-Jordan inverse of a small SPD matrix held in LDS, shared by
// the mode-update kernels and the batched path (device code only).
#pragma once
#include <hip/hip_runtime.h>

namespace cpals {

typedef double gj_f64x4 __attribute__((ext_vector_type(4)));

// In-place inverse of an SPD matrix by blocked Gauss-Jordan elimination
// without pivoting, 16 x 16 blocks, NW waves (64 NW threads).  A is RP x RP in LDS with
// pitch RP + 1 (padded with the identity).  Block step k, with D the
// diagonal block, row panel A_kj, column panel A_ik, rest A_ij:
//   D <- D^-1 (scalar elimination of the 16 pivots by one wave),
//   A_kj <- D^-1 A_kj,  A_ij <- A_ij - A_ik A_kj (new A_kj),  A_ik <- -A_ik D^-1,
// which is the in-place scalar elimination grouped by 16 pivots: the pivots
// met are the same Schur-complement diagonals.  The panels and the trailing
// update run on the f64 matrix cores.  Returns false (uniformly, A then
// undefined) when a pivot is at or below tol.  xb: 144 doubles of LDS,
// fail: an LDS flag.
template <int RP, int NW = 4>
__device__ inline bool gj_inverse_lds(double* A, double tol, double* xb, int* fail) {
  constexpr int NB = RP / 16;
  constexpr int P = RP + 1;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int l16 = lane & 15, g = lane >> 4;
  if (tid == 0) *fail = 0;
  __syncthreads();
  for (int kb = 0; kb < NB; ++kb) {
    const int k0 = 16 * kb;
    // (1) D <- D^-1 by wave 0.  Lane (g, l16) keeps D[g + 4q][l16], q < 4, in
    // registers; per pivot s the lanes holding row s and column s publish
    // them in LDS (two alternating buffers, so one wave-level fence per pivot
    // suffices; the other lanes write a dummy slot, so no lane branches) and
    // every lane reads the pivot, its row entry and its four column entries
    // back.  1 / pivot: the hardware reciprocal refined by two Newton steps
    // y <- y + y (1 - p y) (error a few units in the last place; pivots are
    // positive, far from the exponent limits).
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
    // (3) A_ij <- A_ij - A_ik A_kj for every block i, j != k
    for (int tt = wave; tt < NB * NB; tt += NW) {
      const int ib = tt / NB, jb = tt - ib * NB;
      if (ib == kb || jb == kb) continue;
      const int i0 = 16 * ib, j0 = 16 * jb;
      gj_f64x4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int t = 0; t < 4; ++t)
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(A[(i0 + l16) * P + k0 + 4 * t + g],
                                                   A[(k0 + 4 * t + g) * P + j0 + l16], acc, 0, 0, 0);
#pragma unroll
      for (int v = 0; v < 4; ++v) A[(i0 + g + 4 * v) * P + j0 + l16] -= acc[v];
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
