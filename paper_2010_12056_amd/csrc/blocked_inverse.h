// Blocked Gauss-Jordan inverse of a small SPD matrix held in LDS, shared by
// the mode-update kernels and the batched path (device code only).
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

namespace cpals {

typedef double gj_f64x4 __attribute__((ext_vector_type(4)));

// The double held by lane `src` (the same for every lane) of the wave.
__device__ __forceinline__ double gj_readlane(double v, int src) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)u, src);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), src);
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
// doubles of LDS through which the diagonal elimination passes each pivot's
// row and column (the form with the fewest registers, for the batched path).
template <int RP, int NW>
__device__ __forceinline__ bool gj_inverse_lds(double* A, double tol, int* fail, double* xb) {
  constexpr int NB = RP / 16;
  constexpr int P = RP + 1;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int l16 = lane & 15, g = lane >> 4;
  if (tid == 0) *fail = 0;
  __syncthreads();
  for (int kb = 0; kb < NB; ++kb) {
    const int k0 = 16 * kb;
    // (1) D <- D^-1 by wave 0.  Lane (g, l16) keeps D[g + 4q][l16], q < 4, in
    // registers; each pivot's row and column pass through LDS (two
    // alternating buffers, one wave-level fence per pivot; the other lanes
    // write a dummy slot).  1 / pivot: the hardware reciprocal refined by two
    // Newton steps y <- y + y (1 - p y) (error a few units in the last place;
    // pivots are positive, far from the exponent limits).
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


template <int S, int N, typename F>
__device__ __forceinline__ void gj_static_for(F&& f) {
  if constexpr (S < N) {
    f(std::integral_constant<int, S>{});
    gj_static_for<S + 1, N>(f);
  }
}

// Lane S of each 16-lane row of the wave, to every lane of that row (DPP row
// broadcast).
template <int S>
__device__ __forceinline__ double gj_rowbcast(double v) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)u, 0x150 + S, 0xF, 0xF, false);
  const unsigned hi = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)(u >> 32), 0x150 + S, 0xF, 0xF, false);
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// The value of 16-lane row G at the same position within the row, to every
// row: the 16-lane swap puts rows 0 and 2 (first result) or 1 and 3 (second)
// in both rows of each pair, the 32-lane swap then the lower (first) or upper
// (second) pair in both halves.
template <int G>
__device__ __forceinline__ unsigned gj_rowsel32(unsigned v) {
  const auto p = __builtin_amdgcn_permlane16_swap(v, v, false, false);
  const unsigned y = (G & 1) ? p[1] : p[0];
  const auto q = __builtin_amdgcn_permlane32_swap(y, y, false, false);
  return (G & 2) ? q[1] : q[0];
}
template <int G>
__device__ __forceinline__ double gj_rowsel(double v) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = gj_rowsel32<G>((unsigned)u), hi = gj_rowsel32<G>((unsigned)(u >> 32));
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// In-place Gauss-Jordan inverse of a 16 x 16 block held by one wave (every
// lane active): lane (g = lane / 16, l16 = lane % 16) holds row l16, columns
// 4 g .. 4 g + 3 in x.  Pivot s: its row reaches each row group from lane s
// of that group (DPP broadcast), its column from group s / 4 (lane swaps),
// its value by readlane, so no step goes through LDS.  1 / pivot: the
// hardware reciprocal refined by two Newton steps.  Returns false (uniform)
// when a pivot is at or below tol; x is then undefined.
__device__ __forceinline__ bool gj_block16(double (&x)[4], double tol) {
  const int lane = threadIdx.x & 63;
  const int g = lane >> 4, l16 = lane & 15;
  bool ok = true;
  gj_static_for<0, 16>([&](auto sc) {
    constexpr int s = decltype(sc)::value;
    constexpr int gs = s >> 2, cs = s & 3;
    const double piv = gj_readlane(x[cs], 16 * gs + s);
    double rb[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) rb[c] = gj_rowbcast<s>(x[c]);
    const double col = gj_rowsel<gs>(x[cs]);  // this lane's row, column s
    ok = ok && (piv > tol);
    double rinv = __builtin_amdgcn_rcp(piv);
    rinv = fma(rinv, fma(-piv, rinv, 1.0), rinv);
    rinv = fma(rinv, fma(-piv, rinv, 1.0), rinv);
    const bool prow = (l16 == s);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const double f = rb[c] * rinv;
      if (c == cs && g == gs)  // column s
        x[c] = prow ? rinv : -col * rinv;
      else
        x[c] = prow ? f : fma(-col, f, x[c]);
    }
  });
  return ok;
}

// In-place inverse of an SPD matrix by blocked Gauss-Jordan elimination
// (16 x 16 blocks, as gj_inverse_lds) by four waves with look-ahead.  On
// entry A (RP x RP in LDS, pitch RP + 1, padded with the identity) holds the
// matrix with its first diagonal block already inverted, *fail set for that
// block, and tol is valid in wave 0.  Block step k (after a barrier): wave 0
// forms the next diagonal block's update A_k+1,k+1 - A_k+1,k D^-1 A_k,k+1 and
// inverts it (gj_block16) while waves 1-3 take the columns j != k: the row
// panel tile D^-1 A_kj, every trailing tile A_ij - A_ik (D^-1 A_kj) of the
// column except that next diagonal block, and the column panel tile
// -A_jk D^-1; the panel tiles are kept in registers and written after a
// second barrier, once every old panel has been read.  In the last step
// wave 0 takes columns too.  Returns false (uniformly) when a pivot is at or
// below tol.
template <int RP>
__device__ __forceinline__ bool gj_inverse_la(double* A, double tol, int* fail) {
  constexpr int NB = RP / 16;
  constexpr int P = RP + 1;
  constexpr int MJ = (NB + 1) / 3 > 0 ? (NB + 1) / 3 : 1;  // columns per wave (NB - 1 over three)
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int g = lane >> 4, l16 = lane & 15;
  for (int k = 0; k < NB; ++k) {
    __syncthreads();
    if (*fail) return false;  // uniform
    const int k0 = 16 * k;
    const bool la = k + 1 < NB;
    const int nw = la ? 3 : 4, w0 = la ? 1 : 0;
    gj_f64x4 rp[MJ], cp[MJ];
    int jc[MJ];
#pragma unroll
    for (int q = 0; q < MJ; ++q) {
      jc[q] = -1;
      const int idx = (wave - w0) + nw * q;  // the wave's q-th column among those != k
      if (wave < w0 || idx >= NB - 1) continue;
      const int j = idx < k ? idx : idx + 1;
      const int j0 = 16 * j;
      gj_f64x4 r = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int t = 0; t < 4; ++t)
        r = __builtin_amdgcn_mfma_f64_16x16x4f64(A[(k0 + l16) * P + k0 + 4 * t + g], A[(k0 + 4 * t + g) * P + j0 + l16],
                                                 r, 0, 0, 0);
      // r[t] is row 4 t + g of D^-1 A_kj at column l16: the operand of index slice t
      for (int i = 0; i < NB; ++i) {
        if (i == k || (la && i == k + 1 && j == k + 1)) continue;
        const int i0 = 16 * i;
        gj_f64x4 acc;
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[v] = A[(i0 + g + 4 * v) * P + j0 + l16];
#pragma unroll
        for (int t = 0; t < 4; ++t)
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(-A[(i0 + l16) * P + k0 + 4 * t + g], r[t], acc, 0, 0, 0);
#pragma unroll
        for (int v = 0; v < 4; ++v) A[(i0 + g + 4 * v) * P + j0 + l16] = acc[v];
      }
      gj_f64x4 c = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int t = 0; t < 4; ++t)
        c = __builtin_amdgcn_mfma_f64_16x16x4f64(A[(j0 + l16) * P + k0 + 4 * t + g], A[(k0 + 4 * t + g) * P + k0 + l16],
                                                 c, 0, 0, 0);
      rp[q] = r;
      cp[q] = c;
      jc[q] = j;
    }
    if (la && wave == 0) {
      const int k1 = k0 + 16;
      gj_f64x4 r = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int t = 0; t < 4; ++t)
        r = __builtin_amdgcn_mfma_f64_16x16x4f64(A[(k0 + l16) * P + k0 + 4 * t + g], A[(k0 + 4 * t + g) * P + k1 + l16],
                                                 r, 0, 0, 0);
      gj_f64x4 d;
#pragma unroll
      for (int v = 0; v < 4; ++v) d[v] = A[(k1 + g + 4 * v) * P + k1 + l16];
#pragma unroll
      for (int t = 0; t < 4; ++t)
        d = __builtin_amdgcn_mfma_f64_16x16x4f64(-A[(k1 + l16) * P + k0 + 4 * t + g], r[t], d, 0, 0, 0);
      // to the elimination's layout through LDS (this block is wave 0's alone in this step)
#pragma unroll
      for (int v = 0; v < 4; ++v) A[(k1 + g + 4 * v) * P + k1 + l16] = d[v];
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      double x[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) x[c] = A[(k1 + l16) * P + k1 + 4 * g + c];
      if (gj_block16(x, tol)) {
#pragma unroll
        for (int c = 0; c < 4; ++c) A[(k1 + l16) * P + k1 + 4 * g + c] = x[c];
      } else if (lane == 0) {
        *fail = 1;
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < MJ; ++q) {
      if (jc[q] < 0) continue;
      const int j0 = 16 * jc[q];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        A[(k0 + g + 4 * v) * P + j0 + l16] = rp[q][v];
        A[(j0 + g + 4 * v) * P + k0 + l16] = -cp[q][v];
      }
    }
  }
  __syncthreads();
  return true;
}

}  // namespace cpals
