// Internal launch interface of the gfx950 kernels (not part of the C ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cpals {

// Device-resident scalars of a plan.
struct DevStats {
  double normT2;      // ||T||_F^2
  double fit_num;     // ||T||^2 + <Gamma^(N), S^(N)> - 2 <M^(N), A^(N)>
  double r;           // relative residual, Eq. (3)
  double normA2[8];   // ||A^(i)||_F^2 after its last update
  double normdA2[8];  // ||dA^(i)||_F^2 (per-sweep change, or A - A_p in the PP phase)
  int status;         // bit 0: a Gamma had non-finite entries; bit 1: non-finite residual
  int pinv_pending;   // set by the elimination when a pivot fell below its tolerance
  int pinv_count;     // updates that used the pseudo-inverse (cumulative)
  unsigned ticket;    // arrival counter of k_update (0 between launches)
  int r_clamped;      // the last residual's Eq. (3) numerator was negative (r reported as 0)
};

// A BF16 tensor element: the upper 16 bits of an FP32 value.
struct bf16 {
  uint16_t bits;
  __device__ explicit operator double() const { return (double)__uint_as_float((uint32_t)bits << 16); }
};

// An FP8 E4M3 tensor element (bias 7, no infinities), decoded exactly by the
// hardware conversion.
struct fp8e4m3 {
  uint8_t bits;
  __device__ explicit operator double() const {
    return (double)__builtin_amdgcn_cvt_pk_f32_fp8((int)bits, false)[0];
  }
};

constexpr int kMaxOrder = 8;
constexpr int kMaxRank = 128;

// C[p][q][r] = sum_k X[p][k][q] * B[k][r]  (Q == 1: X is [P][K] row-major).
template <typename T>
hipError_t launch_ttm(const T* X, const T* B, T* C, int64_t P, int64_t K, int64_t Q, int R,
                      hipStream_t st);

// BF16 tensor path of the first contraction (FP32 accumulation, FP32 C):
// the factor is first written transposed in BF16, Bt[c][k] with pitch
// bf16_factor_pitch(K), and, for the split product, its remainder Blo.
int bf16_factor_pitch(int64_t K);
hipError_t launch_split_factor(const float* A, int64_t K, int R, uint16_t* hi, uint16_t* lo, hipStream_t st);
hipError_t launch_ttm_bf16(const uint16_t* X, const uint16_t* Bhi, const uint16_t* Blo, float* C, int64_t P,
                           int64_t K, int64_t Q, int R, hipStream_t st);
// The same with an FP8 (E4M3) tensor, widened exactly to BF16 in registers.
hipError_t launch_ttm_fp8(const uint8_t* X, const uint16_t* Bhi, const uint16_t* Blo, float* C, int64_t P,
                          int64_t K, int64_t Q, int R, hipStream_t st);
// FP8 x FP8 (CP_FP8F8): the factor A (K x R, FP32) quantized per column to
// E4M3 after a power-of-two scale, Bq[c][k] with pitch bf16_factor_pitch(K)
// (zero padded) and inv[c] the scale's inverse; then the FP8 tensor's first
// contraction with it on the FP8 matrix cores, each output column multiplied
// by inv[c].
hipError_t launch_quant_factor_fp8(const float* A, int64_t K, int R, uint8_t* Bq, float* inv, hipStream_t st);
hipError_t launch_ttm_fp8f8(const uint8_t* X, const uint8_t* Bq, const float* inv, float* C, int64_t P, int64_t K,
                            int64_t Q, int R, hipStream_t st);

// FP32 tensor path on the BF16 matrix cores (CP_F32X3): the factor split
// into three BF16 parts, Bt[part][c][k] with pitch bf16_factor_pitch(K)
// (3 R pitch elements), then C = X times the factor with the six leading part
// products accumulated in FP32.  KC (Q == 1) needs K % 8 == 0 and 16-byte
// aligned rows, the other layout a tensor below 4 GiB (ttm_x3_fits).  With
// `parts` (ttm_x3_layers(P, K, Q, R) P Q R floats) a contraction with too few
// row tiles to fill the chip is split over K, its partials added in order;
// null: no split.
bool ttm_x3_fits(int64_t P, int64_t K, int64_t Q, int R, const void* X);
int ttm_x3_layers(int64_t P, int64_t K, int64_t Q, int R);
hipError_t launch_split3_factor(const float* A, int64_t K, int R, uint16_t* Bt, hipStream_t st);
hipError_t launch_ttm_x3(const float* X, const uint16_t* Bt, float* C, int64_t P, int64_t K, int64_t Q, int R,
                         float* parts, hipStream_t st);

// The leading half's first two levels in one pass (k_ttm_kc32f): X is
// (P2 S) x K with K == 128 (contracted with B, K x R), then the mode of size S
// before it (A2, S x R) into C (P2 x R); FP32, S a multiple of 32 up to 256,
// 16 < R <= 64, X 16-byte aligned (ttm_kc_fused_fits).  With Y non-null the
// first-level node ((P2 S) x R) is written too (a tree that keeps it).
bool ttm_kc_fused_fits(const float* X, int64_t K, int64_t S, int R);
hipError_t launch_ttm_kc_fused(const float* X, const float* B, const float* A2, float* C, float* Y, int64_t P2,
                               int64_t S, int R, hipStream_t st);

// A first-level contraction in the q-contiguous layout with the contraction
// over one more index i in its epilogue (k_ttm_qg): element (p', i, k, q) of
// X at p' pstride + i sstride + k kstride + q; q < Q contiguous (Q a
// multiple of 64), k < K (a multiple of 32 up to 256), i < S, p' < nP.
// C[p'][q][r] = sum_i W[i][r] sum_k X[p', i, k, q] B[k][r]; with Y non-null
// also the first-level node Y[p' S + i][q][r].  parts holds
// qg_layers(sh) nP Q R floats of partials when that is above one.
struct QgShape {
  int64_t K, kstride, S, sstride, nP, pstride, Q;
};
bool ttm_qg_shape(const QgShape& sh, int R);  // the fits check without X's alignment
bool ttm_qg_fits(const float* X, const QgShape& sh, int R);
int qg_layers(const QgShape& sh);
hipError_t launch_ttm_qg(const float* X, const float* B, const float* W, float* C, float* Y, const QgShape& sh, int R,
                         float* parts, hipStream_t st);

// A first-level contraction with the contraction over the last mode in the
// epilogue (k_ttm_qr; MSDT's root at mode 0, a PP initialization node whose
// single pair child contracts the last mode): X is P x K x Q (K a multiple
// of 32 up to 256), B (K x R); the last mode has size S (64, 128 or 256; Q a
// multiple of S), W (S x R); C ((P Q / S) x R); Y, when non-null, the
// first-level node (P Q x R).
bool ttm_qr_fits(const float* X, int64_t P, int64_t K, int64_t Q, int64_t S, int R);
hipError_t launch_ttm_qr(const float* X, const float* B, const float* W, float* C, float* Y, int64_t P, int64_t K,
                         int64_t Q, int64_t S, int R, hipStream_t st);

// Y[p][q][r] = sum_i X[p][i][q][r] * A[i][r]; accumulation in the output type.
template <typename TI, typename TO>
hipError_t launch_mttv(const TI* X, const TI* A, TO* Y, int64_t P, int64_t I, int64_t Q, int R,
                       hipStream_t st);

// Two children of a node keeping three modes z, u, v (FP32, rank index
// contiguous; element strides Sz, Su, Sv) from one pass over it:
// Ycv[z][u] = sum_v X Av[v] and Ycu[z][v] = sum_u X Au[u] (rank-wise), with
// output strides (ozv, ouv) and (ozu, ovu).  For R in {16, 32, 64} with sv
// at most 8 (1024 / R) (mttv_pair_fits); hipErrorInvalidValue otherwise.
// With `parts` (mttv_pair_split(sz, su) sz sv R floats), the u range is
// split over that many workgroups per slice and their partial Ycu are added
// in range order; null: one workgroup per slice.
constexpr int kMaxPairSplit = 8;
bool mttv_pair_fits(int64_t sz, int64_t sv, int R);
int mttv_pair_split(int64_t sz, int64_t su);
hipError_t launch_mttv_pair(const float* X, const float* Au, const float* Av, float* Ycv, float* Ycu, int64_t sz,
                            int64_t su, int64_t sv, int64_t Sz, int64_t Su, int64_t Sv, int64_t ozv, int64_t ouv,
                            int64_t ozu, int64_t ovu, int R, float* parts, hipStream_t st);

// dst[i] = (T) src[i] for n elements.
template <typename T>
hipError_t launch_convert(const double* src, T* dst, int64_t n, hipStream_t st);

// Layers of a split-K form of a long-K first-level contraction (X is P x K x
// Q; Q = 1 on any type, Q >= 64 in FP32): 1 when a single pass fills the
// chip; at most kMaxSplitLayers.
constexpr int kMaxSplitLayers = 16;
int ttm_split_layers(int64_t P, int64_t K, int64_t Q, int R, int esz);

// The first-level contraction C[p][q][r] = sum_k X[p][k][q] B[k][r] with K
// split over Z workgroup layers: partials in `parts` (Z P Q R elements),
// added in layer order into C (deterministic).  Z <= 1: launch_ttm.
template <typename T>
hipError_t launch_ttm_split(const T* X, const T* B, T* C, int64_t P, int64_t K, int64_t Q, int R, T* parts, int Z,
                            hipStream_t st);

// B (sa sb x R) = Khatri-Rao product of Aa (sa x R) and Ab (sb x R), row i sb + j.
template <typename T>
hipError_t launch_krp2(const T* Aa, int64_t sa, const T* Ab, int64_t sb, int R, T* B, hipStream_t st);

// FP64 copy, dst[i] = src[i] (n elements).
hipError_t launch_copy_f64(const double* src, double* dst, int64_t n, hipStream_t st);

// ||T||^2 into stats->normT2 (two deterministic passes using `partials`).
template <typename T>
hipError_t launch_norm2(const T* X, int64_t n, double* partials, int nparts, DevStats* stats,
                        hipStream_t st);

// S = A^T A for an s x R FP64 matrix (one workgroup, fixed order).
hipError_t launch_gram(const double* A, int64_t s, int R, double* S, hipStream_t st);

// Gamma^(n) = Hadamard product of S[m], m != n (Eq. (1)) and, when pp != 0,
// W^(n) = the bracket of Eq. (7), both entrywise into Gamma / W.
struct GammaArgs {
  const double* S[kMaxOrder];
  const double* dS[kMaxOrder];
  double* Gamma;
  double* W;
  int N, n, R, pp;
};
hipError_t launch_gamma(const GammaArgs& a, hipStream_t st);

// Ginv = Gamma^dagger (Alg. 1): Gauss-Jordan elimination without pivoting in
// one workgroup; when a pivot is at or below R eps max(diag), the symmetric
// eigendecomposition (cyclic Jacobi, a second one-workgroup kernel that
// returns at once otherwise) gives the pseudo-inverse with eigenvalues at or
// below R eps lambda_max dropped.  Non-finite entries set bit 0 of
// stats->status and zero Ginv.
hipError_t launch_inverse(const double* Gamma, double* Ginv, int R, DevStats* stats, hipStream_t st);

// One mode update (Alg. 1 inner body; Alg. 2 with Eq. (7) in PP) in one
// launch of `groups` workgroups (update_groups): A^(n) <- M~ Ginv with the
// shadows, the Gram S^(n) (and dS^(n)), the norms, after the last mode the
// residual of Eq. (3), Gamma^(nx) and W^(nx) of the next mode
// nx = (n + 1) mod N, and with inv_next also Ginv <- Gamma^(nx)^dagger.
template <typename T>
struct UpdateArgs {
  const double* M;    // s x R right-hand side (exact or first-order PP MTTKRP)
  double* A;          // s x R FP64 factor, read (old) and overwritten (new)
  T* Ash;             // s x R shadow of the new factor in tensor precision
  const double* Ap;   // PP: A_p of this mode (else null)
  T* dAsh;            // PP: shadow of dA = A - A_p (else null)
  double* Ginv;       // in: Gamma^(n)^dagger; out (inv_next): Gamma^(nx)^dagger
  double* partS;      // [groups][R][R] partial Gram matrices
  double* partdS;     // PP: [groups][R][R]
  double* partSc;     // [groups][4]: ||A||^2, ||dA||^2, <M~, A>
  double* S[kMaxOrder];   // S^(m); S[n] is written
  double* dS[kMaxOrder];  // dS^(m); dS[n] is written in PP
  double* Gamma;      // in: Gamma^(n); out: Gamma^(nx)
  double* W;          // in (PP): W^(n); out: W^(nx) from the current dS
  DevStats* stats;    // norms, residual, status
  unsigned* ticket;   // arrival counter: 0 at launch, left at 0
  double* partG;      // split path: [ceil(R * R / 32)] shares of <Gamma^(n), S^(n)>
  int64_t s;          // rows of A^(n)
  int nrb;            // 16-row blocks, ceil(s / 16)
  int R, n, N, last, pp, inv_next;
  int fused;          // 1: the last workgroup reduces (update_shape); 0: launch_update reduces
};
// Launch shape of a mode update: `groups` workgroups and whether the last of
// them does the reductions (few, small partials) or a second, parallel
// kernel does (launch_update then also inverts Gamma^(nx) itself with
// launch_inverse when inv_next is set).
void update_shape(int64_t s, int R, bool pp, int* groups, bool* fused);
// Upper bound of `groups` over all mode sizes up to smax.
int update_groups_max(int64_t smax, int R);
template <typename T>
hipError_t launch_update(const UpdateArgs<T>& a, int groups, hipStream_t st);

// r of Eq. (3) for given factors into stats->r: M is the exact MTTKRP of the
// last mode, A its factor (s x R), Gamma / S of that mode.
hipError_t launch_fitness(const double* M, const double* A, int64_t s, int R, const double* Gamma,
                          const double* S, DevStats* stats, hipStream_t st);

// Zero n doubles; zero `bytes` bytes (a multiple of 4) of any buffer.
hipError_t launch_zero_f64(double* p, int64_t n, hipStream_t st);
hipError_t launch_zero_bytes(void* p, size_t bytes, hipStream_t st);

// Independent small setup operations run by one launch (each takes its own
// range of workgroups): FP64 -> FP32 or FP64 conversion (a copy for FP64),
// zero fill of 32-bit words, Gram matrix S = A^T A of an s x R FP64 factor.
enum SetupKind { kSetupToF32 = 0, kSetupToF64 = 1, kSetupZero32 = 2, kSetupGram = 3 };
struct SetupOp {
  const double* src;  // conversions: source; Gram: A (s x R)
  void* dst;          // destination (S for Gram)
  int64_t n;          // elements (conversions), 32-bit words (zero); Gram: s
  int kind;
  int R;              // Gram only
};
constexpr int kMaxSetupOps = 40;
struct SetupBatch {
  SetupOp op[kMaxSetupOps];
  int nops = 0;
};
hipError_t launch_setup(const SetupBatch& b, hipStream_t st);

// First-order PP MTTKRP, Eqs. (5)-(6) without V:
// M[x][r] = Mp[x][r] + sum_{i != n} sum_y P_(n,i)[x][y][r] dA_i[y][r]
template <typename T>
struct PPArgs {
  const T* pair[kMaxOrder];  // operator of the pair {n, i} (null for i == n)
  int pair_n_first[kMaxOrder];  // 1 if stored with n's axis first
  const T* dA[kMaxOrder];
  int64_t dims[kMaxOrder];
  const double* Mp;
  double* M;
  int N, n, R;
  const double* Gamma;  // with Ginv: Gamma^(n), inverted into Ginv by an extra workgroup
  double* Ginv;         // null: no inverse
  DevStats* stats;
};
template <typename T>
hipError_t launch_pp_mttkrp(const PPArgs<T>& a, hipStream_t st);

}  // namespace cpals
