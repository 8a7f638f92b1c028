/*
 * cpals.h - C ABI of the MI355X (gfx950) CP-ALS hot path: MTTKRP by dimension
 * trees, the multi-sweep dimension tree (MSDT) schedule and pairwise
 * perturbation (PP), after Ma and Solomonik, "Efficient parallel CP
 * decomposition with pairwise perturbation and multi-sweep dimension tree".
 *
 * Conventions shared by every entry point
 *   - Arrays are row-major (C order, last index fastest).  A tensor of order N
 *     has dims s[0..N-1]; factor n is an s[n] x R matrix.
 *   - Every array argument is a DEVICE pointer on the plan's device, owned by
 *     the caller and borrowed for the duration of the call (the tensor is
 *     borrowed from cp_set_tensor until the next cp_set_tensor or destroy).
 *   - Factor matrices are always FP64 (the ALS state).  The tensor is stored
 *     in the plan's precision (FP64, FP32, or BF16 or FP8 for the precision
 *     path); contractions with it run in that precision (BF16 and FP8: on the
 *     BF16 matrix cores with FP32 accumulation), every R x R operation (Gram matrices,
 *     their Hadamard products, the inverse or pseudo-inverse of Gamma, norms,
 *     the residual) runs in FP64.
 *   - All work is enqueued on the plan's HIP stream and the call returns
 *     without waiting, unless it has to read a device result: a non-null
 *     `info`, or cp_pp_sweep in CP_PP_AUTO mode (one small device-to-host
 *     read of the factor-change norms before the sweep).
 *   - Errors are returned as cp_status; nothing is thrown and nothing exits.
 *     cp_last_error() gives a message for the last failing call on a plan.
 *   - A plan is not thread-safe.  The library allocates no device memory: the
 *     caller provides one workspace of the size the plan reports.
 *   - Limits: 3 <= N <= 8, 1 <= R <= 128, every s[n] >= 1, numel < 2^40.
 *     Anything else returns CP_ERR_UNSUPPORTED.
 */
#ifndef CPALS_H
#define CPALS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cp_plan_s* cp_plan;

typedef enum {
  CP_OK = 0,
  CP_ERR_ARG = 1,         /* null pointer, bad mode, bad size */
  CP_ERR_STATE = 2,       /* call out of order (no workspace, no tensor, no PP operators) */
  CP_ERR_UNSUPPORTED = 3, /* outside the stated limits */
  CP_ERR_HIP = 4,         /* a HIP runtime call failed; see cp_last_error */
  CP_ERR_NOT_SPD = 5,     /* a Gamma matrix had non-finite entries (a singular Gamma is
                             handled by its pseudo-inverse, as Alg. 1 writes it) */
  CP_ERR_NUMERIC = 6      /* the residual came out NaN or infinite */
} cp_status;

/* Tensor precision.  CP_F64 and CP_F32: the tensor, the tree intermediates
 * and the factor shadows in that type, FP64 for everything of size R x R and
 * for the factors.  CP_BF16 and CP_BF16X2 (not from the paper): the tensor is
 * stored in BF16 (raw bits, the upper half of an FP32 value) and its first
 * contraction runs on the BF16 matrix cores with FP32 accumulation, the
 * factor rounded to BF16 (CP_BF16) or split into two BF16 parts B_hi + B_lo
 * (CP_BF16X2, about 16 significant bits); the levels below are FP32 as in
 * CP_F32.  CP_FP8 and CP_FP8X2 (not from the paper): the tensor is stored in
 * FP8 E4M3 (raw bytes: sign, 4 exponent bits with bias 7, 3 mantissa bits,
 * no infinities; the OCP "e4m3fn" format) and widened exactly to BF16 in
 * registers, so the first contraction is that of CP_BF16 / CP_BF16X2 on the
 * stored values with half the tensor bytes.  E4M3 spans 2^-9 .. 448: scale
 * the tensor by a power of two so that its largest entry lies near 448
 * before storing it (exact; the relative residual does not depend on the
 * tensor's scale), else small entries round to zero.  CP_F32X3 (not from the
 * paper): as CP_F32, except that the first contraction runs on the BF16
 * matrix cores: every FP32 tensor value and factor entry is split exactly
 * into three BF16 parts (each rounded to nearest) and the six leading part
 * products are accumulated in FP32 (the three dropped ones are below 2^-23
 * of the product), so each product carries an error of the order of one FP32
 * rounding; contracting the last mode with rows not 16-byte aligned or K
 * not a multiple of 8, or another mode of a tensor of 4 GiB or more, takes
 * the FP32 matrix cores instead.  CP_FP8F8 (not from the paper): the tensor
 * stored as for CP_FP8, and the first contraction's factor quantized too:
 * each column scaled by the power of two that puts its largest magnitude in
 * (224, 448] (exponent clamped to [-120, 120]) and rounded to nearest E4M3
 * (ties to even), the products of the two E4M3 operands taken on the FP8
 * matrix cores (each product exact; the instruction sums each group of eight
 * consecutive contraction indices in a fixed-point window under the group's
 * largest product, dropping parts more than about 2^-12 below it, and adds
 * the groups in FP32), and the column's scale removed from the output; the
 * factor then carries about 2^-4 relative rounding per entry instead of 2^-8
 * (CP_FP8).  The levels below are FP32. */
typedef enum {
  CP_F64 = 0, CP_F32 = 1, CP_BF16 = 2, CP_BF16X2 = 3, CP_FP8 = 4, CP_FP8X2 = 5, CP_F32X3 = 6, CP_FP8F8 = 7
} cp_prec;

typedef enum {
  CP_TREE_DT = 0,           /* standard binary dimension tree, two first-level TTMs per sweep (Sec. II-C) */
  CP_TREE_DT_COMBINED = 1,  /* as CP_TREE_DT, with the upper two levels of each half combined (the
                               memory / computation trade-off of Sec. IV), order >= 4: the half that
                               keeps the leading modes starts from the tensor, viewed as
                               (s_0 ... s_{N-3}) x (s_{N-2} s_{N-1}), times the Khatri-Rao product of
                               A^(N-2) and A^(N-1); in FP32 plans the half that keeps the trailing modes
                               starts from the Khatri-Rao product of A^(0) and A^(1) times the tensor
                               viewed as (s_0 s_1) x (s_2 ... s_{N-1}).  The order-(N-1)
                               intermediates are never formed (the same flops, far less memory and
                               traffic); long contractions are split over workgroup layers and summed
                               in a fixed order.  Order 3: identical to CP_TREE_DT.  The PP
                               initialization keeps its own tree (Fig. 1b). */
  CP_TREE_MSDT = 2          /* multi-sweep dimension tree, N first-level TTMs per N-1 sweeps (Sec. III) */
} cp_tree;

typedef enum {
  CP_PP_AUTO = 0,          /* Alg. 2 state machine with tolerance pp_tol */
  CP_PP_FORCE_EXACT = 1,   /* a regular sweep */
  CP_PP_FORCE_APPROX = 2,  /* a PP-approximated sweep with the current operators */
  CP_PP_FORCE_REINIT = 3,  /* PP initialization, then a PP-approximated sweep */
  CP_PP_LEARNED = 4        /* as CP_PP_AUTO, with the test replaced by the learned switch
                              (cp_pp_set_switch); not from the paper */
} cp_pp_mode;

typedef enum { CP_SWEEP_EXACT = 0, CP_SWEEP_PP_INIT = 1, CP_SWEEP_PP_APPROX = 2 } cp_sweep_kind;

typedef struct {
  int kind;              /* cp_sweep_kind actually run */
  int fitness_is_exact;  /* 0 when the residual came from an approximated M~^(N) */
  double fitness;        /* f = 1 - r */
  double r;              /* relative residual from Eq. (3), squared tensor norm */
  double dA_rel[8];      /* ||dA^(i)||_F / ||A^(i)||_F after the sweep (Alg. 2 test inputs);
                            1 for a zero factor, 0 past the tensor order */
  int ttm_count;         /* first-level contractions with the tensor done in this call */
  int pinv_updates;      /* factor updates since the last report whose Gamma^(n) was singular to
                            working precision, so that its pseudo-inverse (Alg. 1) came from the
                            eigendecomposition instead of the elimination */
  int rolled_back;       /* CP_PP_LEARNED only: 1 when the switch's judge undid the PP phase that
                            this call ended (the phase broke down, or the regular sweep closing it
                            found a lower exact fitness than at its start); the factors are then
                            back at their values when the phase began and `fitness` is theirs */
  int r_clamped;         /* 1 when the numerator of Eq. (3) came out negative, so r was reported
                            as 0 (fitness 1).  After an approximated sweep this means the PP
                            estimate broke down (M~^(N) far from the exact MTTKRP); after an exact
                            sweep, that r is below what Eq. (3) resolves in floating point */
} cp_sweep_info;

/* Create a plan for an order-`order` tensor of dims `dims` (host array of
 * `order` entries), CP rank `rank`, tensor precision `prec`, tree schedule
 * `tree`, on HIP stream `hip_stream` (a hipStream_t; NULL is the null stream)
 * of the current device.  *out receives the plan.  (Alg. 1 inputs, Sec. II-B.) */
cp_status cp_plan_create(cp_plan* out, int order, const int64_t* dims, int rank, cp_prec prec,
                         cp_tree tree, void* hip_stream);

/* Bytes of device workspace the plan needs (intermediates of the trees, the
 * PP operators, FP64 R x R state).  */
cp_status cp_plan_workspace_size(cp_plan plan, size_t* bytes);

/* Attach a device workspace of at least cp_plan_workspace_size bytes,
 * 256-byte aligned, owned by the caller and kept alive while the plan is
 * used.  Re-attaching drops every cached intermediate. */
cp_status cp_plan_set_workspace(cp_plan plan, void* dptr, size_t bytes);

/* Borrow the tensor T (device, plan precision, dims of the plan) and compute
 * ||T||_F^2 in FP64, used by the residual (Eq. (3)).  Drops cached state. */
cp_status cp_set_tensor(cp_plan plan, const void* T);

/* M = MTTKRP of mode `mode` (0-based): M^(n) = T_(n) P^(n), the product of
 * the mode-n unfolding with the Khatri-Rao product of every other factor
 * (Sec. II-B).  A: host array of `order` device pointers to FP64 s[i] x R
 * factors (A[mode] is not read); M: device FP64 s[mode] x R output.  Computed
 * along the standard dimension tree path for that mode.  Stateless for the
 * caller, but drops the plan's cached sweep state (as cp_reset). */
cp_status cp_mttkrp(cp_plan plan, const double* const* A, int mode, double* M);

/* Allocation-free MTTKRP, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Computes what cp_mttkrp computes, with the same kernels, for
 * a tensor T of `order` dims `dims` (host array) in precision `prec`, factors
 * A (host array of `order` device FP64 pointers, A[mode] not read) and rank
 * `rank`, into M (device FP64, dims[mode] x rank), enqueued on `hip_stream`
 * of the current device.  No plan, no workspace: the intermediates live in a
 * static device array of 64 MiB that each device holds from library load
 * until the process ends; nothing is allocated or freed.  CP_ERR_UNSUPPORTED
 * when the intermediates would not fit (the factor shadows plus the nodes of
 * the mode's tree path, e.g. order 4, 64^4, R = 32 in FP32 needs 32.5 MiB).
 * Calls that overlap on one device share that array and race: serialize
 * them (one stream, or events).  The error text of a failing call is
 * cp_last_error(NULL) on the same thread. */
cp_status cp_mttkrp_static(int order, const int64_t* dims, int rank, cp_prec prec, const void* T,
                           const double* const* A, int mode, double* M, void* hip_stream);

/* As cp_mttkrp, but the first contraction with the tensor uses mode
 * `root_mode` (!= mode), the rest of the path contracts the remaining modes
 * one at a time in increasing distance from `mode`.  Exercises every
 * first-level layout (Sec. III: T x_m A^(m) serves every MTTKRP except m). */
cp_status cp_mttkrp_rooted(cp_plan plan, const double* const* A, int mode, int root_mode, double* M);

/* One ALS sweep (Alg. 1, one pass of the loop body): for n = 0..N-1,
 * Gamma^(n) by Eq. (1), M^(n) by the plan's tree, A^(n) <- M^(n) Gamma^(n)^-1,
 * S^(n) <- A^(n)T A^(n); then the residual by Eq. (3).  A: host array of N
 * device pointers to the FP64 factors, updated in place.  The factors must be
 * the ones the plan last wrote (or call cp_reset after changing them).
 * info may be NULL (no host synchronization). */
cp_status cp_als_sweep(cp_plan plan, double* const* A, cp_sweep_info* info);

/* One outer step of PP-CP-ALS (Alg. 2): depending on `mode` and, in
 * CP_PP_AUTO, on the test ||dA^(i)||_F < pp_tol ||A^(i)||_F for every i,
 * either a regular sweep with the plan's tree, or PP initialization (A_p <- A,
 * dA <- 0, operators M_p^(i,j), M_p^(n) by the PP dimension tree of Fig. 1b)
 * followed by an approximated sweep, or an approximated sweep alone
 * (M~^(n) by Eqs. (5)-(8)).  Same argument rules as cp_als_sweep. */
cp_status cp_pp_sweep(cp_plan plan, double* const* A, double pp_tol, cp_pp_mode mode,
                      cp_sweep_info* info);

/* Exact fitness f = 1 - r (Eq. (3) with an exact MTTKRP of the last mode)
 * of the given FP64 factors (host array of N device pointers).  Used to audit
 * approximated sweeps.  Synchronizes; drops the plan's cached sweep state. */
cp_status cp_fitness(cp_plan plan, const double* const* A, double* fitness);

/* Learned PP switch (not from the paper; it replaces the hand threshold of
 * Alg. 2 in CP_PP_LEARNED mode).  A perceptron D = N + 3 -> H -> H -> 1 with
 * tanh hidden units and a sigmoid output; parameters theta (device FP32,
 * layout W1 (D x H), b1, W2 (H x H), b2, w3 (H), b3, owned by the caller and
 * kept alive).  Before each outer step (except the first) the plan forms
 *   x_i     = log10(max(||dA_i||_F / ||A_i||_F, 1e-12)),       i < N
 *   x_{N+j} = log10(max(|f_j - f_{j+1}|, 1e-12)), j = 0,1,2,   f_0 the newest
 *             fitness (a delta not yet available counts as 1),
 * normalizes (x - shift) / scale (host arrays of D), and runs a PP step when
 * the network's probability exceeds `threshold`, a regular sweep otherwise.
 * The regular sweep is the judge: when a PP phase breaks down (non-finite
 * state) or the regular sweep that closes it has a lower exact fitness than
 * the one before the phase began, the factors are restored to their values at
 * the phase start (A_p) and the next four outer steps are regular sweeps
 * (cp_sweep_info.rolled_back).  theta == NULL removes the switch. */
cp_status cp_pp_set_switch(cp_plan plan, const float* theta, int hidden, const double* shift,
                           const double* scale, double threshold);

/* Features (unnormalized, D = N + 3 values, host array) and probability of the
 * last learned decision. */
cp_status cp_pp_last_decision(cp_plan plan, double* features, double* probability);

/* Training and inference kernels of the switch network (device FP32 arrays,
 * stream as in cp_plan_create).  D <= 16, H <= 128, B >= 1.
 * cp_mlp_forward: p[b] = sigmoid(net(X[b])) for B rows of X (B x D).
 * cp_mlp_grad: grad[0..n) = gradient of the mean binary cross-entropy over the
 *   B samples (labels y in {0,1}), grad[n] = the loss; n = cp_mlp_param_count;
 *   scratch of cp_mlp_scratch_floats(B, H) floats.  Sums over samples run in
 *   sample order (bitwise reproducible).
 * cp_mlp_adam: one Adam step (Kingma and Ba) on n parameters, t counting from 1. */
size_t cp_mlp_param_count(int D, int H);
size_t cp_mlp_scratch_floats(int B, int H);
cp_status cp_mlp_forward(const float* X, int B, int D, int H, const float* theta, float* p, void* stream);
cp_status cp_mlp_grad(const float* X, const float* y, int B, int D, int H, const float* theta, float* grad,
                      float* scratch, void* stream);
cp_status cp_mlp_adam(float* theta, const float* grad, float* m, float* v, int n, int t, float lr,
                      float beta1, float beta2, float eps, void* stream);

/* Drop cached intermediates, the MSDT position and the PP state: the next
 * sweep re-reads the factors and recomputes their Gram matrices. */
cp_status cp_reset(cp_plan plan);

/* Wait for the plan's stream and report a deferred device-side failure
 * (CP_ERR_NOT_SPD from a solve, CP_ERR_NUMERIC from a residual). */
cp_status cp_sync(cp_plan plan);

/* Phase timers (the per-sweep breakdown of Sec. V-B).  Categories: */
typedef enum {
  CP_PHASE_TTM = 0,     /* first-level contractions of the tensor with one factor */
  CP_PHASE_MTTV = 1,    /* batched TTVs down the trees (incl. PP operator levels) */
  CP_PHASE_UPDATE = 2,  /* Hadamard products of Eqs. (1)/(7), Gamma inverse, solve, Gram, norms */
  CP_PHASE_PP = 3,      /* first-order PP corrections, Eqs. (5)-(6) */
  CP_PHASE_OTHER = 4,
  CP_PHASE_COUNT = 5
} cp_phase;

/* mask: the categories to time from now on, bit (1 << cp_phase) for each
 * (CP_PROFILE_ALL: every one; 0: none).  A HIP event pair is recorded on the
 * plan's stream around every group of launches of a timed category: two
 * event records per group, which on a short sweep cost measurable time (all
 * categories: about a tenth of a 128^4 R = 64 step), so time only what is
 * needed.  CP_ERR_ARG for bits past CP_PHASE_COUNT. */
#define CP_PROFILE_ALL ((1 << CP_PHASE_COUNT) - 1)
cp_status cp_profile_enable(cp_plan plan, int mask);

/* Wait for the plan's stream, then write the summed device time in
 * milliseconds (ms[CP_PHASE_COUNT], host array) and the number of recorded
 * groups (launches[CP_PHASE_COUNT]) since the last read, and reset them. */
cp_status cp_profile_read(cp_plan plan, double* ms, int64_t* launches);

/* Destroy the plan (does not free the caller's workspace). */
cp_status cp_plan_destroy(cp_plan plan);

const char* cp_status_str(cp_status s);
/* Message of the last failing call on `plan`; with plan == NULL, of the last
 * failing plan-free call (cp_mttkrp_static) on this thread. */
const char* cp_last_error(cp_plan plan);

/* ---------------------------------------------------------------------------
 * Batched path (not from the paper): many small independent order-3 dense
 * FP32 tensors, each with its own mode sizes (1 <= s <= 96) and rank
 * (1 <= R <= 32), decomposed by CP-ALS (Alg. 1 with the standard dimension
 * tree of Sec. II-C, residual by Eq. (3)) in ONE persistent kernel launch: a
 * device work queue hands whole tensors, largest first, to free workgroups,
 * which run every requested sweep of a tensor before taking the next.  The
 * call enqueues two kernels (a counter reset and the persistent kernel),
 * allocates nothing and does not synchronize, so it can be captured in a HIP
 * graph and replayed.
 * ------------------------------------------------------------------------- */
typedef struct cp_batch_s* cp_batch;

/* count tensors; dims: host array count x 3; ranks: host array of count.
 * The queue order and the packed layout are fixed here. */
cp_status cp_batch_create(cp_batch* out, int count, const int64_t* dims, const int* ranks, void* hip_stream);

/* Packed layout the caller fills: tensor i (C order) starts at element
 * t_offsets[i] of one FP32 array of t_total elements; its factor m (s_m x R,
 * row-major, FP64) at element a_offsets[3 i + m] of one FP64 array of a_total
 * elements.  Host output arrays (any may be NULL). */
cp_status cp_batch_layout(cp_batch b, int64_t* t_offsets, int64_t* a_offsets, int64_t* t_total, int64_t* a_total);

/* Launch shape: waves per workgroup (4 or 8) and resident workgroups per
 * compute unit (1..4); before cp_batch_set_workspace (the scratch per
 * workgroup is part of the workspace).  Chosen by the autotuner. */
cp_status cp_batch_set_launch(cp_batch b, int waves_per_group, int groups_per_cu);

/* Device workspace (256-byte aligned, caller-owned): queue, counter and one
 * intermediate slot per workgroup. */
cp_status cp_batch_workspace_size(cp_batch b, size_t* bytes);
cp_status cp_batch_set_workspace(cp_batch b, void* dptr, size_t bytes);

/* `sweeps` ALS sweeps on every tensor.  T: packed tensors (device FP32),
 * A: packed factors (device FP64, read as the initial factors and
 * overwritten), fitness: device FP64 count x sweeps (f = 1 - r after each
 * sweep, Eq. (3)), status: device int count (0, or 1 when a Gamma^(n) was not
 * numerically positive definite; that tensor's sweeps stop), ticks: device
 * int64 count x 2 (wall-clock counter at the start and end of the tensor's
 * sweeps; cp_batch_tick_rate gives the rate) or NULL. */
cp_status cp_batch_sweeps(cp_batch b, const float* T, double* A, int sweeps, double* fitness, int* status,
                          long long* ticks);

/* Rate of the device wall clock used by `ticks`, in Hz. */
cp_status cp_batch_tick_rate(cp_batch b, double* hz);

void cp_batch_destroy(cp_batch b);

#ifdef __cplusplus
}
#endif
#endif /* CPALS_H */
