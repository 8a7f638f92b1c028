// Host runtime and C ABI of the CP-ALS hot path (declarations and contracts
// in include/cpals.h).
//
// The plan owns host-side state only: the schedule position, versions of the
// factors, which intermediate sits in which workspace slot, the PP phase.
// Device memory comes from one caller-provided workspace, carved at attach.
//
// Intermediates follow Eq. (4): the tensor contracted with every factor not
// in a kept mode set.  Layout: kept modes in increasing order, rank index
// last (row-major), so every contraction below the first one is the same
// strided batched TTV, Y[p][q][r] = sum_i X[p][i][q][r] A[i][r].
//
// Slot d of the workspace holds one node with N - d kept modes (depth d of
// a root-to-leaf path).  A node stays valid while every factor contracted
// into it keeps the version it had when the node was built; a path reuses
// its deepest valid node.  This gives the standard dimension tree's reuse
// (Sec. II-C) and MSDT's reuse of a first-level node across sweeps
// (Sec. III) from the same mechanism.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/cpals.h"
#include "kernels.h"

using namespace cpals;

namespace {

constexpr size_t kAlign = 256;
constexpr int kNormParts = 1024;

inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Slot {
  uint32_t set = 0;  // bitmask of kept modes
  uint64_t ver[kMaxOrder] = {};
  bool valid = false;
};

}  // namespace

struct cp_plan_s {
  int N = 0, R = 0;
  int64_t dims[kMaxOrder] = {};
  cp_prec prec = CP_F32;
  cp_tree tree = CP_TREE_DT;
  hipStream_t st = nullptr;
  size_t esz = 4;
  std::string err;

  // workspace
  char* ws = nullptr;
  size_t ws_bytes = 0;
  size_t ws_need = 0;
  struct Region {
    size_t off, bytes;
  };
  std::vector<Region> regions;

  void* Ash[kMaxOrder] = {};   // factor shadows, tensor precision
  void* dAsh[kMaxOrder] = {};  // PP: shadows of dA = A - A_p
  double* Ap[kMaxOrder] = {};  // PP: A_p, FP64
  double* S[kMaxOrder] = {};   // Gram matrices, FP64
  double* dS[kMaxOrder] = {};  // PP: A^T dA, FP64
  double* Mp[kMaxOrder] = {};  // PP: M_p^(n), FP64
  void* pair[kMaxOrder][kMaxOrder] = {};  // PP: M_p^(i,j), i < j, axes (s_i, s_j, R)
  double *Gamma = nullptr, *Ginv = nullptr, *W = nullptr, *Mbuf = nullptr;
  double *partS = nullptr, *partdS = nullptr, *partSc = nullptr, *partG = nullptr, *normParts = nullptr;
  DevStats* stats = nullptr;
  void* slot_buf[kMaxOrder] = {};
  size_t slot_cap[kMaxOrder] = {};
  int nblk_max = 0;

  // state
  const void* T = nullptr;
  bool state_ready = false;
  uint64_t ver[kMaxOrder] = {};
  Slot slot[kMaxOrder];
  int64_t msdt_u = 0;
  int phase = 0;  // 0: exact, 1: PP phase
  bool have_ops = false;
  bool fresh = true;  // no sweep since the state was (re)initialized: dA = A
  int ttm_count = 0;
  int ginv_ready = -1;        // mode whose Gamma^dagger the last update left in Ginv
  bool join_pending = false;  // an inverse runs on the second stream

  // learned PP switch (set by cp_pp_set_switch)
  const float* sw_theta = nullptr;
  int sw_H = 0;
  double sw_shift[16] = {}, sw_scale[16] = {};
  double sw_thresh = 0.5;
  bool sw_set = false;
  float* sw_in = nullptr;   // workspace: normalized features
  float* sw_out = nullptr;  // workspace: probability
  void* krp = nullptr;        // CP_TREE_DT_COMBINED (order >= 4): Khatri-Rao product of the last two factors
  void* parts = nullptr;      // split-K partial products of the combined contractions
  int split_z = 1;            // layers of the leading half's combined contraction
  int split_zr = 1;           // layers of the trailing half's
  void* pair_parts = nullptr;  // FP32, order >= 4: partial sums of the fused two-child PP operators
  uint16_t* Bt_hi = nullptr;  // BF16 plans: transposed BF16 factor of the first contraction
  uint16_t* Bt_lo = nullptr;  // BF16X2 plans: its remainder part
  int pinv_seen = 0;         // stats->pinv_count at the last report
  double fit_hist[4] = {};  // fitness after the most recent sweeps, newest first
  int n_hist = 0;
  bool pending_fit = false;  // a sweep ran whose fitness is not in fit_hist yet
  double last_feat[16] = {};
  int last_feat_n = 0;
  double last_prob = -1.0;
  // judge of the learned switch: exact fitness when the open PP phase began,
  // regular sweeps still forced after a rollback
  bool sw_phase_open = false;
  double sw_entry_fit = 0.0;
  int sw_cooldown = 0;

  // second stream: the Gamma / inverse kernel of a mode update runs there,
  // concurrently with that mode's MTTKRP on the plan stream (fork/join events)
  hipStream_t aux = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;

  // phase timers: a HIP event pair around every launch group, by category
  unsigned prof = 0;  // phase categories recorded (bit 1 << cp_phase)
  struct Mark {
    hipEvent_t a, b;
    int cat;
  };
  std::vector<Mark> marks;
  std::vector<hipEvent_t> pool;
};

namespace {

// Low-precision tensors: the first contraction on the BF16 matrix cores with
// a BF16 factor (split in two parts for the X2 variants); FP32 below.
bool lowp(cp_prec q) { return q == CP_BF16 || q == CP_BF16X2 || q == CP_FP8 || q == CP_FP8X2 || q == CP_FP8F8; }
bool split_factor(cp_prec q) { return q == CP_BF16X2 || q == CP_FP8X2; }
bool fp8(cp_prec q) { return q == CP_FP8 || q == CP_FP8X2 || q == CP_FP8F8; }
bool f32_tensor(cp_prec q) { return q == CP_F32 || q == CP_F32X3; }

// The first contraction of a low-precision tensor X (P x K x Q) with the
// FP32 factor shadow A (K x R) into FP32 C.
hipError_t lowp_first_level(cp_plan p, const void* X, const float* A, float* C, int64_t P, int64_t K, int64_t Q);

cp_status fail(cp_plan p, cp_status s, const char* fmt, ...) {
  if (p) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    p->err = buf;
  }
  return s;
}

#define HIP_TRY(p, expr)                                                              \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess)                                                             \
      return fail((p), CP_ERR_HIP, "%s failed: %s", #expr, hipGetErrorString(e_));   \
  } while (0)

#define CP_TRY(expr)              \
  do {                            \
    cp_status s_ = (expr);        \
    if (s_ != CP_OK) return s_;   \
  } while (0)

hipEvent_t get_event(cp_plan p) {
  if (!p->pool.empty()) {
    hipEvent_t e = p->pool.back();
    p->pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Records an event pair around the launches made during its lifetime when
// the plan's phase timers are on.
struct ProfScope {
  cp_plan p;
  int cat;
  hipStream_t st;
  hipEvent_t a = nullptr;
  ProfScope(cp_plan p_, int cat_) : ProfScope(p_, cat_, p_->st) {}
  ProfScope(cp_plan p_, int cat_, hipStream_t st_) : p(p_), cat(cat_), st(st_) {
    if ((p->prof >> cat) & 1u) {
      a = get_event(p);
      if (a && hipEventRecord(a, st) != hipSuccess) a = nullptr;
    }
  }
  ~ProfScope() {
    if (!a) return;
    hipEvent_t b = get_event(p);
    if (b && hipEventRecord(b, st) == hipSuccess) p->marks.push_back({a, b, cat});
  }
};

int64_t node_numel(cp_plan p, uint32_t set) {
  int64_t n = p->R;
  for (int m = 0; m < p->N; ++m)
    if (set & (1u << m)) n *= p->dims[m];
  return n;
}

// CP_TREE_DT_COMBINED: the half of the dimension tree that keeps the leading
// modes starts by contracting the last two modes, N-1 then N-2, and nothing
// but its next level reads the node in between.  Done as one contraction of
// the tensor, viewed as (s_0 ... s_{N-3}) x (s_{N-2} s_{N-1}), with the
// Khatri-Rao product of the two factors: the upper two levels combined (the
// memory / computation trade-off of Sec. IV).  The intermediate of order N-1
// is never formed.  Orders 4 and up (at order 3 that half has one contraction).
int64_t combined_k(cp_plan p) {
  if (p->tree != CP_TREE_DT_COMBINED || p->N < 4) return 0;
  return p->dims[p->N - 2] * p->dims[p->N - 1];
}

// The same for the half that keeps the trailing modes: it starts by
// contracting modes 0 then 1, so its first node is the tensor, viewed as
// (s_0 s_1) x (s_2 ... s_{N-1}), contracted over its leading index with the
// Khatri-Rao product of A^(0) and A^(1).  FP32 plans (the long-K kernel of
// that layout is FP32).
int64_t combined_k_right(cp_plan p) {
  if (p->tree != CP_TREE_DT_COMBINED || p->N < 4 || !f32_tensor(p->prec)) return 0;
  return p->dims[0] * p->dims[1];
}

size_t fused_parts_floats(cp_plan p);

void plan_layout(cp_plan p) {
  const int N = p->N, R = p->R;
  p->regions.clear();
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off += align_up(bytes ? bytes : 1);
    p->regions.push_back({o, bytes});
    return o;
  };
  int64_t smax = 0;
  for (int m = 0; m < N; ++m) smax = std::max(smax, p->dims[m]);
  p->nblk_max = update_groups_max(smax, R);  // workgroups of a mode update
  // fixed order of regions; set_workspace replays it
  for (int m = 0; m < N; ++m) take((size_t)p->dims[m] * R * p->esz);      // Ash
  for (int m = 0; m < N; ++m) take((size_t)p->dims[m] * R * p->esz);      // dAsh
  for (int m = 0; m < N; ++m) take((size_t)p->dims[m] * R * 8);           // Ap
  for (int m = 0; m < N; ++m) take((size_t)R * R * 8);                    // S
  for (int m = 0; m < N; ++m) take((size_t)R * R * 8);                    // dS
  for (int m = 0; m < N; ++m) take((size_t)p->dims[m] * R * 8);           // Mp
  for (int i = 0; i < N; ++i)
    for (int j = i + 1; j < N; ++j) take((size_t)p->dims[i] * p->dims[j] * R * p->esz);  // pairs
  take((size_t)R * R * 8);                       // Gamma
  take((size_t)R * R * 8);                       // Ginv
  take((size_t)R * R * 8);                       // W
  take((size_t)smax * R * 8);                    // Mbuf
  take((size_t)p->nblk_max * R * R * 8);         // partS
  take((size_t)p->nblk_max * R * R * 8);         // partdS
  take((size_t)p->nblk_max * 4 * 8);             // partSc
  take((size_t)(R * R + 31) / 32 * 8);           // partG
  take((size_t)kNormParts * 8);                  // normParts
  take(sizeof(DevStats));                        // stats
  take(16 * sizeof(float));                      // sw_in
  take(16 * sizeof(float));                      // sw_out
  const bool bf = lowp(p->prec);
  const int64_t kc = combined_k(p);         // contraction length of the combined first levels (0: none)
  const int64_t kcr = combined_k_right(p);
  take((size_t)std::max(kc, kcr) * R * p->esz);  // krp (one half at a time)
  {
    int64_t P = 1, Q = 1;
    for (int m = 0; m < N - 2; ++m) P *= p->dims[m];
    for (int m = 2; m < N; ++m) Q *= p->dims[m];
    p->split_z = (kc > 0 && !lowp(p->prec)) ? ttm_split_layers(P, kc, 1, R, (int)p->esz) : 1;
    p->split_zr = kcr > 0 ? ttm_split_layers(1, kcr, Q, R, (int)p->esz) : 1;
    size_t pl = p->split_z > 1 ? (size_t)p->split_z * P : 0;
    size_t pr = p->split_zr > 1 ? (size_t)p->split_zr * Q : 0;
    if (p->prec == CP_F32X3) {  // the three-part contractions' own split over K
      if (kc > 0) pl = std::max(pl, (size_t)ttm_x3_layers(P, kc, 1, R) * P);
      if (kcr > 0) pr = std::max(pr, (size_t)ttm_x3_layers(1, kcr, Q, R) * Q);
    }
    // the fused first and second levels (path_fused_op): one partial node per range
    const size_t pf = fused_parts_floats(p) / R;
    take(std::max(std::max(pl, pr), pf) * R * p->esz);  // parts
  }
  {
    // pair_parts: the largest split partials of launch_mttv_pair over the
    // (slice z, summed u, kept v) mode triples it can take
    size_t pp = 0;
    if (f32_tensor(p->prec) && N >= 4)
      for (int z = 0; z < N; ++z)
        for (int u = 0; u < N; ++u)
          for (int v = 0; v < N; ++v)
            if (z != u && z != v && u != v && mttv_pair_fits(p->dims[z], p->dims[v], R))
              pp = std::max(pp, (size_t)mttv_pair_split(p->dims[z], p->dims[u]) * p->dims[z] * p->dims[v] * R * 4);
    take(pp);
  }
  const int64_t kb = std::max(smax, kc);
  const int64_t kx = std::max(kb, kcr);
  take(bf ? (size_t)R * bf16_factor_pitch(kb) * 2
          : p->prec == CP_F32X3 ? (size_t)3 * R * bf16_factor_pitch(kx) * 2 : 0);   // Bt_hi (all three parts for X3)
  take(split_factor(p->prec) ? (size_t)R * bf16_factor_pitch(kb) * 2 : 0);              // Bt_lo
  // slots for depths 1..N-2 (depth d keeps N - d modes)
  std::vector<int64_t> sorted(p->dims, p->dims + N);
  std::sort(sorted.begin(), sorted.end(), std::greater<int64_t>());
  for (int d = 1; d <= N - 2; ++d) {
    int64_t n = R;
    for (int m = 0; m < N - d; ++m) n *= sorted[m];
    p->slot_cap[d] = (size_t)n * p->esz;
    take(p->slot_cap[d]);
  }
  p->ws_need = off;
}

void plan_carve(cp_plan p) {
  const int N = p->N;
  size_t k = 0;
  auto next = [&]() { return (void*)(p->ws + p->regions[k++].off); };
  for (int m = 0; m < N; ++m) p->Ash[m] = next();
  for (int m = 0; m < N; ++m) p->dAsh[m] = next();
  for (int m = 0; m < N; ++m) p->Ap[m] = (double*)next();
  for (int m = 0; m < N; ++m) p->S[m] = (double*)next();
  for (int m = 0; m < N; ++m) p->dS[m] = (double*)next();
  for (int m = 0; m < N; ++m) p->Mp[m] = (double*)next();
  for (int i = 0; i < N; ++i)
    for (int j = i + 1; j < N; ++j) p->pair[i][j] = next();
  p->Gamma = (double*)next();
  p->Ginv = (double*)next();
  p->W = (double*)next();
  p->Mbuf = (double*)next();
  p->partS = (double*)next();
  p->partdS = (double*)next();
  p->partSc = (double*)next();
  p->partG = (double*)next();
  p->normParts = (double*)next();
  p->stats = (DevStats*)next();
  p->sw_in = (float*)next();
  p->sw_out = (float*)next();
  p->krp = next();
  p->parts = next();
  p->pair_parts = next();
  p->Bt_hi = (uint16_t*)next();
  void* lo = next();
  p->Bt_lo = split_factor(p->prec) ? (uint16_t*)lo : nullptr;
  for (int d = 1; d <= N - 2; ++d) p->slot_buf[d] = next();
}

void drop_cache(cp_plan p) {
  p->ginv_ready = -1;
  p->n_hist = 0;
  p->pending_fit = false;
  p->sw_phase_open = false;  // a PP phase cannot outlive the state it was judged against
  p->sw_cooldown = 0;
  for (int d = 0; d < kMaxOrder; ++d) p->slot[d] = Slot();
  p->msdt_u = 0;
  p->phase = 0;
  p->have_ops = false;
  p->state_ready = false;
  p->fresh = true;
}

uint32_t full_set(int N) { return (N >= 32) ? 0xffffffffu : ((1u << N) - 1u); }

bool slot_valid(cp_plan p, int d, uint32_t set) {
  const Slot& s = p->slot[d];
  if (!s.valid || s.set != set) return false;
  for (int m = 0; m < p->N; ++m)
    if (!(set & (1u << m)) && s.ver[m] != p->ver[m]) return false;
  return true;
}

void slot_record(cp_plan p, int d, uint32_t set) {
  Slot& s = p->slot[d];
  s.set = set;
  s.valid = true;
  for (int m = 0; m < p->N; ++m) s.ver[m] = p->ver[m];
}

// Shape of contracting mode c out of a node keeping `set` (tensor modes in
// increasing order, rank index last): X viewed as [P][I][Q](R).
void contract_shape(cp_plan p, uint32_t set, int c, int64_t* P, int64_t* I, int64_t* Q) {
  int64_t pp = 1, qq = 1;
  for (int m = 0; m < p->N; ++m) {
    if (!(set & (1u << m))) continue;
    if (m < c) pp *= p->dims[m];
    if (m > c) qq *= p->dims[m];
  }
  *P = pp;
  *I = p->dims[c];
  *Q = qq;
}

hipError_t lowp_first_level(cp_plan p, const void* X, const float* A, float* C, int64_t P, int64_t K, int64_t Q) {
  if (p->prec == CP_FP8F8) {
    // the E4M3 factor (R x Kp bytes) and its R column scales share the
    // factor buffer (R x Kp BF16 elements)
    uint8_t* q8 = (uint8_t*)p->Bt_hi;
    float* inv = (float*)(q8 + (size_t)p->R * bf16_factor_pitch(K));
    hipError_t e = launch_quant_factor_fp8(A, K, p->R, q8, inv, p->st);
    if (e != hipSuccess) return e;
    return launch_ttm_fp8f8((const uint8_t*)X, q8, inv, C, P, K, Q, p->R, p->st);
  }
  hipError_t e = launch_split_factor(A, K, p->R, p->Bt_hi, p->Bt_lo, p->st);
  if (e != hipSuccess) return e;
  if (fp8(p->prec)) return launch_ttm_fp8((const uint8_t*)X, p->Bt_hi, p->Bt_lo, C, P, K, Q, p->R, p->st);
  return launch_ttm_bf16((const uint16_t*)X, p->Bt_hi, p->Bt_lo, C, P, K, Q, p->R, p->st);
}

// One contraction: input node `in` (or the tensor when in_set is the full
// set) keeping in_set, contracting mode c, into `out` (tensor precision, or
// FP64 when out_f64).
template <typename TT>
cp_status contract(cp_plan p, const void* in, uint32_t in_set, int c, void* out, bool out_f64) {
  int64_t P, I, Q;
  contract_shape(p, in_set, c, &P, &I, &Q);
  const TT* A = (const TT*)p->Ash[c];
  if (in_set == full_set(p->N)) {
    if (out_f64) return fail(p, CP_ERR_STATE, "internal: first-level contraction into FP64");
    ++p->ttm_count;
    ProfScope ps(p, CP_PHASE_TTM);
    if (lowp(p->prec)) {
      HIP_TRY(p, lowp_first_level(p, in, (const float*)A, (float*)out, P, I, Q));
    } else if (p->prec == CP_F32X3 && ttm_x3_fits(P, I, Q, p->R, in)) {
      HIP_TRY(p, launch_split3_factor((const float*)A, I, p->R, p->Bt_hi, p->st));
      HIP_TRY(p, launch_ttm_x3((const float*)in, p->Bt_hi, (float*)out, P, I, Q, p->R, nullptr, p->st));
    } else {
      HIP_TRY(p, launch_ttm<TT>((const TT*)in, A, (TT*)out, P, I, Q, p->R, p->st));
    }
  } else if (out_f64) {
    ProfScope ps(p, CP_PHASE_MTTV);
    HIP_TRY(p, (launch_mttv<TT, double>((const TT*)in, A, (double*)out, P, I, Q, p->R, p->st)));
  } else {
    ProfScope ps(p, CP_PHASE_MTTV);
    HIP_TRY(p, (launch_mttv<TT, TT>((const TT*)in, A, (TT*)out, P, I, Q, p->R, p->st)));
  }
  return CP_OK;
}

cp_status contract_any(cp_plan p, const void* in, uint32_t in_set, int c, void* out, bool out_f64) {
  if (p->prec == CP_F64) return contract<double>(p, in, in_set, c, out, out_f64);
  return contract<float>(p, in, in_set, c, out, out_f64);
}

// The combined first level of one half.  side 1 (leading half): node
// (modes 0 .. N-3, R) = T viewed as (s_0 ... s_{N-3}) x (s_{N-2} s_{N-1})
// times the Khatri-Rao product of the shadows of A^(N-2) and A^(N-1).
// side 2 (trailing half): node (modes 2 .. N-1, R) = the Khatri-Rao product
// of A^(0) and A^(1), transposed, times T viewed as (s_0 s_1) x (s_2 ...).
template <typename TT>
cp_status contract_combined(cp_plan p, int side, void* out) {
  const int N = p->N;
  ++p->ttm_count;
  ProfScope ps(p, CP_PHASE_TTM);
  if (side == 2) {
    int64_t Q = 1;
    for (int m = 2; m < N; ++m) Q *= p->dims[m];
    const int64_t K = combined_k_right(p);
    HIP_TRY(p, launch_krp2<TT>((const TT*)p->Ash[0], p->dims[0], (const TT*)p->Ash[1], p->dims[1], p->R,
                               (TT*)p->krp, p->st));
    if (p->prec == CP_F32X3 && ttm_x3_fits(1, K, Q, p->R, p->T)) {
      HIP_TRY(p, launch_split3_factor((const float*)p->krp, K, p->R, p->Bt_hi, p->st));
      HIP_TRY(p, launch_ttm_x3((const float*)p->T, p->Bt_hi, (float*)out, 1, K, Q, p->R, (float*)p->parts, p->st));
      return CP_OK;
    }
    HIP_TRY(p, launch_ttm_split<TT>((const TT*)p->T, (const TT*)p->krp, (TT*)out, 1, K, Q, p->R, (TT*)p->parts,
                                    p->split_zr, p->st));
    return CP_OK;
  }
  int64_t P = 1;
  for (int m = 0; m < N - 2; ++m) P *= p->dims[m];
  const int64_t K = combined_k(p);
  HIP_TRY(p, launch_krp2<TT>((const TT*)p->Ash[N - 2], p->dims[N - 2], (const TT*)p->Ash[N - 1], p->dims[N - 1],
                             p->R, (TT*)p->krp, p->st));
  if (lowp(p->prec)) {
    HIP_TRY(p, lowp_first_level(p, p->T, (const float*)p->krp, (float*)out, P, K, 1));
  } else if (p->prec == CP_F32X3 && ttm_x3_fits(P, K, 1, p->R, p->T)) {
    HIP_TRY(p, launch_split3_factor((const float*)p->krp, K, p->R, p->Bt_hi, p->st));
    HIP_TRY(p, launch_ttm_x3((const float*)p->T, p->Bt_hi, (float*)out, P, K, 1, p->R, (float*)p->parts, p->st));
  } else {
    HIP_TRY(p, launch_ttm_split<TT>((const TT*)p->T, (const TT*)p->krp, (TT*)out, P, K, 1, p->R, (TT*)p->parts,
                                    p->split_z, p->st));
  }
  return CP_OK;
}

// Whether a path from the tensor takes a combined first level: 1 when it
// starts with the contractions of modes N-1 and N-2, 2 when with modes 0 and
// 1, and goes on below that node; 0 otherwise.
int path_combines(cp_plan p, const std::vector<int>& seq) {
  if (seq.size() < 3) return 0;
  if (combined_k(p) > 0 && seq[0] == p->N - 1 && seq[1] == p->N - 2) return 1;
  if (combined_k_right(p) > 0 && seq[0] == 0 && seq[1] == 1) return 2;
  return 0;
}

// The first two contractions of a path from the tensor in one pass, where a
// fused kernel takes them (FP32 plans).  Standard tree: a half's first-level
// node feeds only its second-level node, which is formed in the epilogue
// (kind 1: the last mode, then the one before it; kind 2: mode 0, then mode
// 1); the first-level node is not kept.  MSDT: a subtree's first child (the
// mode just before the root) is formed in the epilogue and the first-level
// node is kept for the subtree's later child (kind 1 for the root N-1, kind 2
// for a root in the middle, kind 3 for the root 0, whose first child is the
// last mode).
struct FusedOp {
  int kind = 0;
  bool store = false;
  int64_t P2 = 0, S = 0;  // kinds 1 and 3 (P2: kind 1's output rows, kind 3's slices)
  int64_t K = 0, Q = 0;   // kind 3
  QgShape sh{};           // kind 2
};

int64_t mode_product(cp_plan p, int lo, int hi) {
  int64_t x = 1;
  for (int m = lo; m < hi; ++m) x *= p->dims[m];
  return x;
}

// k_ttm_qg's shape for contracting mode a, then mode b, of the tensor (row
// major, element stride st_j = s_{j+1} ... s_{N-1}): k is mode a (stride
// st_a), i is mode b (stride st_b), q the modes after both (contiguous), and
// p' the remaining modes, which must form one strided run: the modes between
// a and b (when a or b is mode 0) or those before both (when a and b are
// neighbours).  The output node keeps p' then q, as the tree's node layout.
bool qg_pair_shape(cp_plan p, int a, int b, QgShape* sh) {
  const int N = p->N;
  if (a == b || a < 0 || b < 0 || a >= N || b >= N) return false;
  const int lo = std::min(a, b), hi = std::max(a, b);
  auto st = [&](int j) { return mode_product(p, j + 1, N); };
  sh->K = p->dims[a];
  sh->kstride = st(a);
  sh->S = p->dims[b];
  sh->sstride = st(b);
  sh->Q = st(hi);
  if (hi == lo + 1) {  // neighbours: p' = the modes before both
    sh->nP = mode_product(p, 0, lo);
    sh->pstride = lo > 0 ? st(lo - 1) : 0;
    return true;
  }
  if (lo == 0) {  // p' = the modes between
    sh->nP = mode_product(p, 1, hi);
    sh->pstride = st(hi - 1);
    return true;
  }
  return false;
}

// The fused kernel for contracting mode a, then mode b, from the tensor
// (store: the first-level node is written too).
bool fused_op_for(cp_plan p, int a, int b, bool store, FusedOp* op) {
  const int N = p->N;
  if (p->prec != CP_F32 || N < 4) return false;
  op->store = store;
  if (a == N - 1 && b == N - 2 && ttm_kc_fused_fits((const float*)p->T, p->dims[N - 1], p->dims[N - 2], p->R)) {
    op->kind = 1;
    op->P2 = mode_product(p, 0, N - 2);
    op->S = p->dims[N - 2];
    return true;
  }
  if (b == N - 1 && a < N - 1) {
    // the modes before a are the slices, the ones after it the q range (the last one contracted second)
    const int64_t P = mode_product(p, 0, a), Q = mode_product(p, a + 1, N);
    if (ttm_qr_fits((const float*)p->T, P, p->dims[a], Q, p->dims[N - 1], p->R)) {
      op->kind = 3;
      op->P2 = P;
      op->K = p->dims[a];
      op->Q = Q;
      op->S = p->dims[N - 1];
      return true;
    }
  }
  QgShape sh;
  if (!qg_pair_shape(p, a, b, &sh) || !ttm_qg_fits((const float*)p->T, sh, p->R)) return false;
  op->kind = 2;
  op->sh = sh;
  return true;
}

// A path's first two contractions: the standard tree's halves (the node is
// not kept), MSDT's subtree roots with their first child (the node is kept).
bool path_fused_op(cp_plan p, const std::vector<int>& seq, FusedOp* op) {
  const int N = p->N;
  if (seq.size() < 3) return false;
  const int a = seq[0], b = seq[1];
  if (p->tree == CP_TREE_DT && ((a == N - 1 && b == N - 2) || (a == 0 && b == 1)))
    return fused_op_for(p, a, b, false, op);
  if (p->tree == CP_TREE_MSDT && b == (a + N - 1) % N) return fused_op_for(p, a, b, true, op);
  return false;
}

// Launch a fused op into `out` (the second-level node), the first-level node
// into Y when op.store.
cp_status launch_fused(cp_plan p, const FusedOp& op, int a, int b, void* out, void* Y) {
  const float* B = (const float*)p->Ash[a];
  const float* W = (const float*)p->Ash[b];
  float* Yf = op.store ? (float*)Y : nullptr;
  if (op.kind == 1) {
    HIP_TRY(p, launch_ttm_kc_fused((const float*)p->T, B, W, (float*)out, Yf, op.P2, op.S, p->R, p->st));
  } else if (op.kind == 3) {
    HIP_TRY(p, launch_ttm_qr((const float*)p->T, B, W, (float*)out, Yf, op.P2, op.K, op.Q, op.S, p->R, p->st));
  } else {
    HIP_TRY(p, launch_ttm_qg((const float*)p->T, B, W, (float*)out, Yf, op.sh, p->R, (float*)p->parts, p->st));
  }
  return CP_OK;
}

// Partial-node floats the fused kernels of this plan can need (0: none):
// any ordered pair of modes k_ttm_qg takes.
size_t fused_parts_floats(cp_plan p) {
  size_t need = 0;
  if (p->prec != CP_F32 || p->N < 4) return 0;
  for (int a = 0; a < p->N; ++a)
    for (int b = 0; b < p->N; ++b) {
      QgShape sh;
      if (!qg_pair_shape(p, a, b, &sh) || !ttm_qg_shape(sh, p->R)) continue;
      const int nz = qg_layers(sh);
      if (nz > 1) need = std::max(need, (size_t)nz * sh.nP * sh.Q * p->R);
    }
  return need;
}

// Walk a root-to-leaf contraction sequence; M (FP64, s_leaf x R) receives the leaf.
// Depth of the deepest cached node on a path (0: the path starts from the
// tensor).
int path_start(cp_plan p, const std::vector<int>& seq, std::vector<uint32_t>* sets_out = nullptr) {
  const int len = (int)seq.size();
  std::vector<uint32_t> sets(len + 1);
  sets[0] = full_set(p->N);
  for (int d = 1; d <= len; ++d) sets[d] = sets[d - 1] & ~(1u << seq[d - 1]);
  int start = 0;
  for (int d = len - 1; d >= 1; --d)
    if (slot_valid(p, d, sets[d])) {
      start = d;
      break;
    }
  if (sets_out) *sets_out = sets;
  return start;
}

cp_status run_path(cp_plan p, const std::vector<int>& seq, double* M) {
  const int N = p->N;
  const int len = (int)seq.size();
  if (len != N - 1) return fail(p, CP_ERR_STATE, "internal: path of length %d", len);
  std::vector<uint32_t> sets;
  const int start = path_start(p, seq, &sets);
  int d = start + 1;
  const int side = (d == 1) ? path_combines(p, seq) : 0;
  FusedOp op;
  if (!side && d == 1 && len >= 3 && path_fused_op(p, seq, &op)) {
    // the first two contractions in one pass (path_fused_op); the
    // first-level node is written only where the tree keeps it
    if ((size_t)node_numel(p, sets[2]) * p->esz > p->slot_cap[2] ||
        (op.store && (size_t)node_numel(p, sets[1]) * p->esz > p->slot_cap[1]))
      return fail(p, CP_ERR_STATE, "internal: slot too small");
    ++p->ttm_count;
    ProfScope ps(p, CP_PHASE_TTM);
    CP_TRY(launch_fused(p, op, seq[0], seq[1], p->slot_buf[2], p->slot_buf[1]));
    if (op.store) slot_record(p, 1, sets[1]);
    slot_record(p, 2, sets[2]);
    d = 3;
  }
  if (side) {
    if ((size_t)node_numel(p, sets[2]) * p->esz > p->slot_cap[2])
      return fail(p, CP_ERR_STATE, "internal: slot 2 too small");
    CP_TRY(p->prec == CP_F64 ? contract_combined<double>(p, side, p->slot_buf[2])
                             : contract_combined<float>(p, side, p->slot_buf[2]));
    slot_record(p, 2, sets[2]);
    d = 3;
  }
  for (; d <= len; ++d) {
    const void* in = (d == 1) ? p->T : p->slot_buf[d - 1];
    if (d == len) {
      CP_TRY(contract_any(p, in, sets[d - 1], seq[d - 1], M, true));
    } else {
      if ((size_t)node_numel(p, sets[d]) * p->esz > p->slot_cap[d])
        return fail(p, CP_ERR_STATE, "internal: slot %d too small", d);
      CP_TRY(contract_any(p, in, sets[d - 1], seq[d - 1], p->slot_buf[d], false));
      slot_record(p, d, sets[d]);
    }
  }
  return CP_OK;
}

// ---------------------------------------------------------------------------
// Schedules (host).  Positions of an ordered mode list are split in halves,
// the left half taking ceil(len/2); leaving a range for its left child
// contracts the right part from the far end inward, leaving it for its right
// child contracts the left part from the far end inward.
// ---------------------------------------------------------------------------
std::vector<int> tree_path(const std::vector<int>& order, int leaf_pos) {
  std::vector<int> out;
  int lo = 0, hi = (int)order.size() - 1;
  while (lo < hi) {
    const int mid = lo + (hi - lo + 2) / 2 - 1;
    if (leaf_pos <= mid) {
      for (int q = hi; q > mid; --q) out.push_back(order[q]);
      hi = mid;
    } else {
      for (int q = lo; q <= mid; ++q) out.push_back(order[q]);
      lo = mid + 1;
    }
  }
  return out;
}

// Standard dimension tree (Sec. II-C, Fig. 1a).
std::vector<int> dt_path(int N, int n) {
  std::vector<int> order(N);
  for (int i = 0; i < N; ++i) order[i] = i;
  return tree_path(order, n);
}

// MSDT (Sec. III, Fig. 2): subtree j = u / (N-1) has root mode
// N-1 - (j mod N) (0-based) and a binary tree over the next N-1 modes in
// cyclic order.
std::vector<int> msdt_path(int N, int64_t u) {
  const int64_t j = u / (N - 1);
  const int m = (int)((N - 1) - (j % N));
  std::vector<int> order;
  for (int t = 1; t < N; ++t) order.push_back((m + t) % N);
  const int t = (int)(u % (N - 1));
  std::vector<int> out{m};
  std::vector<int> rest = tree_path(order, t);
  out.insert(out.end(), rest.begin(), rest.end());
  return out;
}

// ---------------------------------------------------------------------------
// Mode update (Alg. 1 / Alg. 2 inner body), M in p->Mbuf.
// ---------------------------------------------------------------------------
cp_status ensure_aux(cp_plan p) {
  if (p->aux) return CP_OK;
  HIP_TRY(p, hipStreamCreateWithFlags(&p->aux, hipStreamNonBlocking));
  HIP_TRY(p, hipEventCreateWithFlags(&p->ev_fork, hipEventDisableTiming));
  HIP_TRY(p, hipEventCreateWithFlags(&p->ev_join, hipEventDisableTiming));
  return CP_OK;
}

// Gamma^(n)^-1 on the second stream.  Gamma^(n) (and W^(n)) were formed by
// the previous update (or at state setup), so the inverse depends only on
// the Gram matrices and overlaps the MTTKRP of the same mode.  Nothing to do
// when the previous update already inverted Gamma^(n) itself.
cp_status launch_prep_forked(cp_plan p, int n, bool pp) {
  (void)pp;
  if (p->ginv_ready == n) {
    p->ginv_ready = -1;
    return CP_OK;
  }
  p->ginv_ready = -1;
  p->join_pending = true;
  CP_TRY(ensure_aux(p));
  HIP_TRY(p, hipEventRecord(p->ev_fork, p->st));
  HIP_TRY(p, hipStreamWaitEvent(p->aux, p->ev_fork, 0));
  {
    ProfScope ps(p, CP_PHASE_UPDATE, p->aux);
    HIP_TRY(p, launch_inverse(p->Gamma, p->Ginv, p->R, p->stats, p->aux));
  }
  HIP_TRY(p, hipEventRecord(p->ev_join, p->aux));
  return CP_OK;
}

// Gamma^(n) and W^(n) from the current Gram matrices (state setup).
cp_status form_gamma(cp_plan p, int n, bool pp) {
  p->ginv_ready = -1;
  GammaArgs ga{};
  for (int m = 0; m < p->N; ++m) {
    ga.S[m] = p->S[m];
    ga.dS[m] = p->dS[m];
  }
  ga.Gamma = p->Gamma;
  ga.W = p->W;
  ga.N = p->N;
  ga.n = n;
  ga.R = p->R;
  ga.pp = pp ? 1 : 0;
  HIP_TRY(p, launch_gamma(ga, p->st));
  return CP_OK;
}

// Whether the update of mode n also inverts the next mode's Gamma (inside
// its last workgroup) instead of leaving it to the second stream: worth it
// in exact sweeps when the next MTTKRP is short (the next path starts from a
// cached node), so that nothing would hide the inverse.  In PP sweeps the
// first-order correction kernel of the next mode inverts it in a workgroup
// of its own.  Called after ver[n] moved on.
bool inline_next_inverse(cp_plan p, int n, bool pp) {
  if (pp) return false;  // the next PP correction kernel inverts it alongside
  if (n == p->N - 1) return false;
  const std::vector<int> seq =
      (p->tree == CP_TREE_MSDT) ? msdt_path(p->N, p->msdt_u) : dt_path(p->N, n + 1);
  return path_start(p, seq) >= 1;
}

// Rest of a mode update on the plan stream once the prep has joined:
// A^(n) <- M Gamma^-1 (with V^(n) in PP), shadows, Gram, norms, residual,
// Gamma^(nx) (and its inverse when the next MTTKRP is short).
template <typename TT>
cp_status finish_update_t(cp_plan p, int n, double* A, bool pp) {
  const int R = p->R;
  if (p->join_pending) {
    HIP_TRY(p, hipStreamWaitEvent(p->st, p->ev_join, 0));
    p->join_pending = false;
  }
  ProfScope ps(p, CP_PHASE_UPDATE);
  ++p->ver[n];
  const bool inv_next = inline_next_inverse(p, n, pp);
  UpdateArgs<TT> ua{};
  ua.M = p->Mbuf;
  ua.A = A;
  ua.Ash = (TT*)p->Ash[n];
  ua.Ap = pp ? p->Ap[n] : nullptr;
  ua.dAsh = pp ? (TT*)p->dAsh[n] : nullptr;
  ua.Ginv = p->Ginv;
  ua.partS = p->partS;
  ua.partdS = p->partdS;
  ua.partSc = p->partSc;
  for (int m = 0; m < p->N; ++m) {
    ua.S[m] = p->S[m];
    ua.dS[m] = p->dS[m];
  }
  ua.Gamma = p->Gamma;
  ua.W = p->W;
  ua.stats = p->stats;
  ua.ticket = &p->stats->ticket;
  ua.partG = p->partG;
  ua.s = p->dims[n];
  ua.nrb = (int)((p->dims[n] + 15) / 16);
  ua.R = R;
  ua.n = n;
  ua.N = p->N;
  ua.last = (n == p->N - 1) ? 1 : 0;
  ua.pp = pp ? 1 : 0;
  ua.inv_next = inv_next ? 1 : 0;
  int groups = 1;
  bool fused = true;
  update_shape(p->dims[n], R, pp, &groups, &fused);
  groups = std::min(groups, p->nblk_max);
  ua.fused = fused ? 1 : 0;
  HIP_TRY(p, launch_update<TT>(ua, groups, p->st));
  p->ginv_ready = inv_next ? (n + 1) % p->N : -1;
  return CP_OK;
}

cp_status finish_update(cp_plan p, int n, double* A, bool pp) {
  if (p->prec == CP_F64) return finish_update_t<double>(p, n, A, pp);
  return finish_update_t<float>(p, n, A, pp);
}

cp_status convert_factor(cp_plan p, const double* src, void* dst, int64_t n) {
  if (p->prec == CP_F64) {
    HIP_TRY(p, launch_convert<double>(src, (double*)dst, n, p->st));
  } else {
    HIP_TRY(p, launch_convert<float>(src, (float*)dst, n, p->st));
  }
  return CP_OK;
}

cp_status check_ready(cp_plan p) {
  if (!p) return CP_ERR_ARG;
  if (!p->ws) return fail(p, CP_ERR_STATE, "no workspace attached");
  if (!p->T) return fail(p, CP_ERR_STATE, "no tensor set");
  return CP_OK;
}

// Shadows and Gram matrices from the caller's factors (one setup launch for
// every mode's conversion, Gram matrix and zero dS, and W), then Gamma^(0).
cp_status init_state(cp_plan p, double* const* A) {
  SetupBatch sb;
  const int64_t RR = (int64_t)p->R * p->R;
  for (int m = 0; m < p->N; ++m) {
    sb.op[sb.nops++] = {A[m], p->Ash[m], p->dims[m] * p->R, p->prec == CP_F64 ? kSetupToF64 : kSetupToF32, 0};
    sb.op[sb.nops++] = {A[m], p->S[m], p->dims[m], kSetupGram, p->R};
    sb.op[sb.nops++] = {nullptr, p->dS[m], 2 * RR, kSetupZero32, 0};
    ++p->ver[m];
  }
  sb.op[sb.nops++] = {nullptr, p->W, 2 * RR, kSetupZero32, 0};
  HIP_TRY(p, launch_setup(sb, p->st));
  CP_TRY(form_gamma(p, 0, false));
  p->state_ready = true;
  p->fresh = true;
  return CP_OK;
}

cp_status read_stats(cp_plan p, DevStats* h) {
  HIP_TRY(p, hipMemcpyAsync(h, p->stats, sizeof(DevStats), hipMemcpyDeviceToHost, p->st));
  HIP_TRY(p, hipStreamSynchronize(p->st));
  return CP_OK;
}

void note_fitness(cp_plan p, double r) {
  for (int k = 3; k > 0; --k) p->fit_hist[k] = p->fit_hist[k - 1];
  p->fit_hist[0] = 1.0 - r;
  if (p->n_hist < 4) ++p->n_hist;
  p->pending_fit = false;
}

cp_status fill_info(cp_plan p, cp_sweep_info* info, int kind) {
  DevStats h;
  CP_TRY(read_stats(p, &h));
  if (p->pending_fit) note_fitness(p, h.r);
  const int pinv_seen = p->pinv_seen;
  p->pinv_seen = h.pinv_count;
  if (info) {
    info->kind = kind;
    info->fitness_is_exact = (kind == CP_SWEEP_EXACT) ? 1 : 0;
    info->r = h.r;
    info->fitness = 1.0 - h.r;
    for (int m = 0; m < kMaxOrder; ++m)
      info->dA_rel[m] = m >= p->N ? 0.0 : (h.normA2[m] > 0 ? std::sqrt(h.normdA2[m] / h.normA2[m]) : 1.0);
    info->ttm_count = p->ttm_count;
    info->pinv_updates = h.pinv_count - pinv_seen;
    info->rolled_back = 0;
    info->r_clamped = h.r_clamped;
  }
  if (h.status & 1) return fail(p, CP_ERR_NOT_SPD, "a Gamma matrix had non-finite entries");
  if (h.status & 2) return fail(p, CP_ERR_NUMERIC, "non-finite residual");
  return CP_OK;
}

cp_status exact_sweep(cp_plan p, double* const* A) {
  for (int n = 0; n < p->N; ++n) {
    std::vector<int> seq = (p->tree == CP_TREE_MSDT) ? msdt_path(p->N, p->msdt_u++) : dt_path(p->N, n);
    CP_TRY(launch_prep_forked(p, n, false));
    CP_TRY(run_path(p, seq, p->Mbuf));
    CP_TRY(finish_update(p, n, A[n], false));
  }
  p->phase = 0;
  p->fresh = false;
  return CP_OK;
}

// ---------------------------------------------------------------------------
// PP initialization (Alg. 2; Sec. II-D, Fig. 1b): operators M_p^(i,j) for all
// pairs and M_p^(n) for all n at A_p = A, by the PP dimension tree.  Level l
// keeps N - l modes; its nodes are position i together with the run of
// N-l-1 positions starting at j, 1 <= i < j <= l+2 (C(l+2,2) nodes; the last
// level is every pair).  Positions are mapped to modes through a cyclic
// relabeling chosen so that the first root is the live first-level node of
// the regular sweep when there is one (the footnote's amortized root).
// ---------------------------------------------------------------------------
struct PPNode {
  uint32_t set;
  int parent;  // index into the previous level
};

std::vector<std::vector<PPNode>> pp_tree(int N, const std::vector<int>& order) {
  std::vector<std::vector<PPNode>> levels;
  for (int l = 1; l <= N - 2; ++l) {
    const int w = N - l - 1;
    std::vector<PPNode> nodes;
    for (int i = 1; i <= l + 2; ++i)
      for (int j = i + 1; j <= l + 2; ++j) {
        uint32_t s = 1u << order[i - 1];
        for (int q = j; q < j + w; ++q) s |= 1u << order[q - 1];
        int par = -1;
        if (l > 1) {
          const auto& prev = levels.back();
          for (int k = 0; k < (int)prev.size(); ++k)
            if ((prev[k].set & s) == s) {
              par = k;
              break;
            }
        }
        nodes.push_back({s, par});
      }
    levels.push_back(nodes);
  }
  return levels;
}

int lowest_bit(uint32_t x) {
  for (int b = 0; b < 32; ++b)
    if (x & (1u << b)) return b;
  return -1;
}

int pair_first(uint32_t set) { return lowest_bit(set); }
int pair_second(uint32_t set) { return lowest_bit(set & ~(1u << lowest_bit(set))); }

// Two pair operators of the PP tree from one pass over their parent, a node
// keeping three modes (launch_mttv_pair): child c1 contracts one mode of
// the parent, child c2 another; the third mode is the slice index.  FP32
// plans and the kernel's rank and size limits; *done tells whether it ran.
cp_status pp_pair_fused(cp_plan p, uint32_t pset, uint32_t c1, uint32_t c2, const void* X, bool* done) {
  *done = false;
  if (!f32_tensor(p->prec)) return CP_OK;
  const int m1 = lowest_bit(pset & ~c1), m2 = lowest_bit(pset & ~c2);
  const int z = lowest_bit(pset & ~(1u << m1) & ~(1u << m2));
  if (m1 < 0 || m2 < 0 || z < 0 || m1 == m2) return CP_OK;
  // v: the contracted mode spread over a workgroup's threads (the shorter one)
  const bool swap = p->dims[m1] > p->dims[m2];
  const int v = swap ? m2 : m1, u = swap ? m1 : m2;
  const int R = p->R;
  if (!mttv_pair_fits(p->dims[z], p->dims[v], R)) return CP_OK;
  // element strides of the parent (modes in increasing order, rank last)
  int md[3] = {z, u, v};
  std::sort(md, md + 3);
  int64_t stride[kMaxOrder] = {};
  stride[md[2]] = R;
  stride[md[1]] = p->dims[md[2]] * R;
  stride[md[0]] = p->dims[md[1]] * p->dims[md[2]] * R;
  // output strides of a pair keeping {z, w}: (z's, w's)
  auto pair_strides = [&](int w, int64_t* oz, int64_t* ow) {
    if (z < w) {
      *oz = p->dims[w] * R;
      *ow = R;
    } else {
      *ow = p->dims[z] * R;
      *oz = R;
    }
  };
  int64_t ozv, ouv, ozu, ovu;
  pair_strides(u, &ozv, &ouv);  // contracting v keeps {z, u}
  pair_strides(v, &ozu, &ovu);  // contracting u keeps {z, v}
  float* Ycv = (float*)p->pair[std::min(z, u)][std::max(z, u)];
  float* Ycu = (float*)p->pair[std::min(z, v)][std::max(z, v)];
  ProfScope ps(p, CP_PHASE_MTTV);
  HIP_TRY(p, launch_mttv_pair((const float*)X, (const float*)p->Ash[u], (const float*)p->Ash[v], Ycv, Ycu,
                              p->dims[z], p->dims[u], p->dims[v], stride[z], stride[u], stride[v], ozv, ouv, ozu, ovu,
                              R, (float*)p->pair_parts, p->st));
  *done = true;
  return CP_OK;
}

cp_status pp_node(cp_plan p, const std::vector<std::vector<PPNode>>& lv, int l, int k) {
  const int N = p->N;
  const uint32_t set = lv[l - 1][k].set;
  const bool is_pair = (l == N - 2);
  void* out = is_pair ? p->pair[pair_first(set)][pair_second(set)] : p->slot_buf[l];
  if (l == 1) {
    const int m = lowest_bit(full_set(N) & ~set);
    if (!is_pair && !slot_valid(p, 1, set) && l + 1 == N - 2) {
      // a node whose only child is a pair: the pair straight from the
      // tensor, both contractions in one pass (the node is not formed)
      std::vector<int> kids;
      for (int c = 0; c < (int)lv[l].size(); ++c)
        if (lv[l][c].parent == k) kids.push_back(c);
      FusedOp op;
      if (kids.size() == 1) {
        // the pair is the tensor contracted with both factors, in either
        // order: the node's own mode first, else the child's
        const uint32_t cs = lv[l][kids[0]].set;
        int a = m, b = lowest_bit(set & ~cs);
        bool ok = fused_op_for(p, a, b, false, &op);
        if (!ok) {
          std::swap(a, b);
          ok = fused_op_for(p, a, b, false, &op);
        }
        if (ok) {
          ++p->ttm_count;
          ProfScope ps(p, CP_PHASE_TTM);
          CP_TRY(launch_fused(p, op, a, b, p->pair[pair_first(cs)][pair_second(cs)], nullptr));
          return CP_OK;
        }
      }
    }
    if (!is_pair && slot_valid(p, 1, set)) {
      // live first-level node of the regular sweep: reused, not recomputed
    } else {
      CP_TRY(contract_any(p, p->T, full_set(N), m, out, false));
      if (!is_pair) slot_record(p, 1, set);
    }
  } else {
    const uint32_t pset = lv[l - 2][lv[l - 1][k].parent].set;
    const int m = lowest_bit(pset & ~set);
    CP_TRY(contract_any(p, p->slot_buf[l - 1], pset, m, out, false));
    if (!is_pair) slot_record(p, l, set);
  }
  if (!is_pair) {
    std::vector<int> kids;
    for (int c = 0; c < (int)lv[l].size(); ++c)
      if (lv[l][c].parent == k) kids.push_back(c);
    size_t i = 0;
    // pair children of a node that keeps three modes: two at a time from one
    // pass over the node where the fused kernel applies
    while (l + 1 == N - 2 && i + 1 < kids.size()) {
      bool done = false;
      CP_TRY(pp_pair_fused(p, set, lv[l][kids[i]].set, lv[l][kids[i + 1]].set, p->slot_buf[l], &done));
      if (!done) break;
      i += 2;
    }
    for (; i < kids.size(); ++i) CP_TRY(pp_node(p, lv, l + 1, kids[i]));
  }
  return CP_OK;
}

cp_status pp_init(cp_plan p, double* const* A) {
  const int N = p->N;
  // A_p <- A; dA = 0, so dS = 0, W^(0) = 0 and the shadow of dA (read only by
  // the first-order corrections) is zero; Gamma^(0) is current (S unchanged).
  // One setup launch.
  SetupBatch sb;
  const int64_t RR = (int64_t)p->R * p->R;
  for (int m = 0; m < N; ++m) {
    sb.op[sb.nops++] = {A[m], p->Ap[m], p->dims[m] * p->R, kSetupToF64, 0};
    sb.op[sb.nops++] = {nullptr, p->dS[m], 2 * RR, kSetupZero32, 0};
    sb.op[sb.nops++] = {nullptr, p->dAsh[m], p->dims[m] * p->R * (int64_t)(p->esz / 4), kSetupZero32, 0};
  }
  sb.op[sb.nops++] = {nullptr, p->W, 2 * RR, kSetupZero32, 0};
  HIP_TRY(p, launch_setup(sb, p->st));
  // relabel so that the first root is the live first-level node, if any
  int live = -1;
  for (int m = 0; m < N; ++m)
    if (slot_valid(p, 1, full_set(N) & ~(1u << m))) live = m;
  const int last = (live >= 0) ? live : N - 1;
  std::vector<int> order(N);
  for (int t = 0; t < N; ++t) order[t] = (last + 1 + t) % N;
  auto lv = pp_tree(N, order);
  for (int k = 0; k < (int)lv[0].size(); ++k) CP_TRY(pp_node(p, lv, 1, k));
  // M_p^(n) from the pair {n, n+1 mod N}, contracting the other mode
  for (int n = 0; n < N; ++n) {
    const int x = (n + 1) % N;
    const int a = std::min(n, x), b = std::max(n, x);
    const uint32_t set = (1u << a) | (1u << b);
    CP_TRY(contract_any(p, p->pair[a][b], set, x, p->Mp[n], true));
  }
  p->have_ops = true;
  p->phase = 1;
  return CP_OK;
}

template <typename TT>
cp_status pp_first_order(cp_plan p, int n, bool inv) {
  PPArgs<TT> a{};
  for (int i = 0; i < p->N; ++i) {
    a.dims[i] = p->dims[i];
    a.dA[i] = (const TT*)p->dAsh[i];
    if (i == n) continue;
    const int lo = std::min(n, i), hi = std::max(n, i);
    a.pair[i] = (const TT*)p->pair[lo][hi];
    a.pair_n_first[i] = (n < i) ? 1 : 0;
  }
  a.Mp = p->Mp[n];
  a.M = p->Mbuf;
  a.N = p->N;
  a.n = n;
  a.R = p->R;
  a.Gamma = p->Gamma;
  a.Ginv = inv ? p->Ginv : nullptr;
  a.stats = p->stats;
  ProfScope ps(p, CP_PHASE_PP);
  HIP_TRY(p, launch_pp_mttkrp<TT>(a, p->st));
  return CP_OK;
}

cp_status approx_sweep(cp_plan p, double* const* A) {
  for (int n = 0; n < p->N; ++n) {
    // Gamma^(n)^-1 in a workgroup of the correction kernel, unless the
    // previous update left it
    const bool inv = p->ginv_ready != n;
    p->ginv_ready = -1;
    if (p->prec == CP_F64) {
      CP_TRY(pp_first_order<double>(p, n, inv));
    } else {
      CP_TRY(pp_first_order<float>(p, n, inv));
    }
    CP_TRY(finish_update(p, n, A[n], true));
  }
  p->fresh = false;
  return CP_OK;
}

bool check_factor_ptrs(double* const* A, int N) {
  if (!A) return false;
  for (int m = 0; m < N; ++m)
    if (!A[m]) return false;
  return true;
}

// Learned switch decision: features from the norms of the last updates and
// the fitness history, normalized, through the network on the GPU.
//   x_i = log10(max(||dA_i|| / ||A_i||, 1e-12))            i < N
//   x_{N+j} = log10(max(|f_j - f_{j+1}|, 1e-12))           j = 0, 1, 2 (newest first;
//                                                          a missing delta counts as 1)
cp_status switch_decide(cp_plan p, bool* pp) {
  DevStats h;
  CP_TRY(read_stats(p, &h));
  const int N = p->N, D = N + 3;
  double x[16];
  for (int i = 0; i < N; ++i) {
    const double rel = h.normA2[i] > 0.0 ? std::sqrt(h.normdA2[i] / h.normA2[i]) : 1.0;
    x[i] = std::log10(std::max(rel, 1e-12));
  }
  for (int j = 0; j < 3; ++j) {
    const double d = (p->n_hist >= j + 2) ? std::fabs(p->fit_hist[j] - p->fit_hist[j + 1]) : 1.0;
    x[N + j] = std::log10(std::max(d, 1e-12));
  }
  float xf[16];
  for (int i = 0; i < D; ++i) {
    p->last_feat[i] = x[i];
    xf[i] = (float)((x[i] - p->sw_shift[i]) / p->sw_scale[i]);
  }
  p->last_feat_n = D;
  HIP_TRY(p, hipMemcpyAsync(p->sw_in, xf, D * sizeof(float), hipMemcpyHostToDevice, p->st));
  CP_TRY(cp_mlp_forward(p->sw_in, 1, D, p->sw_H, p->sw_theta, p->sw_out, p->st));
  float prob = 0.f;
  HIP_TRY(p, hipMemcpyAsync(&prob, p->sw_out, sizeof(float), hipMemcpyDeviceToHost, p->st));
  HIP_TRY(p, hipStreamSynchronize(p->st));
  p->last_prob = prob;
  *pp = prob > p->sw_thresh;
  return CP_OK;
}

// Rollback of the learned switch's judge: the factors return to A_p, the
// state at the start of the PP phase (pp_init copied A into A_p), the
// plan's cached state is dropped, and the next kJudgeCooldown outer steps
// are regular sweeps.
constexpr int kJudgeCooldown = 4;

cp_status judge_rollback(cp_plan p, double* const* A) {
  for (int m = 0; m < p->N; ++m)
    HIP_TRY(p, launch_copy_f64(p->Ap[m], A[m], p->dims[m] * p->R, p->st));
  HIP_TRY(p, launch_zero_bytes(&p->stats->status, sizeof(int), p->st));
  const double f = p->sw_entry_fit;
  drop_cache(p);
  p->sw_phase_open = false;
  p->sw_cooldown = kJudgeCooldown;
  p->fit_hist[0] = f;  // the exact fitness of the restored factors
  p->n_hist = 1;
  return CP_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// Allocation-free MTTKRP (cp_mttkrp_static).  Its intermediates (factor
// shadows, the nodes of the dimension-tree path, the BF16 factor parts) live
// in this file-scope device array instead of a caller workspace.  Every
// device the library runs on holds its own copy from module load until the
// process ends.  On the host the array's name is only a stand-in: device
// memory is reached through the address hipGetSymbolAddress gives for the
// current device, looked up once per device and kept.
// ---------------------------------------------------------------------------
constexpr size_t kStaticScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
thread_local std::string g_static_err;

cp_status static_fail(cp_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_static_err = buf;
  return s;
}

// This device's copy of `scratch` (device `dev` must be current).
hipError_t static_scratch(int dev, void** out) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

// Carve the scratch of an MTTKRP of `mode` along the standard tree path:
// the factor shadows, the BF16 factor parts of a low-precision tensor, and
// one node per depth of that path, each region 256-byte aligned.  With
// base == nullptr only the total is computed.
size_t static_layout(cp_plan p, int mode, char* base) {
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char* at = base ? base + off : nullptr;
    off += align_up(bytes ? bytes : 1);
    return at;
  };
  int64_t smax = 0;
  for (int m = 0; m < p->N; ++m) {
    p->Ash[m] = take((size_t)p->dims[m] * p->R * p->esz);
    smax = std::max(smax, p->dims[m]);
  }
  const size_t bt = lowp(p->prec) ? (size_t)p->R * bf16_factor_pitch(smax) * 2 : 0;
  p->Bt_hi = (uint16_t*)take(bt);
  void* lo = take(split_factor(p->prec) ? bt : 0);
  p->Bt_lo = split_factor(p->prec) ? (uint16_t*)lo : nullptr;
  const std::vector<int> seq = dt_path(p->N, mode);
  uint32_t set = full_set(p->N);
  for (int d = 1; d <= p->N - 2; ++d) {
    set &= ~(1u << seq[d - 1]);
    p->slot_cap[d] = (size_t)node_numel(p, set) * p->esz;
    p->slot_buf[d] = take(p->slot_cap[d]);
  }
  return off;
}

}  // namespace

extern "C" {

cp_status cp_plan_create(cp_plan* out, int order, const int64_t* dims, int rank, cp_prec prec,
                         cp_tree tree, void* hip_stream) {
  if (!out || !dims) return CP_ERR_ARG;
  *out = nullptr;
  if (order < 3 || order > kMaxOrder) return CP_ERR_UNSUPPORTED;
  if (rank < 1 || rank > kMaxRank) return CP_ERR_UNSUPPORTED;
  if (prec != CP_F64 && !f32_tensor(prec) && !lowp(prec)) return CP_ERR_UNSUPPORTED;
  if (tree != CP_TREE_DT && tree != CP_TREE_DT_COMBINED && tree != CP_TREE_MSDT) return CP_ERR_UNSUPPORTED;
  double numel = 1.0;
  for (int m = 0; m < order; ++m) {
    if (dims[m] < 1) return CP_ERR_ARG;
    numel *= (double)dims[m];
  }
  if (numel * rank >= 1099511627776.0) return CP_ERR_UNSUPPORTED;
  cp_plan p = new (std::nothrow) cp_plan_s();
  if (!p) return CP_ERR_HIP;
  p->N = order;
  p->R = rank;
  for (int m = 0; m < order; ++m) p->dims[m] = dims[m];
  p->prec = prec;
  p->tree = tree;
  p->st = (hipStream_t)hip_stream;
  p->esz = (prec == CP_F64) ? 8 : 4;
  plan_layout(p);
  *out = p;
  return CP_OK;
}

cp_status cp_plan_workspace_size(cp_plan p, size_t* bytes) {
  if (!p || !bytes) return CP_ERR_ARG;
  *bytes = p->ws_need;
  return CP_OK;
}

cp_status cp_plan_set_workspace(cp_plan p, void* dptr, size_t bytes) {
  if (!p || !dptr) return CP_ERR_ARG;
  if (bytes < p->ws_need) return fail(p, CP_ERR_ARG, "workspace of %zu bytes, need %zu", bytes, p->ws_need);
  if (((uintptr_t)dptr) % kAlign) return fail(p, CP_ERR_ARG, "workspace not 256-byte aligned");
  p->ws = (char*)dptr;
  p->ws_bytes = bytes;
  plan_carve(p);
  drop_cache(p);
  HIP_TRY(p, launch_zero_bytes(p->stats, sizeof(DevStats), p->st));
  return CP_OK;
}

cp_status cp_set_tensor(cp_plan p, const void* T) {
  if (!p || !T) return CP_ERR_ARG;
  if (!p->ws) return fail(p, CP_ERR_STATE, "no workspace attached");
  p->T = T;
  drop_cache(p);
  HIP_TRY(p, launch_zero_bytes(&p->stats->status, sizeof(int), p->st));
  int64_t numel = 1;
  for (int m = 0; m < p->N; ++m) numel *= p->dims[m];
  if (p->prec == CP_F64) {
    HIP_TRY(p, launch_norm2<double>((const double*)T, numel, p->normParts, kNormParts, p->stats, p->st));
  } else if (fp8(p->prec)) {
    HIP_TRY(p, launch_norm2<fp8e4m3>((const fp8e4m3*)T, numel, p->normParts, kNormParts, p->stats, p->st));
  } else if (lowp(p->prec)) {
    HIP_TRY(p, launch_norm2<bf16>((const bf16*)T, numel, p->normParts, kNormParts, p->stats, p->st));
  } else {
    HIP_TRY(p, launch_norm2<float>((const float*)T, numel, p->normParts, kNormParts, p->stats, p->st));
  }
  return CP_OK;
}

cp_status cp_mttkrp(cp_plan p, const double* const* A, int mode, double* M) {
  CP_TRY(check_ready(p));
  if (!A || !M || mode < 0 || mode >= p->N) return fail(p, CP_ERR_ARG, "bad argument");
  for (int m = 0; m < p->N; ++m)
    if (m != mode && !A[m]) return fail(p, CP_ERR_ARG, "null factor %d", m);
  drop_cache(p);
  for (int m = 0; m < p->N; ++m) {
    if (m == mode) continue;
    CP_TRY(convert_factor(p, A[m], p->Ash[m], p->dims[m] * p->R));
    ++p->ver[m];
  }
  p->ttm_count = 0;
  return run_path(p, dt_path(p->N, mode), M);
}

cp_status cp_mttkrp_rooted(cp_plan p, const double* const* A, int mode, int root_mode, double* M) {
  CP_TRY(check_ready(p));
  if (!A || !M || mode < 0 || mode >= p->N || root_mode < 0 || root_mode >= p->N || root_mode == mode)
    return fail(p, CP_ERR_ARG, "bad argument");
  for (int m = 0; m < p->N; ++m)
    if (m != mode && !A[m]) return fail(p, CP_ERR_ARG, "null factor %d", m);
  drop_cache(p);
  for (int m = 0; m < p->N; ++m) {
    if (m == mode) continue;
    CP_TRY(convert_factor(p, A[m], p->Ash[m], p->dims[m] * p->R));
    ++p->ver[m];
  }
  std::vector<int> seq{root_mode};
  for (int m = 0; m < p->N; ++m)
    if (m != mode && m != root_mode) seq.push_back(m);
  p->ttm_count = 0;
  return run_path(p, seq, M);
}

cp_status cp_als_sweep(cp_plan p, double* const* A, cp_sweep_info* info) {
  CP_TRY(check_ready(p));
  if (!check_factor_ptrs(A, p->N)) return fail(p, CP_ERR_ARG, "null factor pointer");
  if (!p->state_ready) CP_TRY(init_state(p, A));
  if (p->sw_set && p->pending_fit) {
    DevStats h;
    CP_TRY(read_stats(p, &h));
    note_fitness(p, h.r);
  }
  p->ttm_count = 0;
  CP_TRY(exact_sweep(p, A));
  p->pending_fit = true;
  if (info) return fill_info(p, info, CP_SWEEP_EXACT);
  return CP_OK;
}

cp_status cp_pp_sweep(cp_plan p, double* const* A, double pp_tol, cp_pp_mode mode, cp_sweep_info* info) {
  CP_TRY(check_ready(p));
  if (!check_factor_ptrs(A, p->N)) return fail(p, CP_ERR_ARG, "null factor pointer");
  if (mode < CP_PP_AUTO || mode > CP_PP_LEARNED) return fail(p, CP_ERR_ARG, "bad PP mode");
  if (mode == CP_PP_LEARNED && !p->sw_set) return fail(p, CP_ERR_STATE, "no learned switch set");
  if (!p->state_ready) CP_TRY(init_state(p, A));
  if ((p->sw_set || mode == CP_PP_LEARNED) && p->pending_fit) {
    DevStats h;
    CP_TRY(read_stats(p, &h));
    note_fitness(p, h.r);
  }
  int kind;
  if (mode == CP_PP_AUTO) {
    if (!(pp_tol > 0.0)) return fail(p, CP_ERR_ARG, "pp_tol must be positive");
    bool ok = false;
    if (!p->fresh) {
      DevStats h;
      CP_TRY(read_stats(p, &h));
      ok = true;
      for (int m = 0; m < p->N; ++m)
        if (!(std::sqrt(h.normdA2[m]) < pp_tol * std::sqrt(h.normA2[m]))) ok = false;
    }
    kind = !ok ? CP_SWEEP_EXACT : (p->phase == 1 ? CP_SWEEP_PP_APPROX : CP_SWEEP_PP_INIT);
  } else if (mode == CP_PP_LEARNED) {
    bool pp = false;
    if (!p->fresh && p->sw_cooldown == 0) CP_TRY(switch_decide(p, &pp));
    if (p->sw_cooldown > 0) --p->sw_cooldown;
    kind = !pp ? CP_SWEEP_EXACT : (p->phase == 1 ? CP_SWEEP_PP_APPROX : CP_SWEEP_PP_INIT);
    if (kind == CP_SWEEP_PP_INIT) {
      // the last sweep was regular: its fitness (noted above) is exact
      p->sw_entry_fit = p->n_hist > 0 ? p->fit_hist[0] : -1e300;
      p->sw_phase_open = true;
    }
  } else if (mode == CP_PP_FORCE_EXACT) {
    kind = CP_SWEEP_EXACT;
  } else if (mode == CP_PP_FORCE_APPROX) {
    if (!p->have_ops || p->phase != 1)
      return fail(p, CP_ERR_STATE, "approximated sweep requested outside the PP phase");
    kind = CP_SWEEP_PP_APPROX;
  } else {
    kind = CP_SWEEP_PP_INIT;
  }
  p->ttm_count = 0;
  if (kind == CP_SWEEP_EXACT) {
    CP_TRY(exact_sweep(p, A));
  } else {
    if (kind == CP_SWEEP_PP_INIT) CP_TRY(pp_init(p, A));
    CP_TRY(approx_sweep(p, A));
  }
  p->pending_fit = true;
  if (mode == CP_PP_LEARNED && p->sw_phase_open) {
    // the judge: a phase that broke down (non-finite state), or that the
    // regular sweep closing it shows to have lost fitness, is undone
    DevStats h;
    CP_TRY(read_stats(p, &h));
    const bool broke = (h.status & 3) != 0;
    const bool closing = (kind == CP_SWEEP_EXACT);
    if (broke || (closing && !(1.0 - h.r >= p->sw_entry_fit))) {
      const int pinv_seen = p->pinv_seen;
      p->pinv_seen = h.pinv_count;
      CP_TRY(judge_rollback(p, A));
      if (info) {
        info->kind = kind;
        info->fitness_is_exact = 1;
        info->fitness = p->fit_hist[0];
        info->r = 1.0 - info->fitness;
        for (int m = 0; m < kMaxOrder; ++m) info->dA_rel[m] = 0.0;
        info->ttm_count = p->ttm_count;
        info->pinv_updates = h.pinv_count - pinv_seen;
        info->rolled_back = 1;
        info->r_clamped = 0;
      }
      return CP_OK;
    }
    if (closing) p->sw_phase_open = false;
  }
  if (info) return fill_info(p, info, kind);
  return CP_OK;
}

cp_status cp_pp_set_switch(cp_plan p, const float* theta, int hidden, const double* shift, const double* scale,
                           double threshold) {
  if (!p) return CP_ERR_ARG;
  if (!theta) {
    p->sw_set = false;
    p->sw_theta = nullptr;
    return CP_OK;
  }
  if (!shift || !scale || hidden < 1 || hidden > 128 || p->N + 3 > 16)
    return fail(p, CP_ERR_ARG, "bad switch arguments");
  const int D = p->N + 3;
  for (int i = 0; i < D; ++i) {
    if (!(scale[i] > 0.0)) return fail(p, CP_ERR_ARG, "feature scale must be positive");
    p->sw_shift[i] = shift[i];
    p->sw_scale[i] = scale[i];
  }
  p->sw_theta = theta;
  p->sw_H = hidden;
  p->sw_thresh = threshold;
  p->sw_set = true;
  return CP_OK;
}

cp_status cp_pp_last_decision(cp_plan p, double* features, double* probability) {
  if (!p || !features || !probability) return CP_ERR_ARG;
  for (int i = 0; i < p->last_feat_n; ++i) features[i] = p->last_feat[i];
  *probability = p->last_prob;
  return CP_OK;
}

cp_status cp_fitness(cp_plan p, const double* const* A, double* fitness) {
  CP_TRY(check_ready(p));
  if (!A || !fitness) return fail(p, CP_ERR_ARG, "bad argument");
  for (int m = 0; m < p->N; ++m)
    if (!A[m]) return fail(p, CP_ERR_ARG, "null factor %d", m);
  drop_cache(p);
  const int n = p->N - 1;
  for (int m = 0; m < p->N; ++m) {
    CP_TRY(convert_factor(p, A[m], p->Ash[m], p->dims[m] * p->R));
    HIP_TRY(p, launch_gram(A[m], p->dims[m], p->R, p->S[m], p->st));
    ++p->ver[m];
  }
  CP_TRY(form_gamma(p, n, false));
  CP_TRY(run_path(p, dt_path(p->N, n), p->Mbuf));
  HIP_TRY(p, launch_fitness(p->Mbuf, A[n], p->dims[n], p->R, p->Gamma, p->S[n], p->stats, p->st));
  DevStats h;
  CP_TRY(read_stats(p, &h));
  *fitness = 1.0 - h.r;
  drop_cache(p);
  return CP_OK;
}

cp_status cp_reset(cp_plan p) {
  if (!p) return CP_ERR_ARG;
  drop_cache(p);
  if (p->ws) HIP_TRY(p, launch_zero_bytes(&p->stats->status, sizeof(int), p->st));
  return CP_OK;
}

cp_status cp_sync(cp_plan p) {
  if (!p) return CP_ERR_ARG;
  if (!p->ws) {
    HIP_TRY(p, hipStreamSynchronize(p->st));
    return CP_OK;
  }
  DevStats h;
  CP_TRY(read_stats(p, &h));
  if (h.status & 1) return fail(p, CP_ERR_NOT_SPD, "a Gamma matrix had non-finite entries");
  if (h.status & 2) return fail(p, CP_ERR_NUMERIC, "non-finite residual");
  return CP_OK;
}

cp_status cp_profile_enable(cp_plan p, int on) {
  if (!p) return CP_ERR_ARG;
  if (on < 0 || on >= (1 << CP_PHASE_COUNT)) return fail(p, CP_ERR_ARG, "bad phase mask %d", on);
  p->prof = (unsigned)on;
  return CP_OK;
}

cp_status cp_profile_read(cp_plan p, double* ms, int64_t* launches) {
  if (!p || !ms || !launches) return CP_ERR_ARG;
  for (int c = 0; c < CP_PHASE_COUNT; ++c) {
    ms[c] = 0.0;
    launches[c] = 0;
  }
  HIP_TRY(p, hipStreamSynchronize(p->st));
  if (p->aux) HIP_TRY(p, hipStreamSynchronize(p->aux));
  cp_status st = CP_OK;
  for (auto& m : p->marks) {
    float t = 0.f;
    hipError_t e = hipEventElapsedTime(&t, m.a, m.b);
    if (e != hipSuccess && st == CP_OK)
      st = fail(p, CP_ERR_HIP, "hipEventElapsedTime failed: %s", hipGetErrorString(e));
    ms[m.cat] += t;
    launches[m.cat] += 1;
    p->pool.push_back(m.a);
    p->pool.push_back(m.b);
  }
  p->marks.clear();
  return st;
}

cp_status cp_plan_destroy(cp_plan p) {
  if (!p) return CP_ERR_ARG;
  for (auto& m : p->marks) {
    hipEventDestroy(m.a);
    hipEventDestroy(m.b);
  }
  for (auto e : p->pool) hipEventDestroy(e);
  if (p->aux) {
    hipStreamSynchronize(p->aux);
    hipStreamDestroy(p->aux);
    hipEventDestroy(p->ev_fork);
    hipEventDestroy(p->ev_join);
  }
  delete p;
  return CP_OK;
}

cp_status cp_mttkrp_static(int order, const int64_t* dims, int rank, cp_prec prec, const void* T,
                           const double* const* A, int mode, double* M, void* hip_stream) {
  g_static_err.clear();
  if (!dims || !T || !A || !M) return static_fail(CP_ERR_ARG, "null argument");
  if (order < 3 || order > kMaxOrder || rank < 1 || rank > kMaxRank)
    return static_fail(CP_ERR_UNSUPPORTED, "order %d / rank %d outside the limits", order, rank);
  if (prec != CP_F64 && prec != CP_F32 && !lowp(prec)) return static_fail(CP_ERR_UNSUPPORTED, "bad precision");
  if (mode < 0 || mode >= order) return static_fail(CP_ERR_ARG, "bad mode %d", mode);
  for (int m = 0; m < order; ++m) {
    if (dims[m] < 1) return static_fail(CP_ERR_ARG, "dims[%d] = %lld", m, (long long)dims[m]);
    if (m != mode && !A[m]) return static_fail(CP_ERR_ARG, "null factor %d", m);
  }
  cp_plan_s pl;
  cp_plan p = &pl;
  p->N = order;
  p->R = rank;
  for (int m = 0; m < order; ++m) p->dims[m] = dims[m];
  p->prec = prec;
  p->tree = CP_TREE_DT;
  p->st = (hipStream_t)hip_stream;
  p->esz = (prec == CP_F64) ? 8 : 4;
  const size_t need = static_layout(p, mode, nullptr);
  if (need > kStaticScratchBytes)
    return static_fail(CP_ERR_UNSUPPORTED, "needs %zu bytes of scratch; the static scratch holds %zu", need,
                       kStaticScratchBytes);
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return static_fail(CP_ERR_HIP, "hipGetDevice failed: %s", hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return static_fail(CP_ERR_UNSUPPORTED, "device %d", dev);
  void* base = nullptr;
  e = static_scratch(dev, &base);
  if (e != hipSuccess) return static_fail(CP_ERR_HIP, "hipGetSymbolAddress failed: %s", hipGetErrorString(e));
  static_layout(p, mode, (char*)base);
  p->ws = (char*)base;
  p->ws_bytes = kStaticScratchBytes;
  p->T = T;
  for (int m = 0; m < order; ++m) {
    if (m == mode) continue;
    const cp_status s = convert_factor(p, A[m], p->Ash[m], p->dims[m] * p->R);
    if (s != CP_OK) return static_fail(s, "%s", p->err.c_str());
    ++p->ver[m];
  }
  const cp_status s = run_path(p, dt_path(order, mode), M);
  if (s != CP_OK) return static_fail(s, "%s", p->err.c_str());
  return CP_OK;
}

const char* cp_status_str(cp_status s) {
  switch (s) {
    case CP_OK: return "ok";
    case CP_ERR_ARG: return "invalid argument";
    case CP_ERR_STATE: return "call out of order";
    case CP_ERR_UNSUPPORTED: return "unsupported size or option";
    case CP_ERR_HIP: return "HIP runtime error";
    case CP_ERR_NOT_SPD: return "Gamma not finite";
    case CP_ERR_NUMERIC: return "non-finite result";
  }
  return "unknown status";
}

const char* cp_last_error(cp_plan p) {
  if (!p) return g_static_err.empty() ? "null plan" : g_static_err.c_str();
  return p->err.c_str();
}

}  // extern "C"
