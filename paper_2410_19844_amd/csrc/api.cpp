// C ABI of libsos (declared in include/sos.h): argument checks, call
// sequencing on the caller's stream, and the host side of the solve loop.
#include <algorithm>
#include <numeric>
#include <cmath>
#include <cstring>
#include <limits>
#include <mutex>
#include <string>
#include <utility>

#include "sos_internal.h"

namespace sos {

static thread_local std::string g_last_error;

int set_error(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

int hip_error(hipError_t e, const char* what) {
  return set_error(SOS_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define SOS_HIP(call, what)                          \
  do {                                               \
    hipError_t e_ = (call);                          \
    if (e_ != hipSuccess) return hip_error(e_, what); \
  } while (0)

// Event pairs around launches while sos_timing is on.
static hipEvent_t take_event(sos_plan_s* p) {
  if (!p->event_pool.empty()) {
    hipEvent_t e = p->event_pool.back();
    p->event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

struct Timer {
  sos_plan_s* p;
  int cls;
  hipStream_t s;
  hipEvent_t a = nullptr, b = nullptr;
  Timer(sos_plan_s* p_, int c, hipStream_t s_) : p(p_), cls(c), s(s_) {
    if (!p->timing) return;
    a = take_event(p);
    b = take_event(p);
    if (a && b) (void)hipEventRecord(a, s);
  }
  void done() {
    if (!p->timing || !a || !b) return;
    (void)hipEventRecord(b, s);
    p->timed.push_back({cls, a, b});
    a = b = nullptr;
  }
  ~Timer() {
    if (a) p->event_pool.push_back(a);
    if (b) p->event_pool.push_back(b);
  }
};

#define TIMED(cls, call, what)   \
  do {                            \
    Timer tm_(p, cls, s);         \
    SOS_HIP(call, what);          \
    tm_.done();                   \
  } while (0)

static int check_bound(const sos_plan_s* p, const char* fn) {
  if (!p) return set_error(SOS_EINVAL, std::string(fn) + ": plan is NULL");
  if (!p->bound) return set_error(SOS_EINVAL, std::string(fn) + ": plan is not bound to a workspace");
  return SOS_OK;
}

static size_t slot_bytes(const sos_plan_s* p) { return p->state_bytes / 4; }
static size_t w_elem(const sos_plan_s* p) { return p->prec == SOS_FP64 ? 8 : 4; }
static double* scal(const sos_plan_s* p) { return (double*)(p->ws + p->lay.scal); }

// r <- coeff(W W^T) - p in the workspace, L = ||r||^2 -> d_loss.
static int fwd_mode(const sos_plan_s* p, int flags) {
  if (p->prec == SOS_FP64) return kFwdFast;
  if (flags & SOS_FLAG_EXACT_FORWARD) return kFwdExact;
  if (flags & SOS_FLAG_OZAKI_FORWARD) return kFwdOzaki;
  if ((flags & SOS_FLAG_FP32_FORWARD) && split_plan(p)) return kFwdF32;
  if ((flags & SOS_FLAG_SINGLE_FORWARD) && split_plan(p)) return kFwdSingle;
  return kFwdFast;
}

// Digit slices of the Ozaki forward.
static int oz_slices(int flags) {
  return (flags & SOS_FLAG_OZAKI_FOUR_SLICES) ? 4 : (flags & SOS_FLAG_OZAKI_FIVE_SLICES) ? 5 : kOzSlices;
}

// grad: a backward follows (so the transposed operand copies are needed).
// reuse: the operand copies already in the workspace were made from this W
// for this mode (by the epilogue of the previous fused step): no preparation.
static int run_forward(sos_plan_s* p, const void* W, const double* d_p, int flags, double* d_loss,
                       bool grad, hipStream_t s, bool reuse = false) {
  const int mode = fwd_mode(p, flags);
  if (!reuse) {
    PrepNeeds need;
    need.a = p->prec == SOS_FP64 || mode == kFwdFast || mode == kFwdSingle;
    need.a_f32 = mode == kFwdF32;
    need.x_f32 = mode == kFwdExact;
    need.t = grad;
    need.t_lo = grad && (flags & SOS_FLAG_SINGLE_BACKWARD) == 0;
    TIMED(SOS_K_PREP, launch_prep(p, W, need, s), "prep");
    p->copies_valid = false;
    p->t_cur = 0;  // the preparation writes the transposed copy into t_hi
  }
  // the int8 slices need the row maxima of W, so no GEMM epilogue leaves them: built every time
  if (mode == kFwdOzaki) TIMED(SOS_K_PREP, launch_oz_slices(p, (const float*)W, s, oz_slices(flags)), "Ozaki slices");
  if ((flags & SOS_FLAG_DETERMINISTIC) && mode == kFwdFast) {
    TIMED(SOS_K_GRAM, launch_gram_det(p, d_p, s), "gram (deterministic)");
  } else if ((flags & SOS_FLAG_UNFUSED_SCATTER) && mode == kFwdFast && p->prec == SOS_BF16X3) {
    TIMED(SOS_K_INIT, launch_init_r(p, d_p, s), "init_r");
    TIMED(SOS_K_GRAM, launch_gram_bf3(p, s, true), "gram (tiles stored)");
    TIMED(SOS_K_SCATTER, launch_scatter_tiles(p, s), "scatter");
  } else {
    TIMED(SOS_K_INIT, launch_init_r(p, d_p, s), "init_r");
    TIMED(SOS_K_GRAM, launch_gram(p, mode, s, (flags & SOS_FLAG_UNMERGED_SCATTER) != 0, oz_slices(flags)), "gram");
  }
  float* r32 = (grad && p->prec != SOS_FP64) ? (float*)(p->ws + p->lay.r32) : nullptr;
  TIMED(SOS_K_LOSS, launch_sumsq(p, (const double*)(p->ws + p->lay.r), p->M, d_loss, s, r32), "loss");
  return SOS_OK;
}

static int run_backward(sos_plan_s* p, void* g, bool split, hipStream_t s) {
  TIMED(SOS_K_GATHER, launch_gather(p, split, s), "gather");
  TIMED(SOS_K_RW, launch_rw(p, g, split, s), "backward");
  return SOS_OK;
}

// One Adam step.  Split plans with the single-product backward and the fast
// or exact forward run the fused backward (Adam and the next step's operand
// copies in the GEMM epilogue); with SOS_FLAG_COPIES_VALID the next such
// step on the same W and mode then skips the preparation.
static int run_step(sos_plan_s* p, void* W, void* state, int64_t t, const double* d_p,
                    const sos_adam_t& h, double* d_loss, int flags, hipStream_t s) {
  const int mode = fwd_mode(p, flags);
  const bool single = (flags & SOS_FLAG_SINGLE_BACKWARD) != 0;
  const bool fuse = split_plan(p) && single &&
                    (mode == kFwdFast || mode == kFwdSingle || mode == kFwdExact || mode == kFwdOzaki);
  const bool reuse = fuse && (flags & SOS_FLAG_COPIES_VALID) && p->copies_valid && p->copies_W == W &&
                     p->copies_mode == mode;
  int rc = run_forward(p, W, d_p, flags, d_loss, true, s, reuse);
  if (rc) return rc;
  char* st = (char*)state;
  if (fuse) {
    TIMED(SOS_K_GATHER, launch_gather(p, false, s), "gather");
    TIMED(SOS_K_RW, launch_rw_adam_bf3(p, W, st, st + slot_bytes(p), t, h, mode, s),
          "backward + Adam");
    p->t_cur ^= 1;
    p->copies_valid = true;
    p->copies_W = W;
    p->copies_mode = mode;
    return SOS_OK;
  }
  void* g = p->ws + p->lay.g;
  rc = run_backward(p, g, !single, s);
  if (rc) return rc;
  TIMED(SOS_K_ADAM, launch_adam(p, W, st, st + slot_bytes(p), g, t, h, s), "adam");
  return SOS_OK;
}

// The deterministic forward replaces the atomic scatter of the plan's own
// (fast) forward in FP32 and FP64 plans that carry pair lists.
static int check_det(const sos_plan_s* p, int flags, const char* fn) {
  if (!(flags & SOS_FLAG_DETERMINISTIC)) return SOS_OK;
  if (!p->det_ok)
    return set_error(SOS_EINVAL, std::string(fn) + ": SOS_FLAG_DETERMINISTIC needs an FP32 or FP64 plan with N <= " +
                                     std::to_string(SOS_BATCH_MAX_N));
  if (fwd_mode(p, flags) != kFwdFast)
    return set_error(SOS_EINVAL, std::string(fn) + ": SOS_FLAG_DETERMINISTIC covers the plan's own forward only");
  return SOS_OK;
}

// The unfused scatter is a measurement variant of the split plans' fast forward.
static int check_unfused(const sos_plan_s* p, int flags, const char* fn) {
  if (!(flags & SOS_FLAG_UNFUSED_SCATTER)) return SOS_OK;
  if (p->prec != SOS_BF16X3 || fwd_mode(p, flags) != kFwdFast)
    return set_error(SOS_EINVAL, std::string(fn) + ": SOS_FLAG_UNFUSED_SCATTER needs a split plan's fast forward");
  return SOS_OK;
}

// The unmerged scatter is a measurement variant of the split plans' fused fast forward.
static int check_unmerged(const sos_plan_s* p, int flags, const char* fn) {
  if (!(flags & SOS_FLAG_UNMERGED_SCATTER)) return SOS_OK;
  if (!split_plan(p) || fwd_mode(p, flags) != kFwdFast || (flags & SOS_FLAG_UNFUSED_SCATTER))
    return set_error(SOS_EINVAL, std::string(fn) + ": SOS_FLAG_UNMERGED_SCATTER needs a split plan's fused fast forward");
  return SOS_OK;
}

// The single-product forward is a variant of the split plans' fused fast forward.
static int check_single(const sos_plan_s* p, int flags, const char* fn) {
  if (!(flags & SOS_FLAG_SINGLE_FORWARD)) return SOS_OK;
  if (!split_plan(p))
    return set_error(SOS_EINVAL, std::string(fn) + ": SOS_FLAG_SINGLE_FORWARD needs a SOS_BF16X3 or SOS_FP16X3 plan");
  if (flags & (SOS_FLAG_UNFUSED_SCATTER | SOS_FLAG_UNMERGED_SCATTER | SOS_FLAG_DETERMINISTIC))
    return set_error(SOS_EINVAL, std::string(fn) + ": SOS_FLAG_SINGLE_FORWARD does not combine with the "
                                                   "measurement variants of the scatter");
  return SOS_OK;
}

// The Ozaki forward needs an FP32 master W and a K extent whose level sums stay exact in int32.
static int check_ozaki(const sos_plan_s* p, int flags, const char* fn) {
  if ((flags & SOS_FLAG_OZAKI_FIVE_SLICES) && !(flags & SOS_FLAG_OZAKI_FORWARD))
    return set_error(SOS_EINVAL, std::string(fn) + ": SOS_FLAG_OZAKI_FIVE_SLICES needs SOS_FLAG_OZAKI_FORWARD");
  if ((flags & SOS_FLAG_OZAKI_FOUR_SLICES) && (!(flags & SOS_FLAG_OZAKI_FORWARD) || (flags & SOS_FLAG_OZAKI_FIVE_SLICES)))
    return set_error(SOS_EINVAL, std::string(fn) + ": SOS_FLAG_OZAKI_FOUR_SLICES needs SOS_FLAG_OZAKI_FORWARD "
                                                   "and excludes SOS_FLAG_OZAKI_FIVE_SLICES");
  if (!(flags & SOS_FLAG_OZAKI_FORWARD) || (flags & SOS_FLAG_EXACT_FORWARD)) return SOS_OK;
  if (p->prec == SOS_FP64)
    return set_error(SOS_EINVAL, std::string(fn) + ": SOS_FLAG_OZAKI_FORWARD needs an FP32 or split plan");
  if (!ozaki_supported(p))
    return set_error(SOS_ERANGE, std::string(fn) + ": SOS_FLAG_OZAKI_FORWARD needs rank <= " +
                                     std::to_string(kOzMaxK / kPadK * kPadK));
  return SOS_OK;
}

static int check_adam(const sos_adam_t* h, const char* fn) {
  if (!h) return set_error(SOS_EINVAL, std::string(fn) + ": adam is NULL");
  if (!(h->lr > 0) || !(h->beta1 >= 0 && h->beta1 < 1) || !(h->beta2 >= 0 && h->beta2 < 1) || !(h->eps >= 0))
    return set_error(SOS_EINVAL, std::string(fn) + ": Adam needs lr > 0, 0 <= beta < 1, eps >= 0");
  return SOS_OK;
}

}  // namespace sos

using namespace sos;

sos_plan_s::~sos_plan_s() {
  for (auto& t : timed) {
    (void)hipEventDestroy(t.a);
    (void)hipEventDestroy(t.b);
  }
  for (auto e : event_pool) (void)hipEventDestroy(e);
}

extern "C" {

int sos_timing(sos_plan_t p, int enable) {
  if (!p) return set_error(SOS_EINVAL, "sos_timing: plan is NULL");
  if (enable) {
    for (auto& t : p->timed) {
      p->event_pool.push_back(t.a);
      p->event_pool.push_back(t.b);
    }
    p->timed.clear();
  }
  p->timing = enable != 0;
  return SOS_OK;
}

int sos_timing_read(sos_plan_t p, double* h_ms, int64_t* h_calls) {
  if (!p || !h_ms) return set_error(SOS_EINVAL, "sos_timing_read: NULL argument");
  for (int c = 0; c < SOS_K_COUNT; ++c) {
    h_ms[c] = 0;
    if (h_calls) h_calls[c] = 0;
  }
  for (auto& t : p->timed) {
    float ms = 0;
    SOS_HIP(hipEventSynchronize(t.b), "sos_timing_read");
    SOS_HIP(hipEventElapsedTime(&ms, t.a, t.b), "sos_timing_read");
    h_ms[t.cls] += ms;
    if (h_calls) h_calls[t.cls] += 1;
    p->event_pool.push_back(t.a);
    p->event_pool.push_back(t.b);
  }
  p->timed.clear();
  return SOS_OK;
}

int sos_plan(int n, int d, int rank, int precision, sos_plan_t* out) {
  try {
    return plan_create(n, d, rank, precision, out);
  } catch (...) {
    return set_error(SOS_ENOMEM, "sos_plan: host allocation failed");
  }
}

int sos_plan_query(sos_plan_t p, int64_t* N, int64_t* M, size_t* ws_bytes, size_t* state_bytes) {
  if (!p) return set_error(SOS_EINVAL, "sos_plan_query: plan is NULL");
  if (N) *N = p->N;
  if (M) *M = p->M;
  if (ws_bytes) *ws_bytes = p->lay.bytes;
  if (state_bytes) *state_bytes = p->state_bytes;
  return SOS_OK;
}

int sos_plan_bind(sos_plan_t p, void* d_ws, size_t ws_bytes, void* stream) {
  if (!p) return set_error(SOS_EINVAL, "sos_plan_bind: plan is NULL");
  if (!d_ws) return set_error(SOS_EINVAL, "sos_plan_bind: workspace is NULL");
  if (((uintptr_t)d_ws) % 256) return set_error(SOS_EINVAL, "sos_plan_bind: workspace must be 256-byte aligned");
  if (ws_bytes < p->lay.bytes)
    return set_error(SOS_ENOMEM, "sos_plan_bind: workspace smaller than sos_plan_query's ws_bytes");
  hipStream_t s = (hipStream_t)stream;
  p->ws = (char*)d_ws;
  p->ws_size = ws_bytes;
  SOS_HIP(hipMemcpyAsync(p->ws + p->lay.codes, p->codes.data(), p->codes.size() * 4, hipMemcpyHostToDevice, s),
          "sos_plan_bind: codes");
  SOS_HIP(hipMemcpyAsync(p->ws + p->lay.tables, p->tables.data(), p->tables.size() * 4, hipMemcpyHostToDevice, s),
          "sos_plan_bind: tables");
  SOS_HIP(hipMemcpyAsync(p->ws + p->lay.tiles, p->tile_list.data(), p->tile_list.size() * 4, hipMemcpyHostToDevice, s),
          "sos_plan_bind: tiles");
  if (p->det_ok) {
    SOS_HIP(hipMemcpyAsync(p->ws + p->lay.pair_off, p->pair_off.data(), p->pair_off.size() * 4,
                           hipMemcpyHostToDevice, s), "sos_plan_bind: pair offsets");
    SOS_HIP(hipMemcpyAsync(p->ws + p->lay.pair_idx, p->pair_idx.data(), p->pair_idx.size() * 4,
                           hipMemcpyHostToDevice, s), "sos_plan_bind: pair lists");
  }
  if (p->batchable) {
    SOS_HIP(hipMemcpyAsync(p->ws + p->lay.pair_pos, p->pair_pos.data(), p->pair_pos.size() * 4,
                           hipMemcpyHostToDevice, s), "sos_plan_bind: pair positions");
    SOS_HIP(hipMemcpyAsync(p->ws + p->lay.rank_map, p->rank_map.data(), p->rank_map.size() * 4,
                           hipMemcpyHostToDevice, s), "sos_plan_bind: rank map");
    SOS_HIP(hipMemsetAsync(p->ws + p->lay.bcount, 0, 4, s), "sos_plan_bind: block counter");
    SOS_HIP(hipMemcpyAsync(p->ws + p->lay.bhdr, &p->bhdr, sizeof(BatchHeader), hipMemcpyHostToDevice, s),
            "sos_plan_bind: batch header");
  }
  p->merge_ready = false;
  if (split_plan(p)) SOS_HIP(launch_merge_maps(p, s), "sos_plan_bind: merge maps of the gram epilogue");
  SOS_HIP(hipStreamSynchronize(s), "sos_plan_bind");
  if (split_plan(p) && p->ntiles256 > 0) {
    // merge only where it saves atomics (the counts the map kernel left)
    const size_t segs = (size_t)p->ntiles256 * kMergeSegs;
    std::vector<int32_t> issued(segs);
    SOS_HIP(hipMemcpy(issued.data(), p->ws + p->lay.mg_count + segs * 4, segs * 4, hipMemcpyDeviceToHost),
            "sos_plan_bind: merge counts");
    double atomics = 0;
    for (int32_t c : issued) atomics += c;
    const double pairs = 0.5 * (double)p->N * (double)(p->N + 1);
    p->merge_ready = pairs >= kMergeMinRatio * atomics;
  }
  p->bound = true;
  return SOS_OK;
}

void sos_plan_destroy(sos_plan_t p) { delete p; }

int sos_exponents(sos_plan_t p, int which, uint8_t* h_out) {
  if (!p || !h_out) return set_error(SOS_EINVAL, "sos_exponents: NULL argument");
  if (which == 0) {
    std::memcpy(h_out, p->basis.data(), p->basis.size());
    return SOS_OK;
  }
  if (which == 1) {
    std::vector<uint8_t> e;
    try {
      enumerate_monomials(p->n, 2 * p->d, e);
    } catch (...) {
      return set_error(SOS_ENOMEM, "sos_exponents: host allocation failed");
    }
    std::memcpy(h_out, e.data(), e.size());
    return SOS_OK;
  }
  return set_error(SOS_EINVAL, "sos_exponents: which must be 0 (basis) or 1 (coefficients)");
}

int sos_pair_ranks(sos_plan_t p, int32_t* d_out, void* stream) {
  if (int rc = check_bound(p, "sos_pair_ranks")) return rc;
  if (!d_out) return set_error(SOS_EINVAL, "sos_pair_ranks: d_out is NULL");
  SOS_HIP(launch_pair_ranks(p, d_out, (hipStream_t)stream), "sos_pair_ranks");
  return SOS_OK;
}

int sos_loss_grad(sos_plan_t p, const void* d_W, const double* d_p, double* d_loss, void* d_grad,
                  double* d_r, int flags, void* stream) {
  if (int rc = check_bound(p, "sos_loss_grad")) return rc;
  if (!d_W || !d_p || !d_loss) return set_error(SOS_EINVAL, "sos_loss_grad: d_W, d_p and d_loss are required");
  if (flags & ~(int)(SOS_FLAG_EXACT_FORWARD | SOS_FLAG_SINGLE_BACKWARD | SOS_FLAG_FP32_FORWARD |
                     SOS_FLAG_OZAKI_FORWARD | SOS_FLAG_DETERMINISTIC | SOS_FLAG_UNFUSED_SCATTER |
                     SOS_FLAG_UNMERGED_SCATTER | SOS_FLAG_OZAKI_FIVE_SLICES | SOS_FLAG_SINGLE_FORWARD |
                     SOS_FLAG_OZAKI_FOUR_SLICES))
    return set_error(SOS_EINVAL, "sos_loss_grad: unknown flags");
  if (int rc = check_single(p, flags, "sos_loss_grad")) return rc;
  if (int rc = check_unmerged(p, flags, "sos_loss_grad")) return rc;
  if (int rc = check_ozaki(p, flags, "sos_loss_grad")) return rc;
  if (int rc = check_unfused(p, flags, "sos_loss_grad")) return rc;
  if (int rc = check_det(p, flags, "sos_loss_grad")) return rc;
  hipStream_t s = (hipStream_t)stream;
  int rc = run_forward(p, d_W, d_p, flags, d_loss, d_grad != nullptr, s);
  if (rc) return rc;
  if (d_grad && (rc = run_backward(p, d_grad, (flags & SOS_FLAG_SINGLE_BACKWARD) == 0, s))) return rc;
  if (d_r)
    SOS_HIP(hipMemcpyAsync(d_r, p->ws + p->lay.r, p->M * 8, hipMemcpyDeviceToDevice, s), "sos_loss_grad: r");
  return SOS_OK;
}

int sos_step(sos_plan_t p, void* d_W, void* d_state, int64_t t, const double* d_p, const sos_adam_t* adam,
             double* d_loss, int flags, void* stream) {
  if (int rc = check_bound(p, "sos_step")) return rc;
  if (int rc = check_adam(adam, "sos_step")) return rc;
  if (!d_W || !d_state || !d_p || !d_loss) return set_error(SOS_EINVAL, "sos_step: NULL device pointer");
  if (t < 1) return set_error(SOS_EINVAL, "sos_step: t is 1-based");
  if (flags & ~(int)(SOS_FLAG_EXACT_FORWARD | SOS_FLAG_COPIES_VALID | SOS_FLAG_SINGLE_BACKWARD |
                     SOS_FLAG_FP32_FORWARD | SOS_FLAG_OZAKI_FORWARD | SOS_FLAG_DETERMINISTIC |
                     SOS_FLAG_UNFUSED_SCATTER | SOS_FLAG_UNMERGED_SCATTER | SOS_FLAG_OZAKI_FIVE_SLICES |
                     SOS_FLAG_SINGLE_FORWARD | SOS_FLAG_OZAKI_FOUR_SLICES))
    return set_error(SOS_EINVAL, "sos_step: unknown flags");
  if (int rc = check_single(p, flags, "sos_step")) return rc;
  if (int rc = check_unmerged(p, flags, "sos_step")) return rc;
  if (int rc = check_ozaki(p, flags, "sos_step")) return rc;
  if (int rc = check_unfused(p, flags, "sos_step")) return rc;
  if (int rc = check_det(p, flags, "sos_step")) return rc;
  return run_step(p, d_W, d_state, t, d_p, *adam, d_loss, flags, (hipStream_t)stream);
}

int sos_verify(sos_plan_t p, const void* d_W, const double* d_p, double* h_rel, double* d_r, void* stream) {
  if (int rc = check_bound(p, "sos_verify")) return rc;
  if (!d_W || !d_p || !h_rel) return set_error(SOS_EINVAL, "sos_verify: NULL argument");
  hipStream_t s = (hipStream_t)stream;
  double* sc = scal(p);
  int rc = run_forward(p, d_W, d_p, SOS_FLAG_EXACT_FORWARD, sc + 0, false, s);
  if (rc) return rc;
  SOS_HIP(launch_sumsq(p, d_p, p->M, sc + 1, s), "sos_verify: ||p||");
  double h[2];
  SOS_HIP(hipMemcpyAsync(h, sc, sizeof(h), hipMemcpyDeviceToHost, s), "sos_verify: readback");
  if (d_r) SOS_HIP(hipMemcpyAsync(d_r, p->ws + p->lay.r, p->M * 8, hipMemcpyDeviceToDevice, s), "sos_verify: r");
  SOS_HIP(hipStreamSynchronize(s), "sos_verify");
  const double np = std::sqrt(h[1]);
  *h_rel = std::sqrt(h[0]) / (np > 0 ? np : 1.0);
  return SOS_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Allocation-free loss and gradient: the workspace is the library's own
// static device array instead of caller memory.
// ---------------------------------------------------------------------------
namespace sos {

// One copy per GPU, alive until the process ends.  In host code the name is
// only a stand-in for the symbol: kernels and copies get the device address
// that hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) char scratch[SOS_NOALLOC_MAX_WS];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_at[kMaxDevices];

// Device address of `scratch` on the device that runs `stream` (looked up once
// per device, with that device current).
static int scratch_for_stream(hipStream_t s, char** out) {
  int cur = 0, dev = 0;
  SOS_HIP(hipGetDevice(&cur), "sos_loss_grad_noalloc: current device");
  dev = cur;
  if (s) SOS_HIP(hipStreamGetDevice(s, &dev), "sos_loss_grad_noalloc: device of the stream");
  if (dev < 0 || dev >= kMaxDevices) return set_error(SOS_ERANGE, "sos_loss_grad_noalloc: device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_at[dev]) {
    if (dev != cur) SOS_HIP(hipSetDevice(dev), "sos_loss_grad_noalloc: select the stream's device");
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (dev != cur) (void)hipSetDevice(cur);
    if (e != hipSuccess) return hip_error(e, "sos_loss_grad_noalloc: address of the static workspace");
    if (!ptr) return set_error(SOS_EHIP, "sos_loss_grad_noalloc: static workspace has no device address");
    g_scratch_at[dev] = ptr;
  }
  *out = (char*)g_scratch_at[dev];
  return SOS_OK;
}

// Points an unbound plan at the static workspace for one call and detaches it
// again on every return path; event timing stays off meanwhile (it would
// create HIP events).
struct ScratchBinding {
  sos_plan_s* p;
  bool timing;
  ScratchBinding(sos_plan_s* p_, char* base) : p(p_), timing(p_->timing) {
    p->ws = base;
    p->ws_size = SOS_NOALLOC_MAX_WS;
    p->bound = true;
    p->timing = false;
  }
  ~ScratchBinding() {
    p->ws = nullptr;
    p->ws_size = 0;
    p->bound = false;
    p->copies_valid = false;
    p->timing = timing;
  }
};

}  // namespace sos

extern "C" {

int sos_loss_grad_noalloc(sos_plan_t p, const void* d_W, const double* d_p, double* d_loss, void* d_grad,
                          double* d_r, int flags, void* stream) {
  if (!p) return set_error(SOS_EINVAL, "sos_loss_grad_noalloc: plan is NULL");
  if (p->bound)
    return set_error(SOS_EINVAL, "sos_loss_grad_noalloc: plan is bound to a workspace (use sos_loss_grad)");
  if (!d_W || !d_p || !d_loss)
    return set_error(SOS_EINVAL, "sos_loss_grad_noalloc: d_W, d_p and d_loss are required");
  if (flags & ~(int)(SOS_FLAG_EXACT_FORWARD | SOS_FLAG_SINGLE_BACKWARD | SOS_FLAG_FP32_FORWARD |
                     SOS_FLAG_OZAKI_FORWARD | SOS_FLAG_OZAKI_FIVE_SLICES | SOS_FLAG_OZAKI_FOUR_SLICES))
    return set_error(SOS_EINVAL, "sos_loss_grad_noalloc: unknown flags");
  if (int rc = check_ozaki(p, flags, "sos_loss_grad_noalloc")) return rc;
  if (p->lay.bytes > (size_t)SOS_NOALLOC_MAX_WS)
    return set_error(SOS_ERANGE, "sos_loss_grad_noalloc: the plan needs a workspace of " +
                                     std::to_string(p->lay.bytes) + " bytes, above the static " +
                                     std::to_string((size_t)SOS_NOALLOC_MAX_WS) + " (use sos_loss_grad)");
  hipStream_t s = (hipStream_t)stream;
  char* base = nullptr;
  if (int rc = scratch_for_stream(s, &base)) return rc;
  ScratchBinding bind(p, base);
  // the ranking tables and the tile list, as sos_plan_bind uploads them; every
  // other region the kernels read is written earlier in the same call
  SOS_HIP(hipMemcpyAsync(p->ws + p->lay.codes, p->codes.data(), p->codes.size() * 4, hipMemcpyHostToDevice, s),
          "sos_loss_grad_noalloc: codes");
  SOS_HIP(hipMemcpyAsync(p->ws + p->lay.tables, p->tables.data(), p->tables.size() * 4, hipMemcpyHostToDevice, s),
          "sos_loss_grad_noalloc: tables");
  SOS_HIP(hipMemcpyAsync(p->ws + p->lay.tiles, p->tile_list.data(), p->tile_list.size() * 4, hipMemcpyHostToDevice,
                         s), "sos_loss_grad_noalloc: tiles");
  int rc = run_forward(p, d_W, d_p, flags, d_loss, d_grad != nullptr, s);
  if (rc) return rc;
  if (d_grad && (rc = run_backward(p, d_grad, (flags & SOS_FLAG_SINGLE_BACKWARD) == 0, s))) return rc;
  if (d_r)
    SOS_HIP(hipMemcpyAsync(d_r, p->ws + p->lay.r, p->M * 8, hipMemcpyDeviceToDevice, s), "sos_loss_grad_noalloc: r");
  return SOS_OK;
}

int sos_solve(sos_plan_t p, void* d_W, void* d_state, const double* d_p, const sos_adam_t* adam,
              const sos_solve_opts_t* o, sos_result_t* res, void* stream) {
  if (int rc = check_bound(p, "sos_solve")) return rc;
  if (int rc = check_adam(adam, "sos_solve")) return rc;
  if (!d_W || !d_state || !d_p || !o || !res) return set_error(SOS_EINVAL, "sos_solve: NULL argument");
  if (o->max_steps < 0 || o->check_every < 1 || !(o->tol >= 0) || !(o->lr_exact >= 0) ||
      !(o->rollback_ratio >= 0) || o->stall_checks < 0 || !(o->single_rel >= 0) || !(o->four_rel >= 0))
    return set_error(SOS_EINVAL, "sos_solve: needs max_steps >= 0, check_every >= 1, tol, lr_exact, "
                                 "rollback_ratio, single_rel, four_rel >= 0 and stall_checks >= 0");
  if (o->finisher < 0 || o->finisher > 2) return set_error(SOS_EINVAL, "sos_solve: finisher must be 0, 1 or 2");
  if (o->step_flags & ~(int)SOS_FLAG_DETERMINISTIC)
    return set_error(SOS_EINVAL, "sos_solve: step_flags may be SOS_FLAG_DETERMINISTIC");
  if (int rc = check_det(p, o->step_flags, "sos_solve")) return rc;
  if (o->finisher && o->ladder)
    if (int rc = check_ozaki(p, SOS_FLAG_OZAKI_FORWARD, "sos_solve")) return rc;
  hipStream_t s = (hipStream_t)stream;
  std::memset(res, 0, sizeof(*res));
  const size_t slot = slot_bytes(p), wbytes = (size_t)p->N * p->k * w_elem(p);
  char* st = (char*)d_state;
  char* best = st + 2 * slot;
  char* cand = st + 3 * slot;
  SOS_HIP(hipMemsetAsync(st, 0, 2 * slot, s), "sos_solve: zero state");
  double* sc = scal(p);
  SOS_HIP(launch_sumsq(p, d_p, p->M, sc + 1, s), "sos_solve: ||p||");
  double pn2 = 0;
  SOS_HIP(hipMemcpyAsync(&pn2, sc + 1, 8, hipMemcpyDeviceToHost, s), "sos_solve: readback");
  SOS_HIP(hipStreamSynchronize(s), "sos_solve");
  const double pnorm = pn2 > 0 ? std::sqrt(pn2) : 1.0;
  const double inf = std::numeric_limits<double>::infinity();

  const bool can_ladder = o->ladder && p->prec != SOS_FP64;
  sos_adam_t h = *adam;
  int phase = 0;
  double best_rel = inf, ref_rel = inf;
  bool have_best = false;
  int stall = 0;
  int64_t t = 0, exact_steps = 0;
  double last_loss = 0;
  bool done = false;
  const bool has_mid = can_ladder && split_plan(p) && o->mid_rel > 0;
  // fast start: the first part of phase 0 with the single-product forward
  bool fast_start = can_ladder && split_plan(p) && o->single_rel > 0;
  // the five-slice finisher's first part with four slices
  bool four = o->finisher == 2 && o->four_rel > 0;
  auto next_phase = [&]() {
    phase = (phase == 0 && has_mid) ? 1 : 2;
    stall = 0;
    if (o->lr_exact > 0) h.lr = o->lr_exact;
    best_rel = ref_rel = inf;  // values of the more accurate forward from here on
  };
  bool w_moved = true;  // W changed outside a step (start, rollback): operand copies must be rebuilt
  int64_t t_adam = 0;   // Adam's step count since the moments were last zeroed
  double done_rel = 0;  // the certificate of `best` that ended the loop
  while (t < o->max_steps && !done) {
    ++t;
    ++t_adam;
    const bool check = (t % o->check_every == 0) || t == o->max_steps;
    if (check) SOS_HIP(hipMemcpyAsync(cand, d_W, wbytes, hipMemcpyDeviceToDevice, s), "sos_solve: snapshot");
    const int exact_flag = o->finisher == 2
                               ? SOS_FLAG_OZAKI_FORWARD | (four ? SOS_FLAG_OZAKI_FOUR_SLICES : SOS_FLAG_OZAKI_FIVE_SLICES)
                           : o->finisher == 1 ? SOS_FLAG_OZAKI_FORWARD
                                              : SOS_FLAG_EXACT_FORWARD;
    const int fast_flags = (o->step_flags & SOS_FLAG_DETERMINISTIC) | (fast_start ? SOS_FLAG_SINGLE_FORWARD : 0);
    const int flags = (phase == 2 ? exact_flag : phase == 1 ? SOS_FLAG_FP32_FORWARD : fast_flags) |
                      (o->single_backward ? SOS_FLAG_SINGLE_BACKWARD : 0) |
                      (w_moved ? 0 : SOS_FLAG_COPIES_VALID);
    int rc = run_step(p, d_W, st, t_adam, d_p, h, sc + 0, flags, s);
    if (rc) return rc;
    w_moved = false;
    if (phase == 2) ++exact_steps;
    if (!check) continue;
    SOS_HIP(hipMemcpyAsync(&last_loss, sc + 0, 8, hipMemcpyDeviceToHost, s), "sos_solve: loss");
    SOS_HIP(hipStreamSynchronize(s), "sos_solve");
    const double rel = std::isfinite(last_loss) ? std::sqrt(last_loss) / pnorm : inf;
    if (!std::isfinite(rel) && !have_best) {
      res->steps = t;
      res->exact_steps = exact_steps;
      res->loss = last_loss;
      res->phase = phase;
      return set_error(SOS_ENUMERIC, "sos_solve: loss is not finite");
    }
    if (rel < best_rel) {
      best_rel = rel;
      std::swap(best, cand);  // the snapshot is the iterate this loss belongs to
      have_best = true;
    }
    if (have_best && (!std::isfinite(rel) || (o->rollback_ratio > 0 && rel > o->rollback_ratio * best_rel))) {
      // diverging: back to the best iterate with half the step size and a
      // fresh start of Adam.  The moments belong to the diverging iterates
      // (after a non-finite loss they hold its NaN or Inf gradient), so they
      // are zeroed and the bias correction restarts.
      SOS_HIP(hipMemcpyAsync(d_W, best, wbytes, hipMemcpyDeviceToDevice, s), "sos_solve: rollback");
      SOS_HIP(hipMemsetAsync(st, 0, 2 * slot, s), "sos_solve: zero moments");
      t_adam = 0;
      w_moved = true;
      h.lr *= 0.5;
      stall = 0;
      ref_rel = best_rel;
      continue;
    }
    if (rel < o->stall_ratio * ref_rel) {
      ref_rel = rel;
      stall = 0;
    } else {
      ++stall;
    }
    if (fast_start) {
      // on to the three products once the single product's rounding (~2^-7 of
      // the coefficients' scale) could start to matter, or on a stall; the
      // Adam state and step size carry over
      if (rel <= o->single_rel || (o->stall_checks > 0 && stall >= o->stall_checks)) {
        fast_start = false;
        stall = 0;
        best_rel = ref_rel = inf;  // values of the three-product forward from here on
      }
      continue;
    }
    if (phase == 2 && four && (rel <= o->four_rel || (o->stall_checks > 0 && stall >= o->stall_checks))) {
      // on to five slices once the four-slice forward's rounding (~4e-8 of
      // the coefficients' scale for Gaussian rows) could start to matter
      four = false;
      stall = 0;
      best_rel = ref_rel = inf;
      continue;
    }
    const double target = phase == 0 ? o->switch_rel : o->mid_rel;
    bool switch_phase = can_ladder && phase < 2 &&
                        ((o->stall_checks > 0 && stall >= o->stall_checks) || (target > 0 && rel <= target));
    if (rel <= o->tol) {
      double vrel = 0;
      int vrc = sos_verify(p, best, d_p, &vrel, nullptr, stream);
      if (vrc) return vrc;
      if (vrel <= o->tol) {
        done = true;
        done_rel = vrel;
      } else if (can_ladder && phase < 2) {
        switch_phase = true;
      }
    }
    if (switch_phase && !done) next_phase();
  }
  if (have_best) SOS_HIP(hipMemcpyAsync(d_W, best, wbytes, hipMemcpyDeviceToDevice, s), "sos_solve: best W");
  // the returned W is `best`: when its certificate ended the loop, that is the result's
  double vrel = done_rel;
  if (!done) {
    int vrc = sos_verify(p, d_W, d_p, &vrel, nullptr, stream);
    if (vrc) return vrc;
  }
  res->steps = t;
  res->exact_steps = exact_steps;
  res->loss = last_loss;
  res->rel = vrel;
  res->best_rel = best_rel;
  res->phase = phase;
  res->status = vrel <= o->tol ? SOS_OK : SOS_NOT_CONVERGED;
  return res->status;
}

static int check_batch(const sos_plan_t* plans, const void* const* W, const double* const* d_p, double* losses,
                       int count, const char* what) {
  if (count < 0) return set_error(SOS_EINVAL, std::string(what) + ": count < 0");
  if (count > 0 && (!plans || !W || !d_p || !losses)) return set_error(SOS_EINVAL, std::string(what) + ": NULL array");
  for (int q = 0; q < count; ++q) {
    if (int rc = check_bound(plans[q], what)) return rc;
    if (plans[q]->prec != SOS_FP32)
      return set_error(SOS_EINVAL, std::string(what) + ": grouped calls take SOS_FP32 plans");
    if (!plans[q]->batchable)
      return set_error(SOS_ERANGE, std::string(what) + ": plan has N > SOS_BATCH_MAX_N");
    if (!W[q] || !d_p[q]) return set_error(SOS_EINVAL, std::string(what) + ": NULL W or p");
  }
  // every problem writes its residual, partial sums and loss partials into its
  // plan's workspace, so two problems of one call must not share one
  std::vector<const char*> ws(count);
  for (int q = 0; q < count; ++q) ws[q] = plans[q]->ws;
  std::sort(ws.begin(), ws.end());
  if (std::adjacent_find(ws.begin(), ws.end()) != ws.end())
    return set_error(SOS_EINVAL, std::string(what) + ": two problems share one plan workspace");
  return SOS_OK;
}

// The problems of a grouped call in launch order: largest basis first
// (stable), so that each group holds problems of similar size and a group of
// small problems is not held up by one large problem.  A problem's results
// do not depend on its group, so the order changes only the time.
struct BatchOrder {
  std::vector<sos_plan_s*> P;
  std::vector<void*> W, S;
  std::vector<int64_t> T;
  std::vector<const double*> p;
  std::vector<int> slot;
  BatchOrder(const sos_plan_t* plans, void* const* d_W, void* const* d_state, const int64_t* t,
             const double* const* d_p, int count)
      : slot(count) {
    std::iota(slot.begin(), slot.end(), 0);
    std::stable_sort(slot.begin(), slot.end(), [&](int a, int b) { return plans[a]->N > plans[b]->N; });
    for (int q : slot) {
      P.push_back(plans[q]);
      W.push_back(d_W[q]);
      p.push_back(d_p[q]);
      if (d_state) S.push_back(d_state[q]);
      if (t) T.push_back(t[q]);
    }
  }
};

int sos_step_batch(const sos_plan_t* plans, void* const* d_W, void* const* d_state, const int64_t* t,
                   const double* const* d_p, const sos_adam_t* adam, double* d_losses, int count,
                   void* stream) {
  if (int rc = check_batch(plans, (const void* const*)d_W, d_p, d_losses, count, "sos_step_batch")) return rc;
  if (count == 0) return SOS_OK;
  if (!d_state || !t) return set_error(SOS_EINVAL, "sos_step_batch: NULL state or t");
  if (int rc = check_adam(adam, "sos_step_batch")) return rc;
  for (int q = 0; q < count; ++q) {
    if (!d_state[q]) return set_error(SOS_EINVAL, "sos_step_batch: NULL state");
    if (t[q] < 1) return set_error(SOS_EINVAL, "sos_step_batch: t is 1-based");
  }
  const BatchOrder o(plans, (void* const*)d_W, d_state, t, d_p, count);
  const int cap = batch_capacity();
  for (int q0 = 0; q0 < count; q0 += cap) {
    const int c = std::min(cap, count - q0);
    SOS_HIP(launch_step_group(o.P.data() + q0, o.W.data() + q0, o.S.data() + q0, o.T.data() + q0, o.p.data() + q0,
                              adam, d_losses, o.slot.data() + q0, c, (hipStream_t)stream),
            "sos_step_batch");
  }
  return SOS_OK;
}

int sos_loss_batch(const sos_plan_t* plans, const void* const* d_W, const double* const* d_p, double* d_losses,
                   int count, void* stream) {
  if (int rc = check_batch(plans, d_W, d_p, d_losses, count, "sos_loss_batch")) return rc;
  const BatchOrder o(plans, (void* const*)d_W, nullptr, nullptr, d_p, count);
  const int cap = batch_capacity();
  for (int q0 = 0; q0 < count; q0 += cap) {
    const int c = std::min(cap, count - q0);
    SOS_HIP(launch_step_group(o.P.data() + q0, o.W.data() + q0, nullptr, nullptr, o.p.data() + q0, nullptr,
                              d_losses, o.slot.data() + q0, c, (hipStream_t)stream),
            "sos_loss_batch");
  }
  return SOS_OK;
}

// ---------------------------------------------------------------------------
// Two-layer network (Section 2): W = net(At, Bt), then the plan's path
// ---------------------------------------------------------------------------

namespace {
struct NetLayout {
  size_t rowpair, rowmap, mA, vA, mB, vB, W, P, gW, dA, dB, dAz;
  size_t snapA[2], snapB[2];  // sos_net_solve: the best weights and the snapshot of a check step
  size_t bytes;
};

NetLayout net_layout(const sos_plan_s* p, int n, int m) {
  NetLayout L;
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off = (off + bytes + 255) / 256 * 256; return o; };
  const size_t N = (size_t)p->N, k = (size_t)p->k, nm = (size_t)n * m;
  const size_t we = p->prec == SOS_FP64 ? 8 : 4;  // W, P and dW in the plan's W type
  L.rowpair = take(N * 4);
  L.rowmap = take((size_t)n * n * 4);
  L.mA = take(nm * 4);
  L.vA = take(nm * 4);
  L.mB = take(nm * k * 4);
  L.vB = take(nm * k * 4);
  L.W = take(N * k * we);
  L.P = take((size_t)n * n * k * we);
  L.gW = take(N * k * we);
  L.dA = take(nm * 4);
  L.dB = take(nm * k * 4);
  L.dAz = take((size_t)n * nm * we);
  for (int q = 0; q < 2; ++q) {
    L.snapA[q] = take(nm * 4);
    L.snapB[q] = take(nm * k * 4);
  }
  L.bytes = off;
  return L;
}

// plan (n - 1, 2); builds the row maps on first use
int net_check(sos_plan_s* p, int n, int m, const char* fn) {
  if (n < 2 || m < 1) return set_error(SOS_EINVAL, std::string(fn) + ": needs n >= 2 and m >= 1");
  if (p->n != n - 1 || p->d != 2)
    return set_error(SOS_EINVAL, std::string(fn) + ": quartic forms in n variables need a plan (n - 1, 2)");
  if ((int64_t)n * n * p->k >= (int64_t(1) << 31) || (int64_t)n * m * p->k >= (int64_t(1) << 31))
    return set_error(SOS_ERANGE, std::string(fn) + ": n^2 k and n m k must stay below 2^31");
  if (p->net_rowpair.empty()) {
    // basis row i is x_a x_c with the homogenising variable x_{n-1} filling the degree up to 2
    p->net_rowpair.assign(p->N, 0);
    p->net_rowmap.assign((size_t)n * n, 0);
    for (int64_t i = 0; i < p->N; ++i) {
      int v[2] = {n - 1, n - 1}, q = 0;
      for (int u = 0; u < n - 1; ++u)
        for (int e = 0; e < p->basis[i * (n - 1) + u]; ++e) v[q++] = u;
      const int a = std::min(v[0], v[1]), c = std::max(v[0], v[1]);
      p->net_rowpair[i] = a * n + c;
      p->net_rowmap[(size_t)a * n + c] = p->net_rowmap[(size_t)c * n + a] = (int32_t)i;
    }
  }
  return SOS_OK;
}

int net_upload_maps(sos_plan_s* p, char* st, const NetLayout& L, hipStream_t s) {
  if (p->net_maps_at == st) return SOS_OK;
  SOS_HIP(hipMemcpyAsync(st + L.rowpair, p->net_rowpair.data(), p->net_rowpair.size() * 4, hipMemcpyHostToDevice, s),
          "net: row pairs");
  SOS_HIP(hipMemcpyAsync(st + L.rowmap, p->net_rowmap.data(), p->net_rowmap.size() * 4, hipMemcpyHostToDevice, s),
          "net: row map");
  p->net_maps_at = st;
  return SOS_OK;
}

int net_forward_W(sos_plan_s* p, int n, int m, const float* At, const float* Bt, char* st, const NetLayout& L,
                  void* W, hipStream_t s) {
  if (int rc = net_upload_maps(p, st, L, s)) return rc;
  SOS_HIP(launch_net_forward(p->prec == SOS_FP64, n, m, p->k, (int)p->N, At, Bt, st + L.P,
                             (const int32_t*)(st + L.rowpair), W, s), "net: forward");
  return SOS_OK;
}

// L and dL/dAt (when dA != nullptr), dL/dBt of the weights
int net_grad(sos_plan_s* p, int n, int m, const float* At, const float* Bt, char* st, const NetLayout& L,
             const double* d_p, double* d_loss, int flags, float* dA, float* dB, hipStream_t s) {
  void* W = st + L.W;
  void* gW = st + L.gW;
  if (int rc = net_forward_W(p, n, m, At, Bt, st, L, W, s)) return rc;
  if (int rc = run_forward(p, W, d_p, flags, d_loss, true, s)) return rc;
  if (int rc = run_backward(p, gW, (flags & SOS_FLAG_SINGLE_BACKWARD) == 0, s)) return rc;
  SOS_HIP(launch_net_backward(p->prec == SOS_FP64, n, m, p->k, At, Bt, gW, (const int32_t*)(st + L.rowmap),
                              st + L.P, dA, dB, st + L.dAz, dA != nullptr, s), "net: backward");
  return SOS_OK;
}

int net_step(sos_plan_s* p, int n, int m, float* At, float* Bt, char* st, const NetLayout& L, int64_t t,
             const double* d_p, const sos_adam_t& h, double* d_loss, int flags, bool train_first, hipStream_t s) {
  float* dA = (float*)(st + L.dA);
  float* dB = (float*)(st + L.dB);
  if (int rc = net_grad(p, n, m, At, Bt, st, L, d_p, d_loss, flags, train_first ? dA : nullptr, dB, s)) return rc;
  const int64_t nm = (int64_t)n * m;
  if (train_first)
    SOS_HIP(launch_adam_f32(At, (float*)(st + L.mA), (float*)(st + L.vA), dA, nm, t, h, s), "net: Adam A");
  SOS_HIP(launch_adam_f32(Bt, (float*)(st + L.mB), (float*)(st + L.vB), dB, nm * p->k, t, h, s), "net: Adam B");
  return SOS_OK;
}
}  // namespace

extern "C" {

int sos_net_query(sos_plan_t p, int n, int m, size_t* state_bytes) {
  if (!p || !state_bytes) return set_error(SOS_EINVAL, "sos_net_query: NULL argument");
  if (int rc = net_check(p, n, m, "sos_net_query")) return rc;
  *state_bytes = net_layout(p, n, m).bytes;
  return SOS_OK;
}

int sos_net_weights(sos_plan_t p, int n, int m, const float* d_At, const float* d_Bt, void* d_W, void* d_state,
                    void* stream) {
  if (int rc = check_bound(p, "sos_net_weights")) return rc;
  if (int rc = net_check(p, n, m, "sos_net_weights")) return rc;
  if (!d_At || !d_Bt || !d_W || !d_state) return set_error(SOS_EINVAL, "sos_net_weights: NULL argument");
  return net_forward_W(p, n, m, d_At, d_Bt, (char*)d_state, net_layout(p, n, m), d_W, (hipStream_t)stream);
}

int sos_net_grad(sos_plan_t p, int n, int m, const float* d_At, const float* d_Bt, void* d_state, const double* d_p,
                 double* d_loss, float* d_dAt, float* d_dBt, int flags, void* stream) {
  if (int rc = check_bound(p, "sos_net_grad")) return rc;
  if (int rc = net_check(p, n, m, "sos_net_grad")) return rc;
  if (!d_At || !d_Bt || !d_state || !d_p || !d_loss || !d_dBt)
    return set_error(SOS_EINVAL, "sos_net_grad: NULL argument");
  if (flags & ~(int)(SOS_FLAG_EXACT_FORWARD | SOS_FLAG_SINGLE_BACKWARD))
    return set_error(SOS_EINVAL, "sos_net_grad: flags may be SOS_FLAG_EXACT_FORWARD | SOS_FLAG_SINGLE_BACKWARD");
  return net_grad(p, n, m, d_At, d_Bt, (char*)d_state, net_layout(p, n, m), d_p, d_loss, flags, d_dAt, d_dBt,
                  (hipStream_t)stream);
}

int sos_net_step(sos_plan_t p, int n, int m, float* d_At, float* d_Bt, void* d_state, int64_t t, const double* d_p,
                 const sos_adam_t* adam, double* d_loss, int flags, int train_first, void* stream) {
  if (int rc = check_bound(p, "sos_net_step")) return rc;
  if (int rc = net_check(p, n, m, "sos_net_step")) return rc;
  if (int rc = check_adam(adam, "sos_net_step")) return rc;
  if (!d_At || !d_Bt || !d_state || !d_p || !d_loss) return set_error(SOS_EINVAL, "sos_net_step: NULL argument");
  if (t < 1) return set_error(SOS_EINVAL, "sos_net_step: t is 1-based");
  if (flags & ~(int)(SOS_FLAG_EXACT_FORWARD | SOS_FLAG_SINGLE_BACKWARD))
    return set_error(SOS_EINVAL, "sos_net_step: flags may be SOS_FLAG_EXACT_FORWARD | SOS_FLAG_SINGLE_BACKWARD");
  return net_step(p, n, m, d_At, d_Bt, (char*)d_state, net_layout(p, n, m), t, d_p, *adam, d_loss, flags,
                  train_first != 0, (hipStream_t)stream);
}

int sos_net_solve(sos_plan_t p, int n, int m, float* d_At, float* d_Bt, void* d_state, const double* d_p,
                  const sos_adam_t* adam, const sos_solve_opts_t* o, int train_first, sos_result_t* res,
                  void* stream) {
  if (int rc = check_bound(p, "sos_net_solve")) return rc;
  if (int rc = net_check(p, n, m, "sos_net_solve")) return rc;
  if (int rc = check_adam(adam, "sos_net_solve")) return rc;
  if (!d_At || !d_Bt || !d_state || !d_p || !o || !res) return set_error(SOS_EINVAL, "sos_net_solve: NULL argument");
  if (o->max_steps < 0 || o->check_every < 1 || !(o->tol >= 0) || !(o->lr_exact >= 0) || !(o->rollback_ratio >= 0))
    return set_error(SOS_EINVAL, "sos_net_solve: needs max_steps >= 0, check_every >= 1, tol, lr_exact and "
                                 "rollback_ratio >= 0");
  hipStream_t s = (hipStream_t)stream;
  std::memset(res, 0, sizeof(*res));
  const NetLayout L = net_layout(p, n, m);
  char* st = (char*)d_state;
  SOS_HIP(hipMemsetAsync(st + L.mA, 0, L.mB - L.mA, s), "sos_net_solve: zero moments of A");
  SOS_HIP(hipMemsetAsync(st + L.mB, 0, L.W - L.mB, s), "sos_net_solve: zero moments of B");
  double* sc = scal(p);
  SOS_HIP(launch_sumsq(p, d_p, p->M, sc + 1, s), "sos_net_solve: ||p||");
  double pn2 = 0;
  SOS_HIP(hipMemcpyAsync(&pn2, sc + 1, 8, hipMemcpyDeviceToHost, s), "sos_net_solve: readback");
  SOS_HIP(hipStreamSynchronize(s), "sos_net_solve");
  const double pnorm = pn2 > 0 ? std::sqrt(pn2) : 1.0;
  sos_adam_t h = *adam;
  const bool can_ladder = o->ladder != 0;
  const int64_t nm = (int64_t)n * m;
  const size_t abytes = (size_t)nm * 4, bbytes = (size_t)nm * p->k * 4;
  // best weights (as measured at a check) and the snapshot of the weights a
  // check step starts from; the two swap roles when the snapshot is better
  int best = 0;
  bool have_best = false;
  int phase = 0;
  int64_t t = 0, exact_steps = 0;
  double loss = 0, best_rel = std::numeric_limits<double>::infinity();
  bool done = false;
  double done_rel = 0;  // the certificate of the best weights that ended the loop
  int64_t t_adam = 0;  // Adam's step count since the moments were last zeroed
  auto verify = [&](int which, double* vrel) -> int {
    void* W = st + L.W;
    const float* A = which < 0 ? d_At : (const float*)(st + L.snapA[which]);
    const float* B = which < 0 ? d_Bt : (const float*)(st + L.snapB[which]);
    if (int rc = net_forward_W(p, n, m, A, B, st, L, W, s)) return rc;
    return sos_verify(p, W, d_p, vrel, nullptr, stream);
  };
  while (t < o->max_steps && !done) {
    ++t;
    ++t_adam;
    const bool check = t % o->check_every == 0 || t == o->max_steps;
    if (check) {  // the loss this step reports belongs to the weights it starts from
      SOS_HIP(hipMemcpyAsync(st + L.snapA[1 - best], d_At, abytes, hipMemcpyDeviceToDevice, s), "net: snapshot A");
      SOS_HIP(hipMemcpyAsync(st + L.snapB[1 - best], d_Bt, bbytes, hipMemcpyDeviceToDevice, s), "net: snapshot B");
    }
    const int flags = (phase ? SOS_FLAG_EXACT_FORWARD : 0) | (o->single_backward ? SOS_FLAG_SINGLE_BACKWARD : 0);
    if (int rc = net_step(p, n, m, d_At, d_Bt, st, L, t_adam, d_p, h, sc + 0, flags, train_first != 0, s))
      return rc;
    if (phase) ++exact_steps;
    if (!check) continue;
    SOS_HIP(hipMemcpyAsync(&loss, sc + 0, 8, hipMemcpyDeviceToHost, s), "sos_net_solve: loss");
    SOS_HIP(hipStreamSynchronize(s), "sos_net_solve");
    const double rel = std::isfinite(loss) ? std::sqrt(std::max(loss, 0.0)) / pnorm
                                           : std::numeric_limits<double>::infinity();
    if (!std::isfinite(rel) && !have_best) return set_error(SOS_ENUMERIC, "sos_net_solve: loss is not finite");
    if (rel < best_rel) {
      best_rel = rel;
      best = 1 - best;
      have_best = true;
    }
    if (!std::isfinite(rel) || (o->rollback_ratio > 0 && rel > o->rollback_ratio * best_rel)) {
      // diverging: back to the best weights with half the step size and
      // zeroed Adam moments (they hold the diverging iterates' gradients)
      SOS_HIP(hipMemcpyAsync(d_At, st + L.snapA[best], abytes, hipMemcpyDeviceToDevice, s), "net: rollback A");
      SOS_HIP(hipMemcpyAsync(d_Bt, st + L.snapB[best], bbytes, hipMemcpyDeviceToDevice, s), "net: rollback B");
      SOS_HIP(hipMemsetAsync(st + L.mA, 0, L.mB - L.mA, s), "net: zero moments of A");
      SOS_HIP(hipMemsetAsync(st + L.mB, 0, L.W - L.mB, s), "net: zero moments of B");
      t_adam = 0;
      h.lr *= 0.5;
      continue;
    }
    if (can_ladder && phase == 0 && rel <= o->switch_rel) {
      phase = 1;
      if (o->lr_exact > 0) h.lr = o->lr_exact;
    }
    if (rel <= o->tol) {
      // certify the best weights: W = net(A, B), FP64 forward
      double vrel = 0;
      if (int rc = verify(best, &vrel)) return rc;
      if (vrel <= o->tol) {
        done = true;
        done_rel = vrel;
      } else if (can_ladder && phase == 0) {
        phase = 1;
        if (o->lr_exact > 0) h.lr = o->lr_exact;
      }
    }
  }
  if (have_best) {  // return the best weights
    SOS_HIP(hipMemcpyAsync(d_At, st + L.snapA[best], abytes, hipMemcpyDeviceToDevice, s), "net: best A");
    SOS_HIP(hipMemcpyAsync(d_Bt, st + L.snapB[best], bbytes, hipMemcpyDeviceToDevice, s), "net: best B");
  }
  // the returned weights are the best ones: when their certificate ended the loop, that is the result's
  double vrel = done_rel;
  if (!done)
    if (int rc = verify(-1, &vrel)) return rc;
  res->steps = t;
  res->exact_steps = exact_steps;
  res->loss = loss;
  res->rel = vrel;
  res->best_rel = best_rel;
  res->phase = phase ? 2 : 0;
  res->status = vrel <= o->tol ? SOS_OK : SOS_NOT_CONVERGED;
  return res->status;
}

}  // extern "C"

const char* sos_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
