// Grouped kernels for many small problems at once (serving): one Adam step
// (forward, loss, backward, update) of up to kMaxBatch independent problems
// per launch of each kernel.  Each problem keeps its own plan workspace
// (pair lists, partial-result scratch, residual r, R), its own W and its own
// Adam state; the kernels read all of them through a descriptor table passed
// by value in the kernel arguments (a few pointers per problem; the plan's
// sizes and array places come from a header in its workspace, written at
// bind), so a call allocates nothing.
//
// Every block works on one problem, and every sum runs in an order fixed by
// that problem's shape alone (no floating-point atomics), so a problem's
// results do not depend on the other problems in the launch.  No block
// contracts over more than kBatchSlice (Gram) or kBatchSliceJ (backward)
// elements: longer contractions are
// split into slices with one partial result each, summed in slice order by
// the consumer, which keeps every block's dependent-load chain short.
//
//   k_b_gram   partial G = W W^T per K slice, upper-triangle 32 x 32 tiles,
//              FP32 entries converted to FP64 (exact products) on
//              v_mfma_f64_16x16x4, the next K chunk prefetched into
//              registers while the current one is multiplied; each entry
//              stored at its pair's place in the coefficient-ordered lists
//   k_b_coeff  r_m = sum over the pairs (i <= j) of monomial m of
//              (2 - [i = j]) G_ij (G_ij summed over slices), minus p_m, in
//              the plan's pair order (a block's pairs staged through LDS in
//              coalesced chunks); L = sum r_m^2 by a fixed-order block
//              sum and a fixed-order sum of the block partials in the block
//              that arrives last
//   k_b_rw     partial g = 4 R W per slice of the contraction index, FP32 MFMA,
//              R_ij = r[rank of alpha_i + alpha_j] through the plan's map
//   k_b_adam   g = sum of the slices, bias-corrected Adam in FP32
#include <hip/hip_runtime.h>

#include <cstdint>

#include "sos_internal.h"

namespace sos {
namespace bat {

typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr int kMaxBatch = 64;
constexpr int kCoeffChunk = 2048;   // pair values staged in LDS per round of k_b_coeff

struct Req {
  const float* W;            // N x k
  float* m;                  // Adam state
  float* v;
  const double* p;           // M
  double* r;                 // M
  double* Gp;                // sg x P partial Gram, P = N (N + 1) / 2 entries in pair-list order
  const int32_t* pair_pos;   // N x N: position of a pair in the pair lists
  const int32_t* rank_map;   // N x N: R_ij = r[rank_map[i N + j]]
  float* gp;                 // sr x N x k partial gradient
  double* part;              // loss partials, one per coefficient block
  unsigned* count;           // blocks of k_b_coeff done (returns to zero)
  const int32_t* pair_off;
  const int32_t* pair_idx;
  double* loss;
  int N, M, k, sg, sr;       // sg = K slices of the gram, sr = j slices of the backward
  float bc1, bc2;
};

// What a launch passes per problem; the plan's constants and array places
// come from the BatchHeader in its workspace (expand() below).
struct Desc {
  const float* W;            // N x k
  float* m;                  // Adam state (v follows at the header's offset)
  const double* p;           // M
  const char* hdr;           // the plan's BatchHeader in its workspace
  double* loss;
  float bc1, bc2;
};

struct Args {
  int count;
  int fwd_off[kMaxBatch + 1];  // prefix sums of gram blocks
  int bwd_off[kMaxBatch + 1];  // prefix sums of backward blocks
  float lr, b1, b2, eps;
  Desc q[kMaxBatch];
};
static_assert(sizeof(Args) <= 4000, "kernel argument block too large");

__device__ __forceinline__ Req expand(const Desc& d) {
  const BatchHeader& h = *(const BatchHeader*)d.hdr;
  char* b = const_cast<char*>(d.hdr);
  Req R;
  R.W = d.W;
  R.m = d.m;
  R.v = (float*)((char*)d.m + h.v);
  R.p = d.p;
  R.r = (double*)(b + h.r);
  R.Gp = (double*)(b + h.Gp);
  R.pair_pos = (const int32_t*)(b + h.pair_pos);
  R.rank_map = (const int32_t*)(b + h.rank_map);
  R.gp = (float*)(b + h.gp);
  R.part = (double*)(b + h.part);
  R.count = (unsigned*)(b + h.count);
  R.pair_off = (const int32_t*)(b + h.pair_off);
  R.pair_idx = (const int32_t*)(b + h.pair_idx);
  R.loss = d.loss;
  R.N = h.N;
  R.M = h.M;
  R.k = h.k;
  R.sg = h.sg;
  R.sr = h.sr;
  R.bc1 = d.bc1;
  R.bc2 = d.bc2;
  return R;
}

// problem owning flat block b (off: prefix sums, off[count] = total)
__device__ __forceinline__ int find_req(const int* off, int count, int b) {
  int q = 0;
  while (q + 1 < count && off[q + 1] <= b) ++q;
  return q;
}

// Gram slices.  Block (tile t, slice s) of a problem: tile t is (I, J),
// I <= J, numbered column by column; slice s covers K in
// [s kBatchSlice, min(k, (s + 1) kBatchSlice)).  Four waves, each one
// 16 x 16 block of the 32 x 32 tile; K in chunks of 32 through LDS, each
// chunk 8 MFMA k-steps of 4.  MFMA f64 16x16x4 operand: lane l holds row
// l % 16 at k = l / 16; result register q of lane l is row l / 16 + 4 q,
// column l % 16.
constexpr int TF = 32, TK = 32;
__global__ __launch_bounds__(256) void k_b_gram(Args a) {
  __shared__ float As[TF][TK + 1], Bs[TF][TK + 1];
  const int q = find_req(a.fwd_off, a.count, blockIdx.x);
  const Req R = expand(a.q[q]);
  const int local = blockIdx.x - a.fwd_off[q];
  const int t = local / R.sg, s = local % R.sg;
  int J = 0;
  while ((J + 1) * (J + 2) / 2 <= t) ++J;
  const int I = t - J * (J + 1) / 2;
  const int kb = s * kBatchSlice;
  const int ke = min(R.k, kb + kBatchSlice);
  const int wave = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int wm = wave >> 1, wn = wave & 1;
  // this thread's share of a chunk: elements tid + 256 u, row e / 32, column e % 32
  float ra[TF * TK / 256], rb[TF * TK / 256];
  auto load = [&](int k0) {
#pragma unroll
    for (int u = 0; u < TF * TK / 256; ++u) {
      const int e = threadIdx.x + 256 * u;
      const int rr = e / TK, kk = k0 + e % TK;
      const int i = I * TF + rr, j = J * TF + rr;
      ra[u] = (i < R.N && kk < ke) ? R.W[(size_t)i * R.k + kk] : 0.f;
      rb[u] = (j < R.N && kk < ke) ? R.W[(size_t)j * R.k + kk] : 0.f;
    }
  };
  f64x4 acc = {0.0, 0.0, 0.0, 0.0};
  load(kb);
  for (int k0 = kb; k0 < ke; k0 += TK) {
#pragma unroll
    for (int u = 0; u < TF * TK / 256; ++u) {
      const int e = threadIdx.x + 256 * u;
      As[e / TK][e % TK] = ra[u];
      Bs[e / TK][e % TK] = rb[u];
    }
    __syncthreads();
    if (k0 + TK < ke) load(k0 + TK);  // in flight while this chunk is multiplied
#pragma unroll
    for (int s4 = 0; s4 < TK / 4; ++s4) {
      const double av = As[wm * 16 + (l & 15)][4 * s4 + (l >> 4)];
      const double bv = Bs[wn * 16 + (l & 15)][4 * s4 + (l >> 4)];
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
    }
    __syncthreads();
  }
  // written at the pair's position in the coefficient-ordered pair lists, so
  // that each coefficient later reads its pairs from one contiguous range
  const size_t P = (size_t)R.N * (R.N + 1) / 2;
  double* G = R.Gp + (size_t)s * P;
  const int j = J * TF + wn * 16 + (l & 15);
#pragma unroll
  for (int qq = 0; qq < 4; ++qq) {
    const int i = I * TF + wm * 16 + (l >> 4) + 4 * qq;
    if (i < R.N && j < R.N && i <= j) G[R.pair_pos[(size_t)i * R.N + j]] = acc[qq];
  }
}

// Sum of x over the block's 256 threads, in a fixed order.
__device__ __forceinline__ double block_sum256(double x, double* sh4) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  if ((threadIdx.x & 63) == 0) sh4[threadIdx.x >> 6] = x;
  __syncthreads();
  const double t = (sh4[0] + sh4[1]) + (sh4[2] + sh4[3]);
  __syncthreads();
  return t;
}

// Coefficients, residual and the loss; grid (blocks of 256
// coefficients, problem).
__global__ __launch_bounds__(256) void k_b_coeff(Args a) {
  const Req R = expand(a.q[blockIdx.y]);
  const int nb = (R.M + 255) / 256;
  if ((int)blockIdx.x >= nb) return;
  __shared__ double sh4[4];
  __shared__ int last;
  __shared__ double vals[kCoeffChunk];
  const int m = blockIdx.x * 256 + threadIdx.x;
  const int m0 = blockIdx.x * 256, m1 = min(R.M, m0 + 256);
  const size_t P = (size_t)R.N * (R.N + 1) / 2;
  // G of pair e: the slices in slice order, doubled off the diagonal
  auto pair_val = [&](int e) {
    double gij = R.Gp[e];
    for (int s = 1; s < R.sg; ++s) gij += R.Gp[s * P + e];
    return ((uint32_t)R.pair_idx[e] >> 31) ? 2.0 * gij : gij;
  };
  // The pairs of this block's coefficients are one contiguous range of the
  // pair lists: stage it through LDS in coalesced chunks, then each thread
  // adds its own coefficient's pairs, in pair order.
  const int eb = R.pair_off[m0], ee = R.pair_off[m1];
  const int my0 = m < R.M ? R.pair_off[m] : 0, my1 = m < R.M ? R.pair_off[m + 1] : 0;
  double c = 0.0;
  for (int cb = eb; cb < ee; cb += kCoeffChunk) {
    const int ce = min(ee, cb + kCoeffChunk);
    __syncthreads();
    for (int e = cb + threadIdx.x; e < ce; e += 256) vals[e - cb] = pair_val(e);
    __syncthreads();
    const int lo = max(my0, cb), hi = min(my1, ce);
    for (int e = lo; e < hi; ++e) c += vals[e - cb];
  }
  double rr = 0.0;
  if (m < R.M) {
    rr = c - R.p[m];
    R.r[m] = rr;
  }
  const double b = block_sum256(rr * rr, sh4);
  if (threadIdx.x == 0) {
    R.part[blockIdx.x] = b;
    __threadfence();
    last = (atomicAdd(R.count, 1u) == (unsigned)nb - 1);
  }
  __syncthreads();
  if (!last) return;
  // every other block of this problem has stored its partial: add them in block order
  __threadfence();
  double x = 0.0;
  for (int q = threadIdx.x; q < nb; q += 256)
    x += __hip_atomic_load(R.part + q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const double L = block_sum256(x, sh4);
  if (threadIdx.x == 0) {
    R.loss[0] = L;
    __hip_atomic_store(R.count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// Partial g = 4 R W over j in one slice of kBatchSliceJ on FP32 MFMA
// (v_mfma_f32_32x32x2f32), in tiles of 64 rows (i) x 64 columns (l), one
// 32 x 32 block per wave.  j runs in chunks of 32 through LDS, the next chunk
// prefetched into registers.  Within each group of 8 j, lane half h
// contracts j = 4 h + s in k-step s (s = 0..3), so a lane's operands of four
// k-steps are one 16-byte LDS read from R (rows i) and from W^T (rows l).
// The order of the sum is fixed by the problem's shape alone.  (Tiles of
// 64 x 256 fetch each R value fewer times and are faster on the largest
// problems alone, but slower on the serving mix, where they leave too few
// blocks per problem.)
constexpr int TBI = 64, TBL = 64, TBK = 32, TBS = TBK + 4;
typedef float f32x16 __attribute__((ext_vector_type(16)));
__global__ __launch_bounds__(256) void k_b_rw(Args a) {
  __shared__ __align__(16) float Rs[TBI][TBS];   // R_ij, j within the chunk
  __shared__ __align__(16) float Wt[TBL][TBS];   // W_jl stored at [l][j]
  const int q = find_req(a.bwd_off, a.count, blockIdx.x);
  const Req R = expand(a.q[q]);
  const int local = blockIdx.x - a.bwd_off[q];
  const int t = local / R.sr, s = local % R.sr;
  const int nl = (R.k + TBL - 1) / TBL;
  const int I = t / nl, L = t % nl;
  const int jb = s * kBatchSliceJ;
  const int je = min(R.N, jb + kBatchSliceJ);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int h = lane >> 5, lr = lane & 31;
  const int row0 = (wave >> 1) * 32, col0 = (wave & 1) * 32;
  // R_ij needs two dependent loads (the rank map, then r): the map entries
  // are fetched two chunks ahead, the values and W one chunk ahead.
  constexpr int NR = TBI * TBK / 256;
  int idx[NR];
  float rr[NR], ww[TBK * TBL / 256];
  auto load_idx = [&](int j0) {
#pragma unroll
    for (int u = 0; u < NR; ++u) {
      const int e = threadIdx.x + 256 * u;
      const int i = I * TBI + e / TBK, j = j0 + e % TBK;
      idx[u] = (i < R.N && j < je) ? R.rank_map[(size_t)i * R.N + j] : -1;
    }
  };
  auto load_vals = [&](int j0) {
#pragma unroll
    for (int u = 0; u < NR; ++u) rr[u] = idx[u] >= 0 ? (float)R.r[idx[u]] : 0.f;
#pragma unroll
    for (int u = 0; u < TBK * TBL / 256; ++u) {
      const int e = threadIdx.x + 256 * u;
      const int j = j0 + e / TBL, c = L * TBL + e % TBL;
      ww[u] = (j < je && c < R.k) ? R.W[(size_t)j * R.k + c] : 0.f;
    }
  };
  f32x16 acc = {};
  load_idx(jb);
  load_vals(jb);
  if (jb + TBK < je) load_idx(jb + TBK);
  for (int j0 = jb; j0 < je; j0 += TBK) {
#pragma unroll
    for (int u = 0; u < TBI * TBK / 256; ++u) {
      const int e = threadIdx.x + 256 * u;
      Rs[e / TBK][e % TBK] = rr[u];
    }
#pragma unroll
    for (int u = 0; u < TBK * TBL / 256; ++u) {
      const int e = threadIdx.x + 256 * u;
      Wt[e % TBL][e / TBL] = ww[u];
    }
    __syncthreads();
    if (j0 + TBK < je) load_vals(j0 + TBK);
    if (j0 + 2 * TBK < je) load_idx(j0 + 2 * TBK);
#pragma unroll
    for (int g8 = 0; g8 < TBK / 8; ++g8) {
      const float4 a4 = *(const float4*)&Rs[row0 + lr][g8 * 8 + 4 * h];
      const float4 b4 = *(const float4*)&Wt[col0 + lr][g8 * 8 + 4 * h];
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a4.x, b4.x, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a4.y, b4.y, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a4.z, b4.z, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a4.w, b4.w, acc, 0, 0, 0);
    }
    __syncthreads();
  }
  float* g = R.gp + (size_t)s * R.N * R.k;
  const int c = L * TBL + col0 + lr;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int i = I * TBI + row0 + (r >> 2) * 8 + h * 4 + (r & 3);
    if (i < R.N && c < R.k) g[(size_t)i * R.k + c] = 4.f * acc[r];
  }
}

// g = sum of the slices (in slice order), then Adam; grid.y = problem.
__global__ __launch_bounds__(256) void k_b_adam(Args a) {
  const Req R = expand(a.q[blockIdx.y]);
  float* W = const_cast<float*>(R.W);
  const int n = R.N * R.k;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x) {
    float ge = R.gp[e];
    for (int s = 1; s < R.sr; ++s) ge += R.gp[(size_t)s * n + e];
    const float me = a.b1 * R.m[e] + (1.f - a.b1) * ge;
    const float ve = a.b2 * R.v[e] + (1.f - a.b2) * ge * ge;
    R.m[e] = me;
    R.v[e] = ve;
    W[e] -= a.lr * (me / R.bc1) / (sqrtf(ve / R.bc2) + a.eps);
  }
}

}  // namespace bat

int batch_capacity() { return bat::kMaxBatch; }

// Problems [0, count), count <= kMaxBatch.  state == nullptr: forward and
// loss only (the certificate); otherwise the whole step.  Problem q's loss
// goes to losses[slot[q]] (losses[q] without a slot map).
hipError_t launch_step_group(sos_plan_s* const* plans, void* const* W, void* const* state, const int64_t* t,
                             const double* const* p, const sos_adam_t* h, double* losses, const int* slot,
                             int count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  const bool step = state != nullptr;
  bat::Args a = {};
  a.count = count;
  if (step) {
    a.lr = (float)h->lr;
    a.b1 = (float)h->beta1;
    a.b2 = (float)h->beta2;
    a.eps = (float)h->eps;
  }
  int maxM = 0, maxNK = 0;
  for (int q = 0; q < count; ++q) {
    const sos_plan_s* pl = plans[q];
    bat::Desc& D = a.q[q];
    D.W = (const float*)W[q];
    if (step) {
      D.m = (float*)state[q];
      D.bc1 = (float)(1.0 - pow(h->beta1, (double)t[q]));
      D.bc2 = (float)(1.0 - pow(h->beta2, (double)t[q]));
    }
    D.p = p[q];
    D.hdr = pl->ws + pl->lay.bhdr;
    D.loss = losses + (slot ? slot[q] : q);
    const BatchHeader& H = pl->bhdr;
    const int ti = (H.N + bat::TF - 1) / bat::TF;
    a.fwd_off[q + 1] = a.fwd_off[q] + ti * (ti + 1) / 2 * H.sg;
    const int bi = (H.N + bat::TBI - 1) / bat::TBI, bl = (H.k + bat::TBL - 1) / bat::TBL;
    a.bwd_off[q + 1] = a.bwd_off[q] + bi * bl * H.sr;
    maxM = H.M > maxM ? H.M : maxM;
    maxNK = H.N * H.k > maxNK ? H.N * H.k : maxNK;
  }
  auto blocks = [](int n) {
    const int b = (n + 255) / 256;
    return b < 1 ? 1 : (b > 1024 ? 1024 : b);
  };
  bat::k_b_gram<<<a.fwd_off[count], 256, 0, s>>>(a);
  bat::k_b_coeff<<<dim3((maxM + 255) / 256, count), 256, 0, s>>>(a);
  if (step) {
    bat::k_b_rw<<<a.bwd_off[count], 256, 0, s>>>(a);
    bat::k_b_adam<<<dim3(blocks(maxNK), count), 256, 0, s>>>(a);
  }
  return hipGetLastError();
}

}  // namespace sos
