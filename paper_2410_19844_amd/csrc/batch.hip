// Grouped kernels for many small problems at once (serving): one Adam step
// (forward, loss, backward, update) of up to kMaxBatch independent problems
// per launch of each kernel.  Each problem keeps its own plan workspace
// (ranking codes and tables, pair lists, Gram scratch, residual r, gradient
// scratch), its own W and its own Adam state; the kernels read all of them
// through a descriptor table passed by value in the kernel arguments, so a
// call allocates nothing.
//
// Every block works on one problem, and every sum runs in an order fixed by
// that problem's shape alone (no atomics), so a problem's results do not
// depend on the other problems in the launch.
//
//   k_b_gram   G = W W^T, upper-triangle 32 x 32 tiles, FP32 entries
//              converted to FP64 (exact products) on v_mfma_f64_16x16x4
//   k_b_coeff  r_m = sum over the pairs (i <= j) of monomial m of
//              (2 - [i = j]) G_ij, minus p_m, in the plan's pair order
//   k_b_loss   L = sum r_m^2, one block per problem
//   k_b_rw     g = 4 R W in FP32, R_ij = r[rank(alpha_i + alpha_j)]
//   k_b_adam   bias-corrected Adam in FP32
#include <hip/hip_runtime.h>

#include <cstdint>

#include "sos_internal.h"

namespace sos {
namespace bat {

typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr int kMaxBatch = 24;

struct Req {
  const float* W;
  float* m;
  float* v;
  float* g;
  const double* p;
  double* r;
  double* G;
  const int32_t* pair_off;
  const int32_t* pair_idx;
  double* loss;
  const uint32_t* codes;
  const int32_t* tables;
  int N, M, k, nwords, ngroups;
  float bc1, bc2;
};

struct Args {
  int count;
  int fwd_off[kMaxBatch + 1];  // prefix sums of forward tiles
  int bwd_off[kMaxBatch + 1];  // prefix sums of backward tiles
  float lr, b1, b2, eps;
  Req q[kMaxBatch];
};
static_assert(sizeof(Args) <= 4000, "kernel argument block too large");

// problem owning flat block b (off: prefix sums, off[count] = total)
__device__ __forceinline__ int find_req(const int* off, int count, int b) {
  int q = 0;
  while (q + 1 < count && off[q + 1] <= b) ++q;
  return q;
}

__device__ __forceinline__ int rank_sum(const Req& R, int i, int j) {
  int r = 0;
#pragma unroll
  for (int w = 0; w < kMaxWords; ++w) {
    if (w < R.nwords) {
      const uint32_t s = R.codes[(size_t)i * R.nwords + w] + R.codes[(size_t)j * R.nwords + w];
      r += R.tables[(2 * w) * kGroupEntries + (s & 0xFFFu)];
      if (2 * w + 1 < R.ngroups) r += R.tables[(2 * w + 1) * kGroupEntries + ((s >> 16) & 0xFFFu)];
    }
  }
  return r;
}

// Gram tiles.  Tile t of a problem is (I, J), I <= J, numbered column by
// column.  Four waves, each one 16 x 16 block of the 32 x 32 tile; K in
// chunks of 32 through LDS (FP32), each chunk 8 MFMA k-steps of 4.
// MFMA f64 16x16x4 operand: lane l holds row l % 16 at k = l / 16; result
// register q of lane l is row l / 16 + 4 q, column l % 16.
constexpr int TF = 32, TK = 32;
__global__ __launch_bounds__(256) void k_b_gram(Args a) {
  __shared__ float As[TF][TK + 1], Bs[TF][TK + 1];
  const int q = find_req(a.fwd_off, a.count, blockIdx.x);
  const Req& R = a.q[q];
  const int t = blockIdx.x - a.fwd_off[q];
  int J = 0;
  while ((J + 1) * (J + 2) / 2 <= t) ++J;
  const int I = t - J * (J + 1) / 2;
  const int wave = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int wm = wave >> 1, wn = wave & 1;
  f64x4 acc = {0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < R.k; k0 += TK) {
#pragma unroll
    for (int u = 0; u < TF * TK / 256; ++u) {
      const int e = threadIdx.x + 256 * u;
      const int rr = e / TK, cc = e % TK;
      const int i = I * TF + rr, j = J * TF + rr, kk = k0 + cc;
      As[rr][cc] = (i < R.N && kk < R.k) ? R.W[(size_t)i * R.k + kk] : 0.f;
      Bs[rr][cc] = (j < R.N && kk < R.k) ? R.W[(size_t)j * R.k + kk] : 0.f;
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < TK / 4; ++s) {
      const double av = As[wm * 16 + (l & 15)][4 * s + (l >> 4)];
      const double bv = Bs[wn * 16 + (l & 15)][4 * s + (l >> 4)];
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
    }
    __syncthreads();
  }
  const int j = J * TF + wn * 16 + (l & 15);
#pragma unroll
  for (int qq = 0; qq < 4; ++qq) {
    const int i = I * TF + wm * 16 + (l >> 4) + 4 * qq;
    if (i < R.N && j < R.N && i <= j) R.G[(size_t)i * R.N + j] = acc[qq];
  }
}

// r_m = c_m - p_m, c_m summed over the plan's pair list; grid.y = problem.
__global__ __launch_bounds__(256) void k_b_coeff(Args a) {
  const Req& R = a.q[blockIdx.y];
  for (int m = blockIdx.x * blockDim.x + threadIdx.x; m < R.M; m += gridDim.x * blockDim.x) {
    const int e1 = R.pair_off[m + 1];
    double c = 0.0;
    for (int e = R.pair_off[m]; e < e1; ++e) {
      const uint32_t x = (uint32_t)R.pair_idx[e];
      const double gij = R.G[x & 0x7FFFFFFFu];
      c += (x >> 31) ? 2.0 * gij : gij;
    }
    R.r[m] = c - R.p[m];
  }
}

// L = sum r^2, one block per problem.
__global__ __launch_bounds__(256) void k_b_loss(Args a) {
  const Req& R = a.q[blockIdx.x];
  double s = 0;
  for (int e = threadIdx.x; e < R.M; e += 256) s += R.r[e] * R.r[e];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  __shared__ double part[4];
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) R.loss[0] = (part[0] + part[1]) + (part[2] + part[3]);
}

// g = 4 R W: tiles of 32 rows (i) x 64 columns (l); the contraction index j
// runs in chunks of 32 with R_ij gathered from r into LDS.
constexpr int TBI = 32, TBL = 64, TBK = 32;
__global__ __launch_bounds__(256) void k_b_rw(Args a) {
  __shared__ float Rs[TBI][TBK + 1];
  __shared__ float Ws[TBK][TBL + 1];
  const int q = find_req(a.bwd_off, a.count, blockIdx.x);
  const Req& R = a.q[q];
  const int t = blockIdx.x - a.bwd_off[q];
  const int nl = (R.k + TBL - 1) / TBL;
  const int I = t / nl, L = t % nl;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;  // rows 2 ty, 2 ty + 1; columns tx + 16 w
  float acc[2][4] = {};
  for (int j0 = 0; j0 < R.N; j0 += TBK) {
#pragma unroll
    for (int u = 0; u < TBI * TBK / 256; ++u) {
      const int e = threadIdx.x + 256 * u;
      const int rr = e / TBK, cc = e % TBK;
      const int i = I * TBI + rr, j = j0 + cc;
      Rs[rr][cc] = (i < R.N && j < R.N) ? (float)R.r[rank_sum(R, i, j)] : 0.f;
    }
#pragma unroll
    for (int u = 0; u < TBK * TBL / 256; ++u) {
      const int e = threadIdx.x + 256 * u;
      const int rr = e / TBL, cc = e % TBL;
      const int j = j0 + rr, c = L * TBL + cc;
      Ws[rr][cc] = (j < R.N && c < R.k) ? R.W[(size_t)j * R.k + c] : 0.f;
    }
    __syncthreads();
#pragma unroll 8
    for (int jj = 0; jj < TBK; ++jj) {
      const float r0 = Rs[2 * ty][jj], r1 = Rs[2 * ty + 1][jj];
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        const float x = Ws[jj][tx + 16 * w];
        acc[0][w] = fmaf(r0, x, acc[0][w]);
        acc[1][w] = fmaf(r1, x, acc[1][w]);
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      const int i = I * TBI + 2 * ty + u, c = L * TBL + tx + 16 * w;
      if (i < R.N && c < R.k) R.g[(size_t)i * R.k + c] = 4.f * acc[u][w];
    }
}

// Adam; grid.y = problem.
__global__ __launch_bounds__(256) void k_b_adam(Args a) {
  const Req& R = a.q[blockIdx.y];
  float* W = const_cast<float*>(R.W);
  const int n = R.N * R.k;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x) {
    const float ge = R.g[e];
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
// loss only (the certificate); otherwise the whole step.
hipError_t launch_step_group(sos_plan_s* const* plans, void* const* W, void* const* state, const int64_t* t,
                             const double* const* p, const sos_adam_t* h, double* losses, int count,
                             hipStream_t s) {
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
    bat::Req& R = a.q[q];
    char* ws = pl->ws;
    R.W = (const float*)W[q];
    if (step) {
      R.m = (float*)state[q];
      R.v = (float*)((char*)state[q] + pl->state_bytes / 4);
      R.bc1 = (float)(1.0 - pow(h->beta1, (double)t[q]));
      R.bc2 = (float)(1.0 - pow(h->beta2, (double)t[q]));
    }
    R.g = (float*)(ws + pl->lay.g);
    R.p = p[q];
    R.r = (double*)(ws + pl->lay.r);
    R.G = (double*)(ws + pl->lay.bG);
    R.pair_off = (const int32_t*)(ws + pl->lay.pair_off);
    R.pair_idx = (const int32_t*)(ws + pl->lay.pair_idx);
    R.loss = losses + q;
    R.codes = (const uint32_t*)(ws + pl->lay.codes);
    R.tables = (const int32_t*)(ws + pl->lay.tables);
    R.N = (int)pl->N;
    R.M = (int)pl->M;
    R.k = pl->k;
    R.nwords = pl->nwords;
    R.ngroups = pl->ngroups;
    const int ti = (R.N + bat::TF - 1) / bat::TF;
    a.fwd_off[q + 1] = a.fwd_off[q] + ti * (ti + 1) / 2;
    const int bi = (R.N + bat::TBI - 1) / bat::TBI, bl = (R.k + bat::TBL - 1) / bat::TBL;
    a.bwd_off[q + 1] = a.bwd_off[q] + bi * bl;
    maxM = R.M > maxM ? R.M : maxM;
    maxNK = R.N * R.k > maxNK ? R.N * R.k : maxNK;
  }
  auto blocks = [](int n) {
    const int b = (n + 255) / 256;
    return b < 1 ? 1 : (b > 1024 ? 1024 : b);
  };
  bat::k_b_gram<<<a.fwd_off[count], 256, 0, s>>>(a);
  bat::k_b_coeff<<<dim3(blocks(maxM), count), 256, 0, s>>>(a);
  bat::k_b_loss<<<count, 256, 0, s>>>(a);
  if (step) {
    bat::k_b_rw<<<a.bwd_off[count], 256, 0, s>>>(a);
    bat::k_b_adam<<<dim3(blocks(maxNK), count), 256, 0, s>>>(a);
  }
  return hipGetLastError();
}

}  // namespace sos
