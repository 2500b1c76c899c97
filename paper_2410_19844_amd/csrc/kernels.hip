// gfx950 kernels of the SOS hot path.
//
//   k_prep        operand copies of W (padded, zero-filled; bf16 hi/lo split;
//                 transposed copies for the backward)
//   k_init_r      r <- -p
//   k_gram        forward: Gram tiles G_IJ = W_I W_J^T on MFMA over the upper
//                 triangle of tiles, reduced straight into the FP64 residual
//                 r[rank(alpha_i + alpha_j)] by atomic adds (eq. nonconvex)
//   k_sumsq_*     L = sum r^2 (deterministic two-pass reduction)
//   k_gather      R_ij = r[rank(alpha_i + alpha_j)] in the operand type
//   k_rw          backward: g = 4 R W on MFMA
//   k_adam        bias-corrected Adam (Kingma and Ba), in place
//
// Every GEMM here is "NT": C[i][j] = sum_k A[i][k] * B[j][k], both operands
// K-contiguous, padded so that tiles never read out of bounds.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>

#include <cstdint>

#include "sos_internal.h"

namespace sos {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

__global__ void k_pair_ranks(RankTab c, int N, int32_t* __restrict__ out) {
  const int64_t total = (int64_t)N * N;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / N), j = (int)(e % N);
    out[e] = pair_rank(c, i, j);
  }
}

// ---------------------------------------------------------------------------
// Operand preparation
// ---------------------------------------------------------------------------
struct PrepArgs {
  const void* W;       // N x k, ld k (double for FP64 plans, float otherwise)
  int N, k;
  int64_t Np, Kp;      // forward copies: rows Np, ld Kp
  int64_t Kp2, Np2;    // transposed copies: rows Kp2, ld Np2
  void* a_hi; void* a_lo; float* a_f32; float* x_f32;
  void* t_hi; void* t_lo;
  const int* sx;       // fp16 split (mode 3): sx[0] = sW, the copies hold 2^sW w
};

// fp16 words carried in the bf16-typed operand arrays
__device__ __forceinline__ __bf16 f16_bits(float x) { return __builtin_bit_cast(__bf16, (_Float16)x); }
__device__ __forceinline__ float f16_value(__bf16 h) { return (float)__builtin_bit_cast(_Float16, h); }

// 64 x 64 tiles through LDS so that both the row-major and the transposed
// copies are written with coalesced stores.  Mode: 0 = FP64, 1 = FP32,
// 2 = bf16 hi/lo split, 3 = fp16 hi/lo split of 2^sW w.  Each destination is
// written only when its pointer is set: the caller asks for the copies its
// forward and backward read.
template <int MODE>
__global__ __launch_bounds__(256) void k_prep(PrepArgs a) {
  using WT = typename std::conditional<MODE == 0, double, float>::type;
  __shared__ WT tile[64][65];
  const int64_t i0 = (int64_t)blockIdx.y * 64, l0 = (int64_t)blockIdx.x * 64;
  const float wsc = (MODE == 3) ? pow2f(a.sx[0]) : 1.0f;
  const WT* W = (const WT*)a.W;
  const int tx = threadIdx.x % 64, ty = threadIdx.x / 64;
  for (int r = ty; r < 64; r += 4) {
    const int64_t i = i0 + r, l = l0 + tx;
    WT v = 0;
    if (i < a.N && l < a.k) v = W[i * a.k + l];
    tile[r][tx] = v;
    if (i < a.Np && l < a.Kp) {
      const int64_t o = i * a.Kp + l;
      if (MODE != 0 && a.x_f32) a.x_f32[blk_off(i, l, panel_stride(a.Kp / kBlkK, 4))] = (float)v;
      if (MODE == 0) {
        if (a.a_hi) ((double*)a.a_hi)[o] = (double)v;
      } else if (MODE == 1) {
        if (a.a_hi) ((float*)a.a_hi)[o] = (float)v;
      } else {
        if (a.a_hi) {
          const int64_t ob = blk_off(i, l, panel_stride(a.Kp / kBlkK, 2));
          if (MODE == 3) {
            const float ws = (float)v * wsc;
            const __bf16 h = f16_bits(ws);
            ((__bf16*)a.a_hi)[ob] = h;
            ((__bf16*)a.a_lo)[ob] = f16_bits(ws - f16_value(h));
          } else {
            const __bf16 h = (__bf16)(float)v;
            ((__bf16*)a.a_hi)[ob] = h;
            ((__bf16*)a.a_lo)[ob] = (__bf16)((float)v - (float)h);
          }
        }
        if (a.a_f32) a.a_f32[o] = (float)v;
      }
    }
  }
  if (!a.t_hi) return;
  __syncthreads();
  for (int r = ty; r < 64; r += 4) {
    const int64_t l = l0 + r, i = i0 + tx;
    if (l < a.Kp2 && i < a.Np2) {
      const WT v = tile[tx][r];
      const int64_t o = l * a.Np2 + i;
      if (MODE == 0) ((double*)a.t_hi)[o] = (double)v;
      else if (MODE == 1) ((float*)a.t_hi)[o] = (float)v;
      else if (MODE == 3) {
        const float ws = (float)v * wsc;
        const __bf16 h = f16_bits(ws);
        const int64_t ob = blk_off(l, i, panel_stride(a.Np2 / kBlkK, 2));
        ((__bf16*)a.t_hi)[ob] = h;
        if (a.t_lo) ((__bf16*)a.t_lo)[ob] = f16_bits(ws - f16_value(h));
      } else {
        const __bf16 h = (__bf16)(float)v;
        const int64_t ob = blk_off(l, i, panel_stride(a.Np2 / kBlkK, 2));
        ((__bf16*)a.t_hi)[ob] = h;
        if (a.t_lo) ((__bf16*)a.t_lo)[ob] = (__bf16)((float)v - (float)h);
      }
    }
  }
}

__global__ void k_init_r(const double* __restrict__ p, double* __restrict__ r, int64_t M) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < M;
       e += (int64_t)gridDim.x * blockDim.x)
    r[e] = -p[e];
}

// ---------------------------------------------------------------------------
// Sum of squares (deterministic: fixed grid, fixed order)
// ---------------------------------------------------------------------------
constexpr int kSumBlocks = 512;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ double block_sum(double v) {
  __shared__ double part[16];
  v = wave_sum(v);
  const int w = threadIdx.x / 64, l = threadIdx.x % 64;
  if (l == 0) part[w] = v;
  __syncthreads();
  double s = 0;
  if (threadIdx.x == 0)
    for (int q = 0; q < (int)(blockDim.x / 64); ++q) s += part[q];
  return s;
}

__device__ float block_max(float v) {
  __shared__ float part[16];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
  const int w = threadIdx.x / 64, l = threadIdx.x % 64;
  if (l == 0) part[w] = v;
  __syncthreads();
  float m = 0.f;
  if (threadIdx.x == 0)
    for (int q = 0; q < (int)(blockDim.x / 64); ++q) m = fmaxf(m, part[q]);
  return m;
}

// The exponent s with max * 2^s < 2^top: the power-of-two scale that puts
// the largest magnitude just below 2^top (0 when max is 0 or not finite),
// clamped to [-100, 100] so that every scale and its inverse, and their
// products in the epilogues, stay normal floats.
__device__ __forceinline__ int pow2_exponent(float m, int top) {
  if (!(m > 0.f) || !(m <= FLT_MAX)) return 0;
  int e;
  (void)frexpf(m, &e);  // m < 2^e
  return min(100, max(-100, top - e));
}

// x32 (optional): FP32 copy of x, written on the way (the gather of R reads it);
// pmax (optional): per-block max |x32| (the fp16 gather's scale)
__global__ __launch_bounds__(256) void k_sumsq_partial(const double* __restrict__ x, int64_t M,
                                                       double* __restrict__ partial, float* __restrict__ x32,
                                                       float* __restrict__ pmax) {
  double s = 0;
  float m = 0.f;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < M;
       e += (int64_t)gridDim.x * blockDim.x) {
    const double v = x[e];
    s += v * v;
    if (x32) {
      x32[e] = (float)v;
      m = fmaxf(m, fabsf((float)v));
    }
  }
  s = block_sum(s);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
  if (pmax) {
    m = block_max(m);
    if (threadIdx.x == 0) pmax[blockIdx.x] = m;
  }
}

// rexp (optional): the fp16 gather's scale exponent sR from the block
// maxima, so that 2^sR |R| < 2^14
__global__ __launch_bounds__(256) void k_sumsq_final(const double* __restrict__ partial,
                                                     double* __restrict__ out, const float* __restrict__ pmax,
                                                     int* __restrict__ rexp) {
  double s = 0;
  for (int q = threadIdx.x; q < kSumBlocks; q += blockDim.x) s += partial[q];
  s = block_sum(s);
  if (threadIdx.x == 0) out[0] = s;
  if (pmax) {
    float m = 0.f;
    for (int q = threadIdx.x; q < kSumBlocks; q += blockDim.x) m = fmaxf(m, pmax[q]);
    m = block_max(m);
    if (threadIdx.x == 0) rexp[0] = pow2_exponent(m, 14);
  }
}

// The scale of the fp16 copies of W: 2^sW with 2^sW max|W| < 2^12, leaving a
// factor 16 of headroom below fp16's largest value for W to grow while fused
// steps reuse the scale.  Per-block maxima, then one block.
__global__ __launch_bounds__(256) void k_absmax_partial(const float* __restrict__ W, int64_t n,
                                                        float* __restrict__ pmax) {
  float m = 0.f;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    m = fmaxf(m, fabsf(W[e]));
  m = block_max(m);
  if (threadIdx.x == 0) pmax[blockIdx.x] = m;
}

__global__ __launch_bounds__(256) void k_absmax_final(const float* __restrict__ pmax, int* __restrict__ wexp) {
  float m = 0.f;
  for (int q = threadIdx.x; q < kSumBlocks; q += blockDim.x) m = fmaxf(m, pmax[q]);
  m = block_max(m);
  if (threadIdx.x == 0) wexp[0] = pow2_exponent(m, 12);
}

// ---------------------------------------------------------------------------
// Tiled NT GEMM core: 128 x 128 output tile, 256 threads = 4 waves (2 x 2),
// each wave 64 x 64.  Operands staged through double-buffered LDS.
// ---------------------------------------------------------------------------
constexpr int BM = kGenericTile;
constexpr int kThreads = 256;

// Mode F64: double operands, f64 16x16x4 MFMA.  Output of one 16x16 block:
// lane l, register q holds row (l / 16) + 4 q, column l % 16.
struct MF64 {
  using GT = double;  // global operand element
  using LT = double;  // LDS element
  static constexpr int NARR = 1;
  static constexpr int BK = 16;
  static constexpr int LDS_LD = BK + 2;  // elements per LDS row (padded)
  static constexpr int NACC = 64;        // doubles per lane
  using Acc = double;
};
// Mode EXACT: float operands in memory, converted exactly to double, f64 MFMA.
struct MEX : MF64 {
  using GT = float;
};
// Mode F32: float operands, f32 32x32x2 MFMA.  Output of one 32x32 block:
// lane l, register q holds row (q / 4) * 8 + (l / 32) * 4 + q % 4, column l % 32.
struct MF32 {
  using GT = float;
  using LT = float;
  static constexpr int NARR = 1;
  static constexpr int BK = 32;
  static constexpr int LDS_LD = BK + 4;
  static constexpr int NACC = 64;
  using Acc = float;
};
// Mode BF3: bf16 hi and lo arrays, three 32x32x16 bf16 MFMA products.
struct MBF3 {
  using GT = __bf16;
  using LT = __bf16;
  static constexpr int NARR = 2;
  static constexpr int BK = 32;
  static constexpr int LDS_LD = BK + 8;
  static constexpr int NACC = 64;
  using Acc = float;
};

template <class Md>
struct Stage {
  // one operand tile: NARR arrays of BM rows x LDS_LD elements
  typename Md::LT a[Md::NARR][BM * Md::LDS_LD];
  typename Md::LT b[Md::NARR][BM * Md::LDS_LD];
};

// global -> registers -> LDS.  The tile is BM rows of BK elements; each thread
// moves 16-byte chunks of the global rows.
template <class Md>
struct Loader {
  using GT = typename Md::GT;
  using LT = typename Md::LT;
  static constexpr int ROW_BYTES = Md::BK * (int)sizeof(GT);
  static constexpr int CPR = ROW_BYTES / 16;                       // chunks per row
  static constexpr int CHUNKS = BM * CPR;                          // per array
  static constexpr int PER_THREAD = CHUNKS / kThreads;
  static constexpr int EPC = 16 / (int)sizeof(GT);                 // elements per chunk
  static_assert(CHUNKS % kThreads == 0, "tile must split evenly");
  uint4 reg[Md::NARR][PER_THREAD];

  __device__ __forceinline__ void load(const GT* const* base, int64_t ld, int64_t row0, int64_t k0) {
#pragma unroll
    for (int q = 0; q < Md::NARR; ++q)
#pragma unroll
      for (int c = 0; c < PER_THREAD; ++c) {
        const int ch = threadIdx.x + c * kThreads;
        const int row = ch / CPR, cc = ch % CPR;
        reg[q][c] = *(const uint4*)(base[q] + (row0 + row) * ld + k0 + cc * EPC);
      }
  }
  __device__ __forceinline__ void store(LT (*dst)[BM * Md::LDS_LD]) {
#pragma unroll
    for (int q = 0; q < Md::NARR; ++q)
#pragma unroll
      for (int c = 0; c < PER_THREAD; ++c) {
        const int ch = threadIdx.x + c * kThreads;
        const int row = ch / CPR, cc = ch % CPR;
        LT* d = &dst[q][row * Md::LDS_LD + cc * EPC];
        if constexpr (sizeof(GT) == sizeof(LT)) {
          *(uint4*)d = reg[q][c];
        } else {  // float -> double, exact
          const float* f = (const float*)&reg[q][c];
#pragma unroll
          for (int e = 0; e < EPC; ++e) d[e] = (double)f[e];
        }
      }
  }
};

// MFMA over one LDS stage.  acc is the wave's 64 x 64 block, NACC per lane.
template <class Md>
__device__ __forceinline__ void mma_stage(const Stage<Md>& s, typename Md::Acc* acc, int wm, int wn);

template <>
__device__ __forceinline__ void mma_stage<MF64>(const Stage<MF64>& s, double* acc, int wm, int wn) {
  const int l = threadIdx.x % 64;
#pragma unroll
  for (int kk = 0; kk < MF64::BK / 4; ++kk) {
    double a[4], b[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      a[q] = s.a[0][(wm * 64 + q * 16 + l % 16) * MF64::LDS_LD + kk * 4 + l / 16];
      b[q] = s.b[0][(wn * 64 + q * 16 + l % 16) * MF64::LDS_LD + kk * 4 + l / 16];
    }
#pragma unroll
    for (int bi = 0; bi < 4; ++bi)
#pragma unroll
      for (int bj = 0; bj < 4; ++bj) {
        f64x4 c;
        double* p = acc + (bi * 4 + bj) * 4;
        c[0] = p[0]; c[1] = p[1]; c[2] = p[2]; c[3] = p[3];
        c = __builtin_amdgcn_mfma_f64_16x16x4f64(a[bi], b[bj], c, 0, 0, 0);
        p[0] = c[0]; p[1] = c[1]; p[2] = c[2]; p[3] = c[3];
      }
  }
}

template <>
__device__ __forceinline__ void mma_stage<MEX>(const Stage<MEX>& s, double* acc, int wm, int wn) {
  mma_stage<MF64>(reinterpret_cast<const Stage<MF64>&>(s), acc, wm, wn);
}

template <>
__device__ __forceinline__ void mma_stage<MF32>(const Stage<MF32>& s, float* acc, int wm, int wn) {
  const int l = threadIdx.x % 64;
#pragma unroll
  for (int kk = 0; kk < MF32::BK / 2; ++kk) {
    float a[2], b[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      a[q] = s.a[0][(wm * 64 + q * 32 + l % 32) * MF32::LDS_LD + kk * 2 + l / 32];
      b[q] = s.b[0][(wn * 64 + q * 32 + l % 32) * MF32::LDS_LD + kk * 2 + l / 32];
    }
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int bj = 0; bj < 2; ++bj) {
        f32x16 c;
        float* p = acc + (bi * 2 + bj) * 16;
#pragma unroll
        for (int e = 0; e < 16; ++e) c[e] = p[e];
        c = __builtin_amdgcn_mfma_f32_32x32x2f32(a[bi], b[bj], c, 0, 0, 0);
#pragma unroll
        for (int e = 0; e < 16; ++e) p[e] = c[e];
      }
  }
}

template <>
__device__ __forceinline__ void mma_stage<MBF3>(const Stage<MBF3>& s, float* acc, int wm, int wn) {
  const int l = threadIdx.x % 64;
#pragma unroll
  for (int kk = 0; kk < MBF3::BK / 16; ++kk) {
    bf16x8 ah[2], al[2], bh[2], bl[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int ra = (wm * 64 + q * 32 + l % 32) * MBF3::LDS_LD + kk * 16 + (l / 32) * 8;
      const int rb = (wn * 64 + q * 32 + l % 32) * MBF3::LDS_LD + kk * 16 + (l / 32) * 8;
      ah[q] = *(const bf16x8*)&s.a[0][ra];
      al[q] = *(const bf16x8*)&s.a[1][ra];
      bh[q] = *(const bf16x8*)&s.b[0][rb];
      bl[q] = *(const bf16x8*)&s.b[1][rb];
    }
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int bj = 0; bj < 2; ++bj) {
        f32x16 c;
        float* p = acc + (bi * 2 + bj) * 16;
#pragma unroll
        for (int e = 0; e < 16; ++e) c[e] = p[e];
        c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[bi], bh[bj], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[bi], bl[bj], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[bi], bh[bj], c, 0, 0, 0);
#pragma unroll
        for (int e = 0; e < 16; ++e) p[e] = c[e];
      }
  }
}

// (row, col) inside the wave's 64 x 64 block of accumulator element e.
template <class Md>
__device__ __forceinline__ void acc_pos(int e, int& row, int& col) {
  const int l = threadIdx.x % 64;
  if constexpr (Md::BK == 16) {  // f64 16x16 blocks, 4 x 4 of them
    const int blk = e / 4, q = e % 4;
    row = (blk / 4) * 16 + l / 16 + 4 * q;
    col = (blk % 4) * 16 + l % 16;
  } else {  // 32x32 blocks, 2 x 2 of them
    const int blk = e / 16, q = e % 16;
    row = (blk / 2) * 32 + (q / 4) * 8 + (l / 32) * 4 + q % 4;
    col = (blk % 2) * 32 + l % 32;
  }
}

template <class Md>
__device__ __forceinline__ void gemm_tile(const typename Md::GT* const* A, const typename Md::GT* const* B,
                                          int64_t ld, int64_t K, int64_t a_row0, int64_t b_row0,
                                          Stage<Md>* st, typename Md::Acc* acc) {
  const int wave = threadIdx.x / 64;
  const int wm = wave / 2, wn = wave % 2;
#pragma unroll
  for (int e = 0; e < Md::NACC; ++e) acc[e] = 0;
  Loader<Md> la, lb;
  la.load(A, ld, a_row0, 0);
  lb.load(B, ld, b_row0, 0);
  la.store(st[0].a);
  lb.store(st[0].b);
  __syncthreads();
  const int64_t nk = K / Md::BK;
  for (int64_t kt = 0; kt + 1 < nk; ++kt) {
    const int cur = (int)(kt & 1);
    la.load(A, ld, a_row0, (kt + 1) * Md::BK);
    lb.load(B, ld, b_row0, (kt + 1) * Md::BK);
    mma_stage<Md>(st[cur], acc, wm, wn);
    la.store(st[cur ^ 1].a);
    lb.store(st[cur ^ 1].b);
    __syncthreads();
  }
  mma_stage<Md>(st[(nk - 1) & 1], acc, wm, wn);
}

// ---------------------------------------------------------------------------
// Forward: gram tiles over the upper triangle, scattered into r.
// ---------------------------------------------------------------------------
struct GramArgs {
  const void* A[2];   // operand arrays (hi[, lo]); rows Np, ld Kp
  int64_t ld, K;      // ld = K = Kp
  int64_t kslice;     // contraction length per block (a multiple of 64)
  int N, T;           // T = Np / BM tiles per side
  int tiles;          // T (T + 1) / 2
  RankTab rk;
  double* r;
  double* Gd;         // deterministic forward: store G_ij (i <= j) of slice s at Gd[(s N + i) N + j]
                      // instead of adding into r (nullptr: add)
};

__device__ __forceinline__ void tri_tile(int b, int& I, int& J) {
  // b -> (I, J), I <= J, enumerating column J = 0, 1, ... with I = 0..J
  int j = (int)((sqrtf(8.0f * (float)b + 1.0f) - 1.0f) * 0.5f);
  while ((j + 1) * (j + 2) / 2 <= b) ++j;
  while (j * (j + 1) / 2 > b) --j;
  J = j;
  I = b - j * (j + 1) / 2;
}

// Block b takes tile b % tiles over the contraction slice b / tiles (more
// than one slice only when the tiles alone would leave the chip idle); the
// FP64 atomics sum tiles and slices alike, or, for the deterministic
// forward, each slice's G entries are stored for k_coeff_det to sum.
template <class Md>
__global__ __launch_bounds__(kThreads) void k_gram(GramArgs g) {
  extern __shared__ __align__(16) char smem[];
  Stage<Md>* st = (Stage<Md>*)smem;
  int I, J;
  tri_tile((int)(blockIdx.x % g.tiles), I, J);
  const int64_t k0 = (int64_t)(blockIdx.x / g.tiles) * g.kslice;
  const int64_t klen = g.K - k0 < g.kslice ? g.K - k0 : g.kslice;
  const typename Md::GT* ops[2] = {(const typename Md::GT*)g.A[0] + k0, (const typename Md::GT*)g.A[1] + k0};
  typename Md::Acc acc[Md::NACC];
  gemm_tile<Md>(ops, ops, g.ld, klen, (int64_t)I * BM, (int64_t)J * BM, st, acc);
  const int wave = threadIdx.x / 64;
  const int wm = wave / 2, wn = wave % 2;
  // Epilogue through LDS in two row halves (the stage buffers are free now):
  // the copy-out indexes the accumulators at compile time, so they stay in
  // registers; the rank-and-add loop indexes LDS instead.
  using Acc = typename Md::Acc;
  constexpr int HR = BM / 2;
  static_assert(HR * BM * sizeof(Acc) <= 2 * sizeof(Stage<Md>), "half tile must fit the stage buffers");
  Acc* half = (Acc*)smem;
#pragma unroll
  for (int hh = 0; hh < 2; ++hh) {
    __syncthreads();
    if (wm == hh) {
#pragma unroll
      for (int e = 0; e < Md::NACC; ++e) {
        int row, col;
        acc_pos<Md>(e, row, col);
        half[row * BM + wn * 64 + col] = acc[e];
      }
    }
    __syncthreads();
    if (g.Gd) {
      double* Gs = g.Gd + (int64_t)(blockIdx.x / g.tiles) * g.N * g.N;
      for (int x = threadIdx.x; x < HR * BM; x += kThreads) {
        const int i = I * BM + hh * HR + x / BM, j = J * BM + x % BM;
        if (i < g.N && j < g.N && i <= j) Gs[(int64_t)i * g.N + j] = (double)half[x];
      }
      continue;
    }
    for (int x = threadIdx.x; x < HR * BM; x += kThreads) {
      const int i = I * BM + hh * HR + x / BM, j = J * BM + x % BM;
      if (i < g.N && j < g.N && i <= j) {
        const double w = (i == j) ? 1.0 : 2.0;
        unsafeAtomicAdd(g.r + pair_rank(g.rk, i, j), w * (double)half[x]);
      }
    }
  }
}

// Deterministic coefficients: r_m = sum over the pairs of monomial m, in the
// plan's pair-list order (i, then j, ascending), of w_ij sum_s G_ij^(s)
// (slices in order; w = 2 off the diagonal), minus p_m.  No atomics, so the
// result depends on nothing but W and p.
__global__ __launch_bounds__(256) void k_coeff_det(const double* __restrict__ Gd, int splits, int N,
                                                   const int32_t* __restrict__ off, const int32_t* __restrict__ idx,
                                                   const double* __restrict__ p, double* __restrict__ r, int M) {
  const int m = blockIdx.x * 256 + threadIdx.x;
  if (m >= M) return;
  const int64_t nn = (int64_t)N * N;
  double c = 0.0;
  for (int e = off[m]; e < off[m + 1]; ++e) {
    const uint32_t x = (uint32_t)idx[e];
    const int64_t ij = x & 0x7FFFFFFFu;
    double gsum = 0.0;
    for (int s = 0; s < splits; ++s) gsum += Gd[s * nn + ij];
    c += (x >> 31) ? 2.0 * gsum : gsum;
  }
  r[m] = c - p[m];
}

// ---------------------------------------------------------------------------
// Backward: R from r, then g = 4 R W.
// ---------------------------------------------------------------------------
template <int MODE>  // 0 FP64, 1 FP32, 2 bf16 hi/lo, 3 bf16 hi only
__global__ __launch_bounds__(256) void k_gather(RankTab rk, const double* __restrict__ r, int N,
                                                int64_t Np, int64_t ld, void* R_hi, void* R_lo) {
  const int64_t total = Np * ld;
  const int64_t nkb = ld / kBlkK;
  const int64_t ps = panel_stride(nkb, 2);
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    int i, j;
    int64_t o = e;
    if (MODE >= 2) {  // e walks the blocks of the panel-blocked layout in order (see blk_off)
      const int64_t blk = e / (kBlkRows * kBlkK), in = e % (kBlkRows * kBlkK);
      i = (int)((blk / nkb) * kBlkRows + in / kBlkK);
      j = (int)((blk % nkb) * kBlkK + in % kBlkK);
      o = blk_off(i, j, ps);
    } else {
      i = (int)(e / ld);
      j = (int)(e % ld);
    }
    double v = 0.0;
    if (i < N && j < N) v = r[pair_rank(rk, i, j)];
    if (MODE == 0) ((double*)R_hi)[o] = v;
    else if (MODE == 1) ((float*)R_hi)[o] = (float)v;
    else {
      const float f = (float)v;
      const __bf16 h = (__bf16)f;
      ((__bf16*)R_hi)[o] = h;
      if (MODE == 2) ((__bf16*)R_lo)[o] = (__bf16)(f - (float)h);
    }
  }
}

// Offset of R(i, j) in the gather's output layout, and a 16-value store.
template <int MODE>
__device__ __forceinline__ int64_t gather_off(int64_t i, int64_t j, int64_t ld, int64_t ps) {
  return MODE >= 2 ? blk_off(i, j, ps) : i * ld + j;
}

// Modes: 1 FP32 row-major; 2 bf16 hi and lo, 3 bf16 hi only, 4 fp16 hi and
// lo, 5 fp16 hi only (blocked; fp16 values are 2^sR R, scale applied by the caller)
template <int MODE>
__device__ __forceinline__ void gather_store16(void* R_hi, void* R_lo, int64_t o, const float* v) {
  if (MODE == 1) {
    float4* d = (float4*)((float*)R_hi + o);
#pragma unroll
    for (int q = 0; q < 4; ++q) d[q] = make_float4(v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]);
  } else {
    bf16x8 h[2], lo[2];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      if (MODE >= 4) {
        h[q >> 3][q & 7] = f16_bits(v[q]);
        lo[q >> 3][q & 7] = f16_bits(v[q] - f16_value(h[q >> 3][q & 7]));
      } else {
        h[q >> 3][q & 7] = (__bf16)v[q];
        lo[q >> 3][q & 7] = (__bf16)(v[q] - (float)h[q >> 3][q & 7]);
      }
    }
    bf16x8* dh = (bf16x8*)((__bf16*)R_hi + o);
    dh[0] = h[0];
    dh[1] = h[1];
    if (MODE == 2 || MODE == 4) {
      bf16x8* dl = (bf16x8*)((__bf16*)R_lo + o);
      dl[0] = lo[0];
      dl[1] = lo[1];
    }
  }
}

// R from r32 through the ranking, using R = R^T: each 256-thread block
// takes one 64 x 64 tile (I, J) with I <= J of the T2 x T2 tiles covering the
// N x N matrix (T2 = Np2 / 64), computes its values once, writes them at
// (I, J) and, through LDS, transposed at (J, I).  Blocks past the triangle
// write the zero rows Np2 .. Np - 1.  Per thread: one row, 16 consecutive
// columns (one 32-byte run of a 16-column block in the blocked layouts).
// The ranking's small table (field terms or binomials) and the tile's column
// codes are staged in LDS.  r32 is the FP32 copy of r: R is rounded to FP32
// first in every mode, so reading the copy gives the same bits as reading r.
// Mode 1 = FP32 row-major, 2 = bf16 hi and lo (blocked), 3 = bf16 hi only.
template <int MODE>
__global__ __launch_bounds__(256) void k_gather_sym(RankTab rk, const float* __restrict__ r32, int N, int64_t Np,
                                                    int64_t ld, int T2, int64_t nup, void* R_hi, void* R_lo,
                                                    const int* __restrict__ sx) {
  const float rsc = MODE >= 4 ? pow2f(sx[1]) : 1.0f;  // 2^sR for fp16 operands
  __shared__ float V[64][65];
  __shared__ uint32_t Cj[64 * kMaxWords];          // codes of the tile's 64 columns
  extern __shared__ int32_t Tab[];                 // field terms (dense) or binomials (sparse): ntab entries
  const int64_t ps = panel_stride(ld / kBlkK, 2);
  const int il = threadIdx.x >> 2, jc = (threadIdx.x & 3) * 16;
  const int64_t b = blockIdx.x;
  float v[16];
  if (b >= nup) {  // zero rows past the T2 tiles
    const int64_t z = b - nup;
    const int64_t i = (int64_t)T2 * 64 + (z / T2) * 64 + il, j = (z % T2) * 64 + jc;
#pragma unroll
    for (int q = 0; q < 16; ++q) v[q] = 0.f;
    gather_store16<MODE>(R_hi, R_lo, gather_off<MODE>(i, j, ld, ps), v);
    return;
  }
  // b -> (I, J), I <= J, row-major over the upper triangle
  const double tt = 2.0 * T2 + 1.0;
  int I = (int)((tt - sqrt(tt * tt - 8.0 * (double)b)) * 0.5);
  auto first = [&](int r) { return (int64_t)r * T2 - (int64_t)r * (r - 1) / 2; };
  while (I > 0 && first(I) > b) --I;
  while (first(I + 1) <= b) ++I;
  const int J = I + (int)(b - first(I));
  const int i = I * 64 + il, j0 = J * 64 + jc;
  {
    const int32_t* src = stage_tab(rk);
    for (int e = threadIdx.x; e < rk.ntab; e += 256) Tab[e] = src[e];
    for (int e = threadIdx.x; e < 64 * rk.nwords; e += 256) {
      const int jj = J * 64 + e / rk.nwords;
      Cj[e] = jj < N ? rk.codes[(size_t)jj * rk.nwords + e % rk.nwords] : 0u;
    }
  }
  __syncthreads();
  if (i < N) {
    if (!rk.sparse) {
      uint32_t ci[kMaxWords], cj[kMaxWords];
#pragma unroll
      for (int w = 0; w < kMaxWords; ++w) ci[w] = w < rk.nwords ? rk.codes[(size_t)i * rk.nwords + w] : 0u;
#pragma unroll
      for (int q = 0; q < 16; ++q) {
#pragma unroll
        for (int w = 0; w < kMaxWords; ++w) cj[w] = w < rk.nwords ? Cj[(jc + q) * rk.nwords + w] : 0u;
        v[q] = (j0 + q < N) ? rsc * r32[dense_rank_fields(ci, cj, rk.n, Tab)] : 0.f;
      }
    } else {
      const uint32_t ci = rk.codes[i];
      const int D1 = rk.D + 1;
      auto binom = [&](int x, int y) { return Tab[x * D1 + y]; };
#pragma unroll
      for (int q = 0; q < 16; ++q)
        v[q] = (j0 + q < N) ? rsc * r32[sparse_pair_rank(ci, Cj[jc + q], rk.n, rk.total, binom)] : 0.f;
    }
  } else {
#pragma unroll
    for (int q = 0; q < 16; ++q) v[q] = 0.f;
  }
  gather_store16<MODE>(R_hi, R_lo, gather_off<MODE>(i, j0, ld, ps), v);
  if (I == J) return;
#pragma unroll
  for (int q = 0; q < 16; ++q) V[il][jc + q] = v[q];
  __syncthreads();
  // transposed tile: row J*64 + il, columns I*64 + jc .. + 15
#pragma unroll
  for (int q = 0; q < 16; ++q) v[q] = V[jc + q][il];
  gather_store16<MODE>(R_hi, R_lo, gather_off<MODE>((int64_t)J * 64 + il, (int64_t)I * 64 + jc, ld, ps), v);
}

struct RwArgs {
  const void* A[2];   // R arrays: rows Np, ld K
  const void* B[2];   // W^T arrays: rows Kp2, ld K
  int64_t K;          // = Np2
  int N, k;
  void* g;            // N x k, ld k (double or float)
  bool g_double;
};

template <class Md>
__global__ __launch_bounds__(kThreads) void k_rw(RwArgs a) {
  extern __shared__ __align__(16) char smem[];
  Stage<Md>* st = (Stage<Md>*)smem;
  const int I = blockIdx.y, Lt = blockIdx.x;
  const typename Md::GT* A[2] = {(const typename Md::GT*)a.A[0], (const typename Md::GT*)a.A[1]};
  const typename Md::GT* B[2] = {(const typename Md::GT*)a.B[0], (const typename Md::GT*)a.B[1]};
  typename Md::Acc acc[Md::NACC];
  gemm_tile<Md>(A, B, a.K, a.K, (int64_t)I * BM, (int64_t)Lt * BM, st, acc);
  const int wave = threadIdx.x / 64;
  const int wm = wave / 2, wn = wave % 2;
#pragma unroll
  for (int e = 0; e < Md::NACC; ++e) {
    int row, col;
    acc_pos<Md>(e, row, col);
    const int i = I * BM + wm * 64 + row, l = Lt * BM + wn * 64 + col;
    if (i < a.N && l < a.k) {
      const double v = 4.0 * (double)acc[e];
      if (a.g_double) ((double*)a.g)[(int64_t)i * a.k + l] = v;
      else ((float*)a.g)[(int64_t)i * a.k + l] = (float)v;
    }
  }
}

// ---------------------------------------------------------------------------
// Adam (bias-corrected), in place.  bc1 = 1 - b1^t, bc2 = 1 - b2^t.
// ---------------------------------------------------------------------------
template <class T>
__global__ __launch_bounds__(256) void k_adam(T* __restrict__ W, T* __restrict__ m, T* __restrict__ v,
                                              const T* __restrict__ g, int64_t n, T lr, T b1, T b2,
                                              T eps, T bc1, T bc2) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const T ge = g[e];
    const T me = b1 * m[e] + (T(1) - b1) * ge;
    const T ve = b2 * v[e] + (T(1) - b2) * ge * ge;
    m[e] = me;
    v[e] = ve;
    W[e] -= lr * (me / bc1) / (sqrt(ve / bc2) + eps);
  }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
static inline int grid_for(int64_t n, int threads = 256, int cap = 65536) {
  int64_t b = (n + threads - 1) / threads;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return (int)b;
}

hipError_t launch_pair_ranks(const sos_plan_s* p, int32_t* out, hipStream_t s) {
  k_pair_ranks<<<grid_for(p->N * p->N), 256, 0, s>>>(rank_tab(p), (int)p->N, out);
  return hipGetLastError();
}

hipError_t launch_prep(const sos_plan_s* p, const void* W, const PrepNeeds& need, hipStream_t s) {
  PrepArgs a;
  a.W = W; a.N = (int)p->N; a.k = p->k;
  a.Np = p->Np; a.Kp = p->Kp; a.Kp2 = p->Kp2; a.Np2 = p->Np2;
  const bool split = split_plan(p);
  a.sx = scale_exponents(p);
  a.a_hi = need.a ? p->ws + p->lay.a_hi : nullptr;
  a.a_lo = (need.a && split) ? p->ws + p->lay.a_lo : nullptr;
  a.a_f32 = (split && need.a_f32) ? (float*)(p->ws + p->lay.a_f32) : nullptr;
  a.x_f32 = (p->prec != SOS_FP64 && need.x_f32) ? (float*)(p->ws + p->lay.x_f32) : nullptr;
  a.t_hi = need.t ? p->ws + p->lay.t_hi : nullptr;
  a.t_lo = (need.t && need.t_lo && split) ? p->ws + p->lay.t_lo : nullptr;
  const int64_t rows = p->Np > p->Np2 ? p->Np : p->Np2;
  const int64_t cols = p->Kp2 > p->Kp ? p->Kp2 : p->Kp;
  dim3 grid((unsigned)(cols / 64), (unsigned)(rows / 64));
  if (p->prec == SOS_FP64) k_prep<0><<<grid, 256, 0, s>>>(a);
  else if (p->prec == SOS_FP32) k_prep<1><<<grid, 256, 0, s>>>(a);
  else if (p->prec == SOS_FP16X3) {
    // the scale of the 16-bit copies from max |W| first (the fused steps that
    // follow keep it)
    if (need.a || need.t) {
      float* pmax = (float*)((double*)(p->ws + p->lay.scal) + kScalMax);
      const int64_t n = p->N * (int64_t)p->k;
      k_absmax_partial<<<kSumBlocks, 256, 0, s>>>((const float*)W, n, pmax);
      k_absmax_final<<<1, 256, 0, s>>>(pmax, scale_exponents(p));
    }
    k_prep<3><<<grid, 256, 0, s>>>(a);
  } else k_prep<2><<<grid, 256, 0, s>>>(a);
  return hipGetLastError();
}

hipError_t launch_init_r(const sos_plan_s* p, const double* d_p, hipStream_t s) {
  k_init_r<<<grid_for(p->M), 256, 0, s>>>(d_p, (double*)(p->ws + p->lay.r), p->M);
  return hipGetLastError();
}

hipError_t launch_sumsq(const sos_plan_s* p, const double* x, int64_t M, double* out, hipStream_t s, float* x32) {
  double* sc = (double*)(p->ws + p->lay.scal);
  double* partial = sc + 8;
  // fp16 plans: the block maxima of |r| give the gather's scale when r32 is written
  float* pmax = (x32 && p->prec == SOS_FP16X3) ? (float*)(sc + kScalMax) : nullptr;
  k_sumsq_partial<<<kSumBlocks, 256, 0, s>>>(x, M, partial, x32, pmax);
  k_sumsq_final<<<1, 256, 0, s>>>(partial, out, pmax, scale_exponents(p) + 1);
  return hipGetLastError();
}

template <class Md>
static hipError_t gram_launch(const sos_plan_s* p, const void* a0, const void* a1, hipStream_t s,
                              double* Gd = nullptr) {
  GramArgs g;
  g.A[0] = a0; g.A[1] = a1;
  g.ld = p->Kp; g.K = p->Kp;
  g.N = (int)p->N;
  g.T = (int)(p->Np / BM);
  g.rk = rank_tab(p);
  g.r = (double*)(p->ws + p->lay.r);
  g.Gd = Gd;
  const int tiles = g.T * (g.T + 1) / 2;
  g.tiles = tiles;
  // split the contraction when there are too few tiles to fill the chip
  g.kslice = generic_gram_kslice(p->Np, p->Kp);
  const int64_t splits = generic_gram_splits(p->Np, p->Kp);
  const size_t sm = 2 * sizeof(Stage<Md>);
  // set on every launch (a host-side setting, cheap next to these kernels):
  // no shared flag between threads or devices
  hipError_t e = hipFuncSetAttribute((const void*)k_gram<Md>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm);
  if (e != hipSuccess) return e;
  k_gram<Md><<<(unsigned)(tiles * splits), kThreads, sm, s>>>(g);
  return hipGetLastError();
}

hipError_t launch_gram_det(const sos_plan_s* p, const double* d_p, hipStream_t s) {
  char* ws = p->ws;
  double* Gd = (double*)(ws + p->lay.det_G);
  hipError_t e = (p->prec == SOS_FP64) ? gram_launch<MF64>(p, ws + p->lay.a_hi, nullptr, s, Gd)
                                       : gram_launch<MF32>(p, ws + p->lay.a_hi, nullptr, s, Gd);
  if (e != hipSuccess) return e;
  k_coeff_det<<<(unsigned)((p->M + 255) / 256), 256, 0, s>>>(Gd, (int)generic_gram_splits(p->Np, p->Kp), (int)p->N,
                                                              (const int32_t*)(ws + p->lay.pair_off),
                                                              (const int32_t*)(ws + p->lay.pair_idx), d_p,
                                                              (double*)(ws + p->lay.r), (int)p->M);
  return hipGetLastError();
}

hipError_t launch_gram(const sos_plan_s* p, int mode, hipStream_t s, bool unmerged, int oz_slices) {
  const char* ws = p->ws;
  if (p->prec == SOS_FP64) return gram_launch<MF64>(p, ws + p->lay.a_hi, nullptr, s);
  // FP32 padded row-major copy of W: a_hi in FP32 plans, a_f32 in split plans
  const void* w32 = (p->prec == SOS_FP32) ? ws + p->lay.a_hi : ws + p->lay.a_f32;
  if (mode == kFwdExact) return launch_gram_x64(p, s);
  if (mode == kFwdOzaki) return launch_gram_i8(p, s, oz_slices);
  if (mode == kFwdSingle) return launch_gram_bf3(p, s, false, unmerged, true);
  if (mode == kFwdF32 || p->prec == SOS_FP32) return gram_launch<MF32>(p, w32, nullptr, s);
  return launch_gram_bf3(p, s, false, unmerged);
}

template <class Md>
static hipError_t rw_launch(const sos_plan_s* p, void* g, hipStream_t s) {
  RwArgs a;
  const char* ws = p->ws;
  a.A[0] = ws + p->lay.R_hi; a.A[1] = split_plan(p) ? ws + p->lay.R_lo : nullptr;
  a.B[0] = ws + p->lay.t_hi; a.B[1] = split_plan(p) ? ws + p->lay.t_lo : nullptr;
  a.K = p->Np2; a.N = (int)p->N; a.k = p->k;
  a.g = g; a.g_double = (p->prec == SOS_FP64);
  const size_t sm = 2 * sizeof(Stage<Md>);
  // set on every launch (a host-side setting, cheap next to these kernels):
  // no shared flag between threads or devices
  hipError_t e = hipFuncSetAttribute((const void*)k_rw<Md>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm);
  if (e != hipSuccess) return e;
  dim3 grid((unsigned)(p->Kp2 / BM), (unsigned)(p->Np / BM));
  k_rw<Md><<<grid, kThreads, sm, s>>>(a);
  return hipGetLastError();
}

hipError_t launch_gather(const sos_plan_s* p, bool split, hipStream_t s) {
  char* ws = p->ws;
  const RankTab rk = rank_tab(p);
  const int64_t total = p->Np * p->Np2;
  void* Rh = ws + p->lay.R_hi;
  const bool f16 = p->prec == SOS_FP16X3;
  void* Rl = split_plan(p) ? ws + p->lay.R_lo : nullptr;
  const int* sc = scale_exponents(p);
  if (p->prec == SOS_FP64) {
    const double* r = (const double*)(ws + p->lay.r);
    k_gather<0><<<grid_for(total), 256, 0, s>>>(rk, r, (int)p->N, p->Np, p->Np2, Rh, Rl);
    return hipGetLastError();
  }
  const float* r32 = (const float*)(ws + p->lay.r32);
  const int T2 = (int)(p->Np2 / 64);
  const int64_t nup = (int64_t)T2 * (T2 + 1) / 2;
  const int64_t blocks = nup + (p->Np - p->Np2) / 64 * T2;
  if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
  // the table is sized to the plan (1 KB for dense codes), so more blocks fit a CU
  const size_t tab = (size_t)rk.ntab * 4;
  if (rk.ntab > kStageTabMax) return hipErrorInvalidValue;
  if (p->prec == SOS_FP32)
    k_gather_sym<1><<<(unsigned)blocks, 256, tab, s>>>(rk, r32, (int)p->N, p->Np, p->Np2, T2, nup, Rh, Rl, sc);
  else if (f16 && split)
    k_gather_sym<4><<<(unsigned)blocks, 256, tab, s>>>(rk, r32, (int)p->N, p->Np, p->Np2, T2, nup, Rh, Rl, sc);
  else if (f16)
    k_gather_sym<5><<<(unsigned)blocks, 256, tab, s>>>(rk, r32, (int)p->N, p->Np, p->Np2, T2, nup, Rh, Rl, sc);
  else if (split)
    k_gather_sym<2><<<(unsigned)blocks, 256, tab, s>>>(rk, r32, (int)p->N, p->Np, p->Np2, T2, nup, Rh, Rl, sc);
  else
    k_gather_sym<3><<<(unsigned)blocks, 256, tab, s>>>(rk, r32, (int)p->N, p->Np, p->Np2, T2, nup, Rh, Rl, sc);
  return hipGetLastError();
}

hipError_t launch_rw(const sos_plan_s* p, void* g, bool split, hipStream_t s) {
  if (p->prec == SOS_FP64) return rw_launch<MF64>(p, g, s);
  if (p->prec == SOS_FP32) return rw_launch<MF32>(p, g, s);
  return launch_rw_bf3(p, g, split, s);
}

hipError_t launch_adam_f32(float* W, float* m, float* v, const float* g, int64_t n, int64_t t,
                           const sos_adam_t& h, hipStream_t s) {
  const double bc1 = 1.0 - pow(h.beta1, (double)t), bc2 = 1.0 - pow(h.beta2, (double)t);
  k_adam<float><<<grid_for(n), 256, 0, s>>>(W, m, v, g, n, (float)h.lr, (float)h.beta1, (float)h.beta2,
                                            (float)h.eps, (float)bc1, (float)bc2);
  return hipGetLastError();
}

hipError_t launch_adam(const sos_plan_s* p, void* W, void* m, void* v, const void* g, int64_t t,
                       const sos_adam_t& h, hipStream_t s) {
  const int64_t n = p->N * (int64_t)p->k;
  const double bc1 = 1.0 - pow(h.beta1, (double)t), bc2 = 1.0 - pow(h.beta2, (double)t);
  if (p->prec == SOS_FP64)
    k_adam<double><<<grid_for(n), 256, 0, s>>>((double*)W, (double*)m, (double*)v, (const double*)g, n,
                                               h.lr, h.beta1, h.beta2, h.eps, bc1, bc2);
  else
    k_adam<float><<<grid_for(n), 256, 0, s>>>((float*)W, (float*)m, (float*)v, (const float*)g, n,
                                              (float)h.lr, (float)h.beta1, (float)h.beta2, (float)h.eps,
                                              (float)bc1, (float)bc2);
  return hipGetLastError();
}

}  // namespace sos
