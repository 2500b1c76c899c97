// Ozaki-split forward: an FP64-accurate Gram of the FP32 W from int8 MFMA.
//
// Splitting (Ozaki, Ogita, Oishi and Rump, 2012): row i of W is scaled by
// 2^-e_i, e_i the least power of two above its largest magnitude, and cut
// into S signed digits, x = 2^-6 (d_0 + 2^-7 d_1 + ... + 2^-7(S-1) d_{S-1})
// + remainder, every |d_s| <= 64 (each digit is the rounded value of the
// remainder so far, so the cut is exact in FP32 arithmetic).  A product of
// two rows is then a sum of slice products D_s D_t^T, each an exact int32
// sum over K.  The products of one level l = s + t share the weight
// 2^-7l, so they are summed in one int32 accumulator (at most S products,
// exact while S * K * 64^2 < 2^31); levels l < S are kept, the rest dropped.
// After each level the accumulator is added into an FP64 accumulator with
// its weight (exact: a 31-bit integer times a power of two), and the tile
// scatters G_ij = 2^(e_i - 6) 2^(e_j - 6) sum_l 2^-7l T_l,ij into r in FP64.
//
// Error: per product, the digits left out and the levels dropped amount to
// at most (S + 1.05) 2^-7S of 2^(e_i + e_j), so |G_ij - G~_ij| <=
// (S + 1.05) 2^-7S K 2^(e_i + e_j), plus FP64 rounding (about 1e-12 of the
// Gram entry at S = 6 and Gaussian rows; the errors of individual digits are
// independent, so the actual error is far below this bound).
//
// Kernel shape follows the FP64 gram (gemm_x64.hip): 128 x 256 half tiles of
// the 256 x 256 upper-triangle tiles per 512-thread workgroup, 8 waves of
// 64 x 64 (2 x 2 blocks of v_mfma_i32_32x32x32_i8), a 4-deep LDS ring of
// stages filled by direct global->LDS loads.  A stage is one block of 64 K
// of one slice pair: 128 A rows and 256 B rows of 64 bytes (24 KB).  The K
// loop runs over S(S+1)/2 segments, one per slice pair in level order, each
// the whole K extent.  Registers per lane: 64 int32 level sums and 64 FP64
// level totals (two waves per SIMD).
#include <hip/hip_runtime.h>

#include <cfloat>
#include <cmath>
#include <cstdint>

#include "sos_internal.h"

namespace sos {
namespace i8 {

typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef int i32x16 __attribute__((ext_vector_type(16)));
typedef __attribute__((address_space(3))) void* lds_t;

constexpr int S = kOzSlices;
constexpr int TA = 128;             // A rows per tile (half a 256-row panel)
constexpr int TB = 256;             // B rows per tile (one panel)
constexpr int BK = kOzBK;           // K (bytes) per stage
constexpr int NT = 512;
constexpr int NSTAGE = 4;
constexpr int ROWB = BK;            // 64 bytes per row
constexpr int ABYTES = TA * ROWB;   // 8 KB
constexpr int BBYTES = TB * ROWB;   // 16 KB
constexpr int STAGE = ABYTES + BBYTES;
constexpr int PANEL = 256;
constexpr int kXcds = 8;
constexpr int LOADS = 3;            // 24 KB per stage = 24 loads of 1 KB over 8 waves

__device__ __forceinline__ int xcd_order(int b, int nb) {
  const int q = nb / kXcds, rem = nb % kXcds;
  const int xcd = b % kXcds, local = b / kXcds;
  return (xcd < rem) ? xcd * (q + 1) + local : rem * (q + 1) + (xcd - rem) * q + local;
}

// Direct global->LDS load of 16 bytes per lane; the 64-bit VGPR address and
// the s_nop after the m0 write cover the hazards the compiler cannot see
// inside the asm (see gemm_bf3.hip).
__device__ __forceinline__ void dma16(const char* gaddr, unsigned m0) {
  asm volatile("s_mov_b32 m0, %0\n\ts_nop 1\n\tglobal_load_lds_dwordx4 %1, off"
               :
               : "s"(m0), "v"(gaddr)
               : "memory", "m0");
}

template <int n>
__device__ __forceinline__ void wait_vm_barrier() {
  __builtin_amdgcn_s_waitcnt((n & 0xF) | ((n >> 4) << 14) | (7 << 4) | (0xF << 8));
  __builtin_amdgcn_s_waitcnt((0x3F & 0xF) | ((0x3F >> 4) << 14) | (7 << 4) | (0 << 8));  // lgkmcnt(0)
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

// Position in the segment sequence: segment (s, t) of level s + t, block kb.
// Segments run level by level, s ascending inside a level.
struct Cursor {
  int s = 0, t = 0, lvl = 0;
  int64_t kb = 0;
  __device__ __forceinline__ bool level_ends(int64_t nkb) const { return t == 0 && kb == nkb - 1; }
  __device__ __forceinline__ void advance(int64_t nkb) {
    if (++kb < nkb) return;
    kb = 0;
    if (t > 0) {
      ++s;
      --t;
    } else {
      ++lvl;
      s = 0;
      t = lvl;
    }
  }
};

// Global address of row r (within the tile's operand) of K block kb.
__device__ __forceinline__ const char* row_addr(const int8_t* slice, int64_t pstride, int64_t row0, int r,
                                                int64_t kb) {
  const int64_t row = row0 + r;
  return (const char*)(slice + (row / PANEL) * pstride + (kb * PANEL + row % PANEL) * BK);
}

// LDS slot (l & 3) of row r holds 16-byte chunk (l & 3) ^ ((r >> 2) & 3), so
// 16 consecutive rows read at one chunk fall in 16 distinct bank groups.
__device__ __forceinline__ void issue_stage(unsigned st_lds, const int8_t* a_slice, const int8_t* b_slice,
                                            int64_t pstride, int64_t arow0, int64_t brow0, int64_t kb) {
  const int wave = threadIdx.x >> 6, l = threadIdx.x & 63;
  const unsigned wave_u = __builtin_amdgcn_readfirstlane((unsigned)wave);
#pragma unroll
  for (int q = 0; q < LOADS; ++q) {
    const int ins = wave * LOADS + q;  // 0..7: A rows, 8..23: B rows; 16 rows of 64 B each
    const unsigned ins_u = wave_u * LOADS + q;
    const int r = (ins < 8 ? ins : ins - 8) * 16 + (l >> 2);
    const int chunk = (l & 3) ^ ((r >> 2) & 3);
    const char* g = (ins < 8) ? row_addr(a_slice, pstride, arow0, r, kb) : row_addr(b_slice, pstride, brow0, r, kb);
    const unsigned m0 = st_lds + (ins_u < 8 ? 0u : (unsigned)ABYTES) + (ins_u < 8 ? ins_u : ins_u - 8) * 1024u;
    dma16(g + chunk * 16, m0);
  }
}

// One stage: two k-steps of 32, each four MFMAs (2 x 2 blocks of 32 x 32).
// Lane l supplies row l % 32 of a block and bytes 16 (l / 32) .. +15 of the
// k-step, for both operands alike.
__device__ __forceinline__ void mma_stage(const char* st, int wm, int wn, i32x16 (&acc)[2][2]) {
  const int l = threadIdx.x & 63;
#pragma unroll
  for (int ks = 0; ks < 2; ++ks) {
    const int off = (l & 31) * ROWB + (((2 * ks + (l >> 5)) ^ ((l >> 2) & 3)) << 4);
    i32x4 a[2], b[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      a[q] = *(const i32x4*)(st + (wm * 64 + q * 32) * ROWB + off);
      b[q] = *(const i32x4*)(st + ABYTES + (wn * 64 + q * 32) * ROWB + off);
    }
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int bj = 0; bj < 2; ++bj)
        acc[bi][bj] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[bi], b[bj], acc[bi][bj], 0, 0, 0);
  }
}

struct Args {
  const int8_t* oz;       // slice s at oz + s * slice_bytes
  int64_t slice_bytes;
  int64_t nkb;            // Kp / 64
  int64_t pstride;        // bytes per padded panel
  const int2* tiles;      // 256 x 256 upper-triangle tile list
  int ntiles, N;
  const double* scale;    // 2^(e_i - 6) per row (NaN: the row holds a non-finite entry)
  RankTab rk;
  double* r;
};

__global__ __launch_bounds__(NT) void k_gram_i8(Args g) {
  __shared__ __attribute__((aligned(16))) char ring[NSTAGE * STAGE];
  const int v = xcd_order(blockIdx.x, 2 * g.ntiles);
  const int2 t = g.tiles[v >> 1];
  const int half = v & 1;
  const int64_t arow0 = (int64_t)t.x * PANEL + half * TA, brow0 = (int64_t)t.y * PANEL;
  const int wave = threadIdx.x >> 6;
  const int wm = wave >> 2, wn = wave & 3;  // 2 x 4 waves of 64 x 64
  i32x16 acc[2][2];
  double tot[2][2][16];
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) {
      acc[bi][bj] = i32x16{};
#pragma unroll
      for (int q = 0; q < 16; ++q) tot[bi][bj][q] = 0.0;
    }
  const int64_t nkb = g.nkb;
  const int64_t nv = (int64_t)(S * (S + 1) / 2) * nkb;  // stages over all segments
  const unsigned ring_lds = __builtin_amdgcn_readfirstlane((unsigned)(uintptr_t)(lds_t)ring);
  Cursor in, cu;  // next stage to issue, stage to compute
  for (int s = 0; s < NSTAGE - 1; ++s) {
    if (s < nv) {
      issue_stage(ring_lds + s * STAGE, g.oz + in.s * g.slice_bytes, g.oz + in.t * g.slice_bytes, g.pstride, arow0,
                  brow0, in.kb);
      in.advance(nkb);
    }
  }
  double weight = 1.0;  // 2^-7 lvl of the level being summed
  for (int64_t vt = 0; vt < nv; ++vt) {
    const int64_t ahead = nv - 1 - vt;  // stages after vt that have been issued (at most 2)
    if (ahead >= 2) wait_vm_barrier<2 * LOADS>();
    else if (ahead == 1) wait_vm_barrier<LOADS>();
    else wait_vm_barrier<0>();
    // every wave is past its reads of stage vt-1: refill that buffer
    if (vt + NSTAGE - 1 < nv) {
      issue_stage(ring_lds + (unsigned)((vt + NSTAGE - 1) % NSTAGE) * STAGE, g.oz + in.s * g.slice_bytes,
                  g.oz + in.t * g.slice_bytes, g.pstride, arow0, brow0, in.kb);
      in.advance(nkb);
    }
    mma_stage(ring + (vt % NSTAGE) * STAGE, wm, wn, acc);
    if (cu.level_ends(nkb)) {
#pragma unroll
      for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) {
#pragma unroll
          for (int q = 0; q < 16; ++q) tot[bi][bj][q] = fma((double)acc[bi][bj][q], weight, tot[bi][bj][q]);
          acc[bi][bj] = i32x16{};
        }
      weight *= 0x1p-7;
    }
    cu.advance(nkb);
  }
  // scatter: lane l, register q of 32 x 32 block (bi, bj) holds row
  // 8 (q / 4) + 4 (l / 32) + q % 4 and column l % 32 of the block
  const int l = threadIdx.x & 63;
#pragma unroll
  for (int bj = 0; bj < 2; ++bj) {
    const int j = (int)brow0 + wn * 64 + bj * 32 + (l & 31);
    const double sj = j < g.N ? g.scale[j] : 0.0;
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int i = (int)arow0 + wm * 64 + bi * 32 + (q >> 2) * 8 + (l >> 5) * 4 + (q & 3);
        if (i < g.N && j < g.N && i <= j) {
          const double wgt = (i == j) ? 1.0 : 2.0;
          unsafeAtomicAdd(g.r + pair_rank(g.rk, i, j), wgt * (tot[bi][bj][q] * g.scale[i] * sj));
        }
      }
  }
}

// Row exponents: e_i with max_l |W_il| < 2^e_i (0 for a zero row), and the
// scale 2^(e_i - 6) that the gram's epilogue applies (NaN when the row holds
// a NaN or an infinity, so that the coefficients it touches are NaN).
__global__ __launch_bounds__(256) void k_oz_scale(const float* __restrict__ W, int N, int k, int* __restrict__ ex,
                                                  double* __restrict__ scale) {
  __shared__ float smax[4];
  __shared__ int sbad[4];
  const int i = blockIdx.x;
  const float* row = W + (int64_t)i * k;
  float m = 0.f;
  int bad = 0;
  for (int l = threadIdx.x; l < k; l += 256) {
    const float a = fabsf(row[l]);
    bad |= !(a <= FLT_MAX);
    m = fmaxf(m, a);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    m = fmaxf(m, __shfl_xor(m, o));
    bad |= __shfl_xor(bad, o);
  }
  if ((threadIdx.x & 63) == 0) {
    smax[threadIdx.x >> 6] = m;
    sbad[threadIdx.x >> 6] = bad;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    m = fmaxf(fmaxf(smax[0], smax[1]), fmaxf(smax[2], smax[3]));
    bad = sbad[0] | sbad[1] | sbad[2] | sbad[3];
    int e = 0;
    if (m > 0.f && !bad) (void)frexpf(m, &e);  // m = f 2^e, 0.5 <= f < 1
    ex[i] = e;
    scale[i] = bad ? __builtin_nan("") : ldexp(1.0, e - 6);
  }
}

// Digits of a 64 x 64 tile of W into the S slice arrays (padding rows and
// columns get zero digits).  Loads are coalesced along rows; the digits go
// through LDS so that every slice is written in 16-byte chunks of the
// blocked layout.
__global__ __launch_bounds__(256) void k_oz_slice(const float* __restrict__ W, int N, int k,
                                                  const int* __restrict__ ex, int8_t* __restrict__ oz,
                                                  int64_t slice_bytes, int64_t pstride) {
  __shared__ __attribute__((aligned(16))) int8_t dig[S][64][64];
  const int64_t row0 = (int64_t)blockIdx.y * 64, col0 = (int64_t)blockIdx.x * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int rr = ty; rr < 64; rr += 4) {
    const int64_t i = row0 + rr, l = col0 + tx;
    float x = 0.f;
    if (i < N && l < k) x = ldexpf(W[i * k + l], 6 - ex[i]);  // |x| < 64
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const float d = rintf(x);  // |d| <= 64
      dig[s][rr][tx] = (int8_t)(int)d;
      x = (x - d) * 128.0f;      // exact: the remainder keeps the low bits of x
    }
  }
  __syncthreads();
  const int rr = threadIdx.x >> 2, c = threadIdx.x & 3;
  const int64_t o = oz_off(row0 + rr, col0 + 16 * c, pstride);
#pragma unroll
  for (int s = 0; s < S; ++s)
    *(i32x4*)(oz + s * slice_bytes + o) = *(const i32x4*)&dig[s][rr][16 * c];
}

}  // namespace i8

hipError_t launch_oz_slices(const sos_plan_s* p, const float* W, hipStream_t s) {
  char* ws = p->ws;
  int* ex = (int*)(ws + p->lay.oz_exp);
  i8::k_oz_scale<<<(unsigned)p->N, 256, 0, s>>>(W, (int)p->N, p->k, ex, (double*)(ws + p->lay.oz_scale));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const dim3 grid((unsigned)(p->Kp / 64), (unsigned)(p->Np / 64));
  i8::k_oz_slice<<<grid, 256, 0, s>>>(W, (int)p->N, p->k, ex, (int8_t*)(ws + p->lay.oz), (int64_t)p->lay.oz_slice,
                                      oz_panel_stride(p->Kp));
  return hipGetLastError();
}

hipError_t launch_gram_i8(const sos_plan_s* p, hipStream_t s) {
  i8::Args g;
  const char* ws = p->ws;
  g.oz = (const int8_t*)(ws + p->lay.oz);
  g.slice_bytes = (int64_t)p->lay.oz_slice;
  g.nkb = p->Kp / kOzBK;
  g.pstride = oz_panel_stride(p->Kp);
  g.tiles = (const int2*)(ws + p->lay.tiles);
  g.ntiles = p->ntiles256;
  g.N = (int)p->N;
  g.scale = (const double*)(ws + p->lay.oz_scale);
  g.rk = rank_tab(p);
  g.r = (double*)(ws + p->lay.r);
  i8::k_gram_i8<<<2 * g.ntiles, i8::NT, 0, s>>>(g);
  return hipGetLastError();
}

}  // namespace sos
