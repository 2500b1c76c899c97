// Exact forward: the Gram tiles of an FP32 W in FP64 on v_mfma_f64_16x16x4_f64.
//
// Products of two FP32 numbers are exact in FP64 and the accumulation is
// FP64, so the coefficients come out with FP64 rounding only -- the
// forward that can certify a relative residual far below the FP32 level.
//
// Operands stay FP32 in memory and in LDS (half the bytes of FP64) and are
// converted when a fragment is read.  Output tile 128 x 256 per 512-thread
// workgroup: the upper-triangle list of 256 x 256 tiles is walked in row
// halves (a diagonal tile's lower-left quarter is computed and discarded).
// 8 waves, 2 per SIMD, each 64 x 64 (4 x 4 blocks of 16 x 16).  K advances
// in stages of 16 through a 4-deep LDS ring filled by direct global->LDS
// loads from a panel-blocked FP32 copy of W (256 rows x 16 floats per
// contiguous 16 KB block).
//
// Inside a stage the K order is permuted: at k-step kk lane l uses
// k = 4 (l / 16) + kk instead of 4 kk + l / 16.  Both operands use the same
// permutation, so each dot product is unchanged, and one 16-byte LDS read
// per fragment feeds all four k-steps of the stage.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "sos_internal.h"

namespace sos {
namespace x64 {

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) void* lds_t;

constexpr int TA = 128;             // A rows per tile (half a 256-row panel)
constexpr int TB = 256;             // B rows per tile (one panel)
constexpr int BK = 16;              // K per stage
constexpr int NT = 512;
constexpr int NSTAGE = 4;
constexpr int ROWB = BK * 4;        // 64 bytes per row (FP32)
constexpr int ABYTES = TA * ROWB;   // 8 KB
constexpr int BBYTES = TB * ROWB;   // 16 KB
constexpr int STAGE = ABYTES + BBYTES;
constexpr int PANEL = 256;
constexpr int kXcds = 8;

__device__ __forceinline__ int xcd_order(int b, int nb) {
  const int q = nb / kXcds, rem = nb % kXcds;
  const int xcd = b % kXcds, local = b / kXcds;
  return (xcd < rem) ? xcd * (q + 1) + local : rem * (q + 1) + (xcd - rem) * q + local;
}

// Direct global->LDS load of 16 bytes per lane; see gemm_bf3.hip for why it
// is asm and which hazards it covers (VGPR address, s_nop after m0).
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

// Per stage: A is 128 rows (8 KB, 8 instructions of 1 KB), B 256 rows
// (16 KB, 16 instructions); 24 instructions over 8 waves = 3 per wave.
constexpr int LOADS = 3;

// Global byte address of row r (within the tile's operand) at stage ks.
__device__ __forceinline__ const char* row_addr(const float* w, int64_t pstride, int64_t row0, int r, int64_t ks) {
  const int64_t row = row0 + r;
  return (const char*)(w + (row / PANEL) * pstride + (ks * PANEL + row % PANEL) * BK);
}

// st_lds: wave-uniform LDS address of the stage buffer (scalar register).
__device__ __forceinline__ void issue_stage(unsigned st_lds, const float* w, int64_t pstride, int64_t arow0,
                                            int64_t brow0, int64_t ks) {
  const int wave = threadIdx.x >> 6, l = threadIdx.x & 63;
  const unsigned wave_u = __builtin_amdgcn_readfirstlane((unsigned)wave);
#pragma unroll
  for (int q = 0; q < LOADS; ++q) {
    const int ins = wave * LOADS + q;  // 0..23: 0..7 A, 8..23 B; 16 rows of 64 B each
    const unsigned ins_u = wave_u * LOADS + q;
    const int r = (ins < 8 ? ins : ins - 8) * 16 + (l >> 2);
    // LDS slot l & 3 of row r holds chunk (l & 3) ^ ((r >> 2) & 3): 16 consecutive
    // rows read at one chunk then fall in 16 distinct 16-byte bank groups
    const int chunk = (l & 3) ^ ((r >> 2) & 3);
    const char* g = (ins < 8) ? row_addr(w, pstride, arow0, r, ks) : row_addr(w, pstride, brow0, r, ks);
    const unsigned m0 = st_lds + (ins_u < 8 ? 0u : (unsigned)ABYTES) + (ins_u < 8 ? ins_u : ins_u - 8) * 1024u;
    dma16(g + chunk * 16, m0);
  }
}

struct Frag {
  float4 a[4], b[4];  // per 16-row block: k = 4 (l / 16) .. +3 of the stage
};

__device__ __forceinline__ void load_frag(Frag& f, const char* st, int wm, int wn) {
  const int l = threadIdx.x & 63;
  const int off = (l & 15) * ROWB + (((l >> 4) ^ ((l >> 2) & 3)) << 4);  // chunk l / 16, swizzled
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    f.a[q] = *(const float4*)(st + (wm * 64 + q * 16) * ROWB + off);
    f.b[q] = *(const float4*)(st + ABYTES + (wn * 64 + q * 16) * ROWB + off);
  }
}

__device__ __forceinline__ double comp(const float4& v, int kk) {
  return (double)(kk == 0 ? v.x : kk == 1 ? v.y : kk == 2 ? v.z : v.w);
}

__device__ __forceinline__ void mma_stage(const Frag& f, f64x4 (&acc)[4][4]) {
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) {
    double a[4], b[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      a[q] = comp(f.a[q], kk);
      b[q] = comp(f.b[q], kk);
    }
#pragma unroll
    for (int bi = 0; bi < 4; ++bi)
#pragma unroll
      for (int bj = 0; bj < 4; ++bj)
        acc[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[bi], b[bj], acc[bi][bj], 0, 0, 0);
  }
}


struct Args {
  const float* w;     // panel-blocked FP32 W: rows Np, K extent Kp
  int64_t nkb;        // Kp / 16: stages
  int64_t pstride;    // elements per padded panel (see blk_off)
  const int2* tiles;  // 256 x 256 upper-triangle tile list
  int ntiles, N;
  RankTab rk;
  double* r;
};

__global__ __launch_bounds__(NT) void k_gram_x64(Args g) {
  __shared__ __attribute__((aligned(16))) char ring[NSTAGE * STAGE];
  const int v = xcd_order(blockIdx.x, 2 * g.ntiles);
  const int2 t = g.tiles[v >> 1];
  const int half = v & 1;
  const int64_t arow0 = (int64_t)t.x * PANEL + half * TA, brow0 = (int64_t)t.y * PANEL;
  const int wave = threadIdx.x >> 6;
  const int wm = wave >> 2, wn = wave & 3;  // 2 x 4 waves of 64 x 64
  f64x4 acc[4][4];
#pragma unroll
  for (int bi = 0; bi < 4; ++bi)
#pragma unroll
    for (int bj = 0; bj < 4; ++bj) acc[bi][bj] = f64x4{};
  const int64_t nk = g.nkb;
  const unsigned ring_lds = __builtin_amdgcn_readfirstlane((unsigned)(uintptr_t)(lds_t)ring);
  for (int s = 0; s < NSTAGE - 1; ++s)
    if (s < nk) issue_stage(ring_lds + s * STAGE, g.w, g.pstride, arow0, brow0, s);
  for (int64_t kt = 0; kt < nk; ++kt) {
    const int64_t ahead = nk - 1 - kt;  // stages after kt that have been issued (at most 2)
    if (ahead >= 2) wait_vm_barrier<2 * LOADS>();
    else if (ahead == 1) wait_vm_barrier<LOADS>();
    else wait_vm_barrier<0>();
    // all waves are past their reads of stage kt-1: refill its buffer
    if (kt + NSTAGE - 1 < nk)
      issue_stage(ring_lds + (unsigned)((kt + NSTAGE - 1) % NSTAGE) * STAGE, g.w, g.pstride, arow0, brow0,
                  kt + NSTAGE - 1);
    Frag f;
    load_frag(f, ring + (kt % NSTAGE) * STAGE, wm, wn);
    mma_stage(f, acc);
  }
  // scatter: lane l, register q of 16 x 16 block (bi, bj) holds row l / 16 + 4 q, column l % 16
  const int l = threadIdx.x & 63;
#pragma unroll
  for (int bi = 0; bi < 4; ++bi)
#pragma unroll
    for (int bj = 0; bj < 4; ++bj) {
      const int j = (int)brow0 + wn * 64 + bj * 16 + (l & 15);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = (int)arow0 + wm * 64 + bi * 16 + (l >> 4) + 4 * q;
        if (i < g.N && j < g.N && i <= j) {
          const double wgt = (i == j) ? 1.0 : 2.0;
          unsafeAtomicAdd(g.r + pair_rank(g.rk, i, j), wgt * acc[bi][bj][q]);
        }
      }
    }
}

}  // namespace x64

hipError_t launch_gram_x64(const sos_plan_s* p, hipStream_t s) {
  x64::Args g;
  const char* ws = p->ws;
  g.w = (const float*)(ws + p->lay.x_f32);
  g.nkb = p->Kp / kBlkK;
  g.pstride = panel_stride(g.nkb, 4);
  g.tiles = (const int2*)(ws + p->lay.tiles);
  g.ntiles = p->ntiles256;
  g.N = (int)p->N;
  g.rk = rank_tab(p);
  g.r = (double*)(ws + p->lay.r);
  x64::k_gram_x64<<<2 * g.ntiles, x64::NT, 0, s>>>(g);
  return hipGetLastError();
}

}  // namespace sos
