// Split-bf16 ("bf16x3") contractions on gfx950 MFMA, 256 x 256 output tiles.
//
// Every operand w is held as two bf16 arrays, hi = bf16(w) and
// lo = bf16(w - hi); a product w w' is taken as lo*hi' + hi*lo' + hi*hi' on
// v_mfma_f32_32x32x16_bf16 with FP32 accumulation (lo*lo' is dropped).
//
// Tile: 256 x 256 outputs per 512-thread workgroup; 8 waves in a 4 x 2 grid,
// each wave 64 x 128 (2 x 4 MFMA blocks of 32 x 32).  K advances in stages
// of 16 through a 4-deep ring of LDS stages (4 arrays x 256 rows x 32 B =
// 32 KB each) filled by direct global->LDS loads issued three stages ahead,
// so an L2 miss has about three stages of MFMA work to hide behind.
//
// Tile order is XCD-aware: workgroups are dispatched round-robin over the 8
// XCDs (each with its own L2), so consecutive workgroups of one XCD are
// given tiles that share operand panels.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "sos_internal.h"

namespace sos {
namespace bf3 {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int TM = 256;
constexpr int BK = 16;            // K per pipeline stage (one MFMA k-step)
constexpr int NT = 512;
constexpr int NSTAGE = 4;         // LDS stages; loads run NSTAGE - 1 stages ahead
constexpr int ROWB = BK * 2;      // bytes per row per array (32)
constexpr int ARR = TM * ROWB;    // bytes per array tile (8 KB)
constexpr int STAGE = 4 * ARR;    // A_hi, A_lo, B_hi, B_lo (32 KB)
constexpr int kXcds = 8;

typedef __attribute__((address_space(3))) void* lds_t;

// Row r of an array tile holds two 16-byte chunks; chunk c sits in slot
// c ^ ((r >> 3) & 1), so 16 consecutive rows read at one chunk cover 16
// distinct 16-byte bank groups.
__device__ __forceinline__ int slot_off(int row, int chunk) {
  return row * ROWB + ((chunk ^ ((row >> 3) & 1)) << 4);
}

struct Operands {
  const __bf16* a_hi;
  const __bf16* a_lo;
  const __bf16* b_hi;
  const __bf16* b_lo;
  int64_t ld;  // shared leading dimension (= K extent, padded)
};

// Wait until at most n of this wave's vector-memory operations are pending
// (only vmcnt is constrained), then barrier.  The empty asm keeps the
// compiler from moving LDS accesses across; no __syncthreads here, whose
// fence would also wait for the prefetches still in flight.
template <int n>
__device__ __forceinline__ void wait_vm_barrier() {
  __builtin_amdgcn_s_waitcnt((n & 0xF) | ((n >> 4) << 14) | (7 << 4) | (0xF << 8));
  __builtin_amdgcn_s_waitcnt((0x3F & 0xF) | ((0x3F >> 4) << 14) | (7 << 4) | (0 << 8));  // lgkmcnt(0)
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

// One 16-byte direct global->LDS load per lane (global_load_lds_dwordx4):
// lane l writes lds_base + 16 l, lds_base being uniform across the wave.
// Issued through asm so that the compiler's wait-count bookkeeping, which
// cannot tell the pipeline's LDS buffers apart across the loop back-edge,
// does not drain the whole pipeline before each stage; the waits for these
// loads are explicit (wait_vm_barrier).  The asm has no outputs: the data
// goes to LDS, and the address registers are read when it issues.
__device__ __forceinline__ void dma16(const void* gaddr, char* lds_base) {
  const unsigned off = (unsigned)(uintptr_t)(lds_t)lds_base;
  asm volatile("s_mov_b32 m0, %0\n\tglobal_load_lds_dwordx4 %1, off"
               :
               : "s"(__builtin_amdgcn_readfirstlane(off)), "v"(gaddr)
               : "memory", "m0");
}

// Issue the direct-to-LDS loads of one stage: wave w moves rows
// [32w, 32w + 32) of each of the four arrays, lane l one 16-byte chunk.
__device__ __forceinline__ void issue_stage(char* st, const Operands& o, int64_t arow0, int64_t brow0, int64_t k0) {
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int r = w * 32 + (l >> 1);
  const int c = (l & 1) ^ ((r >> 3) & 1);
  const int64_t ea = (arow0 + r) * o.ld + k0 + c * 8;
  const int64_t eb = (brow0 + r) * o.ld + k0 + c * 8;
  char* base = st + w * 1024;
  dma16(o.a_hi + ea, base + 0 * ARR);
  dma16(o.a_lo + ea, base + 1 * ARR);
  dma16(o.b_hi + eb, base + 2 * ARR);
  dma16(o.b_lo + eb, base + 3 * ARR);
}

__device__ __forceinline__ void mma_stage(const char* st, f32x16 (&acc)[2][4], int wm, int wn) {
  const int l = threadIdx.x & 63;
  const int c = l >> 5;
  bf16x8 ah[2], al[2], bh[4], bl[4];
#pragma unroll
  for (int bi = 0; bi < 2; ++bi) {
    const int off = slot_off(wm * 64 + bi * 32 + (l & 31), c);
    ah[bi] = *(const bf16x8*)(st + 0 * ARR + off);
    al[bi] = *(const bf16x8*)(st + 1 * ARR + off);
  }
#pragma unroll
  for (int bj = 0; bj < 4; ++bj) {
    const int off = slot_off(wn * 128 + bj * 32 + (l & 31), c);
    bh[bj] = *(const bf16x8*)(st + 2 * ARR + off);
    bl[bj] = *(const bf16x8*)(st + 3 * ARR + off);
  }
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 4; ++bj) {
      acc[bi][bj] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[bi], bh[bj], acc[bi][bj], 0, 0, 0);
      acc[bi][bj] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[bi], bl[bj], acc[bi][bj], 0, 0, 0);
      acc[bi][bj] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[bi], bh[bj], acc[bi][bj], 0, 0, 0);
    }
}

// Pipeline slot of stage kt: its own LDS buffer is bufs[B] (B = kt % 4),
// and it refills bufs[(B + 3) % 4], last read by stage kt - 1.  Distinct
// __shared__ arrays per buffer (and B known at compile time) let the
// compiler see that these loads never alias the reads of this stage.
// One pipeline step on stage kt: wait for its buffer (rd), refill the buffer
// of stage kt - 1 (wr) with stage kt + 3, then run the MFMAs on rd.  rd and
// wr are restrict-qualified so that, once inlined, the compiler knows the
// refill cannot alias this step's LDS reads and does not wait for it.
__device__ __forceinline__ void pipe_step(const char* __restrict__ rd, char* __restrict__ wr, const Operands& o,
                                          int64_t kt, int64_t nk, int64_t arow0, int64_t brow0,
                                          f32x16 (&acc)[2][4], int wm, int wn) {
  const int64_t ahead = nk - 1 - kt;
  if (ahead >= 2) wait_vm_barrier<8>();
  else if (ahead == 1) wait_vm_barrier<4>();
  else wait_vm_barrier<0>();
  if (kt + NSTAGE - 1 < nk) issue_stage(wr, o, arow0, brow0, (kt + NSTAGE - 1) * BK);
  mma_stage(rd, acc, wm, wn);
}

// C(256 x 256) = A[arow0 .. +256) x B[brow0 .. +256)^T over K (K % BK == 0).
__device__ __forceinline__ void tile_gemm(const Operands& o, int64_t K, int64_t arow0, int64_t brow0,
                                          char* const (&bufs)[NSTAGE], f32x16 (&acc)[2][4]) {
  const int wave = threadIdx.x >> 6;
  const int wm = wave >> 1, wn = wave & 1;
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 4; ++bj) acc[bi][bj] = f32x16{};
  const int64_t nk = K / BK;
  if (0 < nk) issue_stage(bufs[0], o, arow0, brow0, 0);
  if (1 < nk) issue_stage(bufs[1], o, arow0, brow0, BK);
  if (2 < nk) issue_stage(bufs[2], o, arow0, brow0, 2 * BK);
  for (int64_t kt = 0; kt < nk; kt += NSTAGE) {
    pipe_step(bufs[0], bufs[3], o, kt, nk, arow0, brow0, acc, wm, wn);
    if (kt + 1 < nk) pipe_step(bufs[1], bufs[0], o, kt + 1, nk, arow0, brow0, acc, wm, wn);
    if (kt + 2 < nk) pipe_step(bufs[2], bufs[1], o, kt + 2, nk, arow0, brow0, acc, wm, wn);
    if (kt + 3 < nk) pipe_step(bufs[3], bufs[2], o, kt + 3, nk, arow0, brow0, acc, wm, wn);
  }
}

// (row, col) of accumulator (bi, bj, q) inside the 256 x 256 tile.
__device__ __forceinline__ int acc_row(int wm, int bi, int q) {
  const int l = threadIdx.x & 63;
  return wm * 64 + bi * 32 + (q >> 2) * 8 + (l >> 5) * 4 + (q & 3);
}
__device__ __forceinline__ int acc_col(int wn, int bj) {
  return wn * 128 + bj * 32 + (threadIdx.x & 31);
}

// Block id -> position in a per-XCD-contiguous order (bijective on [0, nb)).
__device__ __forceinline__ int xcd_order(int b, int nb) {
  const int q = nb / kXcds, rem = nb % kXcds;
  const int xcd = b % kXcds, local = b / kXcds;
  return (xcd < rem) ? xcd * (q + 1) + local : rem * (q + 1) + (xcd - rem) * q + local;
}

struct RankTab {
  const uint32_t* __restrict__ codes;
  const int32_t* __restrict__ tables;
  int nwords, ngroups;
};

__device__ __forceinline__ int rank_sum(const RankTab& c, int i, int j) {
  int r = 0;
#pragma unroll
  for (int w = 0; w < kMaxWords; ++w) {
    if (w < c.nwords) {
      const uint32_t s = c.codes[(size_t)i * c.nwords + w] + c.codes[(size_t)j * c.nwords + w];
      r += c.tables[(2 * w) * kGroupEntries + (s & 0xFFFu)];
      if (2 * w + 1 < c.ngroups) r += c.tables[(2 * w + 1) * kGroupEntries + ((s >> 16) & 0xFFFu)];
    }
  }
  return r;
}

struct GramArgs {
  Operands o;
  int64_t K;
  const int2* tiles;  // (I, J) tile pairs, I <= J, in locality order
  int ntiles, N;
  RankTab rk;
  double* r;
};

#define SOS_BF3_BUFFERS                                         \
  __shared__ __attribute__((aligned(16))) char lds0[STAGE];    \
  __shared__ __attribute__((aligned(16))) char lds1[STAGE];    \
  __shared__ __attribute__((aligned(16))) char lds2[STAGE];    \
  __shared__ __attribute__((aligned(16))) char lds3[STAGE];    \
  char* const bufs[NSTAGE] = {lds0, lds1, lds2, lds3}

__global__ __launch_bounds__(NT) void k_gram_bf3(GramArgs g) {
  SOS_BF3_BUFFERS;
  const int v = xcd_order(blockIdx.x, g.ntiles);
  const int2 t = g.tiles[v];
  f32x16 acc[2][4];
  tile_gemm(g.o, g.K, (int64_t)t.x * TM, (int64_t)t.y * TM, bufs, acc);
  const int wave = threadIdx.x >> 6;
  const int wm = wave >> 1, wn = wave & 1;
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 4; ++bj) {
      const int j = t.y * TM + acc_col(wn, bj);
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int i = t.x * TM + acc_row(wm, bi, q);
        if (i < g.N && j < g.N && i <= j) {
          const double w = (i == j) ? 1.0 : 2.0;
          unsafeAtomicAdd(g.r + rank_sum(g.rk, i, j), w * (double)acc[bi][bj][q]);
        }
      }
    }
}

struct RwArgs {
  Operands o;  // A = R (rows Np), B = W^T copies (rows Kp2); ld = Np2
  int64_t K;
  int TI, TL, N, k;
  float* g;    // N x k
};

__global__ __launch_bounds__(NT) void k_rw_bf3(RwArgs a) {
  SOS_BF3_BUFFERS;
  const int nb = a.TI * a.TL;
  const int v = xcd_order(blockIdx.x, nb);
  // grouped order: 8 tile-rows at a time, column-major inside the group
  constexpr int GROUP = 8;
  const int per_group = GROUP * a.TL;
  const int gidx = v / per_group, first = gidx * GROUP;
  const int rows = min(GROUP, a.TI - first);
  const int in = v % per_group;
  const int I = first + in % rows, L = in / rows;
  f32x16 acc[2][4];
  tile_gemm(a.o, a.K, (int64_t)I * TM, (int64_t)L * TM, bufs, acc);
  const int wave = threadIdx.x >> 6;
  const int wm = wave >> 1, wn = wave & 1;
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 4; ++bj) {
      const int l = L * TM + acc_col(wn, bj);
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int i = I * TM + acc_row(wm, bi, q);
        if (i < a.N && l < a.k) a.g[(int64_t)i * a.k + l] = 4.0f * acc[bi][bj][q];
      }
    }
}

}  // namespace bf3

// Host side -----------------------------------------------------------------

hipError_t launch_gram_bf3(const sos_plan_s* p, hipStream_t s) {
  bf3::GramArgs g;
  const char* ws = p->ws;
  g.o.a_hi = g.o.b_hi = (const __bf16*)(ws + p->lay.a_hi);
  g.o.a_lo = g.o.b_lo = (const __bf16*)(ws + p->lay.a_lo);
  g.o.ld = p->Kp;
  g.K = p->Kp;
  g.tiles = (const int2*)(ws + p->lay.tiles);
  g.ntiles = p->ntiles256;
  g.N = (int)p->N;
  g.rk.codes = (const uint32_t*)(ws + p->lay.codes);
  g.rk.tables = (const int32_t*)(ws + p->lay.tables);
  g.rk.nwords = p->nwords;
  g.rk.ngroups = p->ngroups;
  g.r = (double*)(ws + p->lay.r);
  bf3::k_gram_bf3<<<g.ntiles, bf3::NT, 0, s>>>(g);
  return hipGetLastError();
}

hipError_t launch_rw_bf3(const sos_plan_s* p, void* g, hipStream_t s) {
  bf3::RwArgs a;
  const char* ws = p->ws;
  a.o.a_hi = (const __bf16*)(ws + p->lay.R_hi);
  a.o.a_lo = (const __bf16*)(ws + p->lay.R_lo);
  a.o.b_hi = (const __bf16*)(ws + p->lay.t_hi);
  a.o.b_lo = (const __bf16*)(ws + p->lay.t_lo);
  a.o.ld = p->Np2;
  a.K = p->Np2;
  a.TI = (int)(p->Np / bf3::TM);
  a.TL = (int)(p->Kp2 / bf3::TM);
  a.N = (int)p->N;
  a.k = p->k;
  a.g = (float*)g;
  bf3::k_rw_bf3<<<a.TI * a.TL, bf3::NT, 0, s>>>(a);
  return hipGetLastError();
}

}  // namespace sos
