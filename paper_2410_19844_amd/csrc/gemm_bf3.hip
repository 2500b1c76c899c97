// Split 16-bit ("bf16x3", "fp16x3") contractions on gfx950 MFMA, 256 x 256
// output tiles.
//
// Every operand w is held as two 16-bit arrays, hi = round(w) and
// lo = round(w - hi); a product w w' is taken as lo*hi' + hi*lo' + hi*hi' on
// v_mfma_f32_32x32x16_bf16 (or _f16) with FP32 accumulation (lo*lo' is
// dropped).  fp16 operands are scaled by powers of two held in the plan's
// workspace (W copies by 2^sW, R by 2^sR), which the epilogues divide out
// exactly.
//
// Tile: 256 x 256 outputs per workgroup; each wave owns WM x WN of it
// (WM / 32 x WN / 32 MFMA blocks of 32 x 32).  K advances through a 4-deep
// ring of LDS stages (4 slots x 256 rows x 32 B = 32 KB each) filled by
// direct global->LDS loads issued three stages ahead, so an L2 miss has
// about three stages of MFMA work to hide behind.  A stage's four slots
// hold A_hi, A_lo, B_hi, B_lo of one K block of 16 (split products), or,
// for single products, A_hi and B_hi of two consecutive K blocks (32 K per
// stage: twice the MFMA work per barrier).
//
// Tile order is XCD-aware: workgroups are dispatched round-robin over the 8
// XCDs (each with its own L2), so consecutive workgroups of one XCD are
// given tiles that share operand panels.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>

#include "sos_internal.h"

namespace sos {
namespace bf3 {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// One 32 x 32 x 16 product.  The operands travel as 16-bit words whatever
// their format: bf16 (SOS_BF16X3 plans) or fp16 (SOS_FP16X3 plans, scaled by
// powers of two so that the lo halves stay in fp16's normal range).
template <bool F16>
__device__ __forceinline__ f32x16 mfma16(const bf16x8& a, const bf16x8& b, const f32x16& c) {
  if constexpr (F16)
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, a), __builtin_bit_cast(f16x8, b), c, 0, 0,
                                                  0);
  else
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

// A float as the plan's 16-bit operand format, and back.
template <bool F16>
__device__ __forceinline__ __bf16 to16(float x) {
  if constexpr (F16) return __builtin_bit_cast(__bf16, (_Float16)x);
  else return (__bf16)x;
}
template <bool F16>
__device__ __forceinline__ float from16(__bf16 h) {
  if constexpr (F16) return (float)__builtin_bit_cast(_Float16, h);
  else return (float)h;
}

constexpr int TM = 256;
constexpr int BK = 16;            // K per slot (one MFMA k-step, one block of the blocked layout)
constexpr int WM = 128;           // rows of the output tile per wave
constexpr int WN = 64;            // columns of the output tile per wave: 8 waves of 128 x 64, two per SIMD
                                  // (128 accumulator registers each), so one wave's MFMAs cover the
                                  // other's waits
constexpr int BI = WM / 32, BJ = WN / 32;     // 32 x 32 MFMA blocks per wave
constexpr int WGN = TM / WN;                  // waves along the column direction
constexpr int NWAVES = (TM / WM) * WGN;
constexpr int NT = 64 * NWAVES;
constexpr int ROWS_PER_WAVE = TM / NWAVES;    // rows each wave loads per array
constexpr int NSTAGE = 4;         // LDS stages; loads run NSTAGE - 1 stages ahead
constexpr int ROWB = BK * 2;      // bytes per row per array (32)
constexpr int ARR = TM * ROWB;    // bytes per array tile (8 KB)
constexpr int STAGE = 4 * ARR;    // four slots (32 KB)
// K per stage: one block with split products, two blocks with single products
template <bool SPLIT>
constexpr int kstage() { return SPLIT ? BK : 2 * BK; }
constexpr int kXcds = 8;

typedef __attribute__((address_space(3))) void* lds_t;

// Row r of an array tile holds two 16-byte chunks; chunk c sits in slot
// c ^ ((r >> 3) & 1), so 16 consecutive rows read at one chunk cover 16
// distinct 16-byte bank groups.
__device__ __forceinline__ int slot_off(int row, int chunk) {
  return row * ROWB + ((chunk ^ ((row >> 3) & 1)) << 4);
}

// Slot sources.  With single products a_lo / b_lo point one K block past
// a_hi / b_hi (the second K block of the stage), not at lo arrays.
struct Operands {
  const __bf16* a_hi;
  const __bf16* a_lo;
  const __bf16* b_hi;
  const __bf16* b_lo;
  int64_t pstride;  // elements per (padded) panel of the panel-blocked layout, see blk_off
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
// goes to LDS, and the registers are read when it issues.
//
// Hazards the compiler cannot see inside the asm, handled here: the global
// address is a per-lane 64-bit VGPR pair (a VALU-written VGPR read by a
// vector-memory instruction is interlocked, whereas an SGPR base written by
// a VALU instruction would need 5 wait states before the load), and the
// SALU write of m0 is followed by s_nop before the load that reads it.
__device__ __forceinline__ void dma16(const char* gaddr, unsigned m0) {
  asm volatile("s_mov_b32 m0, %0\n\ts_nop 1\n\tglobal_load_lds_dwordx4 %1, off"
               :
               : "s"(m0), "v"(gaddr)
               : "memory", "m0");
}

// LDS byte address of the ring and of this wave's rows in a stage, computed
// once per tile as wave-uniform values (scalar registers), so that each load
// costs one 64-bit address add and the m0 write.
struct RingAddr {
  unsigned ring;   // LDS address of stage buffer 0
  unsigned wrow;   // offset of this wave's first row within an array tile
};

__device__ __forceinline__ RingAddr ring_addr(char* ring) {
  RingAddr a;
  a.ring = __builtin_amdgcn_readfirstlane((unsigned)(uintptr_t)(lds_t)ring);
  a.wrow = __builtin_amdgcn_readfirstlane((unsigned)((threadIdx.x >> 6) * ROWS_PER_WAVE * ROWB));
  return a;
}

// Issue the direct-to-LDS loads of one stage (starting at K = k0) into ring
// buffer `buf`: wave w moves rows [ROWS_PER_WAVE w, ROWS_PER_WAVE (w + 1))
// of each slot, 32 rows (1 KB) per instruction, lane l one 16-byte chunk.
// With the panel-blocked layout a slot is one contiguous 8 KB block, so the
// 1 KB of one instruction is 8 whole 128-byte lines.
template <bool SPLIT>
__device__ __forceinline__ void issue_stage(const RingAddr& ra, int buf, const Operands& o, int64_t arow0,
                                            int64_t brow0, int64_t k0) {
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int64_t ablk = (arow0 / TM) * o.pstride + (k0 / BK) * (TM * BK);  // element offset of the block
  const int64_t bblk = (brow0 / TM) * o.pstride + (k0 / BK) * (TM * BK);
  const unsigned m = ra.ring + (unsigned)buf * STAGE + ra.wrow;
#pragma unroll
  for (int h = 0; h < ROWS_PER_WAVE / 32; ++h) {
    const int r = w * ROWS_PER_WAVE + h * 32 + (l >> 1);
    const int c = (l & 1) ^ ((r >> 3) & 1);
    const int e = r * BK + c * 8;  // element offset inside the block
    const unsigned mh = m + h * 32 * ROWB;
    dma16((const char*)(o.a_hi + ablk + e), mh + 0 * ARR);
    dma16((const char*)(o.a_lo + ablk + e), mh + 1 * ARR);
    dma16((const char*)(o.b_hi + bblk + e), mh + 2 * ARR);
    dma16((const char*)(o.b_lo + bblk + e), mh + 3 * ARR);
  }
}

// MFMA operand fragments of one stage for this wave: per 32-row block of A
// (and of B) one 16-byte chunk per lane of hi (and lo).
struct Frag {
  bf16x8 ah[BI], al[BI], bh[BJ], bl[BJ];
};

// Fragment reads: row = (block base, a multiple of 32) + (lane & 31), so the
// swizzle depends on the lane only and every read is one lane-constant base
// plus a compile-time offset.
template <bool SPLIT>
__device__ __forceinline__ void load_frag(Frag& f, const char* st, int wm, int wn) {
  const int l = threadIdx.x & 63;
  const int lane_off = slot_off(l & 31, l >> 5);
  const char* a = st + wm * WM * ROWB + lane_off;
  const char* b = st + 2 * ARR + wn * WN * ROWB + lane_off;
#pragma unroll
  for (int bi = 0; bi < BI; ++bi) {
    f.ah[bi] = *(const bf16x8*)(a + bi * 32 * ROWB);
    f.al[bi] = *(const bf16x8*)(a + ARR + bi * 32 * ROWB);
  }
#pragma unroll
  for (int bj = 0; bj < BJ; ++bj) {
    f.bh[bj] = *(const bf16x8*)(b + bj * 32 * ROWB);
    f.bl[bj] = *(const bf16x8*)(b + ARR + bj * 32 * ROWB);
  }
}

// MFMAs of A-blocks [b0, b1) against all B-blocks.
template <bool SPLIT, bool F16, int b0, int b1>
__device__ __forceinline__ void mma_rows(const Frag& f, f32x16 (&acc)[BI][BJ]) {
#pragma unroll
  for (int bi = b0; bi < b1; ++bi)
#pragma unroll
    for (int bj = 0; bj < BJ; ++bj) {
      if (SPLIT) {
        acc[bi][bj] = mfma16<F16>(f.al[bi], f.bh[bj], acc[bi][bj]);
        acc[bi][bj] = mfma16<F16>(f.ah[bi], f.bl[bj], acc[bi][bj]);
        acc[bi][bj] = mfma16<F16>(f.ah[bi], f.bh[bj], acc[bi][bj]);
      } else {  // two K blocks: slot pairs (hi, hi) and (lo, lo) hold blocks 0 and 1
        acc[bi][bj] = mfma16<F16>(f.ah[bi], f.bh[bj], acc[bi][bj]);
        acc[bi][bj] = mfma16<F16>(f.al[bi], f.bl[bj], acc[bi][bj]);
      }
    }
}

// One step of the software pipeline.  On entry `cur` holds the fragments of
// stage kt.  The first half of its MFMAs is issued; then, while they run,
// the wave waits for stage kt+1 to land, joins the barrier (after which the
// buffer of stage kt is free: every wave has its fragments in registers),
// issues the loads of stage kt+4 into that buffer and reads the fragments of
// stage kt+1 into `nxt`; the second half of the MFMAs of stage kt covers the
// latency of those reads.
template <bool SPLIT, bool F16>
__device__ __forceinline__ void pipe_step(Frag& cur, Frag& nxt, char* ring, const RingAddr& ra, const Operands& o,
                                          int64_t kt, int64_t nk, int64_t arow0, int64_t brow0,
                                          f32x16 (&acc)[BI][BJ], int wm, int wn) {
  constexpr int per = 4 * (ROWS_PER_WAVE / 32);  // loads per thread per stage
  mma_rows<SPLIT, F16, 0, BI / 2>(cur, acc);
  __builtin_amdgcn_sched_barrier(0);
  if (kt + 1 < nk) {
    // stages issued so far: up to kt + 3; stage kt + 1 must have landed
    const int64_t later = (nk - 1) - (kt + 1) < 2 ? (nk - 1) - (kt + 1) : 2;
    if (later == 2) wait_vm_barrier<2 * per>();
    else if (later == 1) wait_vm_barrier<per>();
    else wait_vm_barrier<0>();
    if (kt + NSTAGE < nk) issue_stage<SPLIT>(ra, (int)(kt % NSTAGE), o, arow0, brow0, (kt + NSTAGE) * kstage<SPLIT>());
    load_frag<SPLIT>(nxt, ring + ((kt + 1) % NSTAGE) * STAGE, wm, wn);
  }
  __builtin_amdgcn_sched_barrier(0);
  mma_rows<SPLIT, F16, BI / 2, BI>(cur, acc);
}

// The same step in the steady state (kt + 4 < nk), ordered differently: the
// barrier comes first (stage kt+1 has landed, and every wave is done reading
// the buffer of stage kt, whose fragments are in registers), then the MFMAs
// of stage kt with the fragment reads of stage kt+1 interleaved among them,
// so that the reads have the whole stage's MFMA time to complete, and last
// the refill of stage kt's buffer with stage kt+4 (issued after the MFMAs
// rather than before them: 1-2% faster here, 7% in the int8 gram).  No
// branches.
template <bool SPLIT, bool F16>
__device__ __forceinline__ void pipe_step_steady(Frag& cur, Frag& nxt, char* ring, const RingAddr& ra, const Operands& o,
                                                 int64_t kt,
                                                 int64_t arow0, int64_t brow0, f32x16 (&acc)[BI][BJ], int wm,
                                                 int wn) {
  constexpr int per = 4 * (ROWS_PER_WAVE / 32);
  constexpr int NMFMA = BI * BJ * (SPLIT ? 3 : 2);
  constexpr int NREAD = 2 * (BI + BJ);
  constexpr int RATIO = NMFMA / NREAD;
  wait_vm_barrier<2 * per>();
  __builtin_amdgcn_sched_barrier(0);
  load_frag<SPLIT>(nxt, ring + ((kt + 1) % NSTAGE) * STAGE, wm, wn);
  mma_rows<SPLIT, F16, 0, BI>(cur, acc);
  // scheduling pattern: RATIO MFMAs (mask 0x008), one LDS read (mask 0x100), ...
#pragma unroll
  for (int q = 0; q < NREAD; ++q) {
    __builtin_amdgcn_sched_group_barrier(0x008, RATIO, 0);
    __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
  }
  __builtin_amdgcn_sched_group_barrier(0x008, NMFMA - RATIO * NREAD, 0);
  __builtin_amdgcn_sched_barrier(0);
  issue_stage<SPLIT>(ra, (int)(kt % NSTAGE), o, arow0, brow0, (kt + NSTAGE) * kstage<SPLIT>());
  __builtin_amdgcn_sched_barrier(0);
}

// C(256 x 256) = A[arow0 .. +256) x B[brow0 .. +256)^T over K (K a multiple of the stage K).
template <bool SPLIT, bool F16>
__device__ __forceinline__ void tile_gemm(const Operands& o, int64_t K, int64_t arow0, int64_t brow0,
                                          char* ring, f32x16 (&acc)[BI][BJ]) {
  const int wave = threadIdx.x >> 6;
  const int wm = wave / WGN, wn = wave % WGN;
#pragma unroll
  for (int bi = 0; bi < BI; ++bi)
#pragma unroll
    for (int bj = 0; bj < BJ; ++bj) acc[bi][bj] = f32x16{};
  constexpr int per = 4 * (ROWS_PER_WAVE / 32);
  const int64_t nk = K / kstage<SPLIT>();
  const RingAddr ra = ring_addr(ring);
  for (int s = 0; s < NSTAGE - 1; ++s)
    if (s < nk) issue_stage<SPLIT>(ra, s, o, arow0, brow0, (int64_t)s * kstage<SPLIT>());
  // stage 0 must have landed; stages 1 and 2 may be in flight
  if (nk >= 3) wait_vm_barrier<2 * per>();
  else if (nk == 2) wait_vm_barrier<per>();
  else wait_vm_barrier<0>();
  if (NSTAGE - 1 < nk) issue_stage<SPLIT>(ra, NSTAGE - 1, o, arow0, brow0, (int64_t)(NSTAGE - 1) * kstage<SPLIT>());
  Frag f0, f1;
  load_frag<SPLIT>(f0, ring, wm, wn);
  int64_t kt = 0;
  for (; kt + 1 + NSTAGE < nk; kt += 2) {
    pipe_step_steady<SPLIT, F16>(f0, f1, ring, ra, o, kt, arow0, brow0, acc, wm, wn);
    pipe_step_steady<SPLIT, F16>(f1, f0, ring, ra, o, kt + 1, arow0, brow0, acc, wm, wn);
  }
  for (; kt < nk; kt += 2) {
    pipe_step<SPLIT, F16>(f0, f1, ring, ra, o, kt, nk, arow0, brow0, acc, wm, wn);
    if (kt + 1 < nk) pipe_step<SPLIT, F16>(f1, f0, ring, ra, o, kt + 1, nk, arow0, brow0, acc, wm, wn);
  }
}

// (row, col) of accumulator (bi, bj, q) inside the 256 x 256 tile.
__device__ __forceinline__ int acc_row(int wm, int bi, int q) {
  const int l = threadIdx.x & 63;
  return wm * WM + bi * 32 + (q >> 2) * 8 + (l >> 5) * 4 + (q & 3);
}
__device__ __forceinline__ int acc_col(int wn, int bj) {
  return wn * WN + bj * 32 + (threadIdx.x & 31);
}

// Block id -> position in a per-XCD-contiguous order (bijective on [0, nb)).
__device__ __forceinline__ int xcd_order(int b, int nb) {
  const int q = nb / kXcds, rem = nb % kXcds;
  const int xcd = b % kXcds, local = b / kXcds;
  return (xcd < rem) ? xcd * (q + 1) + local : rem * (q + 1) + (xcd - rem) * q + local;
}

// Tile-rows per group in the R W GEMMs' order (column-major inside a group).
// Each XCD runs a contiguous run of about 32 tiles, so a group of 6 keeps
// them on about 11 operand panels.  At n = 12, d = 6 (73 x 73 tiles) groups
// of 6 read ~29 GB per fused R W + Adam against ~34 GB for 8 and ran 1%
// faster; 4 read as little but ran as 8, and 12 or 16 ran 2-4% slower.
constexpr int kRwGroup = 6;


struct GramArgs {
  Operands o;
  int64_t K;
  const int2* tiles;  // (I, J) tile pairs, I <= J, in locality order
  int ntiles, N;
  int nfull, parts;   // tail split (see TailSplit): tiles nfull.. run in `parts` K ranges
  RankTab rk;
  double* r;
  float* G;           // unfused variant: tile v stored row-major at G + 65536 v (nullptr: scatter)
  const int* sx;      // fp16 operands: sx[0] = sW, the W copies hold 2^sW w (bf16: unused)
  // the plan's merge maps (see kMergeRows), or nullptr: every entry ranked and added on its own
  const uint16_t* mmap;
  const int* mrank;
  const int* mcount;
};

// FP64 add into LDS (ds_add_f64: no return value is asked for).
__device__ __forceinline__ void lds_add(double* p, double x) {
  __hip_atomic_fetch_add(p, x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Epilogue with the plan's merge maps: the tile in four segments of 64 rows.
// Per segment its accumulators go to LDS in FP32 (64 KB, the first half of
// the pipeline ring); every pair is added, with its weight, into the FP64
// slot its map names (the second half: kMergeSlots slots); then each slot in
// use goes into r by one atomic, at the coefficient of the segment's rank
// list.  About 3.6 pairs share a slot at n = 12, d = 6, so r sees that many
// times fewer atomics than with one per pair.
//
// Loads and atomics share one in-order completion counter: a load issued
// after an atomic can only be waited for once the atomic has completed.  So
// a segment loads its share of the rank list at its start (while the
// previous segment's atomics drain), not one entry per atomic, and its map
// words one ahead of their use.
template <bool F16>
__device__ __forceinline__ void gram_merge_epilogue(const GramArgs& g, int v, int2 t, f32x16 (&acc)[BI][BJ],
                                                    char* lds, double unscale) {
  constexpr int RK = kMergeSlots / NT;  // rank-list entries per thread and segment, at most
  const int wave = threadIdx.x >> 6;
  const int wm = wave / WGN, wn = wave % WGN;
  float* stage = (float*)lds;
  double* slots = (double*)(lds + kMergeSeg * 4);
  static_assert(kMergeSeg * 4 + kMergeSlots * 8 <= NSTAGE * STAGE, "merge buffers exceed the ring");
  static_assert(2 * kMergeRows == WM && BI == 4 && kMergeSeg % (NT * 8) == 0 && kMergeSlots % NT == 0,
                "a segment is half a wave's rows");
  const bool diag = t.x == t.y;
#pragma unroll
  for (int qq = 0; qq < kMergeSegs; ++qq) {
    const int seg = v * kMergeSegs + qq;
    const int ns = g.mcount[seg];
    const uint16_t* mp = g.mmap + (size_t)seg * kMergeSeg;
    const int* rl = g.mrank + (size_t)seg * kMergeSlots;
    // every entry of the segment's list, used or not (q < kMergeSlots: inside
    // it), so that the loads carry no branches and are waited for once
    int rk[RK];
#pragma unroll
    for (int it = 0; it < RK; ++it) rk[it] = rl[threadIdx.x + it * NT];
    uint4 mnext = *(const uint4*)(mp + threadIdx.x * 8);
    __syncthreads();  // nobody reads the ring (or the previous segment's slots) any more
    for (int q = threadIdx.x; q < ns; q += NT) slots[q] = 0.0;
    if (wm == qq / 2) {
#pragma unroll
      for (int bi = 0; bi < BI; ++bi) {
        if (bi / 2 != (qq & 1)) continue;
#pragma unroll
        for (int bj = 0; bj < BJ; ++bj)
#pragma unroll
          for (int q = 0; q < 16; ++q)
            stage[(acc_row(wm, bi, q) - qq * kMergeRows) * TM + acc_col(wn, bj)] = acc[bi][bj][q];
      }
    }
    __syncthreads();
    for (int e0 = threadIdx.x * 8; e0 < kMergeSeg; e0 += NT * 8) {
      const uint4 mw = mnext;
      if (e0 + NT * 8 < kMergeSeg) mnext = *(const uint4*)(mp + e0 + NT * 8);
      const float4 xa = *(const float4*)(stage + e0), xb = *(const float4*)(stage + e0 + 4);
      const uint32_t m2[4] = {mw.x, mw.y, mw.z, mw.w};
      const float xs[8] = {xa.x, xa.y, xa.z, xa.w, xb.x, xb.y, xb.z, xb.w};
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const unsigned sl = (m2[u >> 1] >> (16 * (u & 1))) & 0xFFFFu;
        if (sl == kMergeSkip) continue;
        const int row = qq * kMergeRows + (e0 + u) / TM, col = (e0 + u) % TM;
        const double x = ((diag && row == col) ? unscale : 2.0 * unscale) * (double)xs[u];
        if (sl < kMergeSlots) lds_add(slots + sl, x);
        else unsafeAtomicAdd(g.r + pair_rank(g.rk, t.x * TM + row, t.y * TM + col), x);
      }
    }
    __syncthreads();
    // all of this thread's slot sums first, into registers of their own, then
    // the atomics: no atomic then waits for the previous one to release its
    // data registers
    double xv[RK];
#pragma unroll
    for (int it = 0; it < RK; ++it) {
      const int q = threadIdx.x + it * NT;
      const double x = slots[q];  // q < kMergeSlots: inside the slots, used or not
      xv[it] = q < ns ? x : 0.0;
    }
#pragma unroll
    for (int it = 0; it < RK; ++it)
      if (xv[it] != 0.0) unsafeAtomicAdd(g.r + rk[it], xv[it]);
  }
}

#define SOS_BF3_BUFFERS \
  __shared__ __attribute__((aligned(16))) char lds[NSTAGE * STAGE]

// The gram: one workgroup per upper tile, in the locality order of the tile
// list.  Epilogue with merge maps (above), or without: the accumulator tile
// (fp32, 256 KB) goes out in row-halves of 128 x 256 (128 KB, the pipeline
// buffers being free by now); then every thread takes consecutive elements
// of the half, ranks each (row, col) pair and adds it into r.  Copying out
// with compile-time indices keeps the accumulators in registers; the scatter
// loop indexes LDS instead.
// SINGLE: one product hi hi^T (the lo operands of GramArgs point one K block
// past the hi ones, so a stage carries two K blocks, as in the single-product
// R W GEMM); otherwise the three products of the split form.
template <bool F16, bool SINGLE>
__global__ __launch_bounds__(NT) void k_gram_bf3(GramArgs g) {
  SOS_BF3_BUFFERS;
  constexpr int64_t KS = kstage<!SINGLE>();  // K per pipeline stage
  // whole tiles first (XCD-aware order); then the tail tiles, `parts`
  // contiguous K ranges each (whole stages of every panel: the operands are
  // the same arrays moved k0 stages on)
  int v;
  int64_t k0 = 0, nks = g.K / KS;
  if ((int)blockIdx.x < g.nfull) {
    v = xcd_order(blockIdx.x, g.nfull);
  } else {
    const int u = (int)blockIdx.x - g.nfull, q = u % g.parts;
    v = g.nfull + u / g.parts;
    const int64_t nk = g.K / KS;
    k0 = nk * q / g.parts;
    nks = nk * (q + 1) / g.parts - k0;
  }
  const int2 t = g.tiles[v];
  Operands o = g.o;
  const int64_t shift = k0 * (KS / BK) * (TM * BK);
  o.a_hi += shift;
  o.a_lo += shift;
  o.b_hi += shift;
  o.b_lo += shift;
  f32x16 acc[BI][BJ];
  tile_gemm<!SINGLE, F16>(o, nks * KS, (int64_t)t.x * TM, (int64_t)t.y * TM, lds, acc);
  const double unscale = F16 ? (double)pow2f(-2 * g.sx[0]) : 1.0;  // exact: a power of two
  if (g.mmap) {
    gram_merge_epilogue<F16>(g, v, t, acc, lds, unscale);
    return;
  }
  const int wave = threadIdx.x >> 6;
  const int wm = wave / WGN, wn = wave % WGN;
  float* half = (float*)lds;  // the whole pipeline ring: 128 KB
  constexpr int HROWS = 128;
  static_assert(4 * STAGE == HROWS * TM * 4, "half tile must fill the pipeline buffers");
  static_assert(TM == kBlkRows && BK == kBlkK, "stage = one block of the panel-blocked layout");
#pragma unroll
  for (int hh = 0; hh < TM / HROWS; ++hh) {
    __syncthreads();
    if (wm * WM / HROWS == hh) {
#pragma unroll
      for (int bi = 0; bi < BI; ++bi)
#pragma unroll
        for (int bj = 0; bj < BJ; ++bj)
#pragma unroll
          for (int q = 0; q < 16; ++q) {
            const int row = acc_row(wm, bi, q) - hh * HROWS, col = acc_col(wn, bj);
            half[row * TM + col] = acc[bi][bj][q];
          }
    }
    __syncthreads();
    if (g.G) {  // unfused measurement variant: store the half tile, k_scatter_tiles ranks it
      float* dst = g.G + (size_t)v * (TM * TM) + hh * HROWS * TM;
      for (int e = threadIdx.x * 4; e < HROWS * TM; e += NT * 4) *(float4*)(dst + e) = *(const float4*)(half + e);
      continue;
    }
    // In batches of SB entries per thread: the ranks of a batch first (their
    // loads, with indices clamped into the basis so that none sits in a
    // branch), then its atomics.  Loads and atomics complete in order, so
    // this waits once per batch for the previous atomics, not once per entry.
    constexpr int SB = 8, PER = HROWS * TM / NT;
    static_assert(PER % SB == 0, "whole batches");
    for (int k0 = 0; k0 < PER; k0 += SB) {
      int rk[SB];
      double xv[SB];
#pragma unroll
      for (int u = 0; u < SB; ++u) {
        const int e = threadIdx.x + (k0 + u) * NT;
        const int i = t.x * TM + hh * HROWS + e / TM, j = t.y * TM + e % TM;
        const bool ok = i < g.N && j < g.N && i <= j;
        rk[u] = pair_rank(g.rk, min(i, g.N - 1), min(j, g.N - 1));
        xv[u] = ok ? ((i == j) ? unscale : 2.0 * unscale) * (double)half[e] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < SB; ++u)
        if (xv[u] != 0.0) unsafeAtomicAdd(g.r + rk[u], xv[u]);
    }
  }
}

// Merge maps, one workgroup per segment of 64 rows x 256 columns of a tile:
// the rank of every pair of the segment in the upper triangle (i <= j < N)
// goes with its position into a 64-bit key, the keys are sorted in LDS
// (bitonic), and the distinct ranks numbered in ascending order; the first
// kMergeSlots of them get slots, the rest kMergeDirect.  counts[seg] = slots
// in use; counts[nsegs + seg] = the r atomics the segment then issues (slots
// plus direct pairs).
__global__ __launch_bounds__(512) void k_merge_maps(const int2* __restrict__ tiles, int N, RankTab rk,
                                                    uint16_t* __restrict__ map, int* __restrict__ ranks,
                                                    int* __restrict__ counts) {
  constexpr int NTM = 512, PER = kMergeSeg / NTM;
  constexpr unsigned long long kNone = 1ull << 46;  // above every (rank << 14 | position) key
  static_assert(kMergeSeg == 1 << 14, "positions take 14 bits");
  __shared__ unsigned long long key[kMergeSeg];
  __shared__ int part[NTM + 1];
  const int seg = blockIdx.x, v = seg / kMergeSegs, qq = seg % kMergeSegs;
  const int2 t = tiles[v];
  for (int e = threadIdx.x; e < kMergeSeg; e += NTM) {
    const int i = t.x * TM + qq * kMergeRows + e / TM, j = t.y * TM + e % TM;
    key[e] = (i < N && j < N && i <= j) ? ((unsigned long long)pair_rank(rk, i, j) << 14) | (unsigned)e
                                        : kNone | (unsigned)e;
  }
  __syncthreads();
  for (int size = 2; size <= kMergeSeg; size <<= 1)
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int x = threadIdx.x; x < kMergeSeg / 2; x += NTM) {
        const int lo = 2 * x - (x & (stride - 1)), hi = lo + stride;  // lo has bit `stride` clear
        const unsigned long long a = key[lo], b = key[hi];
        if ((a > b) == ((lo & size) == 0)) {
          key[lo] = b;
          key[hi] = a;
        }
      }
      __syncthreads();
    }
  // each thread numbers PER consecutive keys: count the first key of every
  // rank in its range, scan the counts, then assign
  const int x0 = threadIdx.x * PER;
  int firsts = 0;
  for (int u = 0; u < PER; ++u) {
    const unsigned long long k = key[x0 + u];
    firsts += k < kNone && (x0 + u == 0 || (key[x0 + u - 1] >> 14) != (k >> 14));
  }
  part[threadIdx.x] = firsts;
  __syncthreads();
  if (threadIdx.x == 0) {
    int sum = 0;
    for (int w = 0; w < NTM; ++w) {
      const int c = part[w];
      part[w] = sum;
      sum += c;
    }
    part[NTM] = sum;
  }
  __syncthreads();
  __shared__ int direct;
  if (threadIdx.x == 0) direct = 0;
  __syncthreads();
  int slot = part[threadIdx.x] - 1;  // slot of a rank run continuing from the previous thread's keys
  int ndirect = 0;
  uint16_t* mp = map + (size_t)seg * kMergeSeg;
  int* rl = ranks + (size_t)seg * kMergeSlots;
  for (int u = 0; u < PER; ++u) {
    const int x = x0 + u;
    const unsigned long long k = key[x];
    const int e = (int)(k & 0x3FFFu);
    if (k >= kNone) {
      mp[e] = kMergeSkip;
      continue;
    }
    const bool first = x == 0 || (key[x - 1] >> 14) != (k >> 14);
    slot += first;
    if (slot < kMergeSlots) {
      mp[e] = (uint16_t)slot;
      if (first) rl[slot] = (int)(k >> 14);
    } else {
      mp[e] = kMergeDirect;
      ++ndirect;
    }
  }
  if (ndirect) atomicAdd(&direct, ndirect);
  __syncthreads();
  if (threadIdx.x == 0) {
    counts[seg] = min(part[NTM], kMergeSlots);
    counts[gridDim.x + seg] = min(part[NTM], kMergeSlots) + direct;
  }
}

// The scatter of the unfused variant on its own: quarter tiles (64 x 256) of
// the stored Gram tiles, read coalesced, each upper-triangle entry ranked and
// added into r with its weight, as the fused epilogue does.  Measures what
// the scatter costs outside the GEMM (bytes: the N (N + 1) / 2 FP32 entries
// read, r updated by atomics).
__global__ __launch_bounds__(256) void k_scatter_tiles(const float* __restrict__ G, const int2* __restrict__ tiles,
                                                       int N, RankTab rk, double* __restrict__ r) {
  const int v = blockIdx.x >> 2, qq = blockIdx.x & 3;
  const int2 t = tiles[v];
  const float* src = G + (size_t)v * (TM * TM) + qq * 64 * TM;
  for (int e = threadIdx.x; e < 64 * TM; e += 256) {
    const int i = t.x * TM + qq * 64 + e / TM, j = t.y * TM + e % TM;
    if (i < N && j < N && i <= j) {
      const double w = (i == j) ? 1.0 : 2.0;
      unsafeAtomicAdd(r + pair_rank(rk, i, j), w * (double)src[e]);
    }
  }
}

struct RwArgs {
  Operands o;  // A = R (rows Np), B = W^T copies (rows Kp2); K extent Np2
  int64_t K;
  int TI, TL, N, k;
  float* g;    // N x k
  const int* sx;     // fp16 operands: sx[0] = sW (W copies hold 2^sW w), sx[1] = sR (R holds 2^sR r)
};

template <bool SPLIT, bool F16>
__global__ __launch_bounds__(NT) void k_rw_bf3(RwArgs a) {
  SOS_BF3_BUFFERS;
  const int nb = a.TI * a.TL;
  const int v = xcd_order(blockIdx.x, nb);
  // grouped order: kRwGroup tile-rows at a time, column-major inside the group
  constexpr int GROUP = kRwGroup;
  const int per_group = GROUP * a.TL;
  const int gidx = v / per_group, first = gidx * GROUP;
  const int rows = min(GROUP, a.TI - first);
  const int in = v % per_group;
  const int I = first + in % rows, L = in / rows;
  f32x16 acc[BI][BJ];
  tile_gemm<SPLIT, F16>(a.o, a.K, (int64_t)I * TM, (int64_t)L * TM, lds, acc);
  const float four = F16 ? pow2f(2 - a.sx[0] - a.sx[1]) : 4.0f;  // 4 times a power of two
  // epilogue through LDS in row-halves (as in k_gram_bf3), then coalesced
  // row-major stores of 4 * acc into g
  const int wave = threadIdx.x >> 6;
  const int wm = wave / WGN, wn = wave % WGN;
  float* half = (float*)lds;
  constexpr int HROWS = 128;
#pragma unroll
  for (int hh = 0; hh < TM / HROWS; ++hh) {
    __syncthreads();
    if (wm * WM / HROWS == hh) {
#pragma unroll
      for (int bi = 0; bi < BI; ++bi)
#pragma unroll
        for (int bj = 0; bj < BJ; ++bj)
#pragma unroll
          for (int q = 0; q < 16; ++q)
            half[(acc_row(wm, bi, q) - hh * HROWS) * TM + acc_col(wn, bj)] = acc[bi][bj][q];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < HROWS * TM; e += NT) {
      const int i = I * TM + hh * HROWS + e / TM, l = L * TM + e % TM;
      if (i < a.N && l < a.k) a.g[(int64_t)i * a.k + l] = four * half[e];
    }
  }
}

// The single-product backward with Adam and the next step's operand copies
// in its epilogue.  W (FP32 master) is not an operand of this GEMM (it reads
// the bf16 copies of R and W^T), and every (i, l) belongs to exactly one
// tile, so each tile can update its own W, m and v in place.  From the
// updated W it writes what the next step's forward reads (the split copy, or
// the FP32 blocked copy for the exact forward) and the transposed copy for
// the next backward into the second transposed buffer (the one this GEMM does
// not read).  Padding rows and columns get zeros, as the preparation kernel
// writes them.
struct RwAdamArgs {
  RwArgs rw;
  float* __restrict__ W;
  float* __restrict__ m;
  float* __restrict__ v;
  float lr, b1, b2, eps, bc1, bc2;
  __bf16* a_hi;       // next forward, split copy (fast forward), or nullptr
  __bf16* a_lo;
  float* x_f32;       // next forward, FP32 blocked copy (exact forward), or nullptr
                      // (both nullptr: the next forward builds its own operands)
  __bf16* t_next;     // next backward: transposed copy
  int64_t aps, xps, tps;         // panel strides of those layouts
  int64_t Np, Kp, Np2, Kp2;
};

template <bool F16>
__global__ __launch_bounds__(NT) void k_rw_adam_bf3(RwAdamArgs a) {
  SOS_BF3_BUFFERS;
  const RwArgs& r = a.rw;
  const int nb = r.TI * r.TL;
  const int v = xcd_order(blockIdx.x, nb);
  constexpr int GROUP = kRwGroup;
  const int per_group = GROUP * r.TL;
  const int gidx = v / per_group, first = gidx * GROUP;
  const int rows = min(GROUP, r.TI - first);
  const int in = v % per_group;
  const int I = first + in % rows, L = in / rows;
  f32x16 acc[BI][BJ];
  tile_gemm<false, F16>(r.o, r.K, (int64_t)I * TM, (int64_t)L * TM, lds, acc);
  const float four = F16 ? pow2f(2 - r.sx[0] - r.sx[1]) : 4.0f;  // 4 times a power of two
  const float wsc = F16 ? pow2f(r.sx[0]) : 1.0f;                  // scale of the next W copies
  const int wave = threadIdx.x >> 6;
  const int wm = wave / WGN, wn = wave % WGN;
  constexpr int QROWS = 64;                            // quarter tiles of 64 x 256
  float* stage = (float*)lds;                          // 64 KB
  __bf16* tb = (__bf16*)(lds + QROWS * TM * 4);        // 32 KB: bf16 of the updated W
  static_assert(QROWS * TM * 4 + QROWS * TM * 2 <= NSTAGE * STAGE, "epilogue buffers exceed the ring");
#pragma unroll
  for (int qq = 0; qq < TM / QROWS; ++qq) {
    __syncthreads();
    if (wm == qq / 2) {
#pragma unroll
      for (int bi = 0; bi < BI; ++bi) {
        if (bi / 2 != (qq & 1)) continue;
#pragma unroll
        for (int bj = 0; bj < BJ; ++bj)
#pragma unroll
          for (int q = 0; q < 16; ++q)
            stage[(acc_row(wm, bi, q) - qq * QROWS) * TM + acc_col(wn, bj)] = acc[bi][bj][q];
      }
    }
    __syncthreads();
    // Adam on the quarter (row-major, coalesced in W, m, v), the forward copy,
    // and the bf16 of the new W into tb for the transposed copy.  Each thread
    // takes four consecutive elements of a row at a time (one 16-byte access
    // per array when rows start 16-byte aligned, two 8-byte ones when they
    // start 8-byte aligned; 4-byte accesses measured 5% slower over the whole
    // kernel at n=12, d=6 and 20% at the hundred-variable quartic, k = 5050),
    // and the loads of the next four are issued before the current four are
    // computed, so HBM latency overlaps the work.
    constexpr int PER = QROWS * TM / NT;
    constexpr int EB = 4;   // four consecutive elements of one row per fetch batch (one 16-byte access per array)
    const bool vec = (r.k & 3) == 0;       // rows start 16-byte aligned
    const bool vec2 = !vec && (r.k & 1) == 0;  // rows start 8-byte aligned: two 8-byte accesses
    float4 wv[2], mv[2], vv[2];
    auto fetch = [&](int b8, int buf) {
      const int e0 = EB * (threadIdx.x + NT * b8);
      const int64_t i = (int64_t)I * TM + qq * QROWS + e0 / TM, l0 = (int64_t)L * TM + e0 % TM;
      wv[buf] = mv[buf] = vv[buf] = make_float4(0.f, 0.f, 0.f, 0.f);
      if (i < r.N && l0 < r.k) {
        const int64_t o = i * r.k + l0;
        if (vec) {
          wv[buf] = *(const float4*)(a.W + o);
          mv[buf] = *(const float4*)(a.m + o);
          vv[buf] = *(const float4*)(a.v + o);
        } else if (vec2 && l0 + 3 < r.k) {
          const float2 w0 = *(const float2*)(a.W + o), w1 = *(const float2*)(a.W + o + 2);
          const float2 m0 = *(const float2*)(a.m + o), m1 = *(const float2*)(a.m + o + 2);
          const float2 v0 = *(const float2*)(a.v + o), v1 = *(const float2*)(a.v + o + 2);
          wv[buf] = make_float4(w0.x, w0.y, w1.x, w1.y);
          mv[buf] = make_float4(m0.x, m0.y, m1.x, m1.y);
          vv[buf] = make_float4(v0.x, v0.y, v1.x, v1.y);
        } else {
#pragma unroll
          for (int u = 0; u < EB; ++u)
            if (l0 + u < r.k) {
              (&wv[buf].x)[u] = a.W[o + u];
              (&mv[buf].x)[u] = a.m[o + u];
              (&vv[buf].x)[u] = a.v[o + u];
            }
        }
      }
    };
    fetch(0, 0);
#pragma unroll
    for (int b8 = 0; b8 < PER / EB; ++b8) {
      const int buf = b8 & 1;
      if (b8 + 1 < PER / EB) fetch(b8 + 1, buf ^ 1);
      const int e0 = EB * (threadIdx.x + NT * b8);
      const int64_t i = (int64_t)I * TM + qq * QROWS + e0 / TM, l0 = (int64_t)L * TM + e0 % TM;
      const float4 gs = *(const float4*)(stage + e0);
      float4 wn, mn, vn;
#pragma unroll
      for (int u = 0; u < EB; ++u) {
        const float ge = four * (&gs.x)[u];
        const float me = a.b1 * (&mv[buf].x)[u] + (1.f - a.b1) * ge;
        const float ve = a.b2 * (&vv[buf].x)[u] + (1.f - a.b2) * ge * ge;
        (&mn.x)[u] = me;
        (&vn.x)[u] = ve;
        (&wn.x)[u] = (i < r.N && l0 + u < r.k) ? (&wv[buf].x)[u] - a.lr * (me / a.bc1) / (sqrtf(ve / a.bc2) + a.eps) : 0.f;
      }
      if (i < r.N && l0 < r.k) {
        const int64_t o = i * r.k + l0;
        if (vec) {
          *(float4*)(a.m + o) = mn;
          *(float4*)(a.v + o) = vn;
          *(float4*)(a.W + o) = wn;
        } else if (vec2 && l0 + 3 < r.k) {
          *(float2*)(a.m + o) = make_float2(mn.x, mn.y);
          *(float2*)(a.m + o + 2) = make_float2(mn.z, mn.w);
          *(float2*)(a.v + o) = make_float2(vn.x, vn.y);
          *(float2*)(a.v + o + 2) = make_float2(vn.z, vn.w);
          *(float2*)(a.W + o) = make_float2(wn.x, wn.y);
          *(float2*)(a.W + o + 2) = make_float2(wn.z, wn.w);
        } else {
#pragma unroll
          for (int u = 0; u < EB; ++u)
            if (l0 + u < r.k) {
              a.m[o + u] = (&mn.x)[u];
              a.v[o + u] = (&vn.x)[u];
              a.W[o + u] = (&wn.x)[u];
            }
        }
      }
      if (i < a.Np && l0 < a.Kp) {  // Kp is a multiple of 16: all four columns are inside
        const int64_t ob = a.x_f32 ? blk_off(i, l0, a.xps) : blk_off(i, l0, a.aps);
        if (a.x_f32) {
          *(float4*)(a.x_f32 + ob) = wn;
        } else if (a.a_hi) {
          bf16x4 hv, lv;
#pragma unroll
          for (int u = 0; u < EB; ++u) {
            const float ws = (&wn.x)[u] * wsc;
            const __bf16 h = to16<F16>(ws);
            hv[u] = h;
            lv[u] = to16<F16>(ws - from16<F16>(h));
          }
          *(bf16x4*)(a.a_hi + ob) = hv;
          *(bf16x4*)(a.a_lo + ob) = lv;
        }
      }
      bf16x4 tv;
#pragma unroll
      for (int u = 0; u < EB; ++u) tv[u] = to16<F16>((&wn.x)[u] * wsc);
      *(bf16x4*)(tb + e0) = tv;
    }
    __syncthreads();
    // transposed copy: rows l, K = i; 8 consecutive i of one row per thread (16-byte stores)
    for (int f = threadIdx.x * 8; f < QROWS * TM; f += NT * 8) {
      const int kb = f / (TM * kBlkK), lrow = (f % (TM * kBlkK)) / kBlkK, ii0 = f % kBlkK;
      const int64_t l = (int64_t)L * TM + lrow, i0 = (int64_t)I * TM + qq * QROWS + kb * kBlkK + ii0;
      if (l < a.Kp2 && i0 < a.Np2) {
        bf16x8 hv;
#pragma unroll
        for (int u = 0; u < 8; ++u) hv[u] = tb[(kb * kBlkK + ii0 + u) * TM + lrow];
        *(bf16x8*)(a.t_next + blk_off(l, i0, a.tps)) = hv;
      }
    }
  }
}

}  // namespace bf3

// Host side -----------------------------------------------------------------

hipError_t launch_gram_bf3(const sos_plan_s* p, hipStream_t s, bool store, bool unmerged, bool single) {
  bf3::GramArgs g;
  const bool f16 = p->prec == SOS_FP16X3;
  g.sx = scale_exponents(p);
  const char* ws = p->ws;
  g.o.a_hi = g.o.b_hi = (const __bf16*)(ws + p->lay.a_hi);
  // single product: the second K block of each stage is the next block of the same panel
  g.o.a_lo = g.o.b_lo = single ? g.o.a_hi + bf3::TM * bf3::BK : (const __bf16*)(ws + p->lay.a_lo);
  g.o.pstride = panel_stride(p->Kp / kBlkK, 2);
  g.K = p->Kp;  // a multiple of 64: whole stages in both forms
  g.tiles = (const int2*)(ws + p->lay.tiles);
  g.ntiles = p->ntiles256;
  g.N = (int)p->N;
  g.rk = rank_tab(p);
  g.r = (double*)(ws + p->lay.r);
  g.G = store ? (float*)(ws + p->lay.g) : nullptr;
  // the stored tiles of the unfused variant are whole: no tail split there
  const TailSplit ts = store ? TailSplit{g.ntiles, 1} : gram_tail_split(g.ntiles, g.K / (single ? 2 * bf3::BK : bf3::BK), s);
  g.nfull = ts.nfull;
  g.parts = ts.parts;
  const int grid = ts.nfull + (g.ntiles - ts.nfull) * ts.parts;
  const bool merge = p->merge_ready && !store && !unmerged;
  g.mmap = merge ? (const uint16_t*)(ws + p->lay.mg_map) : nullptr;
  g.mrank = merge ? (const int*)(ws + p->lay.mg_rank) : nullptr;
  g.mcount = merge ? (const int*)(ws + p->lay.mg_count) : nullptr;
  if (single) {
    if (f16) bf3::k_gram_bf3<true, true><<<grid, bf3::NT, 0, s>>>(g);
    else bf3::k_gram_bf3<false, true><<<grid, bf3::NT, 0, s>>>(g);
  } else {
    if (f16) bf3::k_gram_bf3<true, false><<<grid, bf3::NT, 0, s>>>(g);
    else bf3::k_gram_bf3<false, false><<<grid, bf3::NT, 0, s>>>(g);
  }
  return hipGetLastError();
}

TailSplit gram_tail_split(int ntiles, int64_t nstages, hipStream_t s) {
  TailSplit ts;
  ts.nfull = ntiles;
  constexpr int kMaxDev = 64, kMaxParts = 8, kMinStages = 16;
  static std::atomic<int> cus_of[kMaxDev];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return ts;
  if (s && hipStreamGetDevice(s, &dev) != hipSuccess) return ts;
  if (dev < 0 || dev >= kMaxDev) return ts;
  int cus = cus_of[dev].load(std::memory_order_relaxed);
  if (cus <= 0) {
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) return ts;
    cus_of[dev].store(cus, std::memory_order_relaxed);
  }
  const int rem = ntiles % cus;
  if (ntiles < cus || rem == 0) return ts;
  // the split that makes the last round shortest: ceil(rem p / cus) waves of
  // 1/p of a tile each (rem = 141, cus = 256: p = 7, 0.57 of a round)
  double best = 1.0;
  for (int p = 2; p <= kMaxParts && nstages / p >= kMinStages; ++p) {
    const double len = (double)((rem * p + cus - 1) / cus) / p;
    if (len < best - 1e-9) {
      best = len;
      ts.parts = p;
    }
  }
  if (ts.parts > 1) ts.nfull = ntiles - rem;
  return ts;
}

hipError_t launch_merge_maps(const sos_plan_s* p, hipStream_t s) {
  char* ws = p->ws;
  if (p->ntiles256 == 0) return hipSuccess;
  // grid = the number of segments (the kernel places its second count array after the first)
  bf3::k_merge_maps<<<p->ntiles256 * kMergeSegs, 512, 0, s>>>(
      (const int2*)(ws + p->lay.tiles), (int)p->N, rank_tab(p), (uint16_t*)(ws + p->lay.mg_map),
      (int*)(ws + p->lay.mg_rank), (int*)(ws + p->lay.mg_count));
  return hipGetLastError();
}

hipError_t launch_scatter_tiles(const sos_plan_s* p, hipStream_t s) {
  const char* ws = p->ws;
  bf3::k_scatter_tiles<<<4 * p->ntiles256, 256, 0, s>>>((const float*)(ws + p->lay.g), (const int2*)(ws + p->lay.tiles),
                                                         (int)p->N, rank_tab(p), (double*)(ws + p->lay.r));
  return hipGetLastError();
}

hipError_t launch_rw_bf3(const sos_plan_s* p, void* g, bool split, hipStream_t s) {
  bf3::RwArgs a;
  const char* ws = p->ws;
  a.o.a_hi = (const __bf16*)(ws + p->lay.R_hi);
  a.o.b_hi = (const __bf16*)(ws + (p->t_cur ? p->lay.t_lo : p->lay.t_hi));
  if (split) {
    a.o.a_lo = (const __bf16*)(ws + p->lay.R_lo);
    a.o.b_lo = (const __bf16*)(ws + p->lay.t_lo);
  } else {  // second K block of each stage: the next block of the same panel
    a.o.a_lo = a.o.a_hi + bf3::TM * bf3::BK;
    a.o.b_lo = a.o.b_hi + bf3::TM * bf3::BK;
  }
  a.o.pstride = panel_stride(p->Np2 / kBlkK, 2);
  a.K = p->Np2;  // a multiple of 64: whole stages in both modes
  a.TI = (int)(p->Np / bf3::TM);
  a.TL = (int)(p->Kp2 / bf3::TM);
  a.N = (int)p->N;
  a.k = p->k;
  a.g = (float*)g;
  const bool f16 = p->prec == SOS_FP16X3;
  a.sx = scale_exponents(p);
  if (f16) {
    if (split) bf3::k_rw_bf3<true, true><<<a.TI * a.TL, bf3::NT, 0, s>>>(a);
    else bf3::k_rw_bf3<false, true><<<a.TI * a.TL, bf3::NT, 0, s>>>(a);
  } else {
    if (split) bf3::k_rw_bf3<true, false><<<a.TI * a.TL, bf3::NT, 0, s>>>(a);
    else bf3::k_rw_bf3<false, false><<<a.TI * a.TL, bf3::NT, 0, s>>>(a);
  }
  return hipGetLastError();
}

}  // namespace sos

namespace sos {

hipError_t launch_rw_adam_bf3(const sos_plan_s* p, void* W, void* m, void* v, int64_t t, const sos_adam_t& h,
                              int next_mode, hipStream_t s) {
  bf3::RwAdamArgs a;
  bf3::RwArgs& r = a.rw;
  char* ws = p->ws;
  const size_t t_read = p->t_cur ? p->lay.t_lo : p->lay.t_hi;
  const size_t t_write = p->t_cur ? p->lay.t_hi : p->lay.t_lo;
  r.o.a_hi = (const __bf16*)(ws + p->lay.R_hi);
  r.o.b_hi = (const __bf16*)(ws + t_read);
  r.o.a_lo = r.o.a_hi + bf3::TM * bf3::BK;
  r.o.b_lo = r.o.b_hi + bf3::TM * bf3::BK;
  r.o.pstride = panel_stride(p->Np2 / kBlkK, 2);
  r.K = p->Np2;
  r.TI = (int)(p->Np / bf3::TM);
  r.TL = (int)(p->Kp2 / bf3::TM);
  r.N = (int)p->N;
  r.k = p->k;
  r.g = nullptr;
  const bool f16 = p->prec == SOS_FP16X3;
  r.sx = scale_exponents(p);
  a.W = (float*)W;
  a.m = (float*)m;
  a.v = (float*)v;
  a.lr = (float)h.lr;
  a.b1 = (float)h.beta1;
  a.b2 = (float)h.beta2;
  a.eps = (float)h.eps;
  a.bc1 = (float)(1.0 - pow(h.beta1, (double)t));
  a.bc2 = (float)(1.0 - pow(h.beta2, (double)t));
  const bool split_copies = next_mode == kFwdFast || next_mode == kFwdSingle;
  a.a_hi = split_copies ? (__bf16*)(ws + p->lay.a_hi) : nullptr;
  a.a_lo = split_copies ? (__bf16*)(ws + p->lay.a_lo) : nullptr;
  a.x_f32 = next_mode == kFwdExact ? (float*)(ws + p->lay.x_f32) : nullptr;
  a.t_next = (__bf16*)(ws + t_write);
  a.aps = panel_stride(p->Kp / kBlkK, 2);
  a.xps = panel_stride(p->Kp / kBlkK, 4);
  a.tps = panel_stride(p->Np2 / kBlkK, 2);
  a.Np = p->Np;
  a.Kp = p->Kp;
  a.Np2 = p->Np2;
  a.Kp2 = p->Kp2;
  if (f16) bf3::k_rw_adam_bf3<true><<<r.TI * r.TL, bf3::NT, 0, s>>>(a);
  else bf3::k_rw_adam_bf3<false><<<r.TI * r.TL, bf3::NT, 0, s>>>(a);
  return hipGetLastError();
}

}  // namespace sos
