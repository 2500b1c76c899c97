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
// The levels are combined in FP64 with their weights (each term exact: a
// 31-bit integer times a power of two), and the tile scatters
// G_ij = 2^(e_i - 6) 2^(e_j - 6) sum_l 2^-7l T_l,ij into r in FP64.
//
// Error: per product, the digits left out and the levels dropped amount to
// at most (S + 1.05) 2^-7S of 2^(e_i + e_j), so |G_ij - G~_ij| <=
// (S + 1.05) 2^-7S K 2^(e_i + e_j), plus FP64 rounding (about 1e-12 of the
// Gram entry at S = 6 and Gaussian rows; the errors of individual digits are
// independent, so the actual error is far below this bound).
// S is a template argument: 6 (kOzSlices, the FP64-level forward), 5
// (levels s + t < 5: 15 slice products instead of 21, about 128x the error,
// for a finisher whose target lies far above it) or 4 (10 products, another
// 128x, for the start of such a finisher).
//
// Kernel: one 256 x 256 upper-triangle tile per 512-thread workgroup, 8 waves
// of 128 x 64 (4 x 2 blocks of v_mfma_i32_32x32x32_i8, two waves per SIMD),
// a 4-deep LDS ring of 32 KB stages (256 A rows and 256 B rows of 64 bytes:
// one block of 64 K of one slice pair) filled by direct global->LDS loads
// three stages ahead, each stage's loads issued after the MFMAs that follow
// the barrier releasing its buffer (7% faster than right after the barrier);
// each k-step's fragments are read from LDS while the previous k-step's
// MFMAs run.
// The K loop runs over the S(S+1)/2 slice pairs in level order, each over the
// whole K extent.  At the end of a level the lanes park their int32 sums in a
// per-tile level buffer in global memory (contiguous 1 KB stores, 1.25 MB per
// tile, read back once by the epilogue) instead of keeping FP64 totals in
// registers: that leaves room for the 128 x 64 wave tile, which reads 6 LDS
// fragments per 8 MFMAs (64 x 64 would read 4 per 4).
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

constexpr int TM = 256;             // tile rows and columns (one panel each)
constexpr int BK = kOzBK;           // K (bytes) per stage: one block of the slice layout
constexpr int NT = 512;
constexpr int NSTAGE = 4;
constexpr int ROWB = BK;            // 64 bytes per row
constexpr int HALF = TM * ROWB;     // one operand's rows of a stage (16 KB)
constexpr int STAGE = 2 * HALF;     // A and B (32 KB)
constexpr int WM = 128, WN = 64;    // wave tile: 4 x 2 blocks of 32 x 32
constexpr int BI = WM / 32, BJ = WN / 32;
constexpr int kXcds = 8;
constexpr int LOADS = 4;            // 32 KB per stage = 32 loads of 1 KB over 8 waves
constexpr int kLvlInts = TM * TM;   // one level of one tile in the level buffer
constexpr int64_t kLvlTile = (int64_t)(kOzSlices - 1) * kLvlInts;  // a tile's levels (room for the most slices)

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

// Wait until at most n of this wave's vector-memory operations are pending,
// then barrier.  Vector-memory operations complete in issue order, so the
// level-buffer stores issued after a stage's loads are waited for too.
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

// LDS slot (l & 3) of row r holds 16-byte chunk (l & 3) ^ ((r >> 2) & 3), so
// 16 consecutive rows read at one chunk fall in 16 distinct bank groups.
// Wave w moves rows 64 (w % 4) .. +63 of A (w < 4) or of B (w >= 4), 16 rows
// (1 KB) per instruction.
__device__ __forceinline__ void issue_stage(unsigned st_lds, const int8_t* a_slice, const int8_t* b_slice,
                                            int64_t pstride, int64_t arow0, int64_t brow0, int64_t kb) {
  const int wave = threadIdx.x >> 6, l = threadIdx.x & 63;
  const unsigned wave_u = __builtin_amdgcn_readfirstlane((unsigned)wave);
  const bool is_a = wave < 4;
  const int8_t* base = is_a ? a_slice + (arow0 / TM) * pstride : b_slice + (brow0 / TM) * pstride;
  const unsigned m = st_lds + (wave_u < 4 ? 0u : (unsigned)HALF) + (wave_u & 3u) * (64u * ROWB);
#pragma unroll
  for (int q = 0; q < LOADS; ++q) {
    const int r = (wave & 3) * 64 + q * 16 + (l >> 2);
    const int chunk = (l & 3) ^ ((r >> 2) & 3);
    dma16((const char*)(base + (kb * TM + r) * BK + chunk * 16), m + q * 1024u);
  }
}

// Fragments of one k-step of 32: per lane one 16 bytes per 32-row block of
// A and of B (row l % 32 of the block, bytes 16 (l / 32) .. +15 of the
// k-step, for both operands alike).
struct Frag {
  i32x4 a[BI], b[BJ];
};

__device__ __forceinline__ void read_frag(Frag& f, const char* st, int ks, int wm, int wn) {
  const int l = threadIdx.x & 63;
  const int off = (l & 31) * ROWB + (((2 * ks + (l >> 5)) ^ ((l >> 2) & 3)) << 4);
#pragma unroll
  for (int q = 0; q < BI; ++q) f.a[q] = *(const i32x4*)(st + (wm * WM + q * 32) * ROWB + off);
#pragma unroll
  for (int q = 0; q < BJ; ++q) f.b[q] = *(const i32x4*)(st + HALF + (wn * WN + q * 32) * ROWB + off);
}

__device__ __forceinline__ void mma_frag(const Frag& f, i32x16 (&acc)[BI][BJ]) {
#pragma unroll
  for (int bi = 0; bi < BI; ++bi)
#pragma unroll
    for (int bj = 0; bj < BJ; ++bj)
      acc[bi][bj] = __builtin_amdgcn_mfma_i32_32x32x32_i8(f.a[bi], f.b[bj], acc[bi][bj], 0, 0, 0);
}

// Interleave: one MFMA, one LDS read, ... so that the reads of the next
// fragments run under the current MFMAs (masks: 0x008 MFMA, 0x100 LDS read).
__device__ __forceinline__ void interleave_reads() {
  constexpr int NMFMA = BI * BJ, NREAD = BI + BJ;
#pragma unroll
  for (int q = 0; q < NREAD; ++q) {
    __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
    __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
  }
  __builtin_amdgcn_sched_group_barrier(0x008, NMFMA - NREAD, 0);
}

struct Args {
  const int8_t* oz;       // slice s at oz + s * slice_bytes
  int64_t slice_bytes;
  int64_t nkb;            // Kp / 64
  int64_t pstride;        // bytes per padded panel
  const int2* tiles;      // 256 x 256 upper-triangle tile list
  int ntiles, N;
  const double* scale;    // 2^(e_i - 6) per row (NaN: the row holds a non-finite entry)
  int* lvl;               // level buffer: per tile (kLvlTile ints), levels 0 .. S-2 of its int32 sums
  RankTab rk;
  double* r;
  // the plan's merge maps (see kMergeRows), or nullptr: every entry ranked and added on its own
  const uint16_t* mmap;
  const int* mrank;
  const int* mcount;
};

// FP64 add into LDS (ds_add_f64: no return value is asked for).
__device__ __forceinline__ void lds_add(double* p, double x) {
  __hip_atomic_fetch_add(p, x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Accumulator registers (bi, bj, 4 g .. 4 g + 3) of lane l sit at ints
// 4 (((bi BJ + bj) 4 + g) 64 + l) of the wave's 8192-int share of a level, as
// one 4-int vector: one 1 KB contiguous store per (bi, bj, g) across the wave.
// lane_off = wave 8192 + 4 l; the offsets of (bi, bj, g) are constants.
__device__ __forceinline__ int lvl_const(int bi, int bj, int g) { return ((bi * BJ + bj) * 4 + g) * 256; }

// Park the accumulators at `base` (this tile's level buffer for one level).
// The empty asm keeps the per-lane offset from being hoisted into 32
// precomputed addresses that would stay live through the K loop.
__device__ __forceinline__ void park_level(int* base, int lane_off, i32x16 (&acc)[BI][BJ]) {
  asm volatile("" : "+v"(lane_off));
#pragma unroll
  for (int bi = 0; bi < BI; ++bi)
#pragma unroll
    for (int bj = 0; bj < BJ; ++bj) {
#pragma unroll
      for (int gq = 0; gq < 4; ++gq) {
        const i32x4 x = {acc[bi][bj][4 * gq], acc[bi][bj][4 * gq + 1], acc[bi][bj][4 * gq + 2],
                         acc[bi][bj][4 * gq + 3]};
        *(i32x4*)(base + lane_off + lvl_const(bi, bj, gq)) = x;
      }
      acc[bi][bj] = i32x16{};
    }
}

// One pass of the merged epilogue (see k_gram_i8): segments h and 2 + h.
// H is a template argument so that the accumulator blocks 2H, 2H + 1 are
// named by compile-time indices (a run-time pass index would put the
// accumulators in scratch memory).
template <int H, int S>
__device__ __forceinline__ void merge_pass(const Args& g, int v, int wm, int wn, int64_t arow0, int64_t brow0,
                                           const int* lvl_tile, int lane_off, char* ring, double* slots_w,
                                           i32x16 (&acc)[BI][BJ]) {
  constexpr int RK = kMergeSlots / NT;
  constexpr int h = H;
  const int l = threadIdx.x & 63;
  const int sa = v * kMergeSegs + h, sb = v * kMergeSegs + 2 + h;
  asm volatile("" ::: "memory");  // this pass's loads stay in it: registers for one pass at a time
  const int na = g.mcount[sa], nb = g.mcount[sb];
  int rka[RK];
#pragma unroll
  for (int it = 0; it < RK; ++it)  // every entry of the list, used or not (inside it), without branches
    rka[it] = g.mrank[(size_t)sa * kMergeSlots + threadIdx.x + it * NT];
  __syncthreads();  // nobody reads the ring (the last stage, or the previous pass's slots) any more
  double* const s0 = (double*)ring;
  double* const s1 = (double*)(ring + kMergeSlots * 8);
  for (int q = threadIdx.x; q < na; q += NT) s0[q] = 0.0;
  for (int q = threadIdx.x; q < nb; q += NT) s1[q] = 0.0;
  __syncthreads();
  const int seg = 2 * wm + h;
  const uint16_t* mp = g.mmap + (size_t)(v * kMergeSegs + seg) * kMergeSeg;
#pragma unroll
  for (int bj = 0; bj < BJ; ++bj) {
    const int col = wn * WN + bj * 32 + (l & 31);
    const int j = (int)brow0 + col;
    const double sj = j < g.N ? g.scale[j] : 0.0;
#pragma unroll
    for (int bb = 0; bb < 2; ++bb) {
      const int bi = 2 * h + bb;
#pragma unroll
      for (int gq = 0; gq < 4; ++gq) {
        i32x4 lv[S - 1];
#pragma unroll
        for (int q = 0; q < S - 1; ++q)
          lv[q] = *(const i32x4*)(lvl_tile + q * kLvlInts + lane_off + lvl_const(bi, bj, gq));
        unsigned sl[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int row = wm * WM + bi * 32 + gq * 8 + (l >> 5) * 4 + u;
          sl[u] = mp[(row - seg * kMergeRows) * TM + col];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int i = (int)arow0 + wm * WM + bi * 32 + gq * 8 + (l >> 5) * 4 + u;
          if (i < g.N && j < g.N && i <= j) {
            double tot = 0.0, w = 1.0;
#pragma unroll
            for (int q = 0; q < S - 1; ++q) {
              tot = fma((double)lv[q][u], w, tot);
              w *= 0x1p-7;
            }
            tot = fma((double)acc[bi][bj][4 * gq + u], w, tot);
            const double x = ((i == j) ? 1.0 : 2.0) * (tot * g.scale[i] * sj);
            if (sl[u] < (unsigned)kMergeSlots) lds_add(slots_w + sl[u], x);
            else unsafeAtomicAdd(g.r + pair_rank(g.rk, i, j), x);
          }
        }
      }
    }
  }
  // the second list now, still before this pass's first atomic
  int rkb[RK];
#pragma unroll
  for (int it = 0; it < RK; ++it) rkb[it] = g.mrank[(size_t)sb * kMergeSlots + threadIdx.x + it * NT];
  __syncthreads();
  // per segment, all of this thread's slot sums first, into registers of
  // their own, then the atomics
  double x[RK];
#pragma unroll
  for (int it = 0; it < RK; ++it) {
    const int q = threadIdx.x + it * NT;
    const double a = s0[q];  // q < kMergeSlots: inside the slots, used or not
    x[it] = q < na ? a : 0.0;
  }
#pragma unroll
  for (int it = 0; it < RK; ++it)
    if (x[it] != 0.0) unsafeAtomicAdd(g.r + rka[it], x[it]);
#pragma unroll
  for (int it = 0; it < RK; ++it) {
    const int q = threadIdx.x + it * NT;
    const double b = s1[q];
    x[it] = q < nb ? b : 0.0;
  }
#pragma unroll
  for (int it = 0; it < RK; ++it)
    if (x[it] != 0.0) unsafeAtomicAdd(g.r + rkb[it], x[it]);
}

template <bool MERGE, int S>
__global__ __launch_bounds__(NT) void k_gram_i8(Args g) {
  static_assert(S >= 2 && S <= kOzSlices, "the level buffer and the slice arrays hold at most kOzSlices");
  __shared__ __attribute__((aligned(16))) char ring[NSTAGE * STAGE];
  const int v = xcd_order(blockIdx.x, g.ntiles);
  const int2 t = g.tiles[v];
  const int64_t arow0 = (int64_t)t.x * TM, brow0 = (int64_t)t.y * TM;
  const int wave = threadIdx.x >> 6;
  const int wm = wave >> 2, wn = wave & 3;  // 2 x 4 waves of 128 x 64
  i32x16 acc[BI][BJ];
#pragma unroll
  for (int bi = 0; bi < BI; ++bi)
#pragma unroll
    for (int bj = 0; bj < BJ; ++bj) acc[bi][bj] = i32x16{};
  const int64_t nkb = g.nkb;
  const int64_t nv = (int64_t)(S * (S + 1) / 2) * nkb;  // stages over all segments
  const unsigned ring_lds = __builtin_amdgcn_readfirstlane((unsigned)(uintptr_t)(lds_t)ring);
  int* const lvl_tile = g.lvl + (int64_t)v * kLvlTile;
  const int lane_off = wave * (kLvlInts / 8) + 4 * (threadIdx.x & 63);
  Cursor in, cu;  // next stage to issue, stage to compute
  // Software pipeline: the ring holds four stages, loads run three stages
  // ahead, and the fragments of each k-step are read from LDS while the
  // MFMAs of the previous k-step run.  Entering iteration vt, the fragments
  // of (vt, k-step 0) are in registers.
  for (int q = 0; q < NSTAGE; ++q) {
    if (q < nv) {
      issue_stage(ring_lds + q * STAGE, g.oz + in.s * g.slice_bytes, g.oz + in.t * g.slice_bytes, g.pstride, arow0,
                  brow0, in.kb);
      in.advance(nkb);
    }
  }
  // stage 0 must have landed; stages 1 .. 3 may be in flight
  if (nv >= 4) wait_vm_barrier<3 * LOADS>();
  else if (nv == 3) wait_vm_barrier<2 * LOADS>();
  else if (nv == 2) wait_vm_barrier<LOADS>();
  else wait_vm_barrier<0>();
  Frag f0, f1;
  read_frag(f0, ring, 0, wm, wn);
  for (int64_t vt = 0; vt < nv; ++vt) {
    const char* st = ring + (vt % NSTAGE) * STAGE;
    // k-step 0 of stage vt, reading k-step 1
    read_frag(f1, st, 1, wm, wn);
    mma_frag(f0, acc);
    interleave_reads();
    __builtin_amdgcn_sched_barrier(0);
    if (vt + 1 < nv) {
      // stage vt+1 must have landed (up to two later stages may be in flight);
      // after the barrier every wave has read all of stage vt
      const int64_t later = nv - 1 - (vt + 1) < 2 ? nv - 1 - (vt + 1) : 2;
      if (later == 2) wait_vm_barrier<2 * LOADS>();
      else if (later == 1) wait_vm_barrier<LOADS>();
      else wait_vm_barrier<0>();
    }
    __builtin_amdgcn_sched_barrier(0);
    // k-step 1 of stage vt, reading k-step 0 of stage vt+1 (after the last
    // stage this reads a buffer of the ring whose data goes unused)
    read_frag(f0, ring + ((vt + 1) % NSTAGE) * STAGE, 0, wm, wn);
    mma_frag(f1, acc);
    interleave_reads();
    __builtin_amdgcn_sched_barrier(0);
    // refill the buffer of stage vt (free since the barrier) with stage
    // vt + 4, after this k-step's MFMAs rather than before them
    if (vt + NSTAGE < nv) {
      issue_stage(ring_lds + (unsigned)(vt % NSTAGE) * STAGE, g.oz + in.s * g.slice_bytes,
                  g.oz + in.t * g.slice_bytes, g.pstride, arow0, brow0, in.kb);
      in.advance(nkb);
    }
    __builtin_amdgcn_sched_barrier(0);
    // park the level's exact sums in the tile's level buffer and start the next
    if (cu.level_ends(nkb) && cu.lvl < S - 1) park_level(lvl_tile + cu.lvl * kLvlInts, lane_off, acc);
    cu.advance(nkb);
  }
  // With merge maps: the tile in two passes over its 64-row segments, {0, 2}
  // then {1, 3}, so that two segments' FP64 slots (2 x 64 KB) fill the ring.
  // In pass h a wave of row half wm adds its row blocks 2h and 2h + 1 (the
  // rows of segment 2 wm + h), combined as below, into the slot its map names;
  // then each slot in use goes into r by one atomic, at the coefficient of
  // the segment's rank list.  Each pass loads its rank-list entries at its
  // start: loads and atomics complete in order, so the pass waits once for
  // the previous one's atomics, not once per atomic.
  const int l = threadIdx.x & 63;
  if constexpr (MERGE) {
    static_assert(kMergeRows * 2 == WM && BI == 4 && kMergeSlots % NT == 0, "a segment is two row blocks of a wave");
    static_assert(2 * kMergeSlots * 8 <= NSTAGE * STAGE, "two segments' slots fill at most the ring");
    double* const slots_w = (double*)(ring + wm * (kMergeSlots * 8));  // this wave's segment in a pass
    merge_pass<0, S>(g, v, wm, wn, arow0, brow0, lvl_tile, lane_off, ring, slots_w, acc);
    merge_pass<1, S>(g, v, wm, wn, arow0, brow0, lvl_tile, lane_off, ring, slots_w, acc);
  } else {
    // combine the levels in FP64 (each term a 31-bit integer times a power of
    // two), scale by the row exponents, scatter.  Register (bi, bj, 4 gq + u)
    // of lane l holds row 32 bi + 8 gq + 4 (l / 32) + u and column 32 bj + l % 32
    // of the wave's 128 x 64 share.
#pragma unroll
    for (int bj = 0; bj < BJ; ++bj) {
      const int j = (int)brow0 + wn * WN + bj * 32 + (l & 31);
      const double sj = j < g.N ? g.scale[j] : 0.0;
#pragma unroll
      for (int bi = 0; bi < BI; ++bi)
#pragma unroll
        for (int gq = 0; gq < 4; ++gq) {
          i32x4 lv[S - 1];
#pragma unroll
          for (int q = 0; q < S - 1; ++q) lv[q] = *(const i32x4*)(lvl_tile + q * kLvlInts + lane_off + lvl_const(bi, bj, gq));
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int i = (int)arow0 + wm * WM + bi * 32 + gq * 8 + (l >> 5) * 4 + u;
            if (i < g.N && j < g.N && i <= j) {
              double tot = 0.0, w = 1.0;
#pragma unroll
              for (int q = 0; q < S - 1; ++q) {
                tot = fma((double)lv[q][u], w, tot);
                w *= 0x1p-7;
              }
              tot = fma((double)acc[bi][bj][4 * gq + u], w, tot);
              const double wgt = (i == j) ? 1.0 : 2.0;
              unsafeAtomicAdd(g.r + pair_rank(g.rk, i, j), wgt * (tot * g.scale[i] * sj));
            }
          }
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

// Digits of a 64 x 64 tile of W into the first S slice arrays (padding rows
// and columns get zero digits).  Loads are coalesced along rows; the digits
// go through LDS so that every slice is written in 16-byte chunks of the
// blocked layout.
template <int S>
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

hipError_t launch_oz_slices(const sos_plan_s* p, const float* W, hipStream_t s, int slices) {
  if (slices != kOzSlices && slices != 5 && slices != 4) return hipErrorInvalidValue;
  char* ws = p->ws;
  int* ex = (int*)(ws + p->lay.oz_exp);
  i8::k_oz_scale<<<(unsigned)p->N, 256, 0, s>>>(W, (int)p->N, p->k, ex, (double*)(ws + p->lay.oz_scale));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const dim3 grid((unsigned)(p->Kp / 64), (unsigned)(p->Np / 64));
  int8_t* oz = (int8_t*)(ws + p->lay.oz);
  const int64_t sb = (int64_t)p->lay.oz_slice, ps = oz_panel_stride(p->Kp);
  if (slices == 4) i8::k_oz_slice<4><<<grid, 256, 0, s>>>(W, (int)p->N, p->k, ex, oz, sb, ps);
  else if (slices == 5) i8::k_oz_slice<5><<<grid, 256, 0, s>>>(W, (int)p->N, p->k, ex, oz, sb, ps);
  else i8::k_oz_slice<kOzSlices><<<grid, 256, 0, s>>>(W, (int)p->N, p->k, ex, oz, sb, ps);
  return hipGetLastError();
}

hipError_t launch_gram_i8(const sos_plan_s* p, hipStream_t s, int slices) {
  if (slices != kOzSlices && slices != 5 && slices != 4) return hipErrorInvalidValue;
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
  g.lvl = (int*)(ws + p->lay.oz_lvl);
  g.rk = rank_tab(p);
  g.r = (double*)(ws + p->lay.r);
  g.mmap = p->merge_ready ? (const uint16_t*)(ws + p->lay.mg_map) : nullptr;
  g.mrank = p->merge_ready ? (const int*)(ws + p->lay.mg_rank) : nullptr;
  g.mcount = p->merge_ready ? (const int*)(ws + p->lay.mg_count) : nullptr;
  if (slices == 4) {
    if (g.mmap) i8::k_gram_i8<true, 4><<<g.ntiles, i8::NT, 0, s>>>(g);
    else i8::k_gram_i8<false, 4><<<g.ntiles, i8::NT, 0, s>>>(g);
  } else if (slices == 5) {
    if (g.mmap) i8::k_gram_i8<true, 5><<<g.ntiles, i8::NT, 0, s>>>(g);
    else i8::k_gram_i8<false, 5><<<g.ntiles, i8::NT, 0, s>>>(g);
  } else {
    if (g.mmap) i8::k_gram_i8<true, kOzSlices><<<g.ntiles, i8::NT, 0, s>>>(g);
    else i8::k_gram_i8<false, kOzSlices><<<g.ntiles, i8::NT, 0, s>>>(g);
  }
  return hipGetLastError();
}

}  // namespace sos
