// Internal declarations shared by the host plan, the C ABI and the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/sos.h"

namespace sos {

// Ranking code layout.  Every basis monomial alpha gets n 4-bit fields:
//   field 0 = |alpha|, field f (1..n-1) = alpha_{f+1} + ... + alpha_n
// (suffix sums).  Fields are additive, and with 2d <= 15 the sum of two
// codes never carries out of a field, so code(alpha_i) + code(alpha_j) is
// the code of alpha_i + alpha_j.  Fields are packed three to a 12-bit group;
// each 32-bit word holds two groups in its two 16-bit halves.  The rank of a
// degree-<=2d monomial is a sum over groups of a 4096-entry table lookup
// (see plan.cpp for the closed form the tables hold).
constexpr int kFieldsPerGroup = 3;
constexpr int kGroupEntries = 4096;
constexpr int kMaxWords = 3;     // n <= 16  ->  at most 6 groups

// The plan's scalar area (doubles): [0] loss, [1] ||p||^2, [2] two int32
// scale exponents of fp16 plans (sW: the W copies hold 2^sW w; sR: R holds
// 2^sR r), [8 .. 520) the partial sums of the loss reduction, [1024 .. 1280)
// block maxima (as floats) for the fp16 scales.
constexpr int kScalScales = 2;
constexpr int kScalMax = 1024;
constexpr int kScalDoubles = 2048;

// Tile sizes shared by host (padding, grids) and device.
constexpr int kPadRows = 256;    // operand rows padded to this multiple (zero rows)
constexpr int kPadK = 64;        // operand K extents padded to this multiple (zero columns)

// Panel-blocked layout of the split-bf16 operands: rows in panels of 256,
// K in blocks of 16; block (panel, kb) is 256 rows x 16 elements stored
// contiguously (8 KB of bf16), blocks of one panel consecutive in kb.  A
// GEMM stage then reads one contiguous 8 KB block per array.
// Consecutive panels are kPanelPadBytes further apart than their data, so
// the blocks that concurrent tiles read at one K (one per panel) do not all
// sit at the same offset modulo the L2 channel interleave.
constexpr int kBlkRows = 256;
constexpr int kBlkK = 16;
constexpr int kPanelPadBytes = 4096;

// Ozaki-split forward (an FP64-accurate Gram from int8 MFMA): each row i of
// the FP32 W is scaled by 2^-e_i, e_i the least power of two above the row's
// largest magnitude, and cut into kOzSlices signed digits of 7 bits
// (|digit| <= 64), most significant first.  The slices are int8 arrays in a
// panel-blocked layout like the bf16 operands: rows in panels of 256, K in
// blocks of 64, block (panel, kb) = 256 rows x 64 bytes contiguous (16 KB).
// A slice product summed over K is exact in int32 while
// kOzSlices * Kp * 64^2 < 2^31 (the level sums below add up to kOzSlices
// products), i.e. for K extents below 87,381.
constexpr int kOzSlices = 6;
constexpr int kOzBK = 64;
__host__ __device__ inline int64_t oz_panel_stride(int64_t Kp) {  // bytes
  return (Kp / kOzBK) * kBlkRows * kOzBK + kPanelPadBytes;
}
__host__ __device__ inline int64_t oz_off(int64_t row, int64_t k, int64_t pstride) {
  return (row / kBlkRows) * pstride + ((k / kOzBK) * kBlkRows + row % kBlkRows) * kOzBK + k % kOzBK;
}
constexpr int64_t kOzMaxK = ((int64_t(1) << 31) - 1) / (kOzSlices * 64 * 64);

// Merge maps of the split plans' gram epilogue.  Each 256 x 256 tile is taken
// in four segments of 64 rows (16,384 pairs); at n = 12, d = 6 the pairs of
// a segment fall on about 4,600 distinct coefficients (3.6 pairs each, up to
// ~7,900 distinct).  A map gives every pair of a segment its slot: the index
// of its coefficient among the segment's distinct ones in ascending order
// (kMergeSkip: outside the upper triangle or past N; kMergeDirect: beyond the
// slot capacity, ranked and added on its own).  The epilogue adds the pairs
// into FP64 slots in LDS and then each slot into r by one global atomic, to
// the coefficient that the segment's rank list names.  Built on the GPU when
// the plan is bound.
constexpr int kMergeRows = 64;
constexpr int kMergeSeg = kMergeRows * kBlkRows;   // pairs per segment
constexpr int kMergeSegs = kBlkRows / kMergeRows;  // segments per tile
constexpr int kMergeSlots = 8192;                  // FP64 slots per segment (64 KB of LDS)
constexpr uint16_t kMergeSkip = 0xFFFF;
constexpr uint16_t kMergeDirect = 0xFFFE;
// Merging pays where it saves atomics: the plan uses the maps only when the
// pairs of the upper triangle are at least kMergeMinRatio times the atomics
// left after merging (n = 12, d = 6: 3.6; quartics in 99 variables: ~1.1).
constexpr double kMergeMinRatio = 1.5;

// Generic gram (kernels.hip, FP32 and FP64 plans): 128 x 128 upper tiles;
// when they alone give fewer than kGramMinBlocks blocks, the contraction is
// split into slices of kslice (a multiple of 64), one block per (tile, slice).
constexpr int kGenericTile = 128;
constexpr int kGramMinBlocks = 512;
inline int64_t generic_gram_kslice(int64_t Np, int64_t Kp) {
  const int64_t T = Np / kGenericTile, tiles = T * (T + 1) / 2;
  int64_t splits = 1;
  if (tiles < kGramMinBlocks) splits = std::min<int64_t>((kGramMinBlocks + tiles - 1) / tiles, Kp / 64);
  if (splits < 1) splits = 1;
  const int64_t ks = (Kp + splits - 1) / splits;
  return (ks + 63) / 64 * 64;
}
inline int64_t generic_gram_splits(int64_t Np, int64_t Kp) {
  const int64_t ks = generic_gram_kslice(Np, Kp);
  return (Kp + ks - 1) / ks;
}

// Grouped serving kernels: the contraction length a block covers, and the
// number of such slices (each with its own partial result) for length len.
constexpr int kBatchSlice = 256;    // K slices of the Gram
constexpr int kBatchSliceJ = 128;   // slices of the backward's contraction index
__host__ __device__ inline int batch_slices(int len) { return (len + kBatchSlice - 1) / kBatchSlice; }
__host__ __device__ inline int batch_slices_j(int len) { return (len + kBatchSliceJ - 1) / kBatchSliceJ; }
__host__ __device__ inline int64_t panel_stride(int64_t nkb, int elem_bytes) {
  return nkb * kBlkRows * kBlkK + kPanelPadBytes / elem_bytes;
}
__host__ __device__ inline int64_t blk_off(int64_t row, int64_t k, int64_t pstride) {
  return (row / kBlkRows) * pstride + ((k / kBlkK) * kBlkRows + row % kBlkRows) * kBlkK + k % kBlkK;
}

// ---------------------------------------------------------------------------
// Ranking of pair sums on the device.  plan.cpp builds one of two encodings:
//
//  dense (n <= 16): the additive 4-bit suffix-sum codes above; the rank of
//    alpha_i + alpha_j is a sum of group-table lookups at code_i + code_j.
//  sparse (n > 16, 2d <= 8, n <= 255): each basis monomial is its ascending
//    list of variables (byte p holds v_p + 1, 0 = none), the product's list
//    is the merge of the two, and with D = 2d, t the merged length and
//    v_0 = 0, m_p = t - p,
//      rank = C(n+D, D) - C(n+t, t)
//           + sum_{p=1..t} [ C(n - v_{p-1} + m_p, m_p + 1) - C(n - v_p + m_p, m_p + 1) ],
//    the number of higher-degree monomials plus, position by position, the
//    number of same-degree lists that agree before p and are smaller at p
//    (a hockey-stick sum of multiset counts).  Binomials come from a table
//    C[x][y], 0 <= x <= n + D, 0 <= y <= D.
// ---------------------------------------------------------------------------
struct RankTab {
  const uint32_t* __restrict__ codes;   // dense: N x nwords; sparse: N packed lists
  const int32_t* __restrict__ tables;   // dense: ngroups x 4096, then the field terms (16 x 16);
                                        // sparse: binomial table (n + D + 1) x (D + 1)
  int nwords, ngroups;
  int sparse, n, D, total;              // sparse only (total = C(n + D, D))
  int ntab;                             // entries of the table a kernel may stage in LDS:
                                        // dense: the 256 field terms; sparse: the binomial table
};

constexpr int kFieldTerms = 256;        // dense: F[f * 16 + v], f < 16, v < 16
constexpr int kStageTabMax = 2376;      // largest ntab: (255 + 8 + 1) x (8 + 1)

// The field-term table of a dense plan, or the binomial table of a sparse one.
__host__ __device__ inline const int32_t* stage_tab(const RankTab& t) {
  return t.sparse ? t.tables : t.tables + (size_t)t.ngroups * kGroupEntries;
}

// Rank of alpha_i + alpha_j for dense codes from the per-field terms:
// rank = sum over fields f < n of F[f][suffix sum f] (the closed form of
// plan.cpp, field by field).  Field f sits in group f / 3 (4 bits each),
// two groups per word.  At most 2d + 1 distinct values per field, so a
// wave's lookups of one field touch consecutive words.
__device__ __forceinline__ int dense_rank_fields(const uint32_t* ci, const uint32_t* cj, int n, const int32_t* F) {
  uint32_t s[kMaxWords];
#pragma unroll
  for (int w = 0; w < kMaxWords; ++w) s[w] = ci[w] + cj[w];
  int r = 0;
#pragma unroll
  for (int f = 0; f < 16; ++f) {
    if (f < n) {
      const int g = f / kFieldsPerGroup, w = g >> 1, sh = 16 * (g & 1) + 4 * (f % kFieldsPerGroup);
      r += F[f * 16 + ((s[w] >> sh) & 15u)];
    }
  }
  return r;
}

// Rank of the sum of two sparse monomials (ascending variable lists packed
// one byte per factor, byte = variable + 1, at most four factors each) through
// binom(x, y) = C(x, y).  The merged list is walked once, the term of each
// factor added as it is taken; no per-thread array (which would live in
// scratch memory).
__device__ __forceinline__ int packed_len(uint32_t x) {
  return (x != 0u) + ((x >> 8) != 0u) + ((x >> 16) != 0u) + ((x >> 24) != 0u);
}

template <class Binom>
__device__ __forceinline__ int sparse_pair_rank(uint32_t a, uint32_t b, int n, int total, const Binom& binom) {
  const int len = packed_len(a) + packed_len(b);
  int r = total - binom(n + len, len);
  int prev = 0;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    if (q < len) {
      const uint32_t va = a & 0xFFu, vb = b & 0xFFu;
      const bool take_a = va != 0 && (vb == 0 || va <= vb);
      const int v = (int)(take_a ? va : vb) - 1;
      if (take_a) a >>= 8;
      else b >>= 8;
      const int m = len - 1 - q;
      r += binom(n - prev + m, m + 1) - binom(n - v + m, m + 1);
      prev = v;
    }
  }
  return r;
}

// The codes of row i, loaded once for many partners j.
struct RankRow {
  uint32_t c[kMaxWords];
};

__device__ __forceinline__ RankRow rank_row(const RankTab& t, int i) {
  RankRow r;
#pragma unroll
  for (int w = 0; w < kMaxWords; ++w) r.c[w] = (w < t.nwords) ? t.codes[(size_t)i * t.nwords + w] : 0u;
  return r;
}

__device__ __forceinline__ int rank_binom(const RankTab& t, int x, int y) { return t.tables[x * (t.D + 1) + y]; }

__device__ __forceinline__ int pair_rank_row(const RankTab& t, const RankRow& ri, int j) {
  if (!t.sparse) {
    int r = 0;
#pragma unroll
    for (int w = 0; w < kMaxWords; ++w) {
      if (w < t.nwords) {
        const uint32_t s = ri.c[w] + t.codes[(size_t)j * t.nwords + w];
        r += t.tables[(2 * w) * kGroupEntries + (s & 0xFFFu)];
        if (2 * w + 1 < t.ngroups) r += t.tables[(2 * w + 1) * kGroupEntries + ((s >> 16) & 0xFFFu)];
      }
    }
    return r;
  }
  return sparse_pair_rank(ri.c[0], t.codes[j], t.n, t.total, [&](int x, int y) { return rank_binom(t, x, y); });
}

__device__ __forceinline__ int pair_rank(const RankTab& t, int i, int j) {
  return pair_rank_row(t, rank_row(t, i), j);
}

struct Layout {
  // byte offsets into the workspace
  size_t codes = 0, tables = 0, r = 0, scal = 0;
  size_t r32 = 0;                // FP32 copy of r (FP32 and split plans; read by the gather)
  size_t tiles = 0;              // (I, J) pairs of 256-row upper-triangle tiles, int2
  size_t a_hi = 0, a_lo = 0;     // W operand copies, rows = Np, ld = Kp   (forward A/B)
  size_t t_hi = 0, t_lo = 0;     // W^T operand copies, rows = Kp2, ld = Np2 (backward B)
  size_t R_hi = 0, R_lo = 0;     // R operand, rows = Np, ld = Np2           (backward A)
  size_t a_f32 = 0;              // FP32 padded W (split-precision plans), rows = Np, ld = Kp
  size_t x_f32 = 0;              // FP32 W, panel-blocked (exact forward), rows = Np, K extent Kp
  size_t g = 0;                  // gradient scratch, N x k in W's type
  size_t oz = 0;                 // Ozaki slices: kOzSlices arrays of oz_slice bytes (FP32-master plans)
  size_t oz_slice = 0;           // bytes per slice array: (Np / 256) panels of oz_panel_stride(Kp)
  size_t oz_exp = 0;             // N int32: row exponents e_i
  size_t oz_scale = 0;           // N doubles: 2^(e_i - 6), NaN for a row holding a non-finite entry
  size_t oz_lvl = 0;             // int32 level sums 0 .. kOzSlices-2 of every 256 x 256 gram tile
  // grouped (serving) path, FP32 plans with N <= SOS_BATCH_MAX_N only
  size_t bG = 0;                 // FP64 partial Gram per K slice: batch_slices(k) x P, entries in pair-list order
  size_t pair_pos = 0;           // N x N int32: position of pair (min(i,j), max(i,j)) in the pair lists
  size_t rank_map = 0;           // N x N int32: coefficient index of alpha_i + alpha_j (R_ij = r[map])
  size_t bg = 0;                 // FP32 partial gradient per j slice: batch_slices_j(N) x N x k
  size_t bpart = 0;              // FP64 loss partials, one per coefficient block of 256
  size_t bcount = 0;             // u32 arrival counter of those blocks (zero between calls)
  size_t pair_off = 0;           // M + 1 int32: pairs of coefficient m are pair_idx[off[m] .. off[m+1])
  size_t pair_idx = 0;           // N (N + 1) / 2 int32: i * N + j (i <= j), bit 31 set when i < j
  size_t bhdr = 0;               // BatchHeader: sizes and the places of the arrays above
  // deterministic forward of FP32 and FP64 plans with N <= SOS_BATCH_MAX_N
  // (uses pair_off / pair_idx above): the gram's slices, splits x N x N doubles
  size_t det_G = 0;
  // split plans: merge maps of the gram epilogue (ntiles256 x 65,536 u16),
  // the rank list of every segment (kMergeSlots int32 each), its length, and
  // (second array of the same size) the r atomics the segment issues
  size_t mg_map = 0, mg_rank = 0, mg_count = 0;
  size_t bytes = 0;
};

// A serving plan's constants, kept in its workspace (written at bind) so that
// a grouped launch passes only a few pointers per problem.  Array places are
// byte offsets from the header itself; v is the byte offset of the second
// Adam moment from the first inside a problem's state.
struct BatchHeader {
  int32_t N, M, k, sg, sr, pad;
  int64_t v;
  int64_t r, Gp, pair_pos, rank_map, gp, part, count, pair_off, pair_idx;
};

}  // namespace sos

struct sos_plan_s {
  int n = 0, d = 0, k = 0, prec = 0;
  int64_t N = 0, M = 0;
  int ngroups = 0, nwords = 0;
  bool sparse = false;             // sparse ranking encoding (n > 16)
  std::vector<uint8_t> basis;      // N x n exponents, library order
  std::vector<uint32_t> codes;     // N x nwords
  std::vector<int32_t> tables;     // ngroups x 4096
  // padded extents
  int64_t Np = 0;    // N rounded up to kPadRows   (rows of W copies, rows of R)
  int64_t Kp = 0;    // k rounded up to kPadK      (ld of W copies)
  int64_t Np2 = 0;   // N rounded up to kPadK      (ld of R and W^T copies)
  int64_t Kp2 = 0;   // k rounded up to kPadRows   (rows of W^T copies)
  sos::Layout lay;
  int ntiles256 = 0;               // upper-triangle tiles of 256 x 256
  std::vector<int32_t> tile_list;  // 2 * ntiles256
  bool batchable = false;          // grouped (serving) calls supported
  bool det_ok = false;             // SOS_FLAG_DETERMINISTIC supported (pair lists, det_G)
  bool merge_ready = false;        // the workspace holds the gram's merge maps (built at bind)
  sos::BatchHeader bhdr{};         // uploaded to lay.bhdr at bind (batchable plans)
  // operand copies left by the last fused step (single-product backward with
  // Adam in its epilogue): valid for W pointer copies_W and forward mode
  // copies_mode until another call rebuilds the copies
  bool copies_valid = false;
  const void* copies_W = nullptr;
  int copies_mode = 0;
  int t_cur = 0;                   // transposed copy for the next backward: 0 = t_hi, 1 = t_lo
  std::vector<int32_t> pair_off, pair_idx, pair_pos, rank_map;
  // two-layer network (plans (n - 1, 2)): basis row <-> variable pair maps,
  // built on first use; net_maps_at = the state buffer they were uploaded to
  std::vector<int32_t> net_rowpair, net_rowmap;
  const void* net_maps_at = nullptr;
  size_t state_bytes = 0;
  char* ws = nullptr;
  size_t ws_size = 0;
  bool bound = false;
  // kernel timing (sos_timing)
  struct TimedLaunch { int cls; hipEvent_t a, b; };
  bool timing = false;
  std::vector<TimedLaunch> timed;
  std::vector<hipEvent_t> event_pool;
  ~sos_plan_s();
};

namespace sos {

// host plan (plan.cpp)
int plan_create(int n, int d, int rank, int prec, sos_plan_s** out);
void enumerate_monomials(int n, int D, std::vector<uint8_t>& out);  // library order
int64_t rank_closed_form(int n, int D, const uint8_t* e);

// Order of the gram's upper-triangle tiles (I <= J < T, 256 rows each) as
// (I, J) pairs: SB x SB super-blocks, columns J outer and rows I inner inside
// one.  The kernels hand each XCD a contiguous run of this list, so the ~32
// tiles that one XCD runs at a time share few operand panels in its L2.  At
// n = 12, d = 6 (T = 73) super-blocks of 4 read 47 GB from HBM per gram,
// against 55 GB for 8 (which runs 0.9% slower) and 63 GB with no XCD mapping.
constexpr int kGramSuperBlock = 4;
inline void gram_tile_order(int T, std::vector<int32_t>& out) {
  const int SB = kGramSuperBlock;
  out.clear();
  for (int P = 0; P * SB < T; ++P)
    for (int Q = P; Q * SB < T; ++Q)
      for (int J = Q * SB; J < std::min(T, (Q + 1) * SB); ++J)
        for (int I = P * SB; I < std::min(T, (P + 1) * SB); ++I)
          if (I <= J) {
            out.push_back(I);
            out.push_back(J);
          }
}

// error handling (api.cpp)
int set_error(int code, const std::string& msg);
int hip_error(hipError_t e, const char* what);

}  // namespace sos

namespace sos {
// plans whose operands are split into 16-bit hi and lo halves
inline bool split_plan(const sos_plan_s* p) { return p->prec == SOS_BF16X3 || p->prec == SOS_FP16X3; }
// device address of the fp16 scale exponents (sW, sR)
inline int* scale_exponents(const sos_plan_s* p) { return (int*)((double*)(p->ws + p->lay.scal) + kScalScales); }
// 2^e as a float, -126 <= e <= 127 (exact; integer operations only, so a
// wave-uniform e stays in scalar registers)
__host__ __device__ inline float pow2f(int e) {
  const uint32_t b = (uint32_t)(127 + e) << 23;
  float f;
  __builtin_memcpy(&f, &b, 4);
  return f;
}
// device ranking view of a bound plan
inline RankTab rank_tab(const sos_plan_s* p) {
  RankTab t;
  t.codes = (const uint32_t*)(p->ws + p->lay.codes);
  t.tables = (const int32_t*)(p->ws + p->lay.tables);
  t.nwords = p->nwords;
  t.ngroups = p->ngroups;
  t.sparse = p->sparse ? 1 : 0;
  t.n = p->n;
  t.D = 2 * p->d;
  t.total = (int)p->M;
  t.ntab = p->sparse ? (p->n + 2 * p->d + 1) * (2 * p->d + 1) : kFieldTerms;
  return t;
}
// kernel launchers (kernels.hip)
hipError_t launch_pair_ranks(const sos_plan_s* p, int32_t* out, hipStream_t s);
// which operand copies k_prep writes (the ones the coming forward and backward read)
struct PrepNeeds {
  bool a = false;      // forward operands: a_hi (+ a_lo for split plans)
  bool a_f32 = false;  // FP32 row-major copy (FP32 rung of split plans)
  bool x_f32 = false;  // FP32 blocked copy (exact forward)
  bool t = false;      // transposed copy for the backward (t_hi)
  bool t_lo = false;   // its lo half (three-product backward of split plans)
};
hipError_t launch_prep(const sos_plan_s* p, const void* W, const PrepNeeds& need, hipStream_t s);
hipError_t launch_init_r(const sos_plan_s* p, const double* d_p, hipStream_t s);
hipError_t launch_sumsq(const sos_plan_s* p, const double* x, int64_t M, double* out, hipStream_t s,
                        float* x32 = nullptr);
// kFwdSingle: split plans' fast forward with one product (hi hi^T)
enum { kFwdFast = 0, kFwdF32 = 1, kFwdExact = 2, kFwdOzaki = 3, kFwdSingle = 4 };
// oz_slices: digit slices of the Ozaki forward (kOzSlices; 5 or 4 with SOS_FLAG_OZAKI_FIVE_SLICES or
// SOS_FLAG_OZAKI_FOUR_SLICES)
hipError_t launch_gram(const sos_plan_s* p, int mode, hipStream_t s, bool unmerged = false, int oz_slices = kOzSlices);
// deterministic forward (FP32 and FP64 plans with pair lists): the generic
// gram stores its slices, then each coefficient sums its pairs in a fixed order
hipError_t launch_gram_det(const sos_plan_s* p, const double* d_p, hipStream_t s);
hipError_t launch_gather(const sos_plan_s* p, bool split, hipStream_t s);
hipError_t launch_rw(const sos_plan_s* p, void* g, bool split, hipStream_t s);
// store: the unfused measurement variant (tiles stored in the g region for
// launch_scatter_tiles instead of scattered in the epilogue)
// Tail split of the 256-row grams: with one tile per workgroup and one
// workgroup per CU, the last ntiles % CUs tiles run as a partial round on a
// mostly idle chip (141 of 256 CUs at n = 12, d = 6).  Those tiles run
// instead in `parts` contiguous K ranges each, every range scattering its
// partial sum (the scatter is linear), so that the last round is shorter.
// nfull = the tiles that run whole (the first nfull of the tile list);
// parts = 1: no split.
struct TailSplit {
  int nfull = 0, parts = 1;
};
TailSplit gram_tail_split(int ntiles, int64_t nstages, hipStream_t s);

// store: the unfused variant's stored tiles; unmerged: one atomic per Gram entry even where merge maps exist;
// single: one product hi hi^T instead of the three of the split form
hipError_t launch_gram_bf3(const sos_plan_s* p, hipStream_t s, bool store = false, bool unmerged = false,
                           bool single = false);
hipError_t launch_scatter_tiles(const sos_plan_s* p, hipStream_t s);
// the merge maps of a split plan's gram epilogue (into lay.mg_*; reads the ranking tables and the tile list)
hipError_t launch_merge_maps(const sos_plan_s* p, hipStream_t s);
hipError_t launch_gram_x64(const sos_plan_s* p, hipStream_t s);
// Ozaki-split forward (gemm_i8.hip): row exponents and the first `slices`
// int8 slices of W (kOzSlices, 5 or 4), then the gram on as many
hipError_t launch_oz_slices(const sos_plan_s* p, const float* W, hipStream_t s, int slices);
hipError_t launch_gram_i8(const sos_plan_s* p, hipStream_t s, int slices);
inline bool ozaki_supported(const sos_plan_s* p) { return p->prec != SOS_FP64 && p->Kp <= kOzMaxK; }
hipError_t launch_rw_bf3(const sos_plan_s* p, void* g, bool split, hipStream_t s);
hipError_t launch_adam(const sos_plan_s* p, void* W, void* m, void* v, const void* g, int64_t t,
                       const sos_adam_t& h, hipStream_t s);
// single-product backward with Adam and the next step's copies in the epilogue
// next_mode: the forward mode of the next step (kFwdFast: write the split copy,
// kFwdExact: the FP32 blocked copy, otherwise no forward copy)
hipError_t launch_rw_adam_bf3(const sos_plan_s* p, void* W, void* m, void* v, int64_t t, const sos_adam_t& h,
                              int next_mode, hipStream_t s);
// two-layer network (net.hip)
// fp64: P, W and dW are double (FP64 plans), else float
hipError_t launch_net_forward(bool fp64, int n, int m, int k, int N, const float* At, const float* Bt, void* P,
                              const int32_t* rowpair, void* W, hipStream_t s);
hipError_t launch_net_backward(bool fp64, int n, int m, int k, const float* At, const float* Bt, const void* dW,
                               const int32_t* rowmap, void* dP, float* dAt, float* dBt, void* dAz, bool want_dAt,
                               hipStream_t s);
hipError_t launch_adam_f32(float* W, float* m, float* v, const float* g, int64_t n, int64_t t,
                           const sos_adam_t& h, hipStream_t s);
// grouped serving kernels (batch.hip); at most batch_capacity() problems per call
int batch_capacity();
// losses + slot[q] (slot NULL: losses + q) receives problem q's loss
hipError_t launch_step_group(sos_plan_s* const* plans, void* const* W, void* const* state, const int64_t* t,
                             const double* const* p, const sos_adam_t* h, double* losses, const int* slot,
                             int count, hipStream_t s);
}  // namespace sos
