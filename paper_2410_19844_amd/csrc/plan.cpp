// Host-side plan: monomial bases, the additive ranking code, rank tables and
// the workspace layout.
//
// Ranking (Section 1.1 order).  Monomials of degree <= D in n variables are
// ordered by total degree (higher first), then lexicographically (larger
// exponent vector first, x1 most significant).  For gamma with t = |gamma|
// and suffix sums u_f = gamma_{f+1} + ... + gamma_n (f = 1..n-1), the
// position of gamma is
//
//   rank_D(gamma) = [C(D+n, n) - C(t+n, n)]                  (all higher degrees)
//                 + sum_{f=1}^{n-1} C(u_f + n-f-1, n-f)      (same degree, lex-larger)
//
// The f-th term counts the degree-t monomials that agree with gamma on
// x1..x_{f-1} and have a larger exponent of x_f: their remaining u_f - 1 - s
// units (s >= 0) are spread over n-f variables, and summing the counts over s
// gives C(u_f + n-f-1, n-f).  Every term depends on one field of the code
// (t or one u_f), which is what makes per-group table lookups possible.
#include <algorithm>
#include <climits>
#include <cstring>
#include <new>

#include "sos_internal.h"

namespace sos {

static int64_t binom(int64_t a, int64_t b) {
  if (b < 0 || a < b) return 0;
  b = std::min(b, a - b);
  int64_t r = 1;
  for (int64_t i = 1; i <= b; ++i) r = r * (a - b + i) / i;
  return r;
}

static void compositions(int n, int v, int left, std::vector<uint8_t>& cur, std::vector<uint8_t>& out) {
  if (v == n - 1) {
    cur[v] = (uint8_t)left;
    out.insert(out.end(), cur.begin(), cur.end());
    return;
  }
  for (int e = left; e >= 0; --e) {  // larger exponent of x_{v+1} first
    cur[v] = (uint8_t)e;
    compositions(n, v + 1, left - e, cur, out);
  }
}

void enumerate_monomials(int n, int D, std::vector<uint8_t>& out) {
  out.clear();
  std::vector<uint8_t> cur(n, 0);
  for (int t = D; t >= 0; --t) compositions(n, 0, t, cur, out);
}

static int64_t field_term(int n, int D, int f, int value) {
  if (f == 0) return binom(D + n, n) - binom(value + n, n);
  return binom(value + n - f - 1, n - f);
}

int64_t rank_closed_form(int n, int D, const uint8_t* e) {
  int t = 0;
  for (int v = 0; v < n; ++v) t += e[v];
  int64_t r = field_term(n, D, 0, t);
  int u = t;
  for (int f = 1; f < n; ++f) {
    u -= e[f - 1];
    r += field_term(n, D, f, u);
  }
  return r;
}

static inline int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

int plan_create(int n, int d, int rank, int prec, sos_plan_s** out) {
  if (!out) return set_error(SOS_EINVAL, "sos_plan: out is NULL");
  *out = nullptr;
  if (n < 1 || d < 1 || rank < 1)
    return set_error(SOS_EINVAL, "sos_plan: n, d and rank must be >= 1");
  if (prec != SOS_FP64 && prec != SOS_FP32 && prec != SOS_BF16X3 && prec != SOS_FP16X3)
    return set_error(SOS_EINVAL, "sos_plan: unknown precision");
  // dense codes (4-bit suffix-sum fields) for n <= 16, 2d <= 15; sparse
  // variable lists (one byte per factor) for more variables at low degree
  const bool sparse = n > 16;
  if (!sparse && 2 * d > 15)
    return set_error(SOS_ERANGE, "sos_plan: needs 2d <= 15 (4-bit code fields)");
  if (sparse && (2 * d > 8 || n > 255))
    return set_error(SOS_ERANGE, "sos_plan: with n > 16 needs 2d <= 8 and n <= 255");
  const int64_t N = binom(n + d, d), M = binom(n + 2 * d, 2 * d);
  if (M >= (int64_t(1) << 31) || N * N >= (int64_t(1) << 31))
    return set_error(SOS_ERANGE, "sos_plan: M and N*N must stay below 2^31");
  if ((int64_t)rank * N >= (int64_t(1) << 34))
    return set_error(SOS_ERANGE, "sos_plan: N*rank too large");

  sos_plan_s* p = new (std::nothrow) sos_plan_s;
  if (!p) return set_error(SOS_ENOMEM, "sos_plan: host allocation failed");
  p->n = n; p->d = d; p->k = rank; p->prec = prec; p->N = N; p->M = M;
  p->sparse = sparse;
  p->ngroups = sparse ? 0 : (n + kFieldsPerGroup - 1) / kFieldsPerGroup;
  p->nwords = sparse ? 1 : (p->ngroups + 1) / 2;

  enumerate_monomials(n, d, p->basis);
  if ((int64_t)p->basis.size() != N * n) {
    delete p;
    return set_error(SOS_EINVAL, "sos_plan: internal enumeration count mismatch");
  }

  const int D = 2 * d;
  if (sparse) {
    // codes: ascending variable list, byte q = (q-th variable) + 1
    p->codes.assign(N, 0u);
    for (int64_t i = 0; i < N; ++i) {
      const uint8_t* e = &p->basis[i * n];
      uint32_t c = 0;
      int q = 0;
      for (int v = 0; v < n; ++v)
        for (int m = 0; m < e[v]; ++m) c |= (uint32_t)(v + 1) << (8 * q++);
      p->codes[i] = c;
    }
    // binomial table C[x][y], 0 <= x <= n + D, 0 <= y <= D
    p->tables.assign((size_t)(n + D + 1) * (D + 1), 0);
    for (int x = 0; x <= n + D; ++x)
      for (int y = 0; y <= D; ++y) {
        const int64_t c = binom(x, y);
        if (c > INT32_MAX) {
          delete p;
          return set_error(SOS_ERANGE, "sos_plan: binomial table entry exceeds int32");
        }
        p->tables[(size_t)x * (D + 1) + y] = (int32_t)c;
      }
  } else {
    // codes
    p->codes.assign(N * p->nwords, 0u);
    for (int64_t i = 0; i < N; ++i) {
      const uint8_t* e = &p->basis[i * n];
      int t = 0;
      for (int v = 0; v < n; ++v) t += e[v];
      int u = t;
      for (int f = 0; f < n; ++f) {
        if (f > 0) u -= e[f - 1];
        const int val = (f == 0) ? t : u;
        const int g = f / kFieldsPerGroup, w = g / 2;
        const int shift = (g % 2) * 16 + (f % kFieldsPerGroup) * 4;
        p->codes[i * p->nwords + w] |= (uint32_t)val << shift;
      }
    }
    // tables: T_g[idx] = sum over the group's fields of field_term(field value)
    p->tables.assign((size_t)p->ngroups * kGroupEntries, 0);
    for (int g = 0; g < p->ngroups; ++g) {
      for (int idx = 0; idx < kGroupEntries; ++idx) {
        int64_t s = 0;
        bool valid = true;
        for (int q = 0; q < kFieldsPerGroup; ++q) {
          const int f = g * kFieldsPerGroup + q;
          const int val = (idx >> (4 * q)) & 15;
          if (f >= n) {
            if (val != 0) valid = false;
            continue;
          }
          if (val > D) valid = false;
          else s += field_term(n, D, f, val);
        }
        p->tables[(size_t)g * kGroupEntries + idx] = valid ? (int32_t)s : 0;
      }
    }
    // then the field terms one at a time: F[f * 16 + v] = field_term(f, v)
    p->tables.resize((size_t)p->ngroups * kGroupEntries + kFieldTerms, 0);
    int32_t* F = p->tables.data() + (size_t)p->ngroups * kGroupEntries;
    for (int f = 0; f < n; ++f)
      for (int v = 0; v <= D; ++v) F[f * 16 + v] = (int32_t)field_term(n, D, f, v);
  }

  // padded extents and workspace layout
  p->Np = round_up(N, kPadRows);
  p->Kp = round_up(rank, kPadK);
  p->Np2 = round_up(N, kPadK);
  p->Kp2 = round_up(rank, kPadRows);
  const size_t wel = (prec == SOS_FP64) ? 8 : 4;          // W / gradient element
  const size_t oel = (prec == SOS_FP64) ? 8 : (prec == SOS_FP32 ? 4 : 2);  // operand element
  // upper-triangle tiles of 256 rows in the gram's locality order
  sos::gram_tile_order((int)(p->Np / 256), p->tile_list);
  p->ntiles256 = (int)(p->tile_list.size() / 2);
  Layout& L = p->lay;
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off = round_up(off + bytes, 256); return o; };
  L.codes = take((size_t)N * p->nwords * 4);
  L.tables = take(p->tables.size() * 4);
  L.r = take((size_t)M * 8);
  if (prec != SOS_FP64) L.r32 = take((size_t)M * 4);
  L.tiles = take(p->tile_list.size() * 4);
  L.scal = take(kScalDoubles * 8);   // scalars, reduction partials, fp16 scales (see kScalScales)
  // split-bf16 operands are panel-blocked with padded panels (see blk_off)
  const bool blk = prec == SOS_BF16X3 || prec == SOS_FP16X3;
  const size_t a_el = blk ? (size_t)(p->Np / kBlkRows) * panel_stride(p->Kp / kBlkK, 2) : (size_t)p->Np * p->Kp;
  const size_t t_el = blk ? (size_t)(p->Kp2 / kBlkRows) * panel_stride(p->Np2 / kBlkK, 2) : (size_t)p->Kp2 * p->Np2;
  const size_t R_el = blk ? (size_t)(p->Np / kBlkRows) * panel_stride(p->Np2 / kBlkK, 2) : (size_t)p->Np * p->Np2;
  L.a_hi = take(a_el * oel);
  if (blk) L.a_lo = take(a_el * oel);
  L.t_hi = take(t_el * oel);
  if (blk) L.t_lo = take(t_el * oel);
  L.R_hi = take(R_el * oel);
  if (blk) L.R_lo = take(R_el * oel);
  // split-precision plans keep an FP32 padded copy of W for the exact FP64 forward
  // (FP32 plans use a_hi, which already is that copy)
  if (blk) L.a_f32 = take((size_t)p->Np * p->Kp * 4);
  if (prec != SOS_FP64) L.x_f32 = take((size_t)(p->Np / kBlkRows) * panel_stride(p->Kp / kBlkK, 4) * 4);
  // gradient scratch; in split plans also the stored Gram tiles of the unfused
  // scatter variant (256 x 256 FP32 per upper tile)
  L.g = take(std::max((size_t)N * rank * wel, blk ? (size_t)p->ntiles256 * 256 * 256 * 4 : 0));
  if (blk) {  // merge maps of the gram epilogue
    const size_t segs = (size_t)p->ntiles256 * kMergeSegs;
    L.mg_map = take(segs * kMergeSeg * 2);
    L.mg_rank = take(segs * kMergeSlots * 4);
    L.mg_count = take(segs * 2 * 4);
  }
  if (prec != SOS_FP64) {  // Ozaki-split forward: int8 slices, row exponents and scales
    L.oz_slice = (size_t)(p->Np / kBlkRows) * oz_panel_stride(p->Kp);
    L.oz = take(L.oz_slice * kOzSlices);
    L.oz_exp = take((size_t)N * 4);
    L.oz_scale = take((size_t)N * 8);
    L.oz_lvl = take((size_t)p->ntiles256 * (kOzSlices - 1) * kBlkRows * kBlkRows * 4);
  }
  // Grouped serving path: the coefficient of monomial m sums the Gram entries
  // of its pairs (i <= j, alpha_i + alpha_j = m) in one fixed order (i, then
  // j, ascending), so a problem's forward is deterministic.  The pair lists
  // are the inverse of the ranking map, built here once (counting sort).
  if ((prec == SOS_FP32 || prec == SOS_FP64) && N <= SOS_BATCH_MAX_N) {
    p->batchable = prec == SOS_FP32;
    p->det_ok = true;
    // rank of alpha_i + alpha_j by the closed form, one field term per
    // variable looked up in a table (the terms depend on (f, value) only)
    std::vector<int64_t> ft((size_t)n * (D + 1));
    for (int f = 0; f < n; ++f)
      for (int v = 0; v <= D; ++v) ft[(size_t)f * (D + 1) + v] = field_term(n, D, f, v);
    auto rank_of = [&](int64_t i, int64_t j) {
      const uint8_t* a = &p->basis[i * n];
      const uint8_t* b = &p->basis[j * n];
      int u = 0;
      for (int v = 0; v < n; ++v) u += a[v] + b[v];
      int64_t r = 0;
      for (int f = 0; f < n; ++f) {
        if (f > 0) u -= a[f - 1] + b[f - 1];
        r += ft[(size_t)f * (D + 1) + u];
      }
      return r;
    };
    p->pair_off.assign(M + 1, 0);
    p->pair_idx.assign(N * (N + 1) / 2, 0);
    p->pair_pos.assign(N * N, 0);
    p->rank_map.assign(N * N, 0);
    for (int64_t i = 0; i < N; ++i)
      for (int64_t j = i; j < N; ++j) {
        const int64_t m = rank_of(i, j);
        p->rank_map[i * N + j] = p->rank_map[j * N + i] = (int32_t)m;
        ++p->pair_off[m + 1];
      }
    for (int64_t m = 0; m < M; ++m) p->pair_off[m + 1] += p->pair_off[m];
    std::vector<int32_t> fill(p->pair_off.begin(), p->pair_off.end() - 1);
    for (int64_t i = 0; i < N; ++i)
      for (int64_t j = i; j < N; ++j) {
        const int32_t e = fill[p->rank_map[i * N + j]]++;
        p->pair_idx[e] = (int32_t)((uint32_t)(i * N + j) | (i < j ? 0x80000000u : 0u));
        p->pair_pos[i * N + j] = p->pair_pos[j * N + i] = e;
      }
    if (p->batchable) {
      L.bG = take((size_t)batch_slices(rank) * p->pair_idx.size() * 8);
      L.pair_pos = take(p->pair_pos.size() * 4);
      L.rank_map = take(p->rank_map.size() * 4);
      L.bg = take((size_t)batch_slices_j((int)N) * N * rank * 4);
      L.bpart = take((size_t)((M + 255) / 256) * 8);
      L.bcount = take(4);
    }
    L.pair_off = take(p->pair_off.size() * 4);
    L.pair_idx = take(p->pair_idx.size() * 4);
    if (p->batchable) L.bhdr = take(sizeof(BatchHeader));
    L.det_G = take((size_t)generic_gram_splits(p->Np, p->Kp) * N * N * 8);
  }
  L.bytes = off;
  p->state_bytes = round_up((size_t)N * rank * wel, 256) * 4;  // m, v, best W, candidate W
  if (p->batchable) {
    BatchHeader& h = p->bhdr;
    h.N = (int32_t)N;
    h.M = (int32_t)M;
    h.k = rank;
    h.sg = batch_slices(rank);
    h.sr = batch_slices_j((int)N);
    h.v = (int64_t)(p->state_bytes / 4);
    auto rel = [&](size_t at) { return (int64_t)at - (int64_t)L.bhdr; };
    h.r = rel(L.r);
    h.Gp = rel(L.bG);
    h.pair_pos = rel(L.pair_pos);
    h.rank_map = rel(L.rank_map);
    h.gp = rel(L.bg);
    h.part = rel(L.bpart);
    h.count = rel(L.bcount);
    h.pair_off = rel(L.pair_off);
    h.pair_idx = rel(L.pair_idx);
  }
  *out = p;
  return SOS_OK;
}

}  // namespace sos
