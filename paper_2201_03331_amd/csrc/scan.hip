// scan.hip -- the exhaustive search: for every k-combination, its contingency
// table (section 3.2) by AND + population count of genotype-table rows
// (section 3.1), its mutual information (section 3.3, Eq. 1-3) in plain single
// precision with a bound of its rounding error, and a filter that keeps every
// combination that can still be among the best top_n (Algorithm 1's sorted
// list).
//
// Work decomposition (section 4.1 reuses the genotype table of a (k-1)-prefix
// for every last variant j after it; here a wave does exactly that):
//   * a wave owns one (k-1)-prefix (order >= 3) or a run of first variants
//     (order 2); its 64 lanes own 64 consecutive last variants j;
//   * the prefix rows are wave-uniform, so they are loaded with scalar loads
//     and combined in scalar registers; each lane ANDs them with its own
//     variant's rows and accumulates population counts;
//   * only rows g = 0, 1 of the last variant are counted: the g = 2 count of a
//     prefix row is that row's own population count minus the other two
//     (every sample has exactly one genotype);
//   * at order 2 the first variant's g = 2 row is likewise derived from the
//     per-variant class counts, so 4 of the 9 cells are counted directly;
//   * at order 3 (pair tables) and order 4 (triple tables) only the {0,1}^k
//     cells are counted; the others follow by inclusion-exclusion from
//     stored lower-order tables and class counts.
// Tiles (workgroups of kScanWaves waves sharing the same 64 last variants)
// are pulled from a device-wide counter by a persistent grid.
#include "filter.hpp"

namespace fiuncho {

struct Ulong2 {
  u64 x, y;
};

// ---------------------------------------------------------------------------
// Software-pipelined word loop shared by the counting kernels.  The lane's
// rows of the next kAhead words are in flight in a register ring; each step
// forms the current word's prefix rows from scalar registers, issues the
// scalar loads of the next word, then does the vector work, so both kinds of
// load latency overlap with VALU work.  step(wn, L) must hold word w's scalar
// operands on entry and leave word wn's loads issued.
// ---------------------------------------------------------------------------
constexpr int kAhead = 4;

template <typename Step>
__device__ __forceinline__ void word_pipeline(uint32_t wbeg, uint32_t wend,
                                              const FI_GLOBAL Ulong2 *col, uint32_t n_pad,
                                              Step &&step) {
  if (wbeg >= wend) return;
  const uint32_t wlast = wend - 1;
  Ulong2 L[kAhead];
#pragma unroll
  for (int u = 0; u < kAhead; ++u) {
    const uint32_t wl = min(wbeg + u, wlast);
    L[u].x = col[(size_t)wl * n_pad].x;
    L[u].y = col[(size_t)wl * n_pad].y;
  }
  uint32_t w = wbeg;
  // full groups: no branches inside, so loads stay in flight across words
  for (; w + kAhead <= wend; w += kAhead) {
#pragma unroll
    for (int u = 0; u < kAhead; ++u) {
      step(min(w + u + 1, wlast), L[u]);
      // refill the ring slot after its last use, so that the load can target
      // the same registers and stay in flight across the loop back-edge
      const uint32_t wf = min(w + u + kAhead, wlast);
      L[u].x = col[(size_t)wf * n_pad].x;
      L[u].y = col[(size_t)wf * n_pad].y;
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  // the last (wend - w) < kAhead words are already in the ring
#pragma unroll
  for (int u = 0; u < kAhead - 1; ++u)
    if (w + u < wend) step(min(w + u + 1, wlast), L[u]);
}

// ---------------------------------------------------------------------------
// order 1: the contingency table of one variant is its class counts
// ---------------------------------------------------------------------------
__device__ __forceinline__ void tile_order1(const JV &v, u64 lt, uint32_t wave, uint32_t lane) {
  const uint32_t j = (uint32_t)lt * (kScanWaves * 64) + wave * 64 + lane;
  const bool active = j < v.n;
  const uint32_t jj = active ? j : 0;
  const FI_GLOBAL uint32_t *mg = as_global(v.marg) + (size_t)jj * 6;
  const MiConst mc = mi_const(v);
  const FI_GLOBAL float *F = as_global(v.Fh);
  float fs = mc.c;
  if (active) {
#pragma unroll
    for (int gg = 0; gg < 3; ++gg) fs += mi_term(F, mg[2 * gg], mg[2 * gg + 1]);
  }
  emit(v, active, fs * mc.inv_m, (u64)j, current_threshold(v), lane);
}

// ---------------------------------------------------------------------------
// order 2: a wave holds P consecutive first variants a (rows g = 0, 1 in
// scalar registers) against 64 last variants j (one per lane)
// ---------------------------------------------------------------------------
template <int P, int CLS>
__device__ __forceinline__ void count_order2(cu64p Bv, const FI_GLOBAL Ulong2 *col,
                                             uint32_t n_pad, uint32_t a_first, uint32_t wbeg,
                                             uint32_t wend, uint32_t (&acc)[P][2][2][2]) {
  if (wbeg >= wend) return;
  // rows g = 0, 1 of the P consecutive first variants: 16 P contiguous bytes
  u64 A[P][2];
  auto load = [&](uint32_t w) {
    cu64p rows = Bv + ((size_t)w * n_pad + a_first) * 2;
#pragma unroll
    for (int p = 0; p < P; ++p) {
      A[p][0] = rows[2 * p];
      A[p][1] = rows[2 * p + 1];
    }
  };
  load(wbeg);
  word_pipeline(wbeg, wend, col, n_pad, [&](uint32_t wn, const Ulong2 &L) {
    u64 R[P][2];
#pragma unroll
    for (int p = 0; p < P; ++p) {
      R[p][0] = A[p][0];
      R[p][1] = A[p][1];
    }
    load(wn);
#pragma unroll
    for (int p = 0; p < P; ++p) {
      acc[p][CLS][0][0] = add_popc64(acc[p][CLS][0][0], R[p][0] & L.x);
      acc[p][CLS][0][1] = add_popc64(acc[p][CLS][0][1], R[p][0] & L.y);
      acc[p][CLS][1][0] = add_popc64(acc[p][CLS][1][0], R[p][1] & L.x);
      acc[p][CLS][1][1] = add_popc64(acc[p][CLS][1][1], R[p][1] & L.y);
    }
  });
}

template <int P>
__device__ __forceinline__ void tile_order2(const Globals &g, const JV &v, uint32_t a_first,
                                            uint32_t j0, uint32_t lane) {
  const uint32_t n = v.n;
  if (a_first > n - 2) return;
  if (a_first + 1 >= j0 + 64) return;  // every lane has j <= a for all prefixes
  const uint32_t j = j0 + lane;
  const FI_GLOBAL Ulong2 *col = as_global(reinterpret_cast<const Ulong2 *>(v.Bv)) + j;
  uint32_t acc[P][2][2][2];
#pragma unroll
  for (int p = 0; p < P; ++p)
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int x = 0; x < 2; ++x) acc[p][c][x][0] = acc[p][c][x][1] = 0;
  cu64p Bvc = as_const(v.Bv);
  count_order2<P, 0>(Bvc, col, v.n_pad, a_first, 0, v.W0, acc);
  count_order2<P, 1>(Bvc, col, v.n_pad, a_first, v.W0, v.W0 + v.W1, acc);

  const float thr = current_threshold(v);
  const uint32_t jj = j < n ? j : n - 1;
  const FI_GLOBAL uint32_t *mj = as_global(v.marg) + (size_t)jj * 6;
  uint32_t Mj[2][2];
#pragma unroll
  for (int gg = 0; gg < 2; ++gg)
#pragma unroll
    for (int c = 0; c < 2; ++c) Mj[gg][c] = mj[2 * gg + c];
  const MiConst mc = mi_const(v);
  const u64 cn2 = binom(g, n, 2);
  const FI_GLOBAL float *F = as_global(v.Fh);
  cu32p marg = as_const(v.marg);
#pragma unroll
  for (int p = 0; p < P; ++p) {
    const uint32_t ap = a_first + p;
    const bool pvalid = ap <= n - 2;
    const bool active = pvalid && j < n && j > ap;
    const uint32_t apc = pvalid ? ap : n - 2;
    uint32_t t[9][2];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const uint32_t Ma0 = marg[(size_t)apc * 6 + 0 + c];
      const uint32_t Ma1 = marg[(size_t)apc * 6 + 2 + c];
      const uint32_t Ma2 = marg[(size_t)apc * 6 + 4 + c];
      t[0][c] = acc[p][c][0][0];
      t[1][c] = acc[p][c][0][1];
      t[3][c] = acc[p][c][1][0];
      t[4][c] = acc[p][c][1][1];
      t[2][c] = Ma0 - t[0][c] - t[1][c];
      t[5][c] = Ma1 - t[3][c] - t[4][c];
      t[6][c] = Mj[0][c] - t[0][c] - t[3][c];
      t[7][c] = Mj[1][c] - t[1][c] - t[4][c];
      t[8][c] = Ma2 - t[6][c] - t[7][c];
    }
    const u64 rank = cn2 - binom(g, n - apc, 2) + (u64)(j - apc - 1);
    score_table<9>(v, F, t, active, thr, mc, rank, lane);
  }
}

// ---------------------------------------------------------------------------
// order k >= 3: a wave holds one (k-1)-prefix.  Its 3^(k-1) rows are visited
// 9 at a time (one "pass" per genotype assignment of the first k-3 prefix
// variants); the 9 rows of a pass are lead & row_a[ga] & row_b[gb] for the
// last two prefix variants a, b.  Scores are separable over cells, so each
// pass adds its 27 cells to the running estimate and drops its counters.
// ---------------------------------------------------------------------------
// Bs holds, per variant and word, the rows g = 0, 1, 2 and a zero pad word
// (32 bytes), so one scalar load brings a variant's three rows of a word.
template <int K, int CLS>
__device__ __forceinline__ void count_orderk(cu64p Bs, const FI_GLOBAL Ulong2 *col,
                                             uint32_t n_pad, uint32_t wcap,
                                             const uint32_t (&pre)[K - 1],
                                             const uint32_t (&lg)[K - 2], uint32_t wbeg,
                                             uint32_t wend, uint32_t (&acc)[2][9][2],
                                             uint32_t (&pc)[2][9]) {
  if (wbeg >= wend) return;
  cu64p ra = Bs + (size_t)pre[K - 3] * 4 * wcap;
  cu64p rb = Bs + (size_t)pre[K - 2] * 4 * wcap;
  cu64p rl[K - 2];
#pragma unroll
  for (int i = 0; i < K - 2; ++i) rl[i] = Bs + (size_t)pre[i < K - 3 ? i : 0] * 4 * wcap;
  u64 lead[K - 2], A[3], B[3];
  auto load = [&](uint32_t w) {
#pragma unroll
    for (int i = 0; i < K - 3; ++i) lead[i] = rl[i][(size_t)w * 4 + lg[i]];
#pragma unroll
    for (int gg = 0; gg < 3; ++gg) {
      A[gg] = ra[(size_t)w * 4 + gg];
      B[gg] = rb[(size_t)w * 4 + gg];
    }
  };
  load(wbeg);
  word_pipeline(wbeg, wend, col, n_pad, [&](uint32_t wn, const Ulong2 &L) {
    u64 ld = ~0ull;
#pragma unroll
    for (int i = 0; i < K - 3; ++i) ld &= lead[i];
    u64 R[9];
#pragma unroll
    for (int ga = 0; ga < 3; ++ga)
#pragma unroll
      for (int gb = 0; gb < 3; ++gb) R[ga * 3 + gb] = ld & A[ga] & B[gb];
    load(wn);
#pragma unroll
    for (int r = 0; r < 9; ++r) {
      pc[CLS][r] += popc64(R[r]);
      acc[CLS][r][0] = add_popc64(acc[CLS][r][0], R[r] & L.x);
      acc[CLS][r][1] = add_popc64(acc[CLS][r][1], R[r] & L.y);
    }
  });
}

template <int K>
__device__ __forceinline__ void tile_orderk(const Globals &g, const JV &v,
                                            const uint32_t (&pre)[K - 1], uint32_t j0,
                                            uint32_t lane) {
  constexpr int NLEAD = K - 3;
  int npass = 1;
#pragma unroll
  for (int i = 0; i < NLEAD; ++i) npass *= 3;
  const uint32_t n = v.n;
  const uint32_t b = pre[K - 2];
  const uint32_t j = j0 + lane;
  const bool active = j < n;
  const FI_GLOBAL Ulong2 *col = as_global(reinterpret_cast<const Ulong2 *>(v.Bv)) + j;
  cu64p Bsc = as_const(v.Bs);
  const FI_GLOBAL float *F = as_global(v.Fh);
  const MiConst mc = mi_const(v);
  float fs = mc.c;
  for (int pass = 0; pass < npass; ++pass) {
    uint32_t lg[K - 2];
    {
      int rem = pass;
#pragma unroll
      for (int i = NLEAD - 1; i >= 0; --i) {
        lg[i] = (uint32_t)(rem % 3);
        rem /= 3;
      }
      lg[K - 3] = 0;
    }
    uint32_t acc[2][9][2], pc[2][9];
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int r = 0; r < 9; ++r) acc[c][r][0] = acc[c][r][1] = pc[c][r] = 0;
    count_orderk<K, 0>(Bsc, col, v.n_pad, v.wcap, pre, lg, 0, v.W0, acc, pc);
    count_orderk<K, 1>(Bsc, col, v.n_pad, v.wcap, pre, lg, v.W0, v.W0 + v.W1, acc, pc);
    if (active) {
#pragma unroll
      for (int r = 0; r < 9; ++r) {
        const uint32_t a0 = acc[0][r][0], a1 = acc[0][r][1];
        const uint32_t c0 = acc[1][r][0], c1 = acc[1][r][1];
        fs += mi_term(F, a0, c0);
        fs += mi_term(F, a1, c1);
        fs += mi_term(F, pc[0][r] - a0 - a1, pc[1][r] - c0 - c1);
      }
    }
  }
  const u64 rank = lex_rank_prefix(g, n, K, pre) + (u64)(j - b - 1);
  emit(v, active, fs * mc.inv_m, rank, current_threshold(v), lane);
}

// ---------------------------------------------------------------------------
// order 3 by inclusion-exclusion.  Every sample has exactly one genotype per
// variant, so a count with "any genotype" at one position is the sum of the
// counts with 0, 1 and 2 there; hence every cell with a genotype 2 follows
// from the {0,1} cells of the combination and of its sub-combinations.  The
// wave counts only the 8 cells of {0,1}^3 per class (4 prefix rows against
// rows g = 0, 1 of the last variant, i.e. 8 AND+popcounts per word instead of
// 18); the {0,1}^2 cells of every pair come from a table built beforehand by
// the order-2 counting loop, and the {0,1} cells of every variant from the
// per-variant class counts.
// ---------------------------------------------------------------------------

// Pair tables: PT[(a * n_pad + j) * 8 + ga * 4 + gj * 2 + c], a < j; or, for
// jobs of fewer than 16,384 samples on the order-3 matrix-core path, the
// packed form PT4[a * n_pad + j] = 4 x (ga, gj) of (4 c0 | 4 c1 << 16).
// Grid: x = rows of kScanWaves * 8 first variants, y = 64-wide blocks of j,
// z = job.  Jobs without a pair table return at once.
__global__ __launch_bounds__(kScanWaves * 64) void pairs_kernel(Globals g) {
  const JobDesc *jd = g.jobs + blockIdx.z;
  JV v = load_view(jd);
  uint32_t *PT = uni_ptr(as_const(jd)->pairs);
  if (PT == nullptr) return;  // packed tables (pairs4) come from pairs4_kernel
  const JobState *st = v.st;
  if (uni((uint32_t)st->status) != 0) return;
  v.W0 = uni(st->W0);
  v.W1 = uni(st->W1);
  const uint32_t n = v.n;
  const uint32_t wave = uni(threadIdx.x >> 6), lane = lane_id();
  const uint32_t row_first = blockIdx.x * (kScanWaves * 8);
  const uint32_t a_first = row_first + wave * 8;
  const uint32_t j0 = row_first + 1 + blockIdx.y * 64;
  if (row_first + 1 >= n || j0 >= n) return;
  if (a_first > n - 2 || a_first + 1 >= j0 + 64) return;
  const uint32_t j = j0 + lane;
  const FI_GLOBAL Ulong2 *col = as_global(reinterpret_cast<const Ulong2 *>(v.Bv)) + j;
  uint32_t acc[8][2][2][2];
#pragma unroll
  for (int p = 0; p < 8; ++p)
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int x = 0; x < 2; ++x) acc[p][c][x][0] = acc[p][c][x][1] = 0;
  cu64p Bvc = as_const(v.Bv);
  count_order2<8, 0>(Bvc, col, v.n_pad, a_first, 0, v.W0, acc);
  count_order2<8, 1>(Bvc, col, v.n_pad, a_first, v.W0, v.W0 + v.W1, acc);
#pragma unroll
  for (int p = 0; p < 8; ++p) {
    const uint32_t ap = a_first + p;
    if (ap <= n - 2 && j < n && j > ap) {
      uint4 *dst = reinterpret_cast<uint4 *>(PT + ((size_t)ap * v.n_pad + j) * 8);
      dst[0] = make_uint4(acc[p][0][0][0], acc[p][1][0][0], acc[p][0][0][1], acc[p][1][0][1]);
      dst[1] = make_uint4(acc[p][0][1][0], acc[p][1][1][0], acc[p][0][1][1], acc[p][1][1][1]);
    }
  }
}

template <int P, int CLS>
__device__ __forceinline__ void count3p(cu64p rb, const cu64p (&ra)[P], uint32_t wbeg,
                                        uint32_t wend, const FI_GLOBAL Ulong2 *col,
                                        uint32_t n_pad, uint32_t (&acc)[P][2][2][2][2]) {
  if (wbeg >= wend) return;
  u64 B0, B1, A0[P], A1[P];
  auto load = [&](uint32_t w) {
    B0 = rb[(size_t)w * 4 + 0];
    B1 = rb[(size_t)w * 4 + 1];
#pragma unroll
    for (int p = 0; p < P; ++p) {
      A0[p] = ra[p][(size_t)w * 4 + 0];
      A1[p] = ra[p][(size_t)w * 4 + 1];
    }
  };
  load(wbeg);
  word_pipeline(wbeg, wend, col, n_pad, [&](uint32_t wn, const Ulong2 &L) {
    u64 R[P][2][2];
#pragma unroll
    for (int p = 0; p < P; ++p) {
      R[p][0][0] = A0[p] & B0;
      R[p][0][1] = A0[p] & B1;
      R[p][1][0] = A1[p] & B0;
      R[p][1][1] = A1[p] & B1;
    }
    load(wn);
#pragma unroll
    for (int p = 0; p < P; ++p)
#pragma unroll
      for (int ga = 0; ga < 2; ++ga)
#pragma unroll
        for (int gb = 0; gb < 2; ++gb) {
          acc[p][CLS][ga][gb][0] = add_popc64(acc[p][CLS][ga][gb][0], R[p][ga][gb] & L.x);
          acc[p][CLS][ga][gb][1] = add_popc64(acc[p][CLS][ga][gb][1], R[p][ga][gb] & L.y);
        }
  });
}

// score_table for tables produced cell by cell by walk_order3
__device__ __forceinline__ void score_streamed(const JV &v, const FI_GLOBAL float *F,
                                               const Order3Parts &q, bool active, float thr,
                                               const MiConst &mc, u64 rank, uint32_t lane) {
  float fs = mc.c;
  if (active) walk_order3(q, [&](uint32_t n0, uint32_t n1) { fs += mi_term(F, n0, n1); });
  emit(v, active, fs * mc.inv_m, rank, thr, lane);
}

// A wave holds P prefixes (a_first + p, b) with a common last prefix variant
// b; lanes own the last variants j.
template <int P>
__device__ __forceinline__ void tile_order3p(const Globals &g, const JV &v, uint32_t b,
                                             uint32_t a_first, uint32_t j0, uint32_t lane) {
  const uint32_t n = v.n;
  if (a_first >= b) return;
  const uint32_t j = j0 + lane;
  const bool jvalid = j < n;
  const FI_GLOBAL Ulong2 *col = as_global(reinterpret_cast<const Ulong2 *>(v.Bv)) + j;
  cu64p Bsc = as_const(v.Bs);
  cu64p rb = Bsc + (size_t)b * 4 * v.wcap;
  cu64p ra[P];
#pragma unroll
  for (int p = 0; p < P; ++p) ra[p] = Bsc + (size_t)min(a_first + p, b - 1) * 4 * v.wcap;
  uint32_t acc[P][2][2][2][2];
#pragma unroll
  for (int p = 0; p < P; ++p)
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) acc[p][c][x][y][0] = acc[p][c][x][y][1] = 0;
  count3p<P, 0>(rb, ra, 0, v.W0, col, v.n_pad, acc);
  count3p<P, 1>(rb, ra, v.W0, v.W0 + v.W1, col, v.n_pad, acc);

  const float thr = current_threshold(v);
  const MiConst mc = mi_const(v);
  const FI_GLOBAL float *F = as_global(v.Fh);
  cu32p marg = as_const(v.marg);
  const uint32_t jj = jvalid ? j : n - 1;
  const FI_GLOBAL uint32_t *PTg = as_global(v.pairs);
  const FI_CONST uint32_t *PTc = as_const(v.pairs);
  uint32_t bj[8];  // (b, j): [gb][gj][c]
  load_pair(PTg + ((size_t)b * v.n_pad + jj) * 8, bj);
  const FI_GLOBAL uint32_t *mj = as_global(v.marg) + (size_t)jj * 6;
  uint32_t Mj[2][2], Mb[2][2];
#pragma unroll
  for (int gg = 0; gg < 2; ++gg)
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      Mj[gg][c] = mj[2 * gg + c];
      Mb[gg][c] = marg[(size_t)b * 6 + 2 * gg + c];
    }
#pragma unroll
  for (int p = 0; p < P; ++p) {
    // one prefix's table and score at a time (bounds register use)
    __builtin_amdgcn_sched_barrier(0);
    const uint32_t a = min(a_first + p, b - 1);
    const bool active = jvalid && a_first + p < b;
    uint32_t aj[8], ab[8], Ma[2][2];
    load_pair(PTg + ((size_t)a * v.n_pad + jj) * 8, aj);
#pragma unroll
    for (int q = 0; q < 8; ++q) ab[q] = PTc[((size_t)a * v.n_pad + b) * 8 + q];
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int c = 0; c < 2; ++c) Ma[x][c] = marg[(size_t)a * 6 + 2 * x + c];
    const uint32_t pre[2] = {a, b};
    const u64 rank = lex_rank_prefix(g, n, 3, pre) + (u64)(j - b - 1);
    const uint32_t mcls[2] = {v.m0, v.m1};
    const Order3Parts parts = {acc[p], ab, aj, bj, Ma, Mb, Mj, mcls};
    score_streamed(v, F, parts, active, thr, mc, rank, lane);
  }
}

// ---------------------------------------------------------------------------
// order 4 with stored triple tables: only the {0,1}^4 cells of (a, b, c, j)
// are counted (16 word-ops per word instead of 54).  The other cells follow
// by inclusion-exclusion: for g_j in {0, 1}, the cells (., ., ., g_j) form an
// order-3 table over (a, b, c) whose "pairs" are the {0,1}^3 tables of
// (a, b, j), (a, c, j), (b, c, j) at g_j, whose "variants" are the {0,1}^2
// pair tables of (a, j), (b, j), (c, j) at g_j and whose size is the count of
// g_j at j; the cells (., ., ., 2) are the prefix's own order-3 table minus
// those two.
// ---------------------------------------------------------------------------

// Pass over all (a, b, j), a < b < j: their {0,1}^3 counts per class into
// the triple tables [pair_index(a, b)][j][g_a][g_b][g_j][class] (or, packed,
// [pair_index(a, b)][j][g_a] of [g_b][g_j] -> 4 c0 | 4 c1 << 16).  Grid: x =
// group of kScanWaves * 2 first variants a, y = b - 1, z = job; each wave
// owns 2 first variants and walks the blocks of 64 last variants.
__global__ __launch_bounds__(kScanWaves * 64) void triples_kernel(Globals g) {
  const JobDesc *jd = g.jobs + blockIdx.z;
  JV v = load_view(jd);
  uint32_t *TT = uni_ptr(as_const(jd)->triples);
  uint4 *TT4 = uni_ptr(as_const(jd)->triples4);
  if (TT == nullptr && TT4 == nullptr) return;
  const JobState *st = v.st;
  if (uni((uint32_t)st->status) != 0) return;
  v.W0 = uni(st->W0);
  v.W1 = uni(st->W1);
  const uint32_t n = v.n;
  const uint32_t wave = uni(threadIdx.x >> 6), lane = lane_id();
  const uint32_t b = blockIdx.y + 1;
  if (b + 1 >= n) return;
  const uint32_t a_first = blockIdx.x * (kScanWaves * 2) + wave * 2;
  if (a_first >= b) return;
  cu64p Bsc = as_const(v.Bs);
  cu64p rb = Bsc + (size_t)b * 4 * v.wcap;
  cu64p ra[2];
#pragma unroll
  for (int p = 0; p < 2; ++p) ra[p] = Bsc + (size_t)min(a_first + p, b - 1) * 4 * v.wcap;
  for (uint32_t j0 = b + 1; j0 < n; j0 += 64) {
    const uint32_t j = j0 + lane;
    const FI_GLOBAL Ulong2 *col = as_global(reinterpret_cast<const Ulong2 *>(v.Bv)) + j;
    uint32_t acc[2][2][2][2][2];  // [p][c][g_a][g_b][g_j]
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
          for (int y = 0; y < 2; ++y) acc[p][c][x][y][0] = acc[p][c][x][y][1] = 0;
    count3p<2, 0>(rb, ra, 0, v.W0, col, v.n_pad, acc);
    count3p<2, 1>(rb, ra, v.W0, v.W0 + v.W1, col, v.n_pad, acc);
#pragma unroll
    for (int p = 0; p < 2; ++p) {
      const uint32_t a = a_first + p;
      if (a < b && j < n && TT) {
        uint4 *dst = reinterpret_cast<uint4 *>(TT + (pair_index(n, a, b) * v.n_pad + j) * 16);
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
          for (int y = 0; y < 2; ++y)
            dst[x * 2 + y] = make_uint4(acc[p][0][x][y][0], acc[p][1][x][y][0], acc[p][0][x][y][1],
                                        acc[p][1][x][y][1]);
      }
      if (a < b && j < n && TT4) {
        uint4 *dst = TT4 + (pair_index(n, a, b) * v.n_pad + j) * 2;
        auto pk = [&](int x, int y, int z) { return (acc[p][0][x][y][z] << 2) | (acc[p][1][x][y][z] << 18); };
#pragma unroll
        for (int x = 0; x < 2; ++x) dst[x] = make_uint4(pk(x, 0, 0), pk(x, 0, 1), pk(x, 1, 0), pk(x, 1, 1));
      }
    }
  }
}

// {0,1}^4 counts of (a, b, c, j) for one class: the 8 rows of (a, b, c) with
// g in {0, 1} are formed in scalar registers per word
template <int CLS>
__device__ __forceinline__ void count4t(cu64p ra, cu64p rb, cu64p rc, uint32_t wbeg, uint32_t wend,
                                        const FI_GLOBAL Ulong2 *col, uint32_t n_pad,
                                        uint32_t (&acc)[2][2][2][2][2]) {
  if (wbeg >= wend) return;
  u64 A[2], B[2], C[2];
  auto load = [&](uint32_t w) {
#pragma unroll
    for (int x = 0; x < 2; ++x) {
      A[x] = ra[(size_t)w * 4 + x];
      B[x] = rb[(size_t)w * 4 + x];
      C[x] = rc[(size_t)w * 4 + x];
    }
  };
  load(wbeg);
  word_pipeline(wbeg, wend, col, n_pad, [&](uint32_t wn, const Ulong2 &L) {
    u64 R[2][2][2];
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y) {
        const u64 ab = A[x] & B[y];
        R[x][y][0] = ab & C[0];
        R[x][y][1] = ab & C[1];
      }
    load(wn);
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y)
#pragma unroll
        for (int z = 0; z < 2; ++z) {
          acc[CLS][x][y][z][0] = add_popc64(acc[CLS][x][y][z][0], R[x][y][z] & L.x);
          acc[CLS][x][y][z][1] = add_popc64(acc[CLS][x][y][z][1], R[x][y][z] & L.y);
        }
  });
}

__device__ __forceinline__ void tile_order4t(const Globals &g, const JV &v, const uint32_t (&pre)[3],
                                             uint32_t j0, uint32_t lane) {
  const uint32_t n = v.n, a = pre[0], b = pre[1], c = pre[2];
  const uint32_t j = j0 + lane;
  const bool active = j < n;
  const uint32_t jj = active ? j : n - 1;
  const FI_GLOBAL Ulong2 *col = as_global(reinterpret_cast<const Ulong2 *>(v.Bv)) + j;
  cu64p Bsc = as_const(v.Bs);
  cu64p ra = Bsc + (size_t)a * 4 * v.wcap, rb = Bsc + (size_t)b * 4 * v.wcap,
        rc = Bsc + (size_t)c * 4 * v.wcap;
  uint32_t acc[2][2][2][2][2];  // [class][g_a][g_b][g_c][g_j]
#pragma unroll
  for (int q = 0; q < 2; ++q)
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y)
#pragma unroll
        for (int z = 0; z < 2; ++z) acc[q][x][y][z][0] = acc[q][x][y][z][1] = 0;
  count4t<0>(ra, rb, rc, 0, v.W0, col, v.n_pad, acc);
  count4t<1>(ra, rb, rc, v.W0, v.W0 + v.W1, col, v.n_pad, acc);

  const float thr = current_threshold(v);
  const MiConst mc = mi_const(v);
  const float fs = order4_tables_sum<true, true>(v, as_global(v.Fh), acc, a, b, c, jj, active, mc.c);
  const u64 rank = lex_rank_prefix(g, n, 4, pre) + (u64)(j - c - 1);
  emit(v, active, fs * mc.inv_m, rank, thr, lane);
}

// ---------------------------------------------------------------------------
// persistent driver
// ---------------------------------------------------------------------------
template <int K, bool TRIPLES = false>
__device__ __forceinline__ void run_orderk(const Globals &g, const JV &v, uint32_t rho, u64 local,
                                           uint32_t wave, uint32_t lane) {
  const uint32_t n = v.n;
  const uint32_t b = rho + (K - 2);
  const uint32_t nj = (n - 1 - b + 63) / 64;
  const u64 grp = local / nj;
  const uint32_t jb = (uint32_t)(local - grp * nj);
  u64 q = grp * kScanWaves + wave;
  if (q >= binom_small(g, b, K - 2)) return;
  uint32_t pre[K - 1];
  pre[K - 2] = b;
  // colex unrank of the (k-2)-subset of [0, b) with index q
  colex_unrank<K - 2>(g, b, q, pre);
  if constexpr (TRIPLES && K == 4) tile_order4t(g, v, pre, b + 1 + jb * 64, lane);
  else tile_orderk<K>(g, v, pre, b + 1 + jb * 64, lane);
}

// waves per SIMD each variant is compiled for (register budget 512 / waves);
// measured: the order-4 triple-table kernel is fastest at 3 (165 registers,
// no spills; 2 waves: 24.1 ms, 3: 19.6 ms, 4 with spills: 24.3 ms at 200 x
// 4,000)
constexpr int scan_min_waves(int ksel) { return ksel == kSelTriples ? 3 : ksel != 0 ? 4 : 2; }

template <int KSEL>
__global__ __launch_bounds__(kScanWaves * 64, scan_min_waves(KSEL)) void scan_kernel(Globals g) {
  __shared__ u64 s_tile;
  const uint32_t lane = lane_id();
  const uint32_t wave = uni(threadIdx.x >> 6);
  RowHint hint;  // the row of the workgroup's last tile
  for (;;) {
    if (threadIdx.x == 0) s_tile = g.tile_base + atomicAdd(g.tile_counter, 1ull);
    __syncthreads();
    const u64 t = uni64(s_tile);
    __syncthreads();
    if (t >= g.total_tiles) break;
    JV v;
    const FI_CONST JobDesc *jd;
    u64 lt;
    if (!locate_tile(g, t, wave, kPilotEmits, v, jd, lt)) continue;
    const int k = KSEL == kSelPairs ? 3 : KSEL == kSelTriples ? 4 : (KSEL && KSEL != kSel23) ? KSEL : (int)v.k;
    if (k == 1) {
      if (KSEL == 0 || KSEL == 1) tile_order1(v, lt, wave, lane);
      continue;
    }
    cu64p rows = as_const(uni_ptr(jd->row_start));
    const uint32_t rl = hint.find(jd, lt);
    const u64 local = uni64(lt - rows[rl]);
    if (k == 2) {
      if (KSEL == 0 || KSEL == 2 || KSEL == kSel23) {
        const uint32_t a_first = rl * (kScanWaves * kOrder2Prefixes);
        const uint32_t j0 = a_first + 1 + (uint32_t)local * 64;
        tile_order2<kOrder2Prefixes>(g, v, a_first + wave * kOrder2Prefixes, j0, lane);
      }
      continue;
    }
    if (k == 3 && (KSEL == kSelPairs || KSEL == kSel23 || (KSEL == 0 && v.path == kPathPairs))) {
      if (KSEL == 0 || KSEL == kSelPairs || KSEL == kSel23) {
        const uint32_t b = rl + 1;
        const uint32_t nj = (v.n - 1 - b + 63) / 64;
        const u64 grp = local / nj;
        const uint32_t jb = (uint32_t)(local - grp * nj);
        const uint32_t a_first = (uint32_t)grp * (kScanWaves * kOrder3Prefixes) + wave * kOrder3Prefixes;
        tile_order3p<kOrder3Prefixes>(g, v, b, a_first, b + 1 + jb * 64, lane);
      }
      continue;
    }
    switch (k) {
      case 3: if (KSEL == 0 || KSEL == 3) run_orderk<3>(g, v, rl, local, wave, lane); break;
      case 4:
        if (KSEL == kSelTriples || (KSEL == 0 && v.path == kPathTriples))
          run_orderk<4, true>(g, v, rl, local, wave, lane);
        else if (KSEL == 0 || KSEL == 4)
          run_orderk<4>(g, v, rl, local, wave, lane);
        break;
      case 5: if (KSEL == 0 || KSEL == 5) run_orderk<5>(g, v, rl, local, wave, lane); break;
      case 6: if (KSEL == 0 || KSEL == 6) run_orderk<6>(g, v, rl, local, wave, lane); break;
      case 7: if (KSEL == 0 || KSEL == 7) run_orderk<7>(g, v, rl, local, wave, lane); break;
      case 8: if (KSEL == 0 || KSEL == 8) run_orderk<8>(g, v, rl, local, wave, lane); break;
      default: break;
    }
  }
}

template <int KSEL>
static int occupancy_grid() {
  int dev = 0, cus = 0, per = 0;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, scan_kernel<KSEL>,
                                                     kScanWaves * 64, 0);
  if (cus <= 0) cus = 256;
  if (per <= 0) per = 1;
  return cus * per;
}

int scan_grid_size(int ksel) {
  switch (ksel) {
    case 1: return occupancy_grid<1>();
    case 2: return occupancy_grid<2>();
    case 3: return occupancy_grid<3>();
    case 4: return occupancy_grid<4>();
    case 5: return occupancy_grid<5>();
    case kSelPairs: return occupancy_grid<kSelPairs>();
    case kSel23: return occupancy_grid<kSel23>();
    case kSelTriples: return occupancy_grid<kSelTriples>();
    default: return occupancy_grid<0>();
  }
}

void launch_triples(const Globals &g, uint32_t max_n, hipStream_t s) {
  const uint32_t groups = (max_n + kScanWaves * 2 - 1) / (kScanWaves * 2);
  const uint32_t rows = max_n > 2 ? max_n - 2 : 1;
  hipLaunchKernelGGL(triples_kernel, dim3(groups ? groups : 1, rows, g.n_jobs), dim3(kScanWaves * 64), 0,
                     s, g);
}

void launch_pairs(const Globals &g, uint32_t max_n, hipStream_t s) {
  const uint32_t rows = (max_n + kScanWaves * 8 - 2) / (kScanWaves * 8);
  const uint32_t jbs = (max_n + 62) / 64;
  hipLaunchKernelGGL(pairs_kernel, dim3(rows ? rows : 1, jbs ? jbs : 1, g.n_jobs),
                     dim3(kScanWaves * 64), 0, s, g);
}

void launch_scan(const Globals &g, int ksel, int grid, hipStream_t s) {
  dim3 gd(grid), bd(kScanWaves * 64);
  switch (ksel) {
    case 1: hipLaunchKernelGGL(scan_kernel<1>, gd, bd, 0, s, g); break;
    case 2: hipLaunchKernelGGL(scan_kernel<2>, gd, bd, 0, s, g); break;
    case 3: hipLaunchKernelGGL(scan_kernel<3>, gd, bd, 0, s, g); break;
    case 4: hipLaunchKernelGGL(scan_kernel<4>, gd, bd, 0, s, g); break;
    case 5: hipLaunchKernelGGL(scan_kernel<5>, gd, bd, 0, s, g); break;
    case kSelPairs: hipLaunchKernelGGL(scan_kernel<kSelPairs>, gd, bd, 0, s, g); break;
    case kSel23: hipLaunchKernelGGL(scan_kernel<kSel23>, gd, bd, 0, s, g); break;
    case kSelTriples: hipLaunchKernelGGL(scan_kernel<kSelTriples>, gd, bd, 0, s, g); break;
    default: hipLaunchKernelGGL(scan_kernel<0>, gd, bd, 0, s, g); break;
  }
}

}  // namespace fiuncho
