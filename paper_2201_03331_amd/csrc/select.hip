// select.hip -- from the scan's candidates to the exact best top_n.
//
// Algorithm 1 keeps a sorted list of the S best scores; its threads' and
// processes' lists are then joined, sorted and truncated (section 4.2, last
// paragraph).  Here the scan leaves an unordered candidate buffer that
// provably holds every combination that can be among the best top_n, and:
//   1. compact:  drop candidates below the final running bound (all blocks);
//   2. select:   exact top_n-th largest FP32 score by radix selection, then keep
//                every candidate within the FP32 error tolerance of it;
//   3. rescore:  recount each kept combination's table and evaluate Eq. 1-3 in
//                IEEE double, term by term in a fixed order;
//   4. finish:   order by (MI descending, rank ascending), write top_n hits.
// The scan's estimate (plain single precision, or the 32-bit fixed-point sum
// of the FP4 matrix-core kernels of orders 3-5) is within fbound of the MI (a
// bound of its rounding error), so a combination is dropped only when its
// estimate is more than 2 fbound below one that top_n others reach: it cannot
// belong to the exact result.  The reported single-precision score is a
// compensated evaluation made here, beside the double-precision one.
#include <algorithm>

#include "filter.hpp"

namespace fiuncho {

__device__ __forceinline__ float tol_threshold(const JobDesc &J, float tau) {
  return tau - 2.0f * J.fbound;
}

// 1. all workgroups, grid-stride over one job's candidates (blockIdx.y = job)
__global__ __launch_bounds__(256) void compact_kernel(Globals g) {
  const JobDesc &J = g.jobs[blockIdx.y];
  JobState *st = J.state;
  if (st->status != 0 || st->m0 == 0 || st->m1 == 0) return;
  const u64 count = st->cand_count;
  if (count > J.cand_cap) {
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(&st->flags, kFlagCandOverflow);
    return;
  }
  const float thr = tol_threshold(J, __uint_as_float(st->tau_key));
  const uint32_t lane = lane_id();
  for (u64 i0 = (u64)blockIdx.x * blockDim.x; i0 < count; i0 += (u64)gridDim.x * blockDim.x) {
    const u64 i = i0 + threadIdx.x;
    bool keep = false;
    Cand c;
    if (i < count) {
      c = J.cand[i];
      keep = c.est >= thr;
    }
    const u64 mask = ballot(keep);
    if (mask == 0) continue;
    const uint32_t leader = __ffsll((long long)mask) - 1;
    uint32_t base = 0;
    if (lane == leader) base = atomicAdd(&st->l1_count, (uint32_t)popc64(mask));
    base = __shfl(base, leader);
    if (keep) {
      const u64 lt = lane ? (~0ull >> (64 - lane)) : 0ull;
      const uint32_t at = base + popc64(mask & lt);
      if (at < J.l1_cap) J.l1[at] = c;
    }
  }
}

// Radix selection (12 + 12 + 7 bits of a non-negative float's bits) of the
// N-th largest of M > N keys, key(i) for i in [0, M), by one workgroup of
// 1024 threads.  Each pass histograms the keys that match the digits found so
// far, then locates the bin holding the N-th largest with a parallel scan of
// the bin counts from the top.
constexpr uint32_t kRadixThreads = 1024;
struct RadixLds {
  uint32_t hist[4096];
  uint32_t wsum[kRadixThreads / 64];
  uint32_t prefix, need;
};

template <typename KeyAt>
__device__ uint32_t radix_kth_largest(KeyAt key_at, uint32_t M, uint32_t N, RadixLds &s) {
  const uint32_t tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  if (tid == 0) {
    s.prefix = 0;
    s.need = N;  // rank (1-based, from the top) still to locate
  }
  const int shifts[3] = {19, 7, 0};
  const int widths[3] = {12, 12, 7};
  uint32_t known_mask = 0;
  for (int pass = 0; pass < 3; ++pass) {
    for (uint32_t i = tid; i < 4096; i += kRadixThreads) s.hist[i] = 0;
    __syncthreads();
    const uint32_t prefix = s.prefix, need = s.need;
    const uint32_t bins = 1u << widths[pass];
    for (uint32_t i = tid; i < M; i += kRadixThreads) {
      const uint32_t key = key_at(i);
      if ((key & known_mask) == prefix) atomicAdd(&s.hist[(key >> shifts[pass]) & (bins - 1)], 1u);
    }
    __syncthreads();
    // thread t owns `per` consecutive bins counted from the top
    const uint32_t per = (bins + kRadixThreads - 1) / kRadixThreads;
    const uint32_t top = bins - 1 - tid * per;  // highest bin of this thread
    uint32_t mine = 0;
    for (uint32_t q = 0; q < per; ++q)
      if (tid * per + q < bins) mine += s.hist[top - q];
    // inclusive scan over threads (from the top)
    uint32_t inc = mine;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const uint32_t o = __shfl_up(inc, off);
      if (lane >= (uint32_t)off) inc += o;
    }
    if (lane == 63) s.wsum[wv] = inc;
    __syncthreads();
    uint32_t before = 0;
    for (uint32_t q = 0; q < wv; ++q) before += s.wsum[q];
    const uint32_t excl = before + inc - mine;
    // the thread whose range of the running count crosses `need`; bin 0 takes
    // whatever is left (it is the lowest possible digit)
    if (tid * per < bins && excl < need && (excl + mine >= need || tid * per + per >= bins)) {
      uint32_t run = excl;
      uint32_t bin = top;
      for (uint32_t q = 0; q < per && tid * per + q < bins; ++q) {
        bin = top - q;
        if (run + s.hist[bin] >= need || bin == 0) break;
        run += s.hist[bin];
      }
      s.need = need - run;
      s.prefix = prefix | (bin << shifts[pass]);
    }
    known_mask |= (bins - 1) << shifts[pass];
    __syncthreads();
  }
  return s.prefix;
}

// 0. pilot: histogram of the pilot sample's scores (2048 bins of the float
// bits' top, as the scan's survivor histogram), then the lower edge of the
// bin holding the top_n-th largest.  The top_n-th largest score of a sample
// is at most the top_n-th largest score of the whole job, so that edge is a
// valid starting bound for the scan's filter.
__global__ __launch_bounds__(256) void pilot_hist_kernel(Globals g) {
  const JobDesc &J = g.jobs[blockIdx.y];
  JobState *st = J.state;
  if (J.pilot_tiles == 0 || st->status != 0 || st->m0 == 0 || st->m1 == 0) return;
  __shared__ uint32_t h[kHistBins];
  for (uint32_t i = threadIdx.x; i < (uint32_t)kHistBins; i += blockDim.x) h[i] = 0;
  __syncthreads();
  const uint32_t *keys = reinterpret_cast<const uint32_t *>(J.cand);
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < J.pilot_slots; i += gridDim.x * blockDim.x) {
    const uint32_t key = keys[i];
    if (key != 0) atomicAdd(&h[key >> kHistShift], 1u);
  }
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < (uint32_t)kHistBins; i += blockDim.x)
    if (h[i]) atomicAdd(&J.phist[i], h[i]);
}

__global__ __launch_bounds__(64) void pilot_tau_kernel(Globals g) {
  const JobDesc &J = g.jobs[blockIdx.x];
  JobState *st = J.state;
  if (J.pilot_tiles == 0 || st->status != 0 || st->m0 == 0 || st->m1 == 0) return;
  refresh_tau(J.phist, st, J.top_n, lane_id());
}

// 2. one workgroup per job: radix selection of the top_n-th largest key over
// the compacted candidates, then the final candidate set, compacted in place
// to the front of l1 (order kept): a chunk's entries are all read before any
// of its kept entries is written, and a kept entry only moves down.
__global__ __launch_bounds__(1024) void select_kernel(Globals g) {
  const JobDesc &J = g.jobs[blockIdx.x];
  JobState *st = J.state;
  if (st->status != 0 || st->m0 == 0 || st->m1 == 0) return;
  if (st->flags & kFlagCandOverflow) return;
  __shared__ RadixLds s;
  __shared__ uint32_t s_wcnt[kRadixThreads / 64];
  __shared__ uint32_t s_base;
  const uint32_t tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const uint32_t M = min(st->l1_count, J.l1_cap);
  const uint32_t N = J.top_n;
  if (M <= N) {  // every candidate is kept
    if (tid == 0) st->l2_count = M;
    return;
  }
  const uint32_t kth = radix_kth_largest([&](uint32_t i) { return J.l1[i].key; }, M, N, s);
  if (tid == 0) {
    st->kth_key = kth;
    s_base = 0;
  }
  const float thr2 = tol_threshold(J, __uint_as_float(kth));
  __syncthreads();
  const u64 below = lane ? (~0ull >> (64 - lane)) : 0ull;
  for (uint32_t i0 = 0; i0 < M; i0 += blockDim.x) {
    const uint32_t i = i0 + tid;
    Cand c;
    bool keep = false;
    if (i < M) {
      c = J.l1[i];
      keep = c.est >= thr2;
    }
    const u64 mask = ballot(keep);
    if (lane == 0) s_wcnt[wv] = popc64(mask);
    __syncthreads();
    uint32_t at = s_base;
    for (uint32_t q = 0; q < wv; ++q) at += s_wcnt[q];
    if (keep) J.l1[at + popc64(mask & below)] = c;
    __syncthreads();
    if (tid == 0) {
      uint32_t t = s_base;
      for (uint32_t q = 0; q < kRadixThreads / 64; ++q) t += s_wcnt[q];
      s_base = t;
    }
    __syncthreads();
  }
  if (tid == 0) st->l2_count = s_base;
}

// 3. one wave per kept candidate: recount the contingency table with one lane
// per genotype cell (AND of the cell's rows, popcount per class), then MI in
// double precision.  Also used for explicit tables (fiuncho_contingency).
// Orders 2 and 3: one pass over the words, every cell of the table counted
// per lane from the rows loaded once, then one wave sum per cell and class.
template <int K, bool WRITE_TABLE>
__device__ void count_cells_small(const JobDesc &J, const JobState *st, const uint32_t *c,
                                  uint32_t lane, uint32_t *lds_t, uint32_t *table_out) {
  constexpr int NC = K == 2 ? 9 : 27;
  const uint32_t W0 = st->W0, W = st->W0 + st->W1, wcap = J.wcap;
  uint32_t t[NC][2];
#pragma unroll
  for (int x = 0; x < NC; ++x) t[x][0] = t[x][1] = 0;
#pragma unroll
  for (int cls = 0; cls < 2; ++cls) {
    const uint32_t wb = cls ? W0 : 0, we = cls ? W : W0;
    for (uint32_t w = wb + lane; w < we; w += 64) {
      u64 r[K][3];
#pragma unroll
      for (int i = 0; i < K; ++i)
#pragma unroll
        for (int gg = 0; gg < 3; ++gg) r[i][gg] = J.Bs[((size_t)c[i] * wcap + w) * 4 + gg];
#pragma unroll
      for (int x = 0; x < NC; ++x) {
        // cell x = sum_i g_i 3^(K-1-i)
        u64 a = ~0ull;
        int rem = x;
#pragma unroll
        for (int i = K - 1; i >= 0; --i) {
          a &= r[i][rem % 3];
          rem /= 3;
        }
        t[x][cls] += popc64(a);
      }
    }
  }
#pragma unroll
  for (int x = 0; x < NC; ++x)
#pragma unroll
    for (int cls = 0; cls < 2; ++cls) {
      uint32_t v = t[x][cls];
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
      if (lane == 0) {
        if (lds_t) lds_t[2 * x + cls] = v;
        if (WRITE_TABLE) table_out[2 * x + cls] = v;
      }
    }
}

template <bool WRITE_TABLE>
__device__ void count_cells(const JobDesc &J, const JobState *st, const uint32_t *c,
                            uint32_t k, uint32_t lane, uint32_t *lds_t,
                            uint32_t *table_out) {
  if (k == 2) return count_cells_small<2, WRITE_TABLE>(J, st, c, lane, lds_t, table_out);
  if (k == 3) return count_cells_small<3, WRITE_TABLE>(J, st, c, lane, lds_t, table_out);
  uint32_t cells = 1;
  for (uint32_t i = 0; i < k; ++i) cells *= 3;
  const uint32_t W0 = st->W0, W = st->W0 + st->W1, wcap = J.wcap;
  // cell x = sum_i g_i 3^(k-1-i): lanes split the words, a wave sum per class
  uint32_t g[kMaxOrder];
  for (uint32_t i = 0; i < k; ++i) g[i] = 0;
  for (uint32_t x = 0; x < cells; ++x) {
    uint32_t n0 = 0, n1 = 0;
    for (uint32_t w = lane; w < W; w += 64) {
      u64 r = ~0ull;
      for (uint32_t i = 0; i < k; ++i) r &= J.Bs[((size_t)c[i] * wcap + w) * 4 + g[i]];
      if (w < W0) n0 += popc64(r);
      else n1 += popc64(r);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      n0 += __shfl_xor(n0, off);
      n1 += __shfl_xor(n1, off);
    }
    if (lane == 0) {
      if (lds_t) {
        lds_t[2 * x] = n0;
        lds_t[2 * x + 1] = n1;
      }
      if (WRITE_TABLE) {
        table_out[2 * x] = n0;
        table_out[2 * x + 1] = n1;
      }
    }
    // next cell: increment the base-3 digits, last variant fastest
    for (int i = (int)k - 1; i >= 0; --i) {
      if (++g[i] < 3) break;
      g[i] = 0;
    }
  }
}

// H(X) + H(Y) - H(X,Y) with plug-in probabilities (Eq. 1-3), evaluated as
// running differences in a fixed order (cells ascending, then classes); P64
// holds (t/m) ln(t/m) computed on the host.
__device__ double mi64_of_table(const double *__restrict__ P64, const uint32_t *t,
                                uint32_t cells, uint32_t m0, uint32_t m1) {
  double hx = 0.0, hy = 0.0, hxy = 0.0;
  for (uint32_t x = 0; x < cells; ++x) hx = hx - P64[t[2 * x] + t[2 * x + 1]];
  hy = hy - P64[m0];
  hy = hy - P64[m1];
  for (uint32_t x = 0; x < cells; ++x) {
    hxy = hxy - P64[t[2 * x]];
    hxy = hxy - P64[t[2 * x + 1]];
  }
  return (hx + hy) - hxy;
}

// m * MI = [f(m) - f(m0) - f(m1)] + sum_x [f(n_x0) + f(n_x1) - f(n_x0 + n_x1)]
// (Eq. 1-3 multiplied out, f(t) = t ln t) in single precision: f as an
// unevaluated pair hi + lo of floats, accumulated with TwoSum so that the
// cancellation of the m ln m sized terms loses nothing.
__device__ float mi32_compensated(const float2 *__restrict__ F, const uint32_t *t,
                                  uint32_t cells, uint32_t m, uint32_t m0, uint32_t m1) {
  float s = F[m].x, e = 0.f;
  two_sum_add(s, e, -F[m0].x);
  two_sum_add(s, e, -F[m1].x);
  e += (F[m].y - F[m0].y) - F[m1].y;
  for (uint32_t x = 0; x < cells; ++x) {
    const float2 a = F[t[2 * x]], b = F[t[2 * x + 1]], c = F[t[2 * x] + t[2 * x + 1]];
    two_sum_add(s, e, a.x);
    two_sum_add(s, e, b.x);
    two_sum_add(s, e, -c.x);
    e += (a.y + b.y) - c.y;
  }
  return (s + e) / (float)m;
}

constexpr int kMaxCells = 6561;  // 3^8

// 3. one workgroup (one wave) per kept candidate l1[i], i < l2_count: its
// exact table, MI in double precision and compensated single precision,
// written to entry i of the candidate buffer (as Scored)
__global__ __launch_bounds__(64) void rescore_kernel(Globals g) {
  const JobDesc &J = g.jobs[blockIdx.y];
  JobState *st = J.state;
  if (st->status != 0 || st->m0 == 0 || st->m1 == 0) return;
  if (st->flags & kFlagCandOverflow) return;
  extern __shared__ uint32_t lds_t[];
  const uint32_t lane = lane_id();
  const uint32_t count = st->l2_count;
  Scored *sc = reinterpret_cast<Scored *>(J.cand);
  uint32_t cells = 1;
  for (uint32_t q = 0; q < J.k; ++q) cells *= 3;
  for (uint32_t i = blockIdx.x; i < count; i += gridDim.x) {
    const Cand cd = J.l1[i];
    uint32_t c[kMaxOrder];
    lex_unrank(g, J.n, J.k, cd.rank, c);
    count_cells<false>(J, st, c, J.k, lane, lds_t, nullptr);
    __syncthreads();
    if (lane == 0) {
      Scored r;
      r.mi = mi64_of_table(J.P64, lds_t, cells, st->m0, st->m1);
      r.mi32 = mi32_compensated(J.F32, lds_t, cells, J.m, st->m0, st->m1);
      r.pad = 0;
      // the filters assumed |estimate - mi| <= fbound
      if (fabs((double)cd.est - r.mi) > (double)J.fbound) atomicOr(&st->flags, kFlagBound);
      sc[i] = r;
    }
    __syncthreads();
  }
}

// A result as the caller sees it: the combination unranked from its rank
__device__ fiuncho_hit make_hit(const Globals &g, const JobDesc &J, u64 rank, double mi, float mi32,
                                float est) {
  fiuncho_hit h;
  uint32_t c[kMaxOrder];
  lex_unrank(g, J.n, J.k, rank, c);
  for (uint32_t q = 0; q < kMaxOrder; ++q) h.snp[q] = q < J.k ? c[q] : 0xffffffffu;
  h.rank = rank;
  h.mi = mi;
  h.mi32 = mi32;
  const double d = fabs((double)mi32 - mi);
  h.rel_err = mi != 0.0 ? (float)(d / fabs(mi)) : (float)d;
  h.est = est;
  h.reserved = 0;
  return h;
}

// An unsigned integer whose order is the order of the double d (finite d)
__device__ __forceinline__ u64 order_key(double d) {
  const u64 b = (u64)__double_as_longlong(d);
  return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}

// (mi, rank) of a precedes (mi, rank) of b in the output order
__device__ __forceinline__ bool precedes(double ma, u64 ra, double mb, u64 rb) {
  return ma > mb || (ma == mb && ra < rb);
}

// Radix selection of the N-th largest of 64-bit keys among the elements i in
// [0, M) that take part (key_at(i, key) returns whether element i does; at
// least N do), by one workgroup of kRadixThreads threads: six passes of 11,
// 11, 11, 11, 10 and 10 bits, each histogramming the keys that match the
// digits found so far.  Returns the key; *ties_in receives how many of the
// elements equal to it belong to the N largest.
struct RadixLds64 {
  uint32_t hist[2048];
  uint32_t wsum[kRadixThreads / 64];
  u64 prefix;
  uint32_t need;
};

template <typename KeyAt>
__device__ u64 radix_kth_largest64(KeyAt key_at, uint32_t M, uint32_t N, RadixLds64 &s,
                                   uint32_t *ties_in) {
  const uint32_t tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  if (tid == 0) {
    s.prefix = 0;
    s.need = N;
  }
  const int shifts[6] = {53, 42, 31, 20, 10, 0};
  const int widths[6] = {11, 11, 11, 11, 10, 10};
  u64 known = 0;
  for (int pass = 0; pass < 6; ++pass) {
    for (uint32_t i = tid; i < 2048; i += kRadixThreads) s.hist[i] = 0;
    __syncthreads();
    const u64 prefix = s.prefix;
    const uint32_t need = s.need;
    const uint32_t bins = 1u << widths[pass];
    for (uint32_t i = tid; i < M; i += kRadixThreads) {
      u64 key;
      if (key_at(i, key) && (key & known) == prefix)
        atomicAdd(&s.hist[(uint32_t)(key >> shifts[pass]) & (bins - 1)], 1u);
    }
    __syncthreads();
    // thread t owns `per` consecutive bins counted from the top
    const uint32_t per = (bins + kRadixThreads - 1) / kRadixThreads;
    const uint32_t top = bins - 1 - tid * per;
    uint32_t mine = 0;
    for (uint32_t q = 0; q < per; ++q)
      if (tid * per + q < bins) mine += s.hist[top - q];
    uint32_t inc = mine;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const uint32_t o = __shfl_up(inc, off);
      if (lane >= (uint32_t)off) inc += o;
    }
    if (lane == 63) s.wsum[wv] = inc;
    __syncthreads();
    uint32_t before = 0;
    for (uint32_t q = 0; q < wv; ++q) before += s.wsum[q];
    const uint32_t excl = before + inc - mine;
    if (tid * per < bins && excl < need && (excl + mine >= need || tid * per + per >= bins)) {
      uint32_t run = excl;
      uint32_t bin = top;
      for (uint32_t q = 0; q < per && tid * per + q < bins; ++q) {
        bin = top - q;
        if (run + s.hist[bin] >= need || bin == 0) break;
        run += s.hist[bin];
      }
      s.need = need - run;
      s.prefix = prefix | ((u64)bin << shifts[pass]);
    }
    known |= (u64)(bins - 1) << shifts[pass];
    __syncthreads();
  }
  const u64 kth = s.prefix;
  if (ties_in) *ties_in = s.need;
  __syncthreads();
  return kth;
}

// Bitonic sort in LDS of P (a power of two) items by (mi descending, rank
// ascending), carrying a 16-bit index
__device__ void lds_sort(double *s_mi, u64 *s_rank, uint16_t *s_idx, uint32_t P) {
  const uint32_t tid = threadIdx.x;
  for (uint32_t size = 2; size <= P; size <<= 1) {
    for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
      for (uint32_t i = tid; i < P; i += blockDim.x) {
        const uint32_t jx = i ^ stride;
        if (jx > i) {
          const bool up = (i & size) == 0;
          const bool i_first = precedes(s_mi[i], s_rank[i], s_mi[jx], s_rank[jx]);
          if (i_first != up) {
            const double tm = s_mi[i];
            s_mi[i] = s_mi[jx];
            s_mi[jx] = tm;
            const u64 tr = s_rank[i];
            s_rank[i] = s_rank[jx];
            s_rank[jx] = tr;
            const uint16_t ti = s_idx[i];
            s_idx[i] = s_idx[jx];
            s_idx[jx] = ti;
          }
        }
      }
      __syncthreads();
    }
  }
}

// 4. one workgroup per job: the first min(top_n, C(n, k)) results by (mi
// descending, rank ascending).  Up to kSortMax kept candidates are sorted in
// LDS.  More (near-ties at the cut-off, or a large top_n) are first reduced
// to exactly the results by two radix selections (the N-th largest MI, then
// among the candidates with that MI the ranks that complete the N) and
// gathered into sel; those are sorted in LDS when they fit, else left to the
// multi-block sort.
__global__ __launch_bounds__(1024) void finish_kernel(Globals g) {
  const JobDesc &J = g.jobs[blockIdx.x];
  JobState *st = J.state;
  const uint32_t tid = threadIdx.x;
  __shared__ double s_mi[kSortMax];
  __shared__ u64 s_rank[kSortMax];
  __shared__ uint16_t s_idx[kSortMax];
  __shared__ RadixLds64 rs;
  __shared__ uint32_t s_count;
  int32_t status = st->status;
  if (status == 0 && (st->flags & kFlagCandOverflow)) status = FIUNCHO_E_WORKSPACE;
  if (status == 0 && (st->flags & kFlagBound)) status = FIUNCHO_E_INTERNAL;
  const u64 want64 = J.total < (u64)J.top_n ? J.total : (u64)J.top_n;
  const uint32_t want = (uint32_t)want64;
  if (status != 0) {
    if (tid == 0) {
      *J.n_out = 0;
      if (J.status_out) *J.status_out = status;
    }
    return;
  }
  if (st->m0 == 0 || st->m1 == 0) {
    // an empty class: every table is independent of the class, MI = 0, and the
    // total order makes the result the first top_n ranks (of a shard: the
    // first top_n ranks congruent to shard_index modulo shard_count)
    const u64 sc = J.shard_count, si = J.shard_index;
    const u64 share = J.total > si ? (J.total - si + sc - 1) / sc : 0;
    const uint32_t want_e = (uint32_t)(share < (u64)J.top_n ? share : (u64)J.top_n);
    for (uint32_t i = tid; i < want_e; i += blockDim.x) J.out[i] = make_hit(g, J, si + (u64)i * sc, 0.0, 0.f, 0.f);
    if (tid == 0) {
      *J.n_out = want_e;
      if (J.status_out) *J.status_out = 0;
    }
    return;
  }
  const uint32_t M = st->l2_count;
  const Scored *sc = reinterpret_cast<const Scored *>(J.cand);
  const uint32_t outn = min(want, M);
  bool from_sel = false;
  if (M > kSortMax) {
    // reduce the M kept candidates to exactly the outn results, in sel
    u64 kth = 0, rcut = ~0ull;
    if (outn < M) {
      uint32_t ties = 0;
      kth = radix_kth_largest64(
          [&](uint32_t i, u64 &key) {
            key = order_key(sc[i].mi);
            return true;
          },
          M, outn, rs, &ties);
      // among the candidates whose MI has that key, the `ties` smallest ranks
      rcut = ~radix_kth_largest64(
          [&](uint32_t i, u64 &key) {
            key = ~J.l1[i].rank;
            return order_key(sc[i].mi) == kth;
          },
          M, ties, rs, nullptr);
    }
    if (tid == 0) s_count = 0;
    __syncthreads();
    for (uint32_t i = tid; i < M; i += blockDim.x) {
      const double mi = sc[i].mi;
      const u64 key = order_key(mi), rank = J.l1[i].rank;
      if (outn == M || key > kth || (key == kth && rank <= rcut)) {
        const uint32_t at = atomicAdd(&s_count, 1u);
        if (at < J.sel_cap) {
          SortItem it;
          it.mi = mi;
          it.rank = rank;
          it.idx = i;
          it.pad = 0;
          J.sel[at] = it;
        }
      }
    }
    __syncthreads();
    if (outn > kSortMax) {
      // ordered by the multi-block sort, which also writes the hits
      if (tid == 0) st->n_sel = outn;
      return;
    }
    from_sel = true;
  }
  // LDS sort of min(M, kSortMax) items: the kept candidates, or the selected
  // results in sel
  const uint32_t L = from_sel ? outn : M;
  uint32_t P = 1;
  while (P < L) P <<= 1;
  for (uint32_t i = tid; i < P; i += blockDim.x) {
    if (i < L) {
      if (from_sel) {
        const SortItem it = J.sel[i];
        s_mi[i] = it.mi;
        s_rank[i] = it.rank;
      } else {
        s_mi[i] = sc[i].mi;
        s_rank[i] = J.l1[i].rank;
      }
    } else {
      s_mi[i] = -INFINITY;
      s_rank[i] = ~0ull;
    }
    s_idx[i] = (uint16_t)i;
  }
  __syncthreads();
  lds_sort(s_mi, s_rank, s_idx, P);
  for (uint32_t i = tid; i < outn; i += blockDim.x) {
    const uint32_t c = from_sel ? J.sel[s_idx[i]].idx : s_idx[i];
    J.out[i] = make_hit(g, J, s_rank[i], s_mi[i], sc[c].mi32, J.l1[c].est);
  }
  if (tid == 0) {
    *J.n_out = outn;
    if (J.status_out) *J.status_out = 0;
  }
}

// ---------------------------------------------------------------------------
// Multi-block ordering of more than kSortMax results (jobs whose top_n
// exceeds kSortMax; n_sel of them in sel): chunks of kChunkSort sorted in LDS,
// then merge passes of doubling run length (each item finds its place by a
// binary search in the partner run; ranks are unique, so places are too),
// then the hits.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void sort_chunks_kernel(Globals g) {
  const JobDesc &J = g.jobs[blockIdx.y];
  const uint32_t n = J.state->n_sel;
  const uint32_t base = blockIdx.x * kChunkSort;
  if (n == 0 || base >= n) return;
  __shared__ double s_mi[kChunkSort];
  __shared__ u64 s_rank[kChunkSort];
  __shared__ uint32_t s_idx[kChunkSort];
  const uint32_t cnt = min(kChunkSort, n - base);
  const uint32_t tid = threadIdx.x;
  for (uint32_t i = tid; i < kChunkSort; i += blockDim.x) {
    if (i < cnt) {
      const SortItem it = J.sel[base + i];
      s_mi[i] = it.mi;
      s_rank[i] = it.rank;
      s_idx[i] = it.idx;
    } else {
      s_mi[i] = -INFINITY;
      s_rank[i] = ~0ull;
      s_idx[i] = 0;
    }
  }
  __syncthreads();
  for (uint32_t size = 2; size <= kChunkSort; size <<= 1) {
    for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
      for (uint32_t i = tid; i < kChunkSort; i += blockDim.x) {
        const uint32_t jx = i ^ stride;
        if (jx > i) {
          const bool up = (i & size) == 0;
          if (precedes(s_mi[i], s_rank[i], s_mi[jx], s_rank[jx]) != up) {
            const double tm = s_mi[i];
            s_mi[i] = s_mi[jx];
            s_mi[jx] = tm;
            const u64 tr = s_rank[i];
            s_rank[i] = s_rank[jx];
            s_rank[jx] = tr;
            const uint32_t ti = s_idx[i];
            s_idx[i] = s_idx[jx];
            s_idx[jx] = ti;
          }
        }
      }
      __syncthreads();
    }
  }
  for (uint32_t i = tid; i < cnt; i += blockDim.x) {
    SortItem it;
    it.mi = s_mi[i];
    it.rank = s_rank[i];
    it.idx = s_idx[i];
    it.pad = 0;
    J.sel[base + i] = it;
  }
}

// one merge pass: sorted runs of `width` items, from sel to sel2 (to_sel2) or
// back; an item without a partner run keeps its place
__global__ __launch_bounds__(256) void merge_pass_kernel(Globals g, uint32_t width, int to_sel2) {
  const JobDesc &J = g.jobs[blockIdx.y];
  const uint32_t n = J.state->n_sel;
  if (n == 0) return;
  const SortItem *src = to_sel2 ? J.sel : J.sel2;
  SortItem *dst = to_sel2 ? J.sel2 : J.sel;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const SortItem it = src[i];
    const uint32_t r = i / width;
    const uint32_t start = r * width;
    const u64 pstart64 = (u64)(r ^ 1u) * width;
    uint32_t pos = i;
    if (pstart64 < n) {
      const uint32_t pstart = (uint32_t)pstart64;
      const uint32_t plen = min(width, n - pstart);
      // partner items that precede this one
      uint32_t lo = 0, hi = plen;
      while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        const SortItem p = src[pstart + mid];
        if (precedes(p.mi, p.rank, it.mi, it.rank)) lo = mid + 1;
        else hi = mid;
      }
      pos = min(start, pstart) + (i - start) + lo;
    }
    dst[pos] = it;
  }
}

// the hits of the ordered results (in sel or sel2)
__global__ __launch_bounds__(256) void sorted_hits_kernel(Globals g, int in_sel2) {
  const JobDesc &J = g.jobs[blockIdx.y];
  JobState *st = J.state;
  const uint32_t n = st->n_sel;
  if (n == 0) return;
  const SortItem *src = in_sel2 ? J.sel2 : J.sel;
  const Scored *sc = reinterpret_cast<const Scored *>(J.cand);
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const SortItem it = src[i];
    J.out[i] = make_hit(g, J, it.rank, it.mi, sc[it.idx].mi32, J.l1[it.idx].est);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    *J.n_out = n;
    if (J.status_out) *J.status_out = 0;
  }
}

// Tables and scores of explicit combinations (job 0): one wave per rank.
// Any output may be null.  est is the plain single-precision evaluation the
// scan filters with (cells in ascending order), mi32 the compensated one, mi
// the double-precision one.
__global__ __launch_bounds__(64) void tables_kernel(Globals g, const u64 *ranks, u64 n_ranks,
                                                    uint32_t *tables, float *est, float *mi32,
                                                    double *mi) {
  const JobDesc &J = g.jobs[0];
  const JobState *st = J.state;
  if (st->status != 0) return;
  extern __shared__ uint32_t lds_t[];
  uint32_t cells = 1;
  for (uint32_t q = 0; q < J.k; ++q) cells *= 3;
  const u64 stride = (u64)gridDim.x * gridDim.y;
  for (u64 i = blockIdx.x + (u64)blockIdx.y * gridDim.x; i < n_ranks; i += stride) {
    uint32_t c[kMaxOrder];
    lex_unrank(g, J.n, J.k, ranks[i], c);
    if (tables) count_cells<true>(J, st, c, J.k, lane_id(), lds_t, tables + i * 2 * cells);
    else count_cells<false>(J, st, c, J.k, lane_id(), lds_t, nullptr);
    __syncthreads();
    if (lane_id() == 0) {
      if (est) {
        const float *F = J.Fh;
        float fs = (F[J.m] - F[st->m0]) - F[st->m1];
        for (uint32_t x = 0; x < cells; ++x) {
          const uint32_t a = lds_t[2 * x], b = lds_t[2 * x + 1];
          fs += (F[a] + F[b]) - F[a + b];
        }
        est[i] = fs * (1.0f / (float)J.m);
      }
      if (mi32) mi32[i] = mi32_compensated(J.F32, lds_t, cells, J.m, st->m0, st->m1);
      if (mi) mi[i] = mi64_of_table(J.P64, lds_t, cells, st->m0, st->m1);
    }
    __syncthreads();
  }
}

void launch_select(const Globals &g, uint32_t max_cand_cap, hipStream_t s) {
  uint32_t blocks = (max_cand_cap + 255) / 256;
  if (blocks > 1024) blocks = 1024;
  if (blocks == 0) blocks = 1;
  hipLaunchKernelGGL(compact_kernel, dim3(blocks, g.n_jobs), dim3(256), 0, s, g);
  hipLaunchKernelGGL(select_kernel, dim3(g.n_jobs), dim3(1024), 0, s, g);
}

void launch_pilot_select(const Globals &g, uint32_t max_pilot_slots, hipStream_t s) {
  uint32_t blocks = (max_pilot_slots + 4095) / 4096;
  blocks = blocks < 1 ? 1 : (blocks > 256 ? 256 : blocks);
  hipLaunchKernelGGL(pilot_hist_kernel, dim3(blocks, g.n_jobs), dim3(256), 0, s, g);
  hipLaunchKernelGGL(pilot_tau_kernel, dim3(g.n_jobs), dim3(64), 0, s, g);
}

void launch_rescore(const Globals &g, uint32_t max_k, hipStream_t s) {
  uint32_t cells = 1;
  for (uint32_t q = 0; q < max_k; ++q) cells *= 3;
  const size_t lds = sizeof(uint32_t) * 2 * cells;
  // one candidate per workgroup up to 2,048 kept candidates: each one's work
  // is a chain of dependent steps (unrank, count, score)
  hipLaunchKernelGGL(rescore_kernel, dim3(2048, g.n_jobs), dim3(64), lds, s, g);
}

void launch_finish(const Globals &g, hipStream_t s) {
  hipLaunchKernelGGL(finish_kernel, dim3(g.n_jobs), dim3(1024), 0, s, g);
}

void launch_big_sort(const Globals &g, uint32_t max_sel, hipStream_t s) {
  if (max_sel <= kSortMax) return;
  const uint32_t chunks = (max_sel + kChunkSort - 1) / kChunkSort;
  hipLaunchKernelGGL(sort_chunks_kernel, dim3(chunks, g.n_jobs), dim3(1024), 0, s, g);
  const uint32_t blocks = std::min<uint32_t>((max_sel + 255) / 256, 4096);
  int in_sel2 = 0;
  for (uint64_t width = kChunkSort; width < max_sel; width <<= 1) {
    hipLaunchKernelGGL(merge_pass_kernel, dim3(blocks, g.n_jobs), dim3(256), 0, s, g, (uint32_t)width,
                       in_sel2 ? 0 : 1);
    in_sel2 ^= 1;
  }
  hipLaunchKernelGGL(sorted_hits_kernel, dim3(blocks, g.n_jobs), dim3(256), 0, s, g, in_sel2);
}

void launch_tables(const Globals &g, const unsigned long long *ranks, uint64_t n_ranks,
                   uint32_t *tables, float *est, float *mi32, double *mi, uint32_t k,
                   hipStream_t s) {
  uint32_t cells = 1;
  for (uint32_t q = 0; q < k; ++q) cells *= 3;
  const uint64_t gx = n_ranks < 65535 ? (n_ranks ? n_ranks : 1) : 65535;
  const uint64_t gy = std::min<uint64_t>((n_ranks + gx - 1) / gx, 64);
  hipLaunchKernelGGL(tables_kernel, dim3((uint32_t)gx, (uint32_t)(gy ? gy : 1)), dim3(64),
                     sizeof(uint32_t) * 2 * cells, s, g, ranks, (u64)n_ranks, tables, est, mi32, mi);
}

}  // namespace fiuncho
