// filter.hpp -- what every counting kernel shares: the wave-uniform view of a
// job, the single-precision MI estimate of a table (section 3.3, Eq. 1-3) and
// the filter that appends the combinations that may be among the best top_n
// (Algorithm 1's sorted list, kept as a device-wide candidate buffer).
#pragma once

#include <type_traits>

#include "device_common.hpp"

namespace fiuncho {

// Wave-uniform copy of what a tile needs from its job (every field is read
// into scalar registers once per tile).
struct JV {
  uint32_t n, m, k, top_n, n_pad, wcap, cand_cap, m0, m1, W0, W1;
  u64 total;
  const u64 *Bv;
  const u64 *Bs;
  const uint32_t *marg;
  uint32_t *hist;
  Cand *cand;
  JobState *st;
  const uint32_t *pairs;
  const uint4 *pairs4;
  const uint32_t *triples;
  const uint4 *triples4;
  const uint4 *quads4;
  uint32_t path;
  uint32_t fp4;               // matrix-core paths: FP4 operands (else int8)
  const float *Fh;
  const uint32_t *Fq;
  float qscale;
  float fbound;
  mutable uint32_t *pk;       // pilot launch: this wave's next 64 score slots
};

template <typename T>
__device__ __forceinline__ T *uni_ptr(T *p) {
  return reinterpret_cast<T *>(uni64(reinterpret_cast<u64>(p)));
}

__device__ __forceinline__ JV load_view(const JobDesc *jd) {
  const FI_CONST JobDesc *J = as_const(jd);
  JV v;
  v.n = uni(J->n);
  v.m = uni(J->m);
  v.k = uni(J->k);
  v.top_n = uni(J->top_n);
  v.n_pad = uni(J->n_pad);
  v.wcap = uni(J->wcap);
  v.cand_cap = uni(J->cand_cap);
  v.total = uni64(J->total);
  v.Bv = uni_ptr(J->Bv);
  v.Bs = uni_ptr(J->Bs);
  v.marg = uni_ptr(J->marg);
  v.hist = uni_ptr(J->hist);
  v.cand = uni_ptr(J->cand);
  v.st = uni_ptr(J->state);
  v.pairs = uni_ptr(J->pairs);
  v.pairs4 = uni_ptr(J->pairs4);
  v.triples = uni_ptr(J->triples);
  v.triples4 = uni_ptr(J->triples4);
  v.quads4 = uni_ptr(J->quads4);
  v.path = uni(J->path);
  v.fp4 = uni(J->fp4);
  v.Fh = uni_ptr(J->Fh);
  v.Fq = uni_ptr(J->Fq);
  v.qscale = __uint_as_float(uni(__float_as_uint(J->qscale)));
  v.fbound = __uint_as_float(uni(__float_as_uint(J->fbound)));
  v.pk = nullptr;
  return v;
}

// m * MI = [f(m) - f(m0) - f(m1)] + sum_x [f(n_x0) + f(n_x1) - f(n_x0 + n_x1)]
// with f(t) = t ln t: Eq. 1-3 with plug-in probabilities, multiplied out.
// The scan evaluates it in plain single precision from a float table of f
// (or in fixed point, see MiConst); the job's fbound bounds the rounding error
// of the resulting MI, and every filter below widens its threshold by twice
// that bound.
// F is the table in global memory or a copy of it in LDS.
template <typename FP>
__device__ __forceinline__ float mi_term(FP F, uint32_t n0, uint32_t n1) {
  return (F[n0] + F[n1]) - F[n0 + n1];
}

// Lower bound of the top_n-th best score from the survivor histogram: the bin
// where the count from the top reaches top_n holds the top_n-th largest
// appended score, so its lower edge is a valid bound.  One wave.
static __device__ __noinline__ void refresh_tau(uint32_t *hist, JobState *st, uint32_t top_n,
                                         uint32_t lane) {
  constexpr int PER = kHistBins / 64;
  const uint32_t *bins = hist + lane * PER;
  uint32_t tot = 0;
  for (int i = 0; i < PER; ++i) tot += load_relaxed(&bins[i]);
  uint32_t suf = tot;  // sum over lanes >= this lane
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    uint32_t o = __shfl_down(suf, off);
    if (lane + off < 64) suf += o;
  }
  const u64 ok = ballot(suf >= top_n);
  if (ok == 0) return;
  const uint32_t L = 63 - __clzll((long long)ok);
  if (lane == L) {
    uint32_t run = suf - tot;
    uint32_t bin = L * PER;
    for (int i = PER - 1; i >= 0; --i) {
      run += load_relaxed(&bins[i]);
      if (run >= top_n) {
        bin = L * PER + i;
        break;
      }
    }
    atomicMax(&st->tau_key, bin << kHistShift);
  }
}

// A combination is kept iff its estimate is at least tau - 2 fbound: with
// |estimate - MI| <= fbound everywhere, tau <= the top_n-th best estimate
// <= the top_n-th best MI + fbound, so anything lower cannot be in the top_n.
__device__ __forceinline__ float current_threshold(const JV &v) {
  const float tau = __uint_as_float(uni(load_relaxed(&v.st->tau_key)));
  return tau - 2.0f * v.fbound;
}

// The same, read by every lane (no wave-uniform copy): the wave waits for the
// load only where the value is next used, so a refresh between two scores
// does not stall.
__device__ __forceinline__ float current_threshold_lanes(const JV &v) {
  return __uint_as_float(load_relaxed(&v.st->tau_key)) - 2.0f * v.fbound;
}

// Appends every active lane whose score clears the threshold and returns the
// number of lanes that appended (the same in every lane); after appends the
// bound may have risen.  rank_of() gives the lane's combination rank; it is
// evaluated only by lanes that append.
template <typename RankOf>
__device__ __forceinline__ uint32_t emit_with(const JV &v, bool active, float est, RankOf &&rank_of,
                                          float thr, uint32_t lane) {
  if (v.pk) {  // pilot: record the score only
    v.pk[lane] = (active && est > 0.f) ? __float_as_uint(est) : 0u;
    v.pk += 64;
    return 0;
  }
  const bool keep = active && est >= thr;
  const u64 mask = ballot(keep);
  if (mask == 0) return 0;
  const uint32_t cnt = popc64(mask);
  const uint32_t leader = __ffsll((long long)mask) - 1;
  u64 base = 0, old = 0;
  if (lane == leader) {
    base = atomicAdd(&v.st->cand_count, (u64)cnt);
    old = atomicAdd(&v.st->nsurv, (u64)cnt);
  }
  base = __shfl(base, leader);
  old = __shfl(old, leader);
  if (keep) {
    const u64 lt = lane ? (~0ull >> (64 - lane)) : 0ull;
    const u64 idx = base + popc64(mask & lt);
    const uint32_t key = est > 0.f ? __float_as_uint(est) : 0u;
    if (idx < v.cand_cap) {
      Cand c;
      c.rank = rank_of();
      c.key = key;
      c.est = est;
      v.cand[idx] = c;
    }
  }
  // histogram counts: the kept lanes that share the first kept lane's bin
  // (often most of them) add with one atomic, the others with one each
  {
    const uint32_t bin = __float_as_uint(est > 0.f ? est : 0.f) >> kHistShift;
    const uint32_t b0 = __shfl(bin, leader);
    const u64 same = mask & ballot(bin == b0);
    if (lane == leader) atomicAdd(&v.hist[b0], (uint32_t)popc64(same));
    if (keep && bin != b0) atomicAdd(&v.hist[bin], 1u);
  }
  const u64 qs = v.top_n > 64 ? v.top_n : 64;
  if ((old + cnt) / qs != old / qs) refresh_tau(v.hist, v.st, v.top_n, lane);
  return cnt;
}

__device__ __forceinline__ uint32_t emit(const JV &v, bool active, float est, u64 rank, float thr,
                                     uint32_t lane) {
  return emit_with(v, active, est, [&] { return rank; }, thr, lane);
}

// Constants of the score of a job: m * MI starts at f(m) - f(m0) - f(m1).
// The FP4 matrix-core kernels of orders 3 to 5, with the f table in LDS, take
// the same sum in fixed point: with Fq[t] = round(2^qs f(t)) modulo 2^32 (qs: the largest
// shift with 2^qs (m ln 2 + 1) <= 2^30), D = Fq[m] - Fq[m0] - Fq[m1] +
// sum_x (Fq[n_x0] + Fq[n_x1] - Fq[n_x]) in 32-bit integers modulo 2^32.  The
// exact sum 2^qs m MI lies in [0, 2^30] and D is off by at most half a unit
// per table entry (3 + 3^(k+1) of them), so D read as a signed integer is
// that integer sum, and est = D x 2^-qs / m; each cell costs two integer
// additions instead of three floating-point ones, and the error, at most
// (3 + 3^(k+1)) 2^-(qs+1) / m + 3u ln 2 (u = 2^-24), is below the
// single-precision bound the filters use, for k <= 5.
struct MiConst {
  float c;
  float inv_m;
  uint32_t q0;   // Fq[m] - Fq[m0] - Fq[m1] modulo 2^32
  float qscale;  // 2^-qs / m
};

__device__ __forceinline__ MiConst mi_const(const JV &v) {
  const FI_CONST float *F = as_const(v.Fh);
  const FI_CONST uint32_t *Fq = as_const(v.Fq);
  MiConst c;
  c.c = (F[v.m] - F[v.m0]) - F[v.m1];
  c.inv_m = 1.0f / (float)v.m;
  c.q0 = Fq[v.m] - Fq[v.m0] - Fq[v.m1];
  c.qscale = v.qscale;
  return c;
}

// Pins an integer running sum at this point of the program.  Integer
// addition is associative, and left free the compiler regroups a walk's
// additions and lifts its table reads far ahead, holding many more registers
// (spilling) than the same walk in floating point; an empty statement that
// may change the sum keeps each group of terms in its place.
__device__ __forceinline__ void pin_sum(uint32_t &s) { asm volatile("" : "+v"(s)); }

// The estimate from the fixed-point sum D (see MiConst)
__device__ __forceinline__ float mi_fixed(uint32_t D, const MiConst &mc) {
  return (float)(int32_t)D * mc.qscale;
}

// Start and result of a score accumulated in the table's element type:
// float tables the single-precision form, uint32_t tables the fixed-point one
template <typename E>
__device__ __forceinline__ E mi_start(const MiConst &mc) {
  if constexpr (std::is_same_v<E, uint32_t>) return mc.q0;
  else return mc.c;
}
template <typename E>
__device__ __forceinline__ float mi_finish(E s, const MiConst &mc) {
  if constexpr (std::is_same_v<E, uint32_t>) return mi_fixed(s, mc);
  else return s * mc.inv_m;
}

// Scores a complete table of NC cells x 2 classes and appends it if it may be
// among the best.
template <int NC, typename FP>
__device__ __forceinline__ uint32_t score_table(const JV &v, FP F,
                                            const uint32_t (&t)[NC][2], bool active, float thr,
                                            const MiConst &mc, u64 rank, uint32_t lane) {
  float fs = mc.c;
  if (active) {
#pragma unroll
    for (int x = 0; x < NC; ++x) fs += mi_term(F, t[x][0], t[x][1]);
  }
  return emit(v, active, fs * mc.inv_m, rank, thr, lane);
}

// 8 u32 of a pair table entry: [ga][gj][c]
__device__ __forceinline__ void load_pair(const FI_GLOBAL uint32_t *p, uint32_t (&q)[8]) {
  const FI_GLOBAL u64 *p64 = reinterpret_cast<const FI_GLOBAL u64 *>(p);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const u64 x = p64[i];
    q[2 * i] = (uint32_t)x;
    q[2 * i + 1] = (uint32_t)(x >> 32);
  }
}

// lexicographic index of the pair (x, y), x < y, among the pairs of n
__device__ __forceinline__ u64 pair_index(uint32_t n, uint32_t x, uint32_t y) {
  return (u64)x * (n - 1) - (u64)x * (x - 1) / 2 + (y - x - 1);
}

// The inputs of an order-3 table walk, held by value.
struct Tab3 {
  uint32_t D[2][2][2][2];  // [c][x][y][z] over {0,1}^3
  uint32_t xy[8];          // sum over z: [x][y][c]
  uint32_t xz[8];          // sum over y: [x][z][c]
  uint32_t yz[8];          // sum over x: [y][z][c]
  uint32_t Mx[2][2];       // [x][c]
  uint32_t My[2][2];
  uint32_t Mz[2][2];
  uint32_t m[2];
};

// walk_order3 over NT tables at once: visit(cells) sees cell p of every table
// (cells[t][class]), p in the walk's order.
template <int NT, typename Visit>
__device__ __forceinline__ void walk3_zip(const Tab3 (&q)[NT], Visit &&visit) {
  uint32_t sum[NT][2], x2z[NT][2][2][2], t2yz[NT][2][2][2], cell[NT][2];
#pragma unroll
  for (int t = 0; t < NT; ++t) sum[t][0] = sum[t][1] = 0;
  auto emit_cell = [&]() {
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      sum[t][0] += cell[t][0];
      sum[t][1] += cell[t][1];
    }
    visit(cell);
  };
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int z = 0; z < 2; ++z) {
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
          for (int c = 0; c < 2; ++c) cell[t][c] = q[t].D[c][x][y][z];
        emit_cell();
      }
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) {
#pragma unroll
      for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int c = 0; c < 2; ++c)
          cell[t][c] = q[t].xy[x * 4 + y * 2 + c] - q[t].D[c][x][y][0] - q[t].D[c][x][y][1];
      emit_cell();  // (x, y, 2)
    }
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int z = 0; z < 2; ++z) {
#pragma unroll
      for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int c = 0; c < 2; ++c)
          cell[t][c] = x2z[t][c][x][z] =
              q[t].xz[x * 4 + z * 2 + c] - q[t].D[c][x][0][z] - q[t].D[c][x][1][z];
      emit_cell();  // (x, 2, z)
    }
#pragma unroll
  for (int y = 0; y < 2; ++y)
#pragma unroll
    for (int z = 0; z < 2; ++z) {
#pragma unroll
      for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int c = 0; c < 2; ++c)
          cell[t][c] = t2yz[t][c][y][z] =
              q[t].yz[y * 4 + z * 2 + c] - q[t].D[c][0][y][z] - q[t].D[c][1][y][z];
      emit_cell();  // (2, y, z)
    }
#pragma unroll
  for (int x = 0; x < 2; ++x) {
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int c = 0; c < 2; ++c)
        cell[t][c] = q[t].Mx[x][c] - q[t].xy[x * 4 + c] - q[t].xy[x * 4 + 2 + c] - x2z[t][c][x][0] -
                     x2z[t][c][x][1];
    emit_cell();  // (x, 2, 2)
  }
#pragma unroll
  for (int y = 0; y < 2; ++y) {
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int c = 0; c < 2; ++c)
        cell[t][c] = q[t].My[y][c] - q[t].xy[y * 2 + c] - q[t].xy[4 + y * 2 + c] - t2yz[t][c][y][0] -
                     t2yz[t][c][y][1];
    emit_cell();  // (2, y, 2)
  }
#pragma unroll
  for (int z = 0; z < 2; ++z) {
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int c = 0; c < 2; ++c)
        cell[t][c] = q[t].Mz[z][c] - q[t].xz[z * 2 + c] - q[t].xz[4 + z * 2 + c] - t2yz[t][c][0][z] -
                     t2yz[t][c][1][z];
    emit_cell();  // (2, 2, z)
  }
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int c = 0; c < 2; ++c) cell[t][c] = q[t].m[c] - sum[t][c];
  visit(cell);  // (2, 2, 2)
}

// 16 u32 of a triple table entry ([g_x][g_y][g_z][class]) and its slice at g_z
__device__ __forceinline__ void load_triple(const FI_GLOBAL uint32_t *p, uint32_t (&q)[16]) {
  const FI_GLOBAL u64 *p64 = reinterpret_cast<const FI_GLOBAL u64 *>(p);
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const u64 x = p64[i];
    q[2 * i] = (uint32_t)x;
    q[2 * i + 1] = (uint32_t)(x >> 32);
  }
}

// The 27 cells of an order-3 table from its {0,1}^3 counts D, the {0,1}^2
// counts of its three pairs, the {0,1} counts of its variants and the class
// sizes.  With "any" marginalising a position, T[x][y][2] = N[x][y][any] -
// T[x][y][0] - T[x][y][1] and likewise along the other positions; the cells
// are produced in an order where each needs only cells already produced.
struct Order3Parts {
  const uint32_t (&D)[2][2][2][2];   // [c][ga][gb][gj]
  const uint32_t (&ab)[8];           // (a, b): [ga][gb][c]
  const uint32_t (&aj)[8];           // (a, j): [ga][gj][c]
  const uint32_t (&bj)[8];           // (b, j): [gb][gj][c]
  const uint32_t (&Ma)[2][2];        // [g][c]
  const uint32_t (&Mb)[2][2];
  const uint32_t (&Mj)[2][2];
  const uint32_t (&m)[2];            // class sizes
};

template <typename Visit>
__device__ __forceinline__ void walk_order3(const Order3Parts &q, Visit &&visit) {
  uint32_t x2z[2][2][2], t2yz[2][2][2], x22[2][2];  // [c][x or y][z], [c][x]
  auto cell = [&](uint32_t n0, uint32_t n1) { visit(n0, n1); };
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int z = 0; z < 2; ++z) cell(q.D[0][x][y][z], q.D[1][x][y][z]);
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) {
      uint32_t t[2];
#pragma unroll
      for (int c = 0; c < 2; ++c) t[c] = q.ab[x * 4 + y * 2 + c] - q.D[c][x][y][0] - q.D[c][x][y][1];
      cell(t[0], t[1]);  // (x, y, 2)
    }
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int z = 0; z < 2; ++z) {
#pragma unroll
      for (int c = 0; c < 2; ++c)
        x2z[c][x][z] = q.aj[x * 4 + z * 2 + c] - q.D[c][x][0][z] - q.D[c][x][1][z];
      cell(x2z[0][x][z], x2z[1][x][z]);  // (x, 2, z)
    }
#pragma unroll
  for (int y = 0; y < 2; ++y)
#pragma unroll
    for (int z = 0; z < 2; ++z) {
#pragma unroll
      for (int c = 0; c < 2; ++c)
        t2yz[c][y][z] = q.bj[y * 4 + z * 2 + c] - q.D[c][0][y][z] - q.D[c][1][y][z];
      cell(t2yz[0][y][z], t2yz[1][y][z]);  // (2, y, z)
    }
#pragma unroll
  for (int x = 0; x < 2; ++x) {
    uint32_t t[2];
#pragma unroll
    for (int c = 0; c < 2; ++c)
      x22[c][x] = q.Ma[x][c] - q.ab[x * 4 + c] - q.ab[x * 4 + 2 + c] - x2z[c][x][0] - x2z[c][x][1];
    cell(x22[0][x], x22[1][x]);  // (x, 2, 2)
  }
#pragma unroll
  for (int y = 0; y < 2; ++y) {
    uint32_t t[2];
#pragma unroll
    for (int c = 0; c < 2; ++c)
      t[c] = q.Mb[y][c] - q.ab[y * 2 + c] - q.ab[4 + y * 2 + c] - t2yz[c][y][0] - t2yz[c][y][1];
    cell(t[0], t[1]);  // (2, y, 2)
  }
#pragma unroll
  for (int z = 0; z < 2; ++z) {
    uint32_t t[2];
#pragma unroll
    for (int c = 0; c < 2; ++c)
      t[c] = q.Mj[z][c] - q.aj[z * 2 + c] - q.aj[4 + z * 2 + c] - t2yz[c][0][z] - t2yz[c][1][z];
    cell(t[0], t[1]);  // (2, 2, z)
  }
  // (2, 2, 2): the cells (x, 2, 2), x = 0, 1, 2, add up to the (b, j) pair's
  // count at (2, 2), which is the class size less the variants' {0,1} counts
  // plus the pair's {0,1}^2 counts
  uint32_t t[2];
#pragma unroll
  for (int c = 0; c < 2; ++c)
    t[c] = q.m[c] - q.Mb[0][c] - q.Mb[1][c] - q.Mj[0][c] - q.Mj[1][c] + q.bj[c] + q.bj[2 + c] +
           q.bj[4 + c] + q.bj[6 + c] - x22[c][0] - x22[c][1];
  visit(t[0], t[1]);
}

// The same walk on packed counts: both classes of every count in one
// register, lo + 2^16 hi.  Sums and differences of packed values are exact
// modulo 2^32, so a result whose two true halves each lie in [0, 2^16) comes
// out as exactly those halves, whatever borrows cross between them on the
// way; every cell is a count of at most the class size.  The halves may carry
// a common scale (4 x count gives byte offsets into a table of floats: class
// sizes below 16,384).  D[ga][gb][gj], ab[ga][gb], aj[ga][gj], bj[gb][gj],
// Ma/Mb/Mj[g], m = both class sizes.
template <typename Visit>
__device__ __forceinline__ void walk_order3_packed(const uint32_t (&D)[2][2][2],
                                                   const uint32_t (&ab)[2][2],
                                                   const uint32_t (&aj)[2][2],
                                                   const uint32_t (&bj)[2][2],
                                                   const uint32_t (&Ma)[2], const uint32_t (&Mb)[2],
                                                   const uint32_t (&Mj)[2], uint32_t m,
                                                   Visit &&visit) {
  auto cell = [&](uint32_t p) { visit(p); };
  uint32_t x2z[2][2], t2yz[2][2], x22[2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int z = 0; z < 2; ++z) cell(D[x][y][z]);
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) cell(ab[x][y] - D[x][y][0] - D[x][y][1]);  // (x, y, 2)
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int z = 0; z < 2; ++z) {
      x2z[x][z] = aj[x][z] - D[x][0][z] - D[x][1][z];
      cell(x2z[x][z]);  // (x, 2, z)
    }
#pragma unroll
  for (int y = 0; y < 2; ++y)
#pragma unroll
    for (int z = 0; z < 2; ++z) {
      t2yz[y][z] = bj[y][z] - D[0][y][z] - D[1][y][z];
      cell(t2yz[y][z]);  // (2, y, z)
    }
#pragma unroll
  for (int x = 0; x < 2; ++x) {
    x22[x] = Ma[x] - ab[x][0] - ab[x][1] - x2z[x][0] - x2z[x][1];
    cell(x22[x]);  // (x, 2, 2)
  }
#pragma unroll
  for (int y = 0; y < 2; ++y) cell(Mb[y] - ab[0][y] - ab[1][y] - t2yz[y][0] - t2yz[y][1]);  // (2, y, 2)
#pragma unroll
  for (int z = 0; z < 2; ++z) cell(Mj[z] - aj[0][z] - aj[1][z] - t2yz[0][z] - t2yz[1][z]);  // (2, 2, z)
  // (2, 2, 2) from the (b, j) pair's count at (2, 2), as in walk_order3
  visit(m - Mb[0] - Mb[1] - Mj[0] - Mj[1] + bj[0][0] + bj[0][1] + bj[1][0] + bj[1][1] - x22[0] - x22[1]);
}

// Class counts (c0, c1) as one packed register of byte offsets 4 c0 | 4 c1 << 16
__device__ __forceinline__ uint32_t pack_x4(uint32_t c0, uint32_t c1) { return (c0 << 2) | (c1 << 18); }

// Decodes global tile t of a launch: its job (binary search over the job
// tile starts), the job's view with the run state read in, and the job-local
// tile index.  In a pilot launch, pilot tile i of S stands for tile
// floor(i T / S) of the job's T, and the wave's scores go to its slots
// (slots_per_wave per tile and wave).  With shards, the shard's i-th tile is
// the tile at offset (shard_index + i) mod shard_count of block i of
// shard_count consecutive tiles.  Returns false when the job is skipped
// (invalid input or an empty class).
// the job (index into g.jobs) that owns launch tile t
__device__ __forceinline__ uint32_t job_of_tile(const Globals &g, u64 t) {
  cu64p jts = as_const(g.job_tile_start);
  uint32_t lo = 0, hi = g.n_jobs - 1;
  while (lo < hi) {
    const uint32_t mid = (lo + hi + 1) >> 1;
    if (jts[mid] <= t) lo = mid;
    else hi = mid - 1;
  }
  return uni(lo);
}

// Whether any job of a launch satisfies mine(m0, m1, m) (its class sizes,
// known once the partition has run).  The dual and the two-accumulator
// matrix-core kernels of a group are both launched over its tiles and split
// its jobs by class sizes: a launch with none of its own exits at once
// instead of drawing and skipping the tiles.
template <typename Mine>
__device__ __forceinline__ bool any_job(const Globals &g, Mine &&mine) {
  for (uint32_t i = 0; i < g.n_jobs; ++i) {
    const FI_CONST JobDesc *jd = as_const(g.jobs) + i;
    const JobState *st = uni_ptr(jd->state);
    if (mine(uni(st->m0), uni(st->m1), uni(jd->m))) return true;
  }
  return false;
}

// Row of tile-local index lt in a job's row table rows[0 .. nrows] (rows[0] =
// 0 <= lt < rows[nrows]).  hint: the row of an earlier tile of the same job,
// or 0; the tiles a workgroup draws only increase, and so do their local
// indices (pilot sampling and shard dealing are monotone), so rows[hint] <=
// lt, and one load settles the common case of the same row again.
__device__ __forceinline__ uint32_t find_row(cu64p rows, uint32_t nrows, u64 lt, uint32_t hint) {
  if (rows[hint + 1] > lt) return hint;
  uint32_t rl = hint + 1, rh = nrows - 1;
  while (rl < rh) {
    const uint32_t mid = (rl + rh + 1) >> 1;
    if (rows[mid] <= lt) rl = mid;
    else rh = mid - 1;
  }
  return uni(rl);
}

// The hint find_row may use for job descriptor jd: the last row found when
// the workgroup's previous tile was of the same job, else 0
struct RowHint {
  const FI_CONST JobDesc *jd = nullptr;
  uint32_t row = 0;
  __device__ __forceinline__ uint32_t find(const FI_CONST JobDesc *j, u64 lt) {
    if (j != jd) {
      jd = j;
      row = 0;
    }
    row = find_row(as_const(uni_ptr(j->row_start)), uni(j->nrows), lt, row);
    return row;
  }
};

__device__ __forceinline__ bool locate_tile(const Globals &g, u64 t, uint32_t wave,
                                            uint32_t slots_per_wave, JV &v,
                                            const FI_CONST JobDesc *&jd, u64 &lt) {
  cu64p jts = as_const(g.job_tile_start);
  const uint32_t lo = job_of_tile(g, t);
  v = load_view(g.jobs + lo);
  {
    const JobState *st = v.st;
    if (uni((uint32_t)st->status) != 0) return false;
    v.m0 = uni(st->m0);
    v.m1 = uni(st->m1);
    v.W0 = uni(st->W0);
    v.W1 = uni(st->W1);
    if (v.m0 == 0 || v.m1 == 0) return false;
  }
  jd = as_const(g.jobs) + lo;
  lt = uni64(t - jts[lo]);
  if (g.pilot) {
    v.pk = reinterpret_cast<uint32_t *>(v.cand) + (lt * kScanWaves + wave) * (slots_per_wave * 64);
    lt = uni64(lt * uni64(jd->tile_count) / uni(jd->pilot_tiles));
  }
  const uint32_t sc = uni(jd->shard_count);
  if (sc > 1) lt = uni64(lt * sc + (uni(jd->shard_index) + lt % sc) % sc);
  return true;
}

// ---------------------------------------------------------------------------
// Order 4 from stored triple tables.  Only the {0,1}^4 cells of (x, y, z, j)
// are counted; the others follow by inclusion-exclusion: for g_j in {0, 1},
// the cells (., ., ., g_j) form an order-3 table over (x, y, z) whose "pairs"
// are the {0,1}^3 tables of (x, y, j), (x, z, j), (y, z, j) at g_j, whose
// "variants" are the {0,1}^2 pair tables of (x, j), (y, j), (z, j) at g_j and
// whose size is the count of g_j at j; the cells (., ., ., 2) are the
// prefix's own order-3 table (x, y, z) minus those two.
// ---------------------------------------------------------------------------

// Sum of the MI terms of (x, y, z, j) added to `start`, from its {0,1}^4
// counts acc[class][g_x][g_y][g_z][g_j]; jj = j clamped below n.  UNIFORM:
// the prefix is the same in every lane (its tables are read by scalar loads).
// CLAMP: clamp every count to its class size before the table reads (a table
// in global memory; LDS reads cannot fault).
template <bool UNIFORM, bool CLAMP, typename FP>
__device__ __forceinline__ float order4_tables_sum(const JV &v, FP F, const uint32_t (&acc)[2][2][2][2][2],
                                                   uint32_t x, uint32_t y, uint32_t z, uint32_t jj,
                                                   bool active, float start) {
  const uint32_t n = v.n, np = v.n_pad;
  const FI_GLOBAL uint32_t *TTg = as_global(v.triples);
  const FI_GLOBAL uint32_t *PTg = as_global(v.pairs);
  const FI_GLOBAL uint32_t *mgj = as_global(v.marg) + (size_t)jj * 6;
  // prefix tables: scalar loads when wave-uniform
  auto TTp = [&](size_t i) -> uint32_t {
    if constexpr (UNIFORM) return as_const(v.triples)[i];
    else return TTg[i];
  };
  auto PTp = [&](size_t i) -> uint32_t {
    if constexpr (UNIFORM) return as_const(v.pairs)[i];
    else return PTg[i];
  };
  auto Mp = [&](size_t i) -> uint32_t {
    if constexpr (UNIFORM) return as_const(v.marg)[i];
    else return as_global(v.marg)[i];
  };

  Tab3 q[3];  // [0]: (x, y, z) itself; [1], [2]: the cells with g_j = 0, 1
  {
    const size_t e = (pair_index(n, x, y) * np + z) * 16;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
          for (int cl = 0; cl < 2; ++cl) q[0].D[cl][a][b][c] = TTp(e + a * 8 + b * 4 + c * 2 + cl);
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      q[0].xy[i] = PTp(((size_t)x * np + y) * 8 + i);
      q[0].xz[i] = PTp(((size_t)x * np + z) * 8 + i);
      q[0].yz[i] = PTp(((size_t)y * np + z) * 8 + i);
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int cl = 0; cl < 2; ++cl) {
        q[0].Mx[a][cl] = Mp((size_t)x * 6 + 2 * a + cl);
        q[0].My[a][cl] = Mp((size_t)y * 6 + 2 * a + cl);
        q[0].Mz[a][cl] = Mp((size_t)z * 6 + 2 * a + cl);
      }
    q[0].m[0] = v.m0;
    q[0].m[1] = v.m1;
  }
  // the g_j slices (per lane)
  {
    uint32_t txy[16], txz[16], tyz[16], pxj[8], pyj[8], pzj[8];
    load_triple(TTg + (pair_index(n, x, y) * np + jj) * 16, txy);
    load_triple(TTg + (pair_index(n, x, z) * np + jj) * 16, txz);
    load_triple(TTg + (pair_index(n, y, z) * np + jj) * 16, tyz);
    load_pair(PTg + ((size_t)x * np + jj) * 8, pxj);
    load_pair(PTg + ((size_t)y * np + jj) * 8, pyj);
    load_pair(PTg + ((size_t)z * np + jj) * 8, pzj);
#pragma unroll
    for (int gj = 0; gj < 2; ++gj) {
      Tab3 &t = q[1 + gj];
#pragma unroll
      for (int cl = 0; cl < 2; ++cl)
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int c = 0; c < 2; ++c) t.D[cl][a][b][c] = acc[cl][a][b][c][gj];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
          for (int cl = 0; cl < 2; ++cl) {
            t.xy[a * 4 + b * 2 + cl] = txy[a * 8 + b * 4 + gj * 2 + cl];
            t.xz[a * 4 + b * 2 + cl] = txz[a * 8 + b * 4 + gj * 2 + cl];
            t.yz[a * 4 + b * 2 + cl] = tyz[a * 8 + b * 4 + gj * 2 + cl];
          }
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int cl = 0; cl < 2; ++cl) {
          t.Mx[a][cl] = pxj[a * 4 + gj * 2 + cl];
          t.My[a][cl] = pyj[a * 4 + gj * 2 + cl];
          t.Mz[a][cl] = pzj[a * 4 + gj * 2 + cl];
        }
#pragma unroll
      for (int cl = 0; cl < 2; ++cl) t.m[cl] = mgj[2 * gj + cl];
    }
  }
  float fs = start;
  if (active) {
    const uint32_t m0 = v.m0, m1 = v.m1;
    auto cl0 = [&](uint32_t t) { return CLAMP ? min(t, m0) : t; };
    auto cl1 = [&](uint32_t t) { return CLAMP ? min(t, m1) : t; };
    walk3_zip<3>(q, [&](const uint32_t (&cell)[3][2]) {
      const uint32_t n20 = cell[0][0] - cell[1][0] - cell[2][0];
      const uint32_t n21 = cell[0][1] - cell[1][1] - cell[2][1];
      fs += mi_term(F, cl0(cell[1][0]), cl1(cell[1][1]));
      fs += mi_term(F, cl0(cell[2][0]), cl1(cell[2][1]));
      fs += mi_term(F, cl0(n20), cl1(n21));
    });
  }
  return fs;
}

}  // namespace fiuncho
