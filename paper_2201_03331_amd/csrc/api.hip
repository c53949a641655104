// api.hip -- the C ABI of libfiuncho: validation, workspace layout, the plan
// (lookup and tile tables), kernel sequencing and result hand-back.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstddef>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "internal.hpp"

using fiuncho::Cand;
using fiuncho::Globals;
using fiuncho::JobDesc;
using fiuncho::JobState;
using fiuncho::SortItem;

namespace {

typedef unsigned long long u64;

thread_local std::string t_err;
thread_local bool t_profiling = false;

int fail(int code, const std::string &msg) {
  t_err = msg;
  return code;
}

#define HIP_TRY(expr)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fail(FIUNCHO_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

u64 binom_host(u64 n, u64 k) {
  if (k > n) return 0;
  if (k > n - k) k = n - k;
  unsigned __int128 r = 1;
  for (u64 i = 1; i <= k; ++i) {
    r = r * (unsigned __int128)(n - k + i) / i;
    if (r > (unsigned __int128)~0ull) return ~0ull;
  }
  return (u64)r;
}

u64 ceil_div(u64 a, u64 b) { return (a + b - 1) / b; }
size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// ---------------------------------------------------------------------------
// validation of one job's shape (values are checked separately)
// ---------------------------------------------------------------------------
int check_shape(const fiuncho_job &j, bool need_ptrs) {
  if (need_ptrs && (!j.genotypes || !j.phenotype || !j.out || !j.n_out))
    return fail(FIUNCHO_E_NULL, "a required pointer is NULL");
  if (j.snps == 0 || j.samples == 0) return fail(FIUNCHO_E_SHAPE, "snps and samples must be positive");
  if (j.samples >= (1u << 24)) return fail(FIUNCHO_E_SHAPE, "samples must be below 2^24");
  if (j.order < 1 || j.order > FIUNCHO_MAX_ORDER || (uint32_t)j.order > j.snps)
    return fail(FIUNCHO_E_ORDER, "order must be in [1, min(snps, 8)]");
  if (j.top_n == 0 || j.top_n > FIUNCHO_MAX_TOPN)
    return fail(FIUNCHO_E_TOPN, "top_n must be in [1, " + std::to_string(FIUNCHO_MAX_TOPN) + "]");
  if (binom_host(j.snps, (u64)j.order) >= (1ull << 63))
    return fail(FIUNCHO_E_OVERFLOW, "C(snps, order) must be below 2^63");
  return FIUNCHO_OK;
}

int check_values(const uint8_t *G, const uint8_t *y, uint32_t n, uint32_t m) {
  const size_t total = (size_t)n * m;
  for (size_t i = 0; i < total; ++i)
    if (G[i] > 2)
      return fail(FIUNCHO_E_GENOTYPE, "genotype value " + std::to_string(G[i]) + " at variant " +
                                          std::to_string(i / m) + ", sample " + std::to_string(i % m));
  for (uint32_t s = 0; s < m; ++s)
    if (y[s] > 1)
      return fail(FIUNCHO_E_PHENOTYPE, "phenotype value " + std::to_string(y[s]) + " at sample " +
                                           std::to_string(s));
  return FIUNCHO_OK;
}

// ---------------------------------------------------------------------------
// tile tables: rows and tiles per row, as the scan kernel decodes them
// ---------------------------------------------------------------------------
void build_rows(uint32_t n, uint32_t k, uint32_t path, std::vector<u64> &row_start) {
  row_start.clear();
  row_start.push_back(0);
  u64 acc = 0;
  if (k == 1) {
    acc = ceil_div(n, (u64)fiuncho::kScanWaves * 64);
    row_start.push_back(acc);
    return;
  }
  if (path == fiuncho::kPathMfma2) {
    // rows A of the upper triangle of 64-variant blocks: tiles (A, B >= A)
    const u64 nb = ceil_div(n, 64);
    for (u64 A = 0; A < nb; ++A) {
      acc += nb - A;
      row_start.push_back(acc);
    }
    return;
  }
  if (k == 2) {
    const u64 S = (u64)fiuncho::kScanWaves * fiuncho::kOrder2Prefixes;
    const u64 rows = ceil_div(n - 1, S);
    for (u64 r = 0; r < rows; ++r) {
      const u64 a_first = r * S;
      acc += ceil_div(n - 1 - a_first, 64);
      row_start.push_back(acc);
    }
    return;
  }
  if (path == fiuncho::kPathMfma3) {
    // rows (jb, b), jb-major: block jb of 64 last variants j = b + 1 + 64 jb
    // + [0, 64) of middle variant b = 1 .. n-2-64 jb; a row's tiles are its
    // groups of 32 first variants.  Tiles taken in this order work on a
    // narrow band of last variants at a time, so the pair-table entries and
    // bitset rows in use stay within each XCD's L2
    for (u64 jb = 0; 64 * jb + 3 <= n; ++jb)
      for (u64 b = 1; b + 2 + 64 * jb <= n; ++b) {
        acc += ceil_div(b, 32);
        row_start.push_back(acc);
      }
    return;
  }
  if (path == fiuncho::kPathPairs) {
    // rows b = 1 .. n-2; groups of kScanWaves * kOrder3Prefixes first
    // variants x blocks of 64 last variants
    const u64 G = (u64)fiuncho::kScanWaves * fiuncho::kOrder3Prefixes;
    for (u64 b = 1; b + 2 <= n; ++b) {
      const u64 groups = ceil_div(b, G);
      acc += groups * ceil_div(n - 1 - b, 64);
      row_start.push_back(acc);
    }
    return;
  }
  // rows b (last prefix variant): groups of prefixes (one per wave on the
  // popcount kernel, 16 per tile on the order-4 triple-table matrix-core
  // kernel) x blocks of 64 last variants
  const u64 G = path == fiuncho::kPathMfma4t   ? 16
                : path == fiuncho::kPathMfma5q ? 8
                                               : (u64)fiuncho::kScanWaves;
  for (u64 b = k - 2; b + 2 <= n; ++b) {
    const u64 groups = ceil_div(binom_host(b, k - 2), G);
    acc += groups * ceil_div(n - 1 - b, 64);
    row_start.push_back(acc);
  }
}

// Every local tile of a job in tile order with the number of combinations it
// tests, as the scan kernel decodes tiles: fn(tile, combinations).
template <class Fn>
void for_each_tile(uint32_t n, uint32_t k, uint32_t path, Fn fn) {
  const u64 N = n;
  if (k == 1) {
    const u64 S = (u64)fiuncho::kScanWaves * 64;
    for (u64 lt = 0; lt * S < N; ++lt) fn(lt, std::min<u64>(S, N - lt * S));
    return;
  }
  u64 lt = 0;
  if (k == 2 && path == fiuncho::kPathMfma2) {
    for (u64 A = 0; A * 64 < N; ++A)
      for (u64 B = A; B * 64 < N; ++B) {
        u64 c = 0;
        const u64 j_end = std::min<u64>(64 * B + 64, N);
        for (u64 a = 64 * A; a < std::min<u64>(64 * A + 64, N); ++a) {
          const u64 lo = std::max<u64>(64 * B, a + 1);
          if (lo < j_end) c += j_end - lo;
        }
        fn(lt++, c);
      }
    return;
  }
  if (k == 2) {
    const u64 S = (u64)fiuncho::kScanWaves * fiuncho::kOrder2Prefixes;
    for (u64 a_first = 0; a_first + 1 < N; a_first += S) {
      const u64 a_end = std::min<u64>(a_first + S, N - 1);
      for (u64 j0 = a_first + 1; j0 < N; j0 += 64) {
        const u64 j_end = std::min<u64>(j0 + 64, N);
        u64 c = 0;
        for (u64 a = a_first; a < a_end; ++a) {
          const u64 lo = std::max<u64>(j0, a + 1);
          if (lo < j_end) c += j_end - lo;
        }
        fn(lt++, c);
      }
    }
    return;
  }
  if (path == fiuncho::kPathMfma3) {
    // rows (jb, b) jb-major, a row's tiles its groups of 32 first variants
    for (u64 jb = 0; 64 * jb + 3 <= N; ++jb)
      for (u64 b = 1; b + 2 + 64 * jb <= N; ++b) {
        const u64 j0 = b + 1 + 64 * jb;
        for (u64 p0 = 0; p0 < b; p0 += 32) fn(lt++, std::min<u64>(32, b - p0) * std::min<u64>(64, N - j0));
      }
    return;
  }
  // rows b (second-to-last variant): groups of prefixes x blocks of 64 last variants
  const bool by_pairs = path == fiuncho::kPathPairs;
  const u64 G = path == fiuncho::kPathPairs    ? (u64)fiuncho::kScanWaves * fiuncho::kOrder3Prefixes
                : path == fiuncho::kPathMfma4t ? 16
                : path == fiuncho::kPathMfma5q ? 8
                                               : (u64)fiuncho::kScanWaves;
  for (u64 b = (by_pairs ? 1 : k - 2); b + 2 <= N; ++b) {
    const u64 prefixes = by_pairs ? b : binom_host(b, k - 2);
    for (u64 p0 = 0; p0 < prefixes; p0 += G) {
      const u64 pc = std::min<u64>(G, prefixes - p0);
      for (u64 j0 = b + 1; j0 < N; j0 += 64) fn(lt++, pc * std::min<u64>(64, N - j0));
    }
  }
}

// Shards deal the tiles of a job in blocks of shard_count consecutive tiles;
// in block q, shard s takes the tile at offset (s + q) mod shard_count.  The
// rotation keeps the shards from always drawing the same position of a
// periodic tile pattern (such as the partial last block of 64 variants of
// every row).
u64 tile_shard(u64 lt, u64 count) { return (lt % count + count - (lt / count) % count) % count; }

// tiles of shard s among `tiles`
u64 shard_tiles(u64 tiles, u64 count, u64 s) {
  const u64 q = tiles / count, r = tiles % count;
  return q + ((s + q) % count < r ? 1 : 0);
}

// ---------------------------------------------------------------------------
// kernel choice per job shape: environment override, else this thread's
// forced choice (autotuning runs), else the tuned table, else the rule
// ---------------------------------------------------------------------------
typedef std::tuple<uint32_t, uint32_t, uint32_t> ShapeKey;  // order, bit length of snps, of words
// a bucket's configuration: counting kernel, and the most workgroups of 4
// waves (so waves per SIMD) each persistent launch keeps on a compute unit
// (0: as many as fit)
struct TuneEntry {
  int kernel;
  int wps;
};
std::mutex g_tune_mu;
std::map<ShapeKey, TuneEntry> g_tuned;
thread_local int t_force_kernel = FIUNCHO_KERNEL_AUTO;
thread_local int t_force_wps = -1;  // an autotuning trial's waves per SIMD (-1: none)

uint32_t bit_length(u64 x) {
  uint32_t b = 0;
  for (; x; x >>= 1) ++b;
  return b;
}

ShapeKey shape_key(uint32_t n, uint32_t m, uint32_t k) {
  return ShapeKey(k, bit_length(n), bit_length(ceil_div(m, 64)));
}

// bytes of the triple tables of an order-4 job (one 64-byte entry per pair
// and last variant slot)
u64 triple_table_bytes(uint32_t n, bool packed = false) {
  const u64 n_pad = (u64)(n + 63) / 64 * 64 + 64;
  return binom_host(n, 2) * n_pad * (packed ? 32 : 64);
}
constexpr u64 kMaxTripleTableBytes = 16ull << 30;
// packed quad tables (order 5 with lower-order tables): 64 bytes per 4-set
u64 quad_table_bytes(uint32_t n) { return binom_host(n, 4) * 64; }
constexpr u64 kMaxQuadTableBytes = 48ull << 30;

bool kernel_valid(int kernel, uint32_t n, uint32_t k) {
  switch (kernel) {
    case FIUNCHO_KERNEL_POPCOUNT: return true;
    case FIUNCHO_KERNEL_PAIRS: return k == 3 && n >= 3;
    case FIUNCHO_KERNEL_MFMA: return k == 2 || (k == 3 && n >= 3);
    case FIUNCHO_KERNEL_MFMA_FP4: return k == 2 || ((k == 3 || k == 4 || k == 5) && n >= k);
    case FIUNCHO_KERNEL_TRIPLES: return k == 4 && n >= 4 && triple_table_bytes(n) <= kMaxTripleTableBytes;
    case FIUNCHO_KERNEL_MFMA_FP4_TABLES:
      return (k == 4 || k == 5) && n >= k && triple_table_bytes(n, true) <= kMaxTripleTableBytes &&
             (k == 4 || quad_table_bytes(n) <= kMaxQuadTableBytes);
    default: return false;
  }
}

// From timing every kernel on MI355X over 100-4,000 variants and
// 1,000-20,000 samples: order 3 on the matrix cores with FP4 operands
// everywhere (1.1-2.4 times the pair-table kernel); order 2 on the same
// kernel except for 256-4,095 variants with fewer than 128 words, where the
// popcount kernel is up to 25 % faster.  Order 4 counts its {0,1}^4 cells on
// the matrix cores and takes the rest from packed triple tables while they
// fit in 16 GiB and the job has fewer than 16,384 samples (200 x 4,000: 5.7 ms
// a search, triple tables on the popcount kernel 18.8 ms, every prefix row on
// the matrix cores 17.6 ms), else the popcount kernel's triple tables, else
// every prefix row on the matrix cores.  Order 5 likewise with quad tables
// while they fit in 48 GiB (200 x 4,000: 1.21 s, every prefix row on the
// matrix cores 1.93 s, popcount 3.7 s), else every prefix row on the matrix
// cores.  The matrix cores take every prefix row of orders 4 and 5 up to
// 20,447 samples.
int rule_kernel(uint32_t n, uint32_t m, uint32_t k) {
  const u64 words = ceil_div(m, 64);
  const bool rows = m <= fiuncho::mfma_narrow_max_samples() && n >= k;
  if (k == 3 && n >= 3) return FIUNCHO_KERNEL_MFMA_FP4;
  if (k == 4 && m < 16384 && kernel_valid(FIUNCHO_KERNEL_MFMA_FP4_TABLES, n, k))
    return FIUNCHO_KERNEL_MFMA_FP4_TABLES;
  if (k == 4 && kernel_valid(FIUNCHO_KERNEL_TRIPLES, n, k)) return FIUNCHO_KERNEL_TRIPLES;
  if (k == 5 && m < 16384 && kernel_valid(FIUNCHO_KERNEL_MFMA_FP4_TABLES, n, k))
    return FIUNCHO_KERNEL_MFMA_FP4_TABLES;
  if ((k == 4 || k == 5) && rows) return FIUNCHO_KERNEL_MFMA_FP4;
  if (k == 2 && !(n >= 256 && n < 4096 && words < 128)) return FIUNCHO_KERNEL_MFMA_FP4;
  return FIUNCHO_KERNEL_POPCOUNT;
}

int choose_kernel(uint32_t n, uint32_t m, uint32_t k) {
  const char *e3 = std::getenv("FIUNCHO_ORDER3_PAIRS");
  if (k == 3 && e3 && e3[0] == '0') return FIUNCHO_KERNEL_POPCOUNT;
  if (k == 3 && e3 && e3[0] == '1' && n >= 3) return FIUNCHO_KERNEL_PAIRS;
  const char *e4 = std::getenv("FIUNCHO_ORDER4_TRIPLES");
  if (k == 4 && e4 && e4[0] == '0') return FIUNCHO_KERNEL_POPCOUNT;
  if (k == 4 && e4 && e4[0] == '1' && kernel_valid(FIUNCHO_KERNEL_TRIPLES, n, k))
    return FIUNCHO_KERNEL_TRIPLES;
  // matrix-core overrides: 1 = int8 operands, 4 = FP4 operands
  const char *e3m = std::getenv("FIUNCHO_ORDER3_MFMA");
  if (k == 3 && e3m && e3m[0] == '1' && n >= 3) return FIUNCHO_KERNEL_MFMA;
  if (k == 3 && e3m && e3m[0] == '4' && n >= 3) return FIUNCHO_KERNEL_MFMA_FP4;
  const char *e2 = std::getenv("FIUNCHO_ORDER2_MFMA");
  if (k == 2 && e2 && e2[0] == '0') return FIUNCHO_KERNEL_POPCOUNT;
  if (k == 2 && e2 && e2[0] == '1') return FIUNCHO_KERNEL_MFMA;
  if (k == 2 && e2 && e2[0] == '4') return FIUNCHO_KERNEL_MFMA_FP4;
  if (t_force_kernel != FIUNCHO_KERNEL_AUTO && kernel_valid(t_force_kernel, n, k)) return t_force_kernel;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tuned.find(shape_key(n, m, k));
    if (it != g_tuned.end() && kernel_valid(it->second.kernel, n, k)) return it->second.kernel;
  }
  return rule_kernel(n, m, k);
}

// waves per SIMD a job of this shape asks of its counting launch (0: as many
// as fit)
int choose_wps(uint32_t n, uint32_t m, uint32_t k) {
  if (t_force_wps >= 0) return t_force_wps;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_tuned.find(shape_key(n, m, k));
  return it != g_tuned.end() ? it->second.wps : 0;
}

bool on_matrix_cores(uint32_t path) {
  return path == fiuncho::kPathMfma2 || path == fiuncho::kPathMfma3 || path == fiuncho::kPathMfmaRows ||
         path == fiuncho::kPathMfma4t || path == fiuncho::kPathMfma5q;
}

uint32_t kernel_path(int kernel, uint32_t k) {
  switch (kernel) {
    case FIUNCHO_KERNEL_PAIRS: return fiuncho::kPathPairs;
    case FIUNCHO_KERNEL_MFMA: return k == 2 ? fiuncho::kPathMfma2 : fiuncho::kPathMfma3;
    case FIUNCHO_KERNEL_MFMA_FP4:
      return k == 2 ? fiuncho::kPathMfma2 : k == 3 ? fiuncho::kPathMfma3 : fiuncho::kPathMfmaRows;
    case FIUNCHO_KERNEL_TRIPLES: return fiuncho::kPathTriples;
    case FIUNCHO_KERNEL_MFMA_FP4_TABLES: return k == 4 ? fiuncho::kPathMfma4t : fiuncho::kPathMfma5q;
    default: return fiuncho::kPathGeneric;
  }
}

uint32_t job_path(uint32_t n, uint32_t m, uint32_t k) { return kernel_path(choose_kernel(n, m, k), k); }

// ---------------------------------------------------------------------------
// workspace layout
// ---------------------------------------------------------------------------
struct JobLayout {
  uint32_t n, m, k, top_n, n_pad, wcap, nrows, path, fp4, shard_index, shard_count;
  uint32_t wps;  // waves per SIMD asked of the counting launch (0: as many as fit)
  u64 total;
  uint32_t cand_cap, l1_cap, sel_cap;
  size_t off_G, off_y, off_idx, off_Bv, off_Bs, off_marg, off_hist, off_phist, off_cand, off_l1, off_sel,
      off_sel2, off_state, off_out, off_nout, off_status, off_pairs, off_pairs4, off_triples, off_triples4, off_quads4;
  // plan (uploaded)
  size_t off_rows, off_F32, off_Fh, off_Fq, off_P64;
  std::vector<u64> row_start;
  u64 tiles;
  uint32_t pilot_tiles, pilot_slots;
  double cost;  // per-tile cost estimate, for ordering
};

// matrix-core launch group of a job: 3 (order - 2) + operand format (0
// int8, 1 FP4, 2 FP4 with at most mfma_narrow_max_samples() samples, run by
// the kernel variant that keeps counts in 16 bits); -1 for the popcount kernel
int mfma_group(const JobLayout &J) {
  if (!on_matrix_cores(J.path)) return -1;
  if (J.path == fiuncho::kPathMfmaRows) return 6 + (int)J.k - 4;  // orders 4, 5
  if (J.path == fiuncho::kPathMfma4t) return 8;
  if (J.path == fiuncho::kPathMfma5q) return 9;
  const int fmt = !J.fp4 ? 0 : J.m <= fiuncho::mfma_narrow_max_samples() ? 2 : 1;
  return 3 * (J.path == fiuncho::kPathMfma3 ? 1 : 0) + fmt;
}

struct Layout {
  std::vector<JobLayout> jobs;
  std::vector<uint32_t> order;  // tile-space order of the jobs (costliest first)
  uint32_t nmax, kmax, max_n_pad, max_wcap, max_cand_cap, max_sel, max_pairs_n, max_pairs4_n, max_triples_n,
      max_quads_n;
  size_t plan_begin, plan_end;  // uploaded region
  size_t off_desc, off_jts, off_jps, off_binom, off_counter;
  // tile-space order: [0, n_scan) popcount kernel, then the jobs of each
  // matrix-core group (mfma_group order), n_group[q] of group q
  uint32_t n_scan, n_group[fiuncho::kMfmaGroups];
  size_t total;
  int ksel;
};

int make_layout(const fiuncho_job *jobs, uint32_t n_jobs, bool host_inputs, uint32_t cap_mult,
                Layout &L) {
  if (!jobs || n_jobs == 0) return fail(FIUNCHO_E_NULL, "no jobs");
  L.jobs.assign(n_jobs, JobLayout());
  L.nmax = 0;
  L.kmax = 0;
  L.max_n_pad = 0;
  L.max_wcap = 0;
  L.max_cand_cap = 0;
  L.max_sel = 0;
  L.max_pairs_n = 0;
  L.max_pairs4_n = 0;
  L.max_triples_n = 0;
  L.max_quads_n = 0;
  size_t off = 0;
  // per-job data
  for (uint32_t i = 0; i < n_jobs; ++i) {
    int st = check_shape(jobs[i], false);
    if (st) return st;
    JobLayout &J = L.jobs[i];
    J.n = jobs[i].snps;
    J.m = jobs[i].samples;
    J.k = (uint32_t)jobs[i].order;
    J.top_n = jobs[i].top_n;
    J.total = binom_host(J.n, J.k);
    J.n_pad = (uint32_t)((J.n + 63) / 64 * 64 + 64);
    J.wcap = (J.m + 63) / 64 + 2;
    u64 cap = std::max<u64>(1ull << 20, 256ull * J.top_n) * cap_mult;
    cap = std::min<u64>(cap, J.total);
    cap = std::min<u64>(cap, 1ull << 31);
    J.cand_cap = (uint32_t)std::max<u64>(cap, 1);
    J.l1_cap = J.cand_cap;
    // room for every result: the results are gathered here when more than
    // kSortMax candidates are kept
    J.sel_cap = (uint32_t)std::max<u64>(std::min<u64>(J.top_n, J.total), 1);
    const int kern = choose_kernel(J.n, J.m, J.k);
    J.path = kernel_path(kern, J.k);
    J.fp4 = kern == FIUNCHO_KERNEL_MFMA_FP4 || kern == FIUNCHO_KERNEL_MFMA_FP4_TABLES;
    J.wps = (uint32_t)choose_wps(J.n, J.m, J.k);
    // orders 4 and 5 on the matrix cores keep counts in 16 bits and the f
    // table in LDS: larger jobs run on the popcount kernel
    if (J.path == fiuncho::kPathMfmaRows && J.m > fiuncho::mfma_narrow_max_samples()) {
      J.path = fiuncho::kPathGeneric;
      J.fp4 = 0;
    }
    // orders 4 and 5 on the matrix cores with lower-order tables: packed
    // tables, counts below 16,384; larger order-4 jobs use the unpacked
    // triple tables on the popcount kernel, larger order-5 jobs every prefix
    // row on the matrix cores (up to 20,447 samples) or the popcount kernel
    if ((J.path == fiuncho::kPathMfma4t || J.path == fiuncho::kPathMfma5q) && J.m >= 16384) {
      if (J.k == 4) {
        J.path = fiuncho::kPathTriples;
        J.fp4 = 0;
      } else {
        const bool rows = J.m <= fiuncho::mfma_narrow_max_samples();
        J.path = rows ? fiuncho::kPathMfmaRows : fiuncho::kPathGeneric;
        J.fp4 = rows ? 1 : 0;
      }
    }
    build_rows(J.n, J.k, J.path, J.row_start);
    J.nrows = (uint32_t)(J.row_start.size() - 1);
    J.shard_count = jobs[i].shard_count > 1 ? jobs[i].shard_count : 1;
    J.shard_index = J.shard_count > 1 ? jobs[i].shard_index : 0;
    if (J.shard_index >= J.shard_count)
      return fail(FIUNCHO_E_SHAPE, "shard_index must be below shard_count");
    J.tiles = shard_tiles(J.row_start.back(), J.shard_count, J.shard_index);
    // pilot sample: 1/32 of the tiles, between 16 and kPilotTiles, for jobs
    // whose search would otherwise start with a flood of candidates (any job
    // with more combinations than the candidate buffer holds, every job of
    // 512 tiles or more, and jobs of 64 tiles or more with over 64 times
    // top_n combinations); its scores live in the candidate buffer until the
    // scan
    {
      const bool want = J.total > J.cand_cap || J.tiles >= 512 ||
                        (J.tiles >= 64 && J.total > 64ull * J.top_n);
      const u64 s = want ? std::min<u64>({J.tiles, (u64)fiuncho::kPilotTiles,
                                          std::max<u64>(16, J.tiles / 32)})
                         : 0;
      const bool mm = on_matrix_cores(J.path);
      const u64 per = mm ? fiuncho::kMfmaPilotEmits : fiuncho::kPilotEmits;
      const u64 slots = s * fiuncho::kScanWaves * per * 64;
      const bool fits = slots * sizeof(uint32_t) <= (u64)J.cand_cap * sizeof(Cand);
      J.pilot_tiles = (s > 0 && fits) ? (uint32_t)s : 0;
      J.pilot_slots = J.pilot_tiles ? (uint32_t)slots : 0;
    }
    const double words = (double)J.wcap;
    J.cost = J.k == 1 ? 1.0
             : J.path == fiuncho::kPathMfma2 ? words * 4 * 64
             : J.path == fiuncho::kPathMfma3 ? words * 8 * 64
             : J.path == fiuncho::kPathMfmaRows ? words * 64 * std::pow(3.0, (double)J.k - 3)
             : J.k == 2 ? words * 4 * fiuncho::kOrder2Prefixes
             : J.path == fiuncho::kPathPairs ? words * 8 * fiuncho::kOrder3Prefixes
             : J.path == fiuncho::kPathTriples ? words * 20
             : J.path == fiuncho::kPathMfma4t ? words * 16 * 16
             : J.path == fiuncho::kPathMfma5q ? words * 32 * 8
                                             : words * 18 * std::pow(3.0, (double)J.k - 3);
    const bool need_pairs = J.path == fiuncho::kPathPairs || J.path == fiuncho::kPathTriples ||
                            J.path == fiuncho::kPathMfma3 || J.path == fiuncho::kPathMfma4t ||
                            J.path == fiuncho::kPathMfma5q;
    if (J.path == fiuncho::kPathTriples || J.path == fiuncho::kPathMfma4t || J.path == fiuncho::kPathMfma5q)
      L.max_triples_n = std::max(L.max_triples_n, J.n);
    if (J.path == fiuncho::kPathMfma5q) L.max_quads_n = std::max(L.max_quads_n, J.n);
    L.nmax = std::max(L.nmax, J.n);
    L.kmax = std::max(L.kmax, J.k);
    L.max_n_pad = std::max(L.max_n_pad, J.n_pad);
    L.max_wcap = std::max(L.max_wcap, J.wcap);
    L.max_cand_cap = std::max(L.max_cand_cap, J.cand_cap);
    L.max_sel = std::max(L.max_sel, J.sel_cap);

    auto take = [&](size_t bytes) {
      size_t o = off;
      off = align256(off + bytes);
      return o;
    };
    J.off_G = host_inputs ? take((size_t)J.n * J.m) : 0;
    J.off_y = host_inputs ? take(J.m) : 0;
    J.off_idx = take(sizeof(uint32_t) * J.m);
    J.off_Bv = take(sizeof(u64) * (size_t)J.wcap * J.n_pad * 2);
    J.off_Bs = take(sizeof(u64) * (size_t)J.n * 4 * J.wcap);
    J.off_marg = take(sizeof(uint32_t) * (size_t)J.n * 6);
    J.off_hist = take(sizeof(uint32_t) * fiuncho::kHistBins);
    J.off_phist = J.pilot_tiles ? take(sizeof(uint32_t) * fiuncho::kHistBins) : 0;
    J.off_cand = take(sizeof(Cand) * (size_t)J.cand_cap);
    J.off_l1 = take(sizeof(Cand) * (size_t)J.l1_cap);
    J.off_sel = take(sizeof(SortItem) * (size_t)J.sel_cap);
    J.off_sel2 = J.sel_cap > fiuncho::kSortMax ? take(sizeof(SortItem) * (size_t)J.sel_cap) : 0;
    J.off_state = take(sizeof(JobState));
    J.off_out = host_inputs ? take(sizeof(fiuncho_hit) * J.top_n) : 0;
    J.off_nout = host_inputs ? take(sizeof(uint32_t)) : 0;
    J.off_status = host_inputs ? take(sizeof(int32_t)) : 0;
    // the order-3 FP4 matrix-core kernels score from packed pair tables when
    // every count fits 14 bits (fewer than 16,384 samples)
    const bool packed_pairs = (J.path == fiuncho::kPathMfma3 && J.fp4 && J.m < 16384) ||
                              J.path == fiuncho::kPathMfma4t || J.path == fiuncho::kPathMfma5q;
    J.off_pairs = need_pairs && !packed_pairs ? take(sizeof(uint32_t) * 8 * (size_t)J.n * J.n_pad) : 0;
    J.off_pairs4 = packed_pairs ? take(sizeof(uint32_t) * 4 * (size_t)J.n * J.n_pad) : 0;
    if (J.off_pairs) L.max_pairs_n = std::max(L.max_pairs_n, J.n);
    if (J.off_pairs4) L.max_pairs4_n = std::max(L.max_pairs4_n, J.n);
    J.off_triples = J.path == fiuncho::kPathTriples ? take((size_t)triple_table_bytes(J.n)) : 0;
    J.off_triples4 = J.path == fiuncho::kPathMfma4t || J.path == fiuncho::kPathMfma5q
                         ? take((size_t)triple_table_bytes(J.n, true))
                         : 0;
    J.off_quads4 = J.path == fiuncho::kPathMfma5q ? take((size_t)quad_table_bytes(J.n)) : 0;
  }
  // plan region
  L.plan_begin = off;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align256(off + bytes);
    return o;
  };
  L.off_desc = take(sizeof(JobDesc) * n_jobs);
  L.off_jts = take(sizeof(u64) * (n_jobs + 1));
  L.off_jps = take(sizeof(u64) * (n_jobs + 1));
  L.off_binom = take(sizeof(u64) * ((size_t)L.nmax + 1) * fiuncho::kBinomStride);
  for (uint32_t i = 0; i < n_jobs; ++i) {
    JobLayout &J = L.jobs[i];
    J.off_rows = take(sizeof(u64) * J.row_start.size());
    J.off_F32 = take(sizeof(float2) * ((size_t)J.m + 1));
    J.off_Fh = take(sizeof(float) * ((size_t)J.m + 1));
    J.off_Fq = take(sizeof(uint32_t) * ((size_t)J.m + 1));
    J.off_P64 = take(sizeof(double) * ((size_t)J.m + 1));
  }
  L.plan_end = off;
  L.off_counter = take(sizeof(u64) * fiuncho::kTileCounters);
  L.total = off;
  // tile-space order: costliest tiles first, so that cheap ones fill the tail
  L.order.resize(n_jobs);
  for (uint32_t i = 0; i < n_jobs; ++i) L.order[i] = i;
  std::stable_sort(L.order.begin(), L.order.end(),
                   [&](uint32_t a, uint32_t b) { return L.jobs[a].cost > L.jobs[b].cost; });
  // jobs on the matrix cores go last, by group: each group runs in its own
  // launch
  std::stable_sort(L.order.begin(), L.order.end(),
                   [&](uint32_t a, uint32_t b) { return mfma_group(L.jobs[a]) < mfma_group(L.jobs[b]); });
  L.n_scan = 0;
  for (auto &c : L.n_group) c = 0;
  for (auto &J : L.jobs) {
    const int q = mfma_group(J);
    if (q < 0) ++L.n_scan;
    else ++L.n_group[q];
  }
  auto sel = [](const JobLayout &J) {
    return J.path == fiuncho::kPathPairs     ? fiuncho::kSelPairs
           : J.path == fiuncho::kPathTriples ? fiuncho::kSelTriples
                                             : (J.k <= 5 ? (int)J.k : 0);
  };
  L.ksel = -1;
  bool only23 = true;
  for (auto &J : L.jobs) {
    if (on_matrix_cores(J.path)) continue;
    if (L.ksel < 0) L.ksel = sel(J);
    else if (sel(J) != L.ksel) L.ksel = 0;
    only23 = only23 && (J.k == 2 || J.path == fiuncho::kPathPairs);
  }
  if (L.ksel < 0) L.ksel = 0;
  if (L.ksel == 0 && only23) L.ksel = fiuncho::kSel23;
  return FIUNCHO_OK;
}

// Bound of |plain single-precision MI - MI| for tables of 3^k cells and m
// samples.  Let u = 2^-24, f(t) = t ln t, n_x = n_x0 + n_x1.  The scan
// computes c = (F[m] - F[m0]) - F[m1], then s += (F[n_x0] + F[n_x1]) -
// F[n_x] over the cells, then s * (1/m), where each table value F[t] is
// within u f(t) of f(t).  Because f is superadditive (f(a) + f(b) <= f(a+b)),
// sum_x f(n_x) <= f(m); the exact start lies in [0, m ln 2], every exact cell
// term in [-n_x ln 2, 0] and every partial sum in [-m ln 2, m ln 2].  Hence:
//   start:        u (3 f(m) + m ln 2)
//   cells:        sum_x u (3 f(n_x) + n_x ln 2) <= u (3 f(m) + m ln 2)
//   accumulation: 3^k additions of at most u m ln 2 each
//   final scaling: 2u ln 2 on MI
// so |estimate - MI| <= u (6 ln m + (3^k + 4) ln 2) (estimate_bound); the
// filters use twice that (fbound).
double estimate_bound(uint32_t k, uint32_t m) {
  double cells = 1;
  for (uint32_t i = 0; i < k; ++i) cells *= 3;
  const double u = std::ldexp(1.0, -24);
  return u * (6.0 * std::log((double)m) + (cells + 4.0) * std::log(2.0));
}
float fbound(uint32_t k, uint32_t m) { return (float)(2.0 * estimate_bound(k, m) * 1.0001); }

// The shift of the fixed-point f table: the largest qs with 2^qs (m ln 2 + 1)
// <= 2^30, so that 2^qs m MI (MI <= ln 2) and its rounding error stay far
// inside a signed 32-bit integer
int fixed_shift(uint32_t m) {
  const double top = std::ldexp(1.0, 30), span = (double)m * std::log(2.0) + 1.0;
  int qs = 0;
  while (std::ldexp(span, qs + 1) <= top) ++qs;
  return qs;
}

// ---------------------------------------------------------------------------
// plan: descriptors and lookup tables, built on the host
// ---------------------------------------------------------------------------
struct PlanCache {
  std::vector<uint8_t> bytes;  // last uploaded plan region
};
std::mutex g_plan_mu;
std::map<std::pair<int, const void *>, PlanCache> g_plans;

void build_plan(const Layout &L, const fiuncho_job *jobs, uint8_t *ws, bool host_inputs,
                std::vector<uint8_t> &plan) {
  plan.assign(L.plan_end - L.plan_begin, 0);
  auto at = [&](size_t off) { return plan.data() + (off - L.plan_begin); };
  const uint32_t n_jobs = (uint32_t)L.jobs.size();
  // binomial table
  u64 *bt = reinterpret_cast<u64 *>(at(L.off_binom));
  for (uint32_t a = 0; a <= L.nmax; ++a)
    for (int r = 0; r < fiuncho::kBinomStride; ++r)
      bt[(size_t)a * fiuncho::kBinomStride + r] = binom_host(a, (u64)r);
  // job tile starts, in tile-space order
  u64 *jts = reinterpret_cast<u64 *>(at(L.off_jts));
  std::vector<u64> begin(n_jobs);
  u64 acc = 0;
  for (uint32_t p = 0; p < n_jobs; ++p) {
    const uint32_t i = L.order[p];
    jts[p] = acc;
    begin[i] = acc;
    acc += L.jobs[i].tiles;
  }
  jts[n_jobs] = acc;
  u64 *jps = reinterpret_cast<u64 *>(at(L.off_jps));
  acc = 0;
  for (uint32_t p = 0; p < n_jobs; ++p) {
    jps[p] = acc;
    acc += L.jobs[L.order[p]].pilot_tiles;
  }
  jps[n_jobs] = acc;
  JobDesc *desc = reinterpret_cast<JobDesc *>(at(L.off_desc));
  for (uint32_t p = 0; p < n_jobs; ++p) {
    const uint32_t i = L.order[p];
    const JobLayout &J = L.jobs[i];
    JobDesc d;
    std::memset(&d, 0, sizeof(d));
    d.n = J.n;
    d.m = J.m;
    d.k = J.k;
    d.top_n = J.top_n;
    d.n_pad = J.n_pad;
    d.wcap = J.wcap;
    d.nrows = J.nrows;
    d.flags = host_inputs ? 0u : 1u;
    d.total = J.total;
    d.tile_begin = begin[i];
    d.tile_count = J.tiles;
    d.pilot_tiles = J.pilot_tiles;
    d.pilot_slots = J.pilot_slots;
    d.G = host_inputs ? ws + J.off_G : jobs[i].genotypes;
    d.y = host_inputs ? ws + J.off_y : jobs[i].phenotype;
    d.idx = reinterpret_cast<uint32_t *>(ws + J.off_idx);
    d.Bv = reinterpret_cast<u64 *>(ws + J.off_Bv);
    d.Bs = reinterpret_cast<u64 *>(ws + J.off_Bs);
    d.marg = reinterpret_cast<uint32_t *>(ws + J.off_marg);
    d.F32 = reinterpret_cast<const float2 *>(ws + J.off_F32);
    d.Fh = reinterpret_cast<const float *>(ws + J.off_Fh);
    d.Fq = reinterpret_cast<const uint32_t *>(ws + J.off_Fq);
    d.qscale = (float)(std::ldexp(1.0, -fixed_shift(J.m)) / (double)J.m);
    d.fbound = fbound(J.k, J.m);
    d.P64 = reinterpret_cast<const double *>(ws + J.off_P64);
    d.row_start = reinterpret_cast<const u64 *>(ws + J.off_rows);
    d.hist = reinterpret_cast<uint32_t *>(ws + J.off_hist);
    d.phist = J.pilot_tiles ? reinterpret_cast<uint32_t *>(ws + J.off_phist) : nullptr;
    d.cand = reinterpret_cast<Cand *>(ws + J.off_cand);
    d.cand_cap = J.cand_cap;
    d.l1_cap = J.l1_cap;
    d.l1 = reinterpret_cast<Cand *>(ws + J.off_l1);
    d.sel = reinterpret_cast<SortItem *>(ws + J.off_sel);
    d.sel2 = J.off_sel2 ? reinterpret_cast<SortItem *>(ws + J.off_sel2) : nullptr;
    d.sel_cap = J.sel_cap;
    d.path = J.path;
    d.fp4 = J.fp4;
    d.shard_index = J.shard_index;
    d.shard_count = J.shard_count;
    d.pairs = J.off_pairs ? reinterpret_cast<uint32_t *>(ws + J.off_pairs) : nullptr;
    d.pairs4 = J.off_pairs4 ? reinterpret_cast<uint4 *>(ws + J.off_pairs4) : nullptr;
    d.triples = J.off_triples ? reinterpret_cast<uint32_t *>(ws + J.off_triples) : nullptr;
    d.triples4 = J.off_triples4 ? reinterpret_cast<uint4 *>(ws + J.off_triples4) : nullptr;
    d.quads4 = J.off_quads4 ? reinterpret_cast<uint4 *>(ws + J.off_quads4) : nullptr;
    d.state = reinterpret_cast<JobState *>(ws + J.off_state);
    d.out = host_inputs ? reinterpret_cast<fiuncho_hit *>(ws + J.off_out) : jobs[i].out;
    d.n_out = host_inputs ? reinterpret_cast<uint32_t *>(ws + J.off_nout) : jobs[i].n_out;
    d.status_out = host_inputs ? reinterpret_cast<int32_t *>(ws + J.off_status) : jobs[i].status;
    std::memcpy(&desc[p], &d, sizeof(d));
    // tile rows
    std::memcpy(at(J.off_rows), J.row_start.data(), sizeof(u64) * J.row_start.size());
    // f(t) = t ln t as a float pair, and (t/m) ln(t/m) in double
    float2 *F = reinterpret_cast<float2 *>(at(J.off_F32));
    float *Fh = reinterpret_cast<float *>(at(J.off_Fh));
    uint32_t *Fq = reinterpret_cast<uint32_t *>(at(J.off_Fq));
    double *P = reinterpret_cast<double *>(at(J.off_P64));
    const int qs = fixed_shift(J.m);
    F[0] = make_float2(0.f, 0.f);
    Fh[0] = 0.f;
    Fq[0] = 0;
    P[0] = 0.0;
    for (uint32_t t = 1; t <= J.m; ++t) {
      const double f = (double)t * std::log((double)t);
      const float hi = (float)f;
      const float lo = (float)(f - (double)hi);
      F[t] = make_float2(hi, lo);
      Fh[t] = hi;
      // below 2^35 (f(t) 2^qs <= log2(m) 2^30): exact in a 64-bit integer
      Fq[t] = (uint32_t)(unsigned long long)std::llround(std::ldexp(f, qs));
      const double p = (double)t / (double)J.m;
      P[t] = p * std::log(p);
    }
  }
}

Globals make_globals(const Layout &L, uint8_t *ws) {
  Globals g;
  g.binom = reinterpret_cast<const u64 *>(ws + L.off_binom);
  g.nmax = L.nmax;
  g.n_jobs = (uint32_t)L.jobs.size();
  g.jobs = reinterpret_cast<const JobDesc *>(ws + L.off_desc);
  g.job_tile_start = reinterpret_cast<const u64 *>(ws + L.off_jts);
  g.total_tiles = 0;
  for (auto &J : L.jobs) g.total_tiles += J.tiles;
  g.tile_base = 0;
  g.tile_counter = reinterpret_cast<u64 *>(ws + L.off_counter);  // kTileCounters of them
  g.job_pilot_start = reinterpret_cast<const u64 *>(ws + L.off_jps);
  g.total_pilot_tiles = 0;
  for (auto &J : L.jobs) g.total_pilot_tiles += J.pilot_tiles;
  g.pilot = 0;
  g.lds_f_entries = 0;
  return g;
}

// The globals of one counting launch over jobs [first, first + count) of the
// tile-space order; `pilot` selects the pilot tiles.  tiles[] = the host's
// copy of the job tile (or pilot) starts.
Globals launch_globals(const Globals &g, const std::vector<u64> &starts, uint32_t first,
                       uint32_t count, bool pilot, int counter) {
  Globals r = g;
  r.jobs = g.jobs + first;
  r.n_jobs = count;
  r.job_tile_start = (pilot ? g.job_pilot_start : g.job_tile_start) + first;
  r.tile_base = starts[first];
  r.total_tiles = starts[first + count];
  r.tile_counter = g.tile_counter + counter;
  r.pilot = pilot ? 1u : 0u;
  return r;
}

int upload_plan(const Layout &L, const fiuncho_job *jobs, uint8_t *ws, bool host_inputs,
                hipStream_t stream, bool force = false) {
  std::vector<uint8_t> plan;
  build_plan(L, jobs, ws, host_inputs, plan);
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_plan_mu);
  PlanCache &pc = g_plans[std::make_pair(dev, (const void *)ws)];
  if (!force && pc.bytes == plan) return FIUNCHO_OK;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  HIP_TRY(hipStreamIsCapturing(stream, &cs));
  if (cs != hipStreamCaptureStatusNone)
    return fail(FIUNCHO_E_WORKSPACE,
                "the plan for this workspace and job set is not uploaded yet: call once "
                "before capturing the stream");
  HIP_TRY(hipMemcpyAsync(ws + L.plan_begin, plan.data(), plan.size(), hipMemcpyHostToDevice, stream));
  HIP_TRY(hipStreamSynchronize(stream));
  pc.bytes.swap(plan);
  return FIUNCHO_OK;
}

// ---------------------------------------------------------------------------
// device check
// ---------------------------------------------------------------------------
int check_device() {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(FIUNCHO_E_DEVICE, std::string("no HIP device: ") + hipGetErrorString(e));
  hipDeviceProp_t prop;
  e = hipGetDeviceProperties(&prop, dev);
  if (e != hipSuccess) return fail(FIUNCHO_E_DEVICE, hipGetErrorString(e));
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(FIUNCHO_E_DEVICE, std::string("libfiuncho is built for gfx950, device is ") + prop.gcnArchName);
  return FIUNCHO_OK;
}

// ---------------------------------------------------------------------------
// profiling events
// ---------------------------------------------------------------------------
// one profiled call: events before pack, before scan, before select, at end
constexpr int kProfEvents = 6;
struct ProfCall {
  // before pack, after pack (and pair tables), after the pilot pass, after
  // the popcount kernel, after the matrix-core kernel, at the end
  hipEvent_t ev[kProfEvents] = {};
  u64 combos = 0;
  uint32_t kernels = 0;
  JobState *state0 = nullptr;
};
thread_local std::vector<ProfCall> t_calls;   // recorded, not yet collected
thread_local std::vector<hipEvent_t> t_free;  // event pool
thread_local ProfCall *t_cur = nullptr;

int prof_begin(u64 combos, uint32_t kernels, JobState *state0) {
  t_cur = nullptr;
  if (!t_profiling) return FIUNCHO_OK;
  t_calls.emplace_back();
  ProfCall &c = t_calls.back();
  for (int i = 0; i < kProfEvents; ++i) {
    if (!t_free.empty()) {
      c.ev[i] = t_free.back();
      t_free.pop_back();
    } else {
      HIP_TRY(hipEventCreate(&c.ev[i]));
    }
  }
  c.combos = combos;
  c.kernels = kernels;
  c.state0 = state0;
  t_cur = &c;
  return FIUNCHO_OK;
}

int prof_record(int i, hipStream_t s) {
  if (!t_cur) return FIUNCHO_OK;
  HIP_TRY(hipEventRecord(t_cur->ev[i], s));
  return FIUNCHO_OK;
}

// ---------------------------------------------------------------------------
// the pipeline on an uploaded plan
// ---------------------------------------------------------------------------
// Combinations of one shard of a job (a walk over the job's tiles, so the
// counts are kept per shape and shard: repeated profiled calls do not repeat
// the walk)
u64 shard_combinations(const JobLayout &J) {
  typedef std::tuple<uint32_t, uint32_t, uint32_t, uint32_t, uint32_t> Key;
  static std::mutex mu;
  static std::map<Key, u64> memo;
  const Key key(J.n, J.k, J.path, J.shard_count, J.shard_index);
  {
    std::lock_guard<std::mutex> lk(mu);
    auto it = memo.find(key);
    if (it != memo.end()) return it->second;
  }
  u64 combos = 0;
  for_each_tile(J.n, J.k, J.path, [&](u64 lt, u64 c) {
    if (tile_shard(lt, J.shard_count) == J.shard_index) combos += c;
  });
  std::lock_guard<std::mutex> lk(mu);
  memo[key] = combos;
  return combos;
}

int run_pipeline(const Layout &L, uint8_t *ws, hipStream_t s) {
  const Globals g = make_globals(L, ws);
  int st;
  u64 combos = 0;
  if (t_profiling)
    for (auto &J : L.jobs) combos += J.shard_count <= 1 ? J.total : shard_combinations(J);
  uint32_t kernels = 0;
  for (auto &J : L.jobs)
    kernels |= 1u << (J.path == fiuncho::kPathPairs     ? FIUNCHO_KERNEL_PAIRS
                      : J.path == fiuncho::kPathTriples ? FIUNCHO_KERNEL_TRIPLES
                      : J.path == fiuncho::kPathMfma4t || J.path == fiuncho::kPathMfma5q
                          ? FIUNCHO_KERNEL_MFMA_FP4_TABLES
                      : on_matrix_cores(J.path)         ? (J.fp4 ? FIUNCHO_KERNEL_MFMA_FP4 : FIUNCHO_KERNEL_MFMA)
                                                      : FIUNCHO_KERNEL_POPCOUNT);
  if ((st = prof_begin(combos, kernels, reinterpret_cast<JobState *>(ws + L.jobs[0].off_state))))
    return st;
  if ((st = prof_record(0, s))) return st;
  fiuncho::launch_init(g, s);
  fiuncho::launch_pack(g, L.max_n_pad, L.max_wcap, s);
  if (L.max_pairs_n) fiuncho::launch_pairs(g, L.max_pairs_n, s);
  if (L.max_pairs4_n) fiuncho::launch_pairs4(g, L.max_pairs4_n, s);
  if (L.max_triples_n) fiuncho::launch_triples(g, L.max_triples_n, s);
  if (L.max_quads_n) fiuncho::launch_quads(g, L.max_quads_n, s);
  if ((st = prof_record(1, s))) return st;
  // job tile and pilot starts in tile-space order (as uploaded)
  const uint32_t nj = (uint32_t)L.jobs.size();
  std::vector<u64> ts(nj + 1, 0), ps(nj + 1, 0);
  for (uint32_t p = 0; p < nj; ++p) {
    ts[p + 1] = ts[p] + L.jobs[L.order[p]].tiles;
    ps[p + 1] = ps[p] + L.jobs[L.order[p]].pilot_tiles;
  }
  const uint32_t ns = L.n_scan;
  // the grid of a counting launch over jobs [first, first + count) of the
  // tile-space order: at most gmax workgroups (every compute unit at full
  // occupancy), fewer when every one of its jobs asks for fewer waves per
  // SIMD (a workgroup is 4 waves: workgroups per compute unit = waves per SIMD)
  int cus = 0;
  {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  }
  auto capped = [&](const Globals &c, int gmax) {
    const uint32_t first = (uint32_t)(c.jobs - g.jobs);
    uint32_t cap = 0;
    for (uint32_t i = first; i < first + c.n_jobs; ++i) {
      const uint32_t w = L.jobs[L.order[i]].wps;
      if (w == 0) return gmax;
      cap = std::max(cap, w);
    }
    return std::min(gmax, (int)(cap * (uint32_t)cus));
  };
  // f-table entries an orders-4/5 matrix-core launch keeps in LDS: those of
  // the largest job of its jobs [first, first + count) of the tile-space
  // order, up to the kernel's maximum
  auto rows_f_entries = [&](const Globals &c, int order, bool dual) {
    const uint32_t first = (uint32_t)(c.jobs - g.jobs);
    uint32_t m_max = 0;
    for (uint32_t i = first; i < first + c.n_jobs; ++i) m_max = std::max(m_max, L.jobs[L.order[i]].m);
    return std::min(m_max + 1, fiuncho::mfma_rows_max_entries(order, dual));
  };
  // group -1: the popcount kernel; q >= 0: the matrix-core kernel of group q
  auto counting = [&](const Globals &c, int q) {
    if (c.total_tiles <= c.tile_base) return;
    const u64 tiles = c.total_tiles - c.tile_base;
    if (q >= 8) {  // orders 4, 5 with lower-order tables
      const int order = q - 4;
      const int grid = (int)std::min<u64>((u64)capped(c, fiuncho::mfma_sub_grid_size(order, false)), tiles);
      fiuncho::launch_mfma_sub(c, order, false, grid, s);
      return;
    }
    if (q >= 6) {  // orders 4, 5: every prefix row on the matrix cores
      const int order = q - 2;
      Globals r = c;
      r.lds_f_entries = rows_f_entries(c, order, false);
      const int grid =
          (int)std::min<u64>((u64)capped(c, fiuncho::mfma_rows_grid_size(order, false, r.lds_f_entries)), tiles);
      fiuncho::launch_mfma_rows(r, order, false, grid, s);
      return;
    }
    const int order = 2 + q / 3;
    const int fmt = q % 3;
    const int gmax = q >= 0 ? fiuncho::mfma_grid_size(order, fmt) : fiuncho::scan_grid_size(L.ksel);
    const int grid = (int)std::min<u64>((u64)capped(c, gmax), tiles);
    if (q >= 0) fiuncho::launch_mfma(c, order, fmt, grid, s);
    else fiuncho::launch_scan(c, L.ksel, grid, s);
  };
  // the matrix-core groups' launches over their jobs; counters 2 + 2q (counting)
  // and 3 + 2q (pilot).  The narrow FP4 groups (2, 5) and the groups of orders
  // 4 and 5 (6, 7) run the dual kernel first over the same tiles, on counters
  // kDualCounters + 2 slot (+ 1 for the pilot): it takes the jobs whose class
  // sizes allow one accumulator for both classes, the group's kernel the rest
  auto mfma_groups = [&](const std::vector<u64> &starts, bool pilot) {
    uint32_t first = ns;
    for (int q = 0; q < fiuncho::kMfmaGroups; ++q) {
      if (L.n_group[q]) {
        const Globals c = launch_globals(g, starts, first, L.n_group[q], pilot, 2 + 2 * q + pilot);
        const int slot = q == 2 ? 0 : q == 5 ? 1 : q >= 6 ? q - 4 : -1;
        const bool sub = q >= 8;  // orders 4, 5 with lower-order tables
        // no dual launch when no job of the group has few enough samples
        const int order = sub ? q - 4 : q >= 6 ? q - 2 : 2 + q / 3;
        const uint32_t dual_max = sub ? fiuncho::mfma_sub_dual_max_samples() : fiuncho::mfma_dual_max_samples(order);
        uint32_t min_m = ~0u;
        for (uint32_t i = first; i < first + L.n_group[q]; ++i) min_m = std::min(min_m, L.jobs[L.order[i]].m);
        if (slot >= 0 && c.total_tiles > c.tile_base && min_m <= dual_max) {
          Globals d = c;
          d.tile_counter = g.tile_counter + fiuncho::kDualCounters + 2 * slot + pilot;
          const u64 tiles = d.total_tiles - d.tile_base;
          if (sub) {
            const int grid = (int)std::min<u64>((u64)capped(d, fiuncho::mfma_sub_grid_size(order, true)), tiles);
            fiuncho::launch_mfma_sub(d, order, true, grid, s);
          } else if (q >= 6) {
            d.lds_f_entries = rows_f_entries(d, order, true);
            const int grid = (int)std::min<u64>(
                (u64)capped(d, fiuncho::mfma_rows_grid_size(order, true, d.lds_f_entries)), tiles);
            fiuncho::launch_mfma_rows(d, order, true, grid, s);
          } else {
            const int grid = (int)std::min<u64>((u64)capped(d, fiuncho::mfma_grid_size(order, 3)), tiles);
            fiuncho::launch_mfma(d, order, 3, grid, s);
          }
        }
        counting(c, q);
      }
      first += L.n_group[q];
    }
  };
  if (g.total_pilot_tiles) {
    if (ns) counting(launch_globals(g, ps, 0, ns, true, 1), -1);
    mfma_groups(ps, true);
    uint32_t max_slots = 0;
    for (auto &J : L.jobs) max_slots = std::max(max_slots, J.pilot_slots);
    fiuncho::launch_pilot_select(g, max_slots, s);
  }
  if ((st = prof_record(2, s))) return st;
  if (ns) counting(launch_globals(g, ts, 0, ns, false, 0), -1);
  if ((st = prof_record(3, s))) return st;
  mfma_groups(ts, false);
  if ((st = prof_record(4, s))) return st;
  fiuncho::launch_select(g, L.max_cand_cap, s);
  fiuncho::launch_rescore(g, L.kmax, s);
  fiuncho::launch_finish(g, s);
  fiuncho::launch_big_sort(g, L.max_sel, s);
  if ((st = prof_record(5, s))) return st;
  HIP_TRY(hipGetLastError());
  return FIUNCHO_OK;
}

int batch_impl(const fiuncho_job *jobs, uint32_t n_jobs, uint32_t flags, void *workspace,
               size_t ws_bytes, hipStream_t stream, uint32_t cap_mult, bool *cand_overflow) {
  if (cand_overflow) *cand_overflow = false;
  if (!jobs || n_jobs == 0) return fail(FIUNCHO_E_NULL, "no jobs");
  if (!workspace) return fail(FIUNCHO_E_NULL, "workspace is NULL");
  if (((uintptr_t)workspace) & 255) return fail(FIUNCHO_E_WORKSPACE, "workspace must be 256-byte aligned");
  const bool host_inputs = !(flags & FIUNCHO_DEVICE_PTRS);
  for (uint32_t i = 0; i < n_jobs; ++i) {
    int st = check_shape(jobs[i], true);
    if (st) return st;
    if (host_inputs) {
      st = check_values(jobs[i].genotypes, jobs[i].phenotype, jobs[i].snps, jobs[i].samples);
      if (st) return st;
    }
  }
  int st = check_device();
  if (st) return st;
  Layout L;
  st = make_layout(jobs, n_jobs, host_inputs, cap_mult, L);
  if (st) return st;
  if (ws_bytes < L.total)
    return fail(FIUNCHO_E_WORKSPACE, "workspace has " + std::to_string(ws_bytes) + " bytes, needs " +
                                         std::to_string(L.total));
  uint8_t *ws = static_cast<uint8_t *>(workspace);
  st = upload_plan(L, jobs, ws, host_inputs, stream, (flags & FIUNCHO_UPLOAD_PLAN) != 0);
  if (st) return st;
  if (host_inputs) {
    for (uint32_t i = 0; i < n_jobs; ++i) {
      const JobLayout &J = L.jobs[i];
      HIP_TRY(hipMemcpyAsync(ws + J.off_G, jobs[i].genotypes, (size_t)J.n * J.m, hipMemcpyHostToDevice, stream));
      HIP_TRY(hipMemcpyAsync(ws + J.off_y, jobs[i].phenotype, J.m, hipMemcpyHostToDevice, stream));
    }
  }
  st = run_pipeline(L, ws, stream);
  if (st) return st;
  if (!host_inputs) return FIUNCHO_OK;
  // bring the results back
  std::vector<uint32_t> nout(n_jobs);
  std::vector<int32_t> status(n_jobs);
  std::vector<JobState> states(n_jobs);
  for (uint32_t i = 0; i < n_jobs; ++i) {
    const JobLayout &J = L.jobs[i];
    HIP_TRY(hipMemcpyAsync(&nout[i], ws + J.off_nout, sizeof(uint32_t), hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipMemcpyAsync(&status[i], ws + J.off_status, sizeof(int32_t), hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipMemcpyAsync(&states[i], ws + J.off_state, sizeof(JobState), hipMemcpyDeviceToHost, stream));
  }
  HIP_TRY(hipStreamSynchronize(stream));
  int first_err = FIUNCHO_OK;
  for (uint32_t i = 0; i < n_jobs; ++i) {
    const JobLayout &J = L.jobs[i];
    if (status[i] != 0) {
      *jobs[i].n_out = 0;
      if (jobs[i].status) *jobs[i].status = status[i];
      if (states[i].flags & fiuncho::kFlagCandOverflow) {
        if (cand_overflow) *cand_overflow = true;
      }
      if (first_err == FIUNCHO_OK) {
        first_err = status[i];
        if (states[i].flags & fiuncho::kFlagCandOverflow)
          fail(status[i], "candidate buffer overflow in job " + std::to_string(i));
        else if (states[i].flags & fiuncho::kFlagBound)
          fail(status[i], "self-check failed in job " + std::to_string(i) +
                              ": a counting kernel's estimate is farther from the exact MI than its bound");
        else
          fail(status[i], "job " + std::to_string(i) + " failed on the device");
      }
      continue;
    }
    if (nout[i] > J.top_n) return fail(FIUNCHO_E_DEVICE, "device returned too many results");
    HIP_TRY(hipMemcpy(jobs[i].out, ws + J.off_out, sizeof(fiuncho_hit) * nout[i], hipMemcpyDeviceToHost));
    *jobs[i].n_out = nout[i];
    if (jobs[i].status) *jobs[i].status = 0;
  }
  return first_err;
}

// library-owned workspace for the plain (synchronous, host pointer) calls
struct OwnedWs {
  void *ptr = nullptr;
  size_t bytes = 0;
};
std::mutex g_ws_mu;
std::map<int, OwnedWs> g_ws;

// frees device memory that held a workspace, forgetting its plan
int free_workspace(void *p) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  {
    std::lock_guard<std::mutex> lk(g_plan_mu);
    g_plans.erase(std::make_pair(dev, (const void *)p));
  }
  HIP_TRY(hipFree(p));
  return FIUNCHO_OK;
}

int owned_workspace(size_t need, void **out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  OwnedWs &w = g_ws[dev];
  if (w.bytes < need) {
    if (w.ptr) {
      // drop the plan cache entry of the old buffer
      {
        std::lock_guard<std::mutex> lk(g_plan_mu);
        g_plans.erase(std::make_pair(dev, (const void *)w.ptr));
      }
      HIP_TRY(hipFree(w.ptr));
      w.ptr = nullptr;
      w.bytes = 0;
    }
    HIP_TRY(hipMalloc(&w.ptr, need));
    w.bytes = need;
  }
  *out = w.ptr;
  return FIUNCHO_OK;
}

}  // namespace

// Device memory of fiuncho_scan_batch_static: one array per GPU, held until
// the process ends.  In host code its name is only a stand-in for the
// symbol: the array's address on a device comes from hipGetSymbolAddress
// (scratch_on_device), and only that address is handed to kernels.
constexpr size_t kScratchBytes = (size_t)FIUNCHO_STATIC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

std::mutex g_scratch_mu;
std::map<int, void *> g_scratch;  // device -> address of its scratch array

// The current device's scratch address, looked up once per device with that
// device current.
int scratch_on_device(void **out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch.find(dev);
  if (it == g_scratch.end()) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(FIUNCHO_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    it = g_scratch.emplace(dev, p).first;
  }
  *out = it->second;
  return FIUNCHO_OK;
}

}  // namespace

int fiuncho::set_error(int code, const char *msg) { return fail(code, msg); }

extern "C" {

const char *fiuncho_last_error(void) { return t_err.c_str(); }

double fiuncho_estimate_bound(int order, uint32_t samples) {
  if (order < 1 || order > FIUNCHO_MAX_ORDER || samples == 0) return -1.0;
  return estimate_bound((uint32_t)order, samples);
}

void fiuncho_set_profiling(int enable) { t_profiling = enable != 0; }

int fiuncho_get_profile(fiuncho_profile *out) {
  if (!out) return fail(FIUNCHO_E_NULL, "out is NULL");
  if (t_calls.empty()) return fail(FIUNCHO_E_NULL, "no profiled call on this thread");
  // phase i runs from event i to event i + 1; the total from the first to the last
  double ph[kProfEvents] = {0};
  for (ProfCall &pc : t_calls) {
    HIP_TRY(hipEventSynchronize(pc.ev[kProfEvents - 1]));
    for (int i = 0; i + 1 < kProfEvents; ++i) {
      float x = 0;
      HIP_TRY(hipEventElapsedTime(&x, pc.ev[i], pc.ev[i + 1]));
      ph[i] += x;
    }
    float x = 0;
    HIP_TRY(hipEventElapsedTime(&x, pc.ev[0], pc.ev[kProfEvents - 1]));
    ph[kProfEvents - 1] += x;
  }
  const double n = (double)t_calls.size();
  const ProfCall &last = t_calls.back();
  JobState s0;
  HIP_TRY(hipMemcpy(&s0, last.state0, sizeof(JobState), hipMemcpyDeviceToHost));
  out->pack_ms = (float)(ph[0] / n);
  out->pilot_ms = (float)(ph[1] / n);
  out->scan_ms = (float)(ph[2] / n);
  out->mfma_ms = (float)(ph[3] / n);
  out->select_ms = (float)(ph[4] / n);
  out->total_ms = (float)(ph[5] / n);
  out->calls = (uint32_t)t_calls.size();
  out->combinations = last.combos;
  out->candidates = s0.cand_count;
  out->kept = s0.l2_count;
  out->flags = s0.flags;
  out->kernels = last.kernels;
  for (ProfCall &pc : t_calls)
    for (int i = 0; i < kProfEvents; ++i) t_free.push_back(pc.ev[i]);
  t_calls.clear();
  t_cur = nullptr;
  return FIUNCHO_OK;
}

size_t fiuncho_workspace_bytes(const fiuncho_job *jobs, uint32_t n_jobs) {
  Layout L;
  if (make_layout(jobs, n_jobs, false, 1, L) != FIUNCHO_OK) return 0;
  return L.total;
}

int fiuncho_scan_batch(const fiuncho_job *jobs, uint32_t n_jobs, uint32_t flags, void *workspace,
                       size_t ws_bytes, void *hip_stream) {
  t_err.clear();
  try {
    return batch_impl(jobs, n_jobs, flags, workspace, ws_bytes, (hipStream_t)hip_stream, 1, nullptr);
  } catch (const std::exception &e) {
    return fail(FIUNCHO_E_DEVICE, std::string("internal error: ") + e.what());
  } catch (...) {
    return fail(FIUNCHO_E_DEVICE, "internal error");
  }
}

int fiuncho_scan_batch_static(const fiuncho_job *jobs, uint32_t n_jobs, uint32_t flags,
                              void *hip_stream) {
  t_err.clear();
  try {
    // the size check comes first, before any device work
    Layout L;
    int st = make_layout(jobs, n_jobs, !(flags & FIUNCHO_DEVICE_PTRS), 1, L);
    if (st) return st;
    if (L.total > kScratchBytes)
      return fail(FIUNCHO_E_WORKSPACE, "these jobs need " + std::to_string(L.total) +
                                           " bytes of workspace; the static scratch holds " +
                                           std::to_string(kScratchBytes) +
                                           " (use fiuncho_scan_batch with a workspace)");
    void *ws = nullptr;
    st = check_device();
    if (st) return st;
    st = scratch_on_device(&ws);
    if (st) return st;
    return batch_impl(jobs, n_jobs, flags, ws, kScratchBytes, (hipStream_t)hip_stream, 1, nullptr);
  } catch (const std::exception &e) {
    return fail(FIUNCHO_E_DEVICE, std::string("internal error: ") + e.what());
  } catch (...) {
    return fail(FIUNCHO_E_DEVICE, "internal error");
  }
}

int fiuncho_scan(const uint8_t *genotypes, const uint8_t *phenotype, uint32_t snps,
                 uint32_t samples, int order, uint32_t top_n, fiuncho_hit *out,
                 uint32_t *n_out) {
  t_err.clear();
  if (n_out) *n_out = 0;
  try {
    fiuncho_job job;
    std::memset(&job, 0, sizeof(job));
    job.genotypes = genotypes;
    job.phenotype = phenotype;
    job.snps = snps;
    job.samples = samples;
    job.order = order;
    job.top_n = top_n;
    job.out = out;
    job.n_out = n_out;
    job.status = nullptr;
    int st = check_shape(job, true);
    if (st) return st;
    st = check_values(genotypes, phenotype, snps, samples);
    if (st) return st;
    st = check_device();
    if (st) return st;
    std::lock_guard<std::mutex> lk(g_ws_mu);
    for (uint32_t mult = 1; mult <= 64; mult *= 8) {
      Layout L;
      st = make_layout(&job, 1, true, mult, L);
      if (st) return st;
      void *ws = nullptr;
      st = owned_workspace(L.total, &ws);
      if (st) return st;
      bool overflow = false;
      st = batch_impl(&job, 1, 0, ws, L.total, nullptr, mult, &overflow);
      if (!(st == FIUNCHO_E_WORKSPACE && overflow)) return st;
    }
    return st;
  } catch (const std::exception &e) {
    return fail(FIUNCHO_E_DEVICE, std::string("internal error: ") + e.what());
  } catch (...) {
    return fail(FIUNCHO_E_DEVICE, "internal error");
  }
}

}  // extern "C"

namespace {

// tables and/or scores of explicit combinations (fiuncho_contingency,
// fiuncho_score)
int explicit_impl(const uint8_t *genotypes, const uint8_t *phenotype, uint32_t snps,
                  uint32_t samples, int order, const uint64_t *ranks, uint64_t n_ranks,
                  uint32_t *tables, float *est, float *mi32, double *mi) {
  fiuncho_job job;
  std::memset(&job, 0, sizeof(job));
  job.genotypes = genotypes;
  job.phenotype = phenotype;
  job.snps = snps;
  job.samples = samples;
  job.order = order;
  job.top_n = 1;
  if (!genotypes || !phenotype || (n_ranks && !ranks))
    return fail(FIUNCHO_E_NULL, "a required pointer is NULL");
  int st = check_shape(job, false);
  if (st) return st;
  st = check_values(genotypes, phenotype, snps, samples);
  if (st) return st;
  const u64 total = binom_host(snps, (u64)order);
  for (uint64_t i = 0; i < n_ranks; ++i)
    if (ranks[i] >= total)
      return fail(FIUNCHO_E_SHAPE, "rank " + std::to_string(ranks[i]) + " is not below C(snps, order)");
  if (n_ranks == 0) return FIUNCHO_OK;
  st = check_device();
  if (st) return st;
  std::lock_guard<std::mutex> lk(g_ws_mu);
  Layout L;
  st = make_layout(&job, 1, true, 1, L);
  if (st) return st;
  uint64_t cells = 1;
  for (int q = 0; q < order; ++q) cells *= 3;
  const size_t rank_off = align256(L.total);
  const size_t tab_off = align256(rank_off + sizeof(u64) * n_ranks);
  const size_t est_off = align256(tab_off + (tables ? sizeof(uint32_t) * 2 * cells * n_ranks : 0));
  const size_t m32_off = align256(est_off + (est ? sizeof(float) * n_ranks : 0));
  const size_t m64_off = align256(m32_off + (mi32 ? sizeof(float) * n_ranks : 0));
  const size_t need = m64_off + (mi ? sizeof(double) * n_ranks : 0);
  void *wsv = nullptr;
  st = owned_workspace(need, &wsv);
  if (st) return st;
  uint8_t *ws = static_cast<uint8_t *>(wsv);
  hipStream_t s = nullptr;
  st = upload_plan(L, &job, ws, true, s);
  if (st) return st;
  const JobLayout &J = L.jobs[0];
  HIP_TRY(hipMemcpyAsync(ws + J.off_G, genotypes, (size_t)snps * samples, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(ws + J.off_y, phenotype, samples, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(ws + rank_off, ranks, sizeof(u64) * n_ranks, hipMemcpyHostToDevice, s));
  const Globals g = make_globals(L, ws);
  fiuncho::launch_init(g, s);
  fiuncho::launch_pack(g, L.max_n_pad, L.max_wcap, s);
  fiuncho::launch_tables(g, reinterpret_cast<const u64 *>(ws + rank_off), n_ranks,
                         tables ? reinterpret_cast<uint32_t *>(ws + tab_off) : nullptr,
                         est ? reinterpret_cast<float *>(ws + est_off) : nullptr,
                         mi32 ? reinterpret_cast<float *>(ws + m32_off) : nullptr,
                         mi ? reinterpret_cast<double *>(ws + m64_off) : nullptr, (uint32_t)order, s);
  HIP_TRY(hipGetLastError());
  int32_t status = 0;
  HIP_TRY(hipMemcpyAsync(&status, ws + J.off_state + offsetof(JobState, status), sizeof(int32_t),
                         hipMemcpyDeviceToHost, s));
  if (tables)
    HIP_TRY(hipMemcpyAsync(tables, ws + tab_off, sizeof(uint32_t) * 2 * cells * n_ranks,
                           hipMemcpyDeviceToHost, s));
  if (est) HIP_TRY(hipMemcpyAsync(est, ws + est_off, sizeof(float) * n_ranks, hipMemcpyDeviceToHost, s));
  if (mi32) HIP_TRY(hipMemcpyAsync(mi32, ws + m32_off, sizeof(float) * n_ranks, hipMemcpyDeviceToHost, s));
  if (mi) HIP_TRY(hipMemcpyAsync(mi, ws + m64_off, sizeof(double) * n_ranks, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (status != 0) return fail(status, "the device rejected the input");
  return FIUNCHO_OK;
}

}  // namespace

extern "C" {

int fiuncho_contingency(const uint8_t *genotypes, const uint8_t *phenotype, uint32_t snps,
                        uint32_t samples, int order, const uint64_t *ranks, uint64_t n_ranks,
                        uint32_t *tables) {
  t_err.clear();
  try {
    if (n_ranks && !tables) return fail(FIUNCHO_E_NULL, "tables is NULL");
    return explicit_impl(genotypes, phenotype, snps, samples, order, ranks, n_ranks, tables,
                         nullptr, nullptr, nullptr);
  } catch (const std::exception &e) {
    return fail(FIUNCHO_E_DEVICE, std::string("internal error: ") + e.what());
  } catch (...) {
    return fail(FIUNCHO_E_DEVICE, "internal error");
  }
}

int fiuncho_shard_counts(uint32_t snps, uint32_t samples, int order, uint32_t units, int scheme,
                         uint64_t *counts) {
  t_err.clear();
  if (!counts) return fail(FIUNCHO_E_NULL, "counts is NULL");
  if (units == 0) return fail(FIUNCHO_E_SHAPE, "units must be positive");
  if (scheme != 0 && scheme != 1) return fail(FIUNCHO_E_SHAPE, "scheme must be 0 or 1");
  if (snps == 0) return fail(FIUNCHO_E_SHAPE, "snps must be positive");
  if (order < 1 || order > FIUNCHO_MAX_ORDER || (uint32_t)order > snps)
    return fail(FIUNCHO_E_ORDER, "order must be in [1, min(snps, 8)]");
  if (binom_host(snps, (u64)order) >= (1ull << 63))
    return fail(FIUNCHO_E_OVERFLOW, "C(snps, order) must be below 2^63");
  for (uint32_t u = 0; u < units; ++u) counts[u] = 0;
  const uint32_t k = (uint32_t)order;
  if (scheme == 1) {
    for_each_tile(snps, k, job_path(snps, samples, k),
                  [&](u64 lt, u64 c) { counts[tile_shard(lt, units)] += c; });
    return FIUNCHO_OK;
  }
  if (k == 1) {  // a single, empty prefix
    counts[0] = snps;
    return FIUNCHO_OK;
  }
  // (k-1)-prefixes with a possible extension are the (k-1)-subsets of
  // [0, snps-2]; in ascending lexicographic order, prefix i goes to unit
  // i mod units and brings the snps - 1 - (its last variant) extensions
  const uint32_t r = k - 1, top = snps - 2;
  std::vector<uint32_t> c(r);
  for (uint32_t q = 0; q < r; ++q) c[q] = q;
  uint32_t unit = 0;
  for (;;) {
    counts[unit] += snps - 1 - c[r - 1];
    unit = unit + 1 == units ? 0 : unit + 1;
    int q = (int)r - 1;
    while (q >= 0 && c[q] == top - (r - 1 - (uint32_t)q)) --q;
    if (q < 0) break;
    ++c[q];
    for (uint32_t z = (uint32_t)q + 1; z < r; ++z) c[z] = c[z - 1] + 1;
  }
  return FIUNCHO_OK;
}

int fiuncho_get_kernel(uint32_t snps, uint32_t samples, int order) {
  t_err.clear();
  if (order < 1 || order > FIUNCHO_MAX_ORDER || (uint32_t)order > snps)
    return fail(FIUNCHO_E_ORDER, "order must be in [1, min(snps, 8)]");
  return choose_kernel(snps, samples, (uint32_t)order);
}

int fiuncho_set_config(uint32_t snps, uint32_t samples, int order, int kernel, int waves_per_simd) {
  t_err.clear();
  if (order < 1 || order > FIUNCHO_MAX_ORDER || (uint32_t)order > snps)
    return fail(FIUNCHO_E_ORDER, "order must be in [1, min(snps, 8)]");
  if (waves_per_simd < 0 || waves_per_simd > 8)
    return fail(FIUNCHO_E_SHAPE, "waves_per_simd must be in [0, 8]");
  std::lock_guard<std::mutex> lk(g_tune_mu);
  const ShapeKey key = shape_key(snps, samples, (uint32_t)order);
  if (kernel == FIUNCHO_KERNEL_AUTO) {
    g_tuned.erase(key);
    return FIUNCHO_OK;
  }
  if (!kernel_valid(kernel, snps, (uint32_t)order))
    return fail(FIUNCHO_E_SHAPE, "kernel " + std::to_string(kernel) + " does not handle order " +
                                     std::to_string(order));
  g_tuned[key] = TuneEntry{kernel, waves_per_simd};
  return FIUNCHO_OK;
}

int fiuncho_set_kernel(uint32_t snps, uint32_t samples, int order, int kernel) {
  return fiuncho_set_config(snps, samples, order, kernel, 0);
}

int fiuncho_get_config(uint32_t snps, uint32_t samples, int order, int *kernel, int *waves_per_simd) {
  t_err.clear();
  if (!kernel || !waves_per_simd) return fail(FIUNCHO_E_NULL, "kernel and waves_per_simd must not be NULL");
  if (order < 1 || order > FIUNCHO_MAX_ORDER || (uint32_t)order > snps)
    return fail(FIUNCHO_E_ORDER, "order must be in [1, min(snps, 8)]");
  *kernel = choose_kernel(snps, samples, (uint32_t)order);
  *waves_per_simd = choose_wps(snps, samples, (uint32_t)order);
  return FIUNCHO_OK;
}

int fiuncho_autotune(uint32_t snps, uint32_t samples, int order, uint32_t reps, int *kernel) {
  t_err.clear();
  try {
    if (!kernel) return fail(FIUNCHO_E_NULL, "kernel is NULL");
    fiuncho_job job;
    std::memset(&job, 0, sizeof(job));
    job.snps = snps;
    job.samples = samples;
    job.order = order;
    job.top_n = 16;
    int st = check_shape(job, false);
    if (st) return st;
    st = check_device();
    if (st) return st;
    const uint32_t k = (uint32_t)order;
    std::vector<int> cands;
    for (int c : {FIUNCHO_KERNEL_POPCOUNT, FIUNCHO_KERNEL_PAIRS, FIUNCHO_KERNEL_MFMA, FIUNCHO_KERNEL_TRIPLES,
                  FIUNCHO_KERNEL_MFMA_FP4, FIUNCHO_KERNEL_MFMA_FP4_TABLES})
      if (kernel_valid(c, snps, k)) cands.push_back(c);
    int best = cands[0], best_wps = 0;
    {
      // seeded synthetic data of this shape: uniform genotypes, alternating classes
      std::vector<uint8_t> G((size_t)snps * samples), y(samples);
      u64 x = 0x9E3779B97F4A7C15ull ^ ((u64)snps << 32 | samples);
      for (auto &g : G) {
        x ^= x << 13;
        x ^= x >> 7;
        x ^= x << 17;
        g = (uint8_t)((x >> 11) % 3);
      }
      for (uint32_t s2 = 0; s2 < samples; ++s2) y[s2] = (uint8_t)(s2 & 1);
      struct Dev {
        void *p = nullptr;
        ~Dev() {
          if (p) (void)hipFree(p);
        }
      } dG, dy, dout, dn, dst;
      HIP_TRY(hipMalloc(&dG.p, G.size()));
      HIP_TRY(hipMalloc(&dy.p, y.size()));
      HIP_TRY(hipMalloc(&dout.p, sizeof(fiuncho_hit) * job.top_n));
      HIP_TRY(hipMalloc(&dn.p, sizeof(uint32_t)));
      HIP_TRY(hipMalloc(&dst.p, sizeof(int32_t)));
      HIP_TRY(hipMemcpy(dG.p, G.data(), G.size(), hipMemcpyHostToDevice));
      HIP_TRY(hipMemcpy(dy.p, y.data(), y.size(), hipMemcpyHostToDevice));
      job.genotypes = static_cast<const uint8_t *>(dG.p);
      job.phenotype = static_cast<const uint8_t *>(dy.p);
      job.out = static_cast<fiuncho_hit *>(dout.p);
      job.n_out = static_cast<uint32_t *>(dn.p);
      job.status = static_cast<int32_t *>(dst.p);
      struct Force {
        ~Force() {
          t_force_kernel = FIUNCHO_KERNEL_AUTO;
          t_force_wps = -1;
        }
      } restore;
      hipEvent_t e0, e1;
      HIP_TRY(hipEventCreate(&e0));
      HIP_TRY(hipEventCreate(&e1));
      float best_ms = 0.f;
      bool timed = false;
      // every kernel, at full occupancy and at 2 and 1 waves per SIMD
      for (int c : cands) {
        for (int wps : {0, 2, 1}) {
          t_force_kernel = c;
          t_force_wps = wps;
          Layout L;
          st = make_layout(&job, 1, false, 1, L);
          if (st) break;
          void *ws = nullptr;
          if (hipMalloc(&ws, L.total) != hipSuccess) {
            st = fail(FIUNCHO_E_DEVICE, "autotune: no device memory for the workspace");
            break;
          }
          st = batch_impl(&job, 1, FIUNCHO_DEVICE_PTRS, ws, L.total, nullptr, 1, nullptr);
          if (st == FIUNCHO_OK && hipEventRecord(e0, nullptr) != hipSuccess) st = FIUNCHO_E_DEVICE;
          for (uint32_t r = 0; st == FIUNCHO_OK && r < std::max<uint32_t>(reps, 1); ++r)
            st = batch_impl(&job, 1, FIUNCHO_DEVICE_PTRS, ws, L.total, nullptr, 1, nullptr);
          float ms = 0.f;
          if (st == FIUNCHO_OK && (hipEventRecord(e1, nullptr) != hipSuccess ||
                                   hipEventSynchronize(e1) != hipSuccess ||
                                   hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
            st = fail(FIUNCHO_E_DEVICE, "autotune: event timing failed");
          int32_t status = 0;
          if (st == FIUNCHO_OK &&
              hipMemcpy(&status, dst.p, sizeof(status), hipMemcpyDeviceToHost) != hipSuccess)
            st = fail(FIUNCHO_E_DEVICE, "autotune: status copy failed");
          const int fst = free_workspace(ws);
          if (st == FIUNCHO_OK) st = fst;
          if (st == FIUNCHO_OK && status != 0) st = fail(status, "autotune: the search failed");
          if (st) break;
          if (!timed || ms < best_ms) {
            best_ms = ms;
            best = c;
            best_wps = wps;
            timed = true;
          }
        }
        if (st) break;
      }
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      if (st) return st;
    }
    {
      std::lock_guard<std::mutex> lk(g_tune_mu);
      g_tuned[shape_key(snps, samples, k)] = TuneEntry{best, best_wps};
    }
    *kernel = best;
    return FIUNCHO_OK;
  } catch (const std::exception &e) {
    return fail(FIUNCHO_E_DEVICE, std::string("internal error: ") + e.what());
  } catch (...) {
    return fail(FIUNCHO_E_DEVICE, "internal error");
  }
}

int fiuncho_score(const uint8_t *genotypes, const uint8_t *phenotype, uint32_t snps,
                  uint32_t samples, int order, const uint64_t *ranks, uint64_t n_ranks,
                  float *est, float *mi32, double *mi) {
  t_err.clear();
  try {
    return explicit_impl(genotypes, phenotype, snps, samples, order, ranks, n_ranks, nullptr, est,
                         mi32, mi);
  } catch (const std::exception &e) {
    return fail(FIUNCHO_E_DEVICE, std::string("internal error: ") + e.what());
  } catch (...) {
    return fail(FIUNCHO_E_DEVICE, "internal error");
  }
}

}  // extern "C"
