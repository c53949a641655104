// internal.hpp -- data structures shared by the host orchestration and the
// gfx950 kernels of libfiuncho.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "fiuncho.h"

namespace fiuncho {

constexpr int kMaxOrder = FIUNCHO_MAX_ORDER;
constexpr int kBinomStride = kMaxOrder + 2;   // C(a, r) for r in [0, 9]
constexpr int kWave = 64;                     // gfx950 wavefront
constexpr int kJBlock = 64;                   // last variants per tile (one per lane)
constexpr int kHistShift = 20;                // survivor histogram bin = key >> 20
constexpr int kHistBins = 1 << (31 - kHistShift);
constexpr uint32_t kSortMax = 8192;           // candidates ordered in one LDS sort
constexpr uint32_t kChunkSort = 4096;         // items per LDS sort of the multi-block sort
constexpr int kScanWaves = 4;                 // waves per workgroup in the scan
constexpr int kOrder2Prefixes = 4;            // first variants per wave at order 2
constexpr int kOrder3Prefixes = 2;            // prefixes per wave, order-3 pair path
constexpr int kPilotEmits = 4;                // score batches a wave emits per tile, at most
constexpr int kMfmaPilotEmits = 16;           // the same for the order-2 matrix-core kernel
constexpr uint32_t kPilotTiles = 256;         // tiles of a job scored by the pilot pass
static_assert(kOrder2Prefixes <= kPilotEmits && kOrder3Prefixes <= kPilotEmits, "pilot slots");

// scan paths of a job
constexpr uint32_t kPathGeneric = 0;          // rows g = 0, 1 of the last variant
constexpr uint32_t kPathPairs = 1;            // order 3, {0,1}^3 cells + pair tables
constexpr int kSelPairs = 31;                 // scan_kernel selector: order-3 pair path only
constexpr int kSel23 = 23;                    // scan_kernel selector: orders 2 and 3 (pair path)
constexpr uint32_t kPathMfma2 = 2;            // order 2 on the matrix cores (mfma_kernel<2>)
constexpr uint32_t kPathTriples = 3;          // order 4, {0,1}^4 cells + triple and pair tables
constexpr uint32_t kPathMfma3 = 4;            // order 3 on the matrix cores (mfma_kernel<3>)
constexpr uint32_t kPathMfmaRows = 5;         // orders 4, 5 on the matrix cores, every prefix row (mfma_rows_kernel)
constexpr int kSelTriples = 41;               // scan_kernel selector: order-4 triple-table path only
constexpr uint32_t kPathMfma4t = 6;           // order 4, {0,1}^4 cells on the matrix cores + triple and pair tables
constexpr uint32_t kPathMfma5q = 7;           // order 5, {0,1}^5 cells on the matrix cores + quad, triple, pair tables
// matrix-core launch groups, in tile-space order: order 2 with int8, FP4 and
// narrow FP4 operands, then order 3 likewise (group = 3 (order - 2) +
// format), then orders 4 and 5 with every prefix row (groups 6, 7), then
// orders 4 and 5 with lower-order tables (groups 8, 9)
constexpr int kMfmaGroups = 10;
// tile counters: the popcount kernel and its pilot, then each matrix-core
// group's counting launch and its pilot
// (the narrow FP4 groups of orders 2 and 3, the groups of orders 4 and 5 and
// the lower-order-table groups run a second kernel, the dual one, over the
// same tiles: 2 more counters each, after the groups')
constexpr int kTileCounters = 2 + 2 * kMfmaGroups + 12;
constexpr int kDualCounters = 2 + 2 * kMfmaGroups;

// state the device writes during one run of a job (cleared at the start)
struct JobState {
  uint32_t m0, m1;            // class sizes
  uint32_t W0, W1;            // 64-bit words per class
  int32_t status;             // FIUNCHO_OK or a negative code
  uint32_t tau_key;           // float bits of the running N-th-best lower bound
  unsigned long long cand_count;  // candidates appended (may exceed the capacity)
  unsigned long long nsurv;       // appended survivors, for histogram refreshes
  uint32_t l1_count;          // candidates above the final running bound
  uint32_t l2_count;          // candidates within the tolerance of the N-th best
  uint32_t kth_key;           // exact N-th largest FP32 key among candidates
  uint32_t flags;             // kFlag* bits
  uint32_t n_sel;             // results left to the multi-block sort (0: none)
  uint32_t pad[3];
};

constexpr uint32_t kFlagCandOverflow = 1u;    // candidate buffer too small
constexpr uint32_t kFlagBound = 4u;           // |estimate - mi| exceeded the stated bound

struct Cand {                 // one appended candidate
  unsigned long long rank;
  uint32_t key;               // float bits of max(est, 0)
  float est;                  // the scan's MI estimate (within fbound of MI)
};

// Exact scores of kept candidate i, written over entry i of the candidate
// buffer (dead once the candidates are compacted into l1)
struct Scored {
  double mi;                  // IEEE double, Eq. 1-3 term by term
  float mi32;                 // compensated single precision
  uint32_t pad;
};
static_assert(sizeof(Scored) <= sizeof(Cand), "scores overlay the candidate buffer");

struct SortItem {             // a result being ordered by (mi desc, rank asc)
  double mi;
  unsigned long long rank;
  uint32_t idx;               // index of the candidate in l1 (and its Scored)
  uint32_t pad;
};

// everything the kernels need about one job; built by the host, uploaded once
struct JobDesc {
  uint32_t n, m, k, top_n;
  uint32_t n_pad;             // n rounded up to a multiple of 64
  uint32_t wcap;              // word stride of the bitsets (>= W0 + W1)
  uint32_t nrows;             // rows of the tile table
  uint32_t flags;             // bit0: outputs are device pointers
  unsigned long long total;   // C(n, k)
  unsigned long long tile_begin;  // first global tile of this job
  unsigned long long tile_count;
  // inputs (device)
  const uint8_t *G;
  const uint8_t *y;
  // derived data (device, workspace)
  uint32_t *idx;              // [m]: sample index of each class position
  unsigned long long *Bv;     // [wcap][n_pad][2] planes g=0,1; variant fastest
  unsigned long long *Bs;     // [n][wcap][4] planes g=0,1,2 and a zero word
  uint32_t *marg;             // [n][3][2] per-variant class marginals
  const float2 *F32;          // (hi, lo) of t ln t for t in [0, m]
  const float *Fh;            // t ln t rounded to float, t in [0, m]
  const uint32_t *Fq;         // round(2^qs t ln t) mod 2^32, t in [0, m]: the fixed-point table of the
                              // FP4 matrix-core kernels of orders 3 to 5 (qs: fixed_shift(m))
  float qscale;               // 2^-qs / m rounded to float
  float fbound;               // bound of |plain single-precision MI - MI|
  const double *P64;          // (t/m) ln(t/m) for t in [0, m]
  const unsigned long long *row_start;  // [nrows + 1] tile offsets
  uint32_t *hist;             // [kHistBins]
  uint32_t *phist;            // [kHistBins] pilot scores (a job with a pilot sample)
  Cand *cand;
  uint32_t cand_cap;
  uint32_t l1_cap;
  Cand *l1;                   // compacted candidates; its first l2_count are kept
  SortItem *sel;              // [sel_cap] the selected results, when more than kSortMax
  SortItem *sel2;             // [sel_cap] second buffer of the multi-block sort (top_n > kSortMax)
  uint32_t sel_cap;
  uint32_t path;              // kPathGeneric or kPathPairs
  JobState *state;
  uint32_t *pairs;            // kPathPairs, kPathTriples: [n][n_pad][g_a 0..1][g_j 0..1][class] counts
  uint4 *pairs4;              // order 3 on the matrix cores with FP4 operands and fewer than 16,384
                              // samples, instead of pairs: [n][n_pad] of [g_a][g_j] -> 4 c0 | 4 c1 << 16
  uint32_t *triples;          // kPathTriples: [pair (a, b)][n_pad][g_a][g_b][g_j][class] counts
  uint4 *triples4;            // kPathMfma4t, kPathMfma5q instead of triples: [pair (a, b)][n_pad][g_a]
                              // of [g_b][g_j] -> 4 c0 | 4 c1 << 16 (fewer than 16,384 samples)
  uint4 *quads4;              // kPathMfma5q: per 4-set a < b < c < j (triples in colex order, each
                              // with j = c + 1 .. n - 1): [g_a][g_b] of [g_c][g_j] -> 4 c0 | 4 c1 << 16
  uint32_t shard_index;       // local tile = launch tile * shard_count + shard_index
  uint32_t shard_count;       // 1 = every tile
  uint32_t pilot_tiles;       // tiles sampled by the pilot pass (0: none)
  uint32_t pilot_slots;       // score slots of the pilot pass (at the start of cand)
  uint32_t fp4;               // kPathMfma2, kPathMfma3: 1 = FP4 operands, 0 = int8
  // outputs
  fiuncho_hit *out;
  uint32_t *n_out;
  int32_t *status_out;
};

struct Globals {
  const unsigned long long *binom;       // [(nmax + 1) * kBinomStride]
  uint32_t nmax;
  uint32_t n_jobs;
  const JobDesc *jobs;
  const unsigned long long *job_tile_start;  // [n_jobs + 1]
  unsigned long long tile_base;    // first global tile of this launch
  unsigned long long total_tiles;  // end of this launch's global tiles
  unsigned long long *tile_counter;
  // pilot pass: an evenly spaced sample of every job's tiles is scored first
  // and only its scores are kept (in the candidate buffer, as float bits), to
  // start the search with a lower bound of the top_n-th best score
  const unsigned long long *job_pilot_start;  // [n_jobs + 1]
  unsigned long long total_pilot_tiles;
  uint32_t pilot;             // 1 in the pilot launch of scan_kernel
  uint32_t lds_f_entries;     // orders 4 and 5 on the matrix cores: f-table entries this launch's
                              // LDS holds (at least m + 1 of every job it counts)
};

// launchers (kernels.hip)
void launch_init(const Globals &g, hipStream_t s);
void launch_pack(const Globals &g, uint32_t max_n_pad, uint32_t max_wcap, hipStream_t s);
void launch_pairs(const Globals &g, uint32_t max_n, hipStream_t s);
void launch_triples(const Globals &g, uint32_t max_n, hipStream_t s);
void launch_scan(const Globals &g, int ksel, int grid, hipStream_t s);
// fmt: 0 int8, 1 FP4, 2 narrow FP4 (jobs of at most mfma_narrow_max_samples()
// samples: table in LDS, counts in 16 bits), 3 dual FP4 (launched over the
// narrow group's tiles; takes the jobs whose class sizes fit 24 bits together)
void launch_mfma(const Globals &g, int order, int fmt, int grid, hipStream_t s);
int mfma_grid_size(int order, int fmt);
uint32_t mfma_narrow_max_samples();
// orders 4 and 5, every prefix genotype row on the matrix cores (FP4
// operands; jobs of at most mfma_narrow_max_samples() samples)
// dual: the kernel that takes the jobs whose class sizes fit 24 bits together
// (both classes in one accumulator); it and the other run over the same tiles
// (g.lds_f_entries: f-table entries of the launch's LDS, at most
// mfma_rows_max_entries(order, dual))
void launch_mfma_rows(const Globals &g, int order, bool dual, int grid, hipStream_t s);
// the most samples a job of this order may have for the dual kernel
uint32_t mfma_dual_max_samples(int order);
uint32_t mfma_rows_max_entries(int order, bool dual);
int mfma_rows_grid_size(int order, bool dual, uint32_t f_entries);
// orders 4 and 5, {0,1}^k cells on the matrix cores (FP4 operands) and the
// other cells from the packed lower-order tables (jobs of fewer than 16,384
// samples); dual as for the rows kernels (jobs of at most
// mfma_sub_dual_max_samples() samples whose class sizes fit 24 bits
// together)
void launch_mfma_sub(const Globals &g, int order, bool dual, int grid, hipStream_t s);
int mfma_sub_grid_size(int order, bool dual);
uint32_t mfma_sub_dual_max_samples();
// the quad tables of the order-5 jobs with lower-order tables
void launch_quads(const Globals &g, uint32_t max_n, hipStream_t s);
// the packed pair tables (pairs4) of the jobs that have them, on the matrix
// cores; the other jobs' pair tables come from launch_pairs
void launch_pairs4(const Globals &g, uint32_t max_n, hipStream_t s);
void launch_select(const Globals &g, uint32_t max_cand_cap, hipStream_t s);
void launch_pilot_select(const Globals &g, uint32_t max_pilot_slots, hipStream_t s);
void launch_rescore(const Globals &g, uint32_t max_k, hipStream_t s);
void launch_finish(const Globals &g, hipStream_t s);
// ordering of more than kSortMax results (jobs with top_n > kSortMax): chunk
// sorts, merge passes up to max_sel items, then the hits
void launch_big_sort(const Globals &g, uint32_t max_sel, hipStream_t s);
void launch_tables(const Globals &g, const unsigned long long *ranks, uint64_t n_ranks,
                   uint32_t *tables, float *est, float *mi32, double *mi, uint32_t k,
                   hipStream_t s);
int scan_grid_size(int ksel);

// records msg as the calling thread's last error (fiuncho_last_error) and
// returns code
int set_error(int code, const char *msg);

}  // namespace fiuncho
