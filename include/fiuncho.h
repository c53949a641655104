/*
 * fiuncho.h -- C ABI of libfiuncho.so, an MI355X (gfx950) implementation of the
 * exhaustive mutual-information epistasis scan described in
 *   C. Ponte-Fernandez, J. Gonzalez-Dominguez, M. J. Martin,
 *   "Fiuncho: a program for any-order epistasis detection in CPU clusters",
 *   arXiv 2201.03331.
 *
 * Problem (section 4, first paragraph; Algorithm 1): given genotypes of n
 * variants for m samples split into cases and controls, test every combination
 * of `order` variants for association with the class and report the best.
 *   - genotype tables / contingency tables: section 3.1 (Fig. 2) and 3.2 (Fig. 3);
 *   - association score: mutual information, section 3.3 (Eq. 1-3), in nats;
 *   - result: the `top_n` best combinations (Algorithm 1's output list of S).
 *
 * Conventions shared by every entry point
 *   - genotypes: uint8, row-major [snps][samples], values 0, 1, 2 (number of
 *     minor alleles); any other value is an error (no missing-data code).
 *   - phenotype: uint8 [samples], 0 = control, 1 = case; anything else is an error.
 *   - a combination is a strictly increasing list of 0-based variant indices;
 *     its rank is its position in lexicographic order among all C(snps, order)
 *     combinations (the enumeration order of Algorithm 1).
 *   - contingency table of a combination: 3^order cells x 2 classes, uint32,
 *     laid out [cell][class]; cell = sum_i g_i * 3^(order-1-i), so the first
 *     (lowest-index) variant is the most significant digit -- the row order of
 *     Fig. 2/3.  Class index = phenotype value (Fig. 3 prints cases first).
 *   - results are ordered by (mi descending, rank ascending); this total order
 *     makes the kept set unique when scores tie.
 *   - every call returns FIUNCHO_OK (0) or a negative FIUNCHO_E_* code;
 *     fiuncho_last_error() then describes the failure.  No C++ exception
 *     crosses the ABI.  On error *n_out is set to 0 and `out` is not written.
 *   - the caller owns every buffer; the library keeps no pointer after a call
 *     returns (plain calls) or after the stream has finished the call's work
 *     (asynchronous batch calls).
 *   - the library works on the calling thread's current HIP device.
 */
#ifndef FIUNCHO_H
#define FIUNCHO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FIUNCHO_MAX_ORDER 8

enum {
  FIUNCHO_OK = 0,
  FIUNCHO_E_NULL = -1,      /* a required pointer is NULL */
  FIUNCHO_E_SHAPE = -2,     /* snps == 0, samples == 0 or samples >= 2^24 */
  FIUNCHO_E_GENOTYPE = -3,  /* a genotype value is not 0, 1 or 2 */
  FIUNCHO_E_PHENOTYPE = -4, /* a phenotype value is not 0 or 1 */
  FIUNCHO_E_ORDER = -5,     /* order < 1, order > 8 or order > snps */
  FIUNCHO_E_TOPN = -6,      /* top_n == 0 or top_n > FIUNCHO_MAX_TOPN */
  FIUNCHO_E_OVERFLOW = -7,  /* C(snps, order) >= 2^63 */
  FIUNCHO_E_WORKSPACE = -8, /* workspace too small, or (batched calls) more
                               candidates than the candidate buffer holds;
                               fiuncho_scan enlarges its buffer and retries */
  FIUNCHO_E_DEVICE = -9,    /* a HIP runtime error or no usable gfx950 device */
  FIUNCHO_E_INTERNAL = -10, /* a self-check failed: the counting kernel's
                               estimate of a rescored combination was
                               farther from its exact MI than twice
                               fiuncho_estimate_bound (never expected; the
                               result is withheld) */
  FIUNCHO_E_IO = -11        /* a file could not be opened, read or written */
};

/* Largest supported top_n.  The device workspace grows with it: the
 * candidate buffers hold about 32 * min(C(snps, order), max(2^20, 256 top_n))
 * bytes and the results 64 + 48 bytes per result. */
#define FIUNCHO_MAX_TOPN (1u << 24)

/* One reported combination (64 bytes). */
typedef struct {
  uint32_t snp[FIUNCHO_MAX_ORDER]; /* ascending variant indices; unused = UINT32_MAX */
  uint64_t rank;                   /* lexicographic rank in [0, C(snps, order)) */
  double mi;                       /* mutual information, IEEE double, nats */
  float mi32;                      /* compensated single-precision MI of the exact table */
  float rel_err;                   /* |mi32 - mi| / mi, |mi32 - mi| when mi == 0 */
  float est;                       /* the MI estimate the counting kernel
                                      computed from its own counts, the score the
                                      search filtered on (single precision, or a
                                      32-bit fixed-point sum in the FP4
                                      matrix-core kernels of orders 3 to 5);
                                      within fiuncho_estimate_bound(order,
                                      samples) of mi (0 for a dataset with an
                                      empty class) */
  uint32_t reserved;               /* 0 */
} fiuncho_hit;

/*
 * fiuncho_estimate_bound -- bound of |est - mi| for any combination of this
 * order in a dataset of this many samples (section 3.3, Eq. 1-3 evaluated in
 * single precision as m MI = [f(m) - f(m0) - f(m1)] + sum over cells of
 * [f(n0) + f(n1) - f(n0 + n1)], f(t) = t ln t from a float table):
 * u (6 ln m + (3^order + 4) ln 2), u = 2^-24.  The search keeps every
 * combination whose estimate lies within 4 times this bound of the top_n-th
 * best estimate, so none of the exact best top_n is lost.  The fixed-point
 * form of the same sum (FP4 matrix-core kernels, orders 3 to 5) errs by less
 * for every sample count.  Returns a negative value for an order outside
 * [1, 8] or samples == 0.
 */
double fiuncho_estimate_bound(int order, uint32_t samples);

/*
 * fiuncho_scan -- the whole exhaustive search on one dataset (Fig. 1,
 * Algorithm 1), synchronous.
 *   genotypes  host pointer, [snps][samples] uint8 (see conventions)
 *   phenotype  host pointer, [samples] uint8
 *   order      interaction order k, 1..8
 *   top_n      how many combinations to report, 1..FIUNCHO_MAX_TOPN (any number
 *              of exact ties at the cut-off is resolved by rank)
 *   out        host array of at least top_n hits, written best first
 *   n_out      receives min(top_n, C(snps, order))
 * All inputs are validated on the host before any device work.  A dataset with
 * an empty class has MI = 0 for every combination; the result is then the
 * first top_n combinations by rank.
 */
int fiuncho_scan(const uint8_t *genotypes, const uint8_t *phenotype,
                 uint32_t snps, uint32_t samples, int order, uint32_t top_n,
                 fiuncho_hit *out, uint32_t *n_out);

/* One dataset of a batched call. */
typedef struct {
  const uint8_t *genotypes; /* [snps][samples]; device pointer with FIUNCHO_DEVICE_PTRS */
  const uint8_t *phenotype; /* [samples]; device pointer with FIUNCHO_DEVICE_PTRS */
  uint32_t snps, samples;
  int order;
  uint32_t top_n;
  fiuncho_hit *out;   /* >= top_n hits; device pointer with FIUNCHO_DEVICE_PTRS */
  uint32_t *n_out;    /* device pointer with FIUNCHO_DEVICE_PTRS */
  int32_t *status;    /* optional (may be NULL): per-job FIUNCHO_* code; device
                         pointer with FIUNCHO_DEVICE_PTRS */
  uint32_t shard_index; /* with shard_count > 1: search only this shard's work   */
  uint32_t shard_count; /* tiles (one GPU's share of a search split across
                           shard_count GPUs): the job's tiles are dealt in blocks of
                           shard_count consecutive tiles, and in block q shard s takes
                           the tile at offset (s + q) mod shard_count.  The result is
                           the best top_n of that share, and merging the lists of
                           all shards under the total order gives the full result.
                           With an empty class every MI is 0 and the share is the
                           ranks congruent to shard_index modulo shard_count.
                           shard_count 0 or 1: the whole search.
                           shard_index >= shard_count: FIUNCHO_E_SHAPE */
} fiuncho_job;

/* Flags of fiuncho_scan_batch. */
#define FIUNCHO_DEVICE_PTRS 1u /* all job pointers are device pointers and the
                                  call returns as soon as the work is queued */
#define FIUNCHO_UPLOAD_PLAN 2u /* upload the plan even if this workspace already
                                  holds it (see fiuncho_scan_batch) */

/*
 * fiuncho_workspace_bytes -- device workspace needed by fiuncho_scan_batch for
 * these jobs (bitsets, tables, candidate buffers, plan).  Depends on the
 * shapes (snps, samples, order, top_n) of the jobs and on the kernel each
 * shape is given (fiuncho_get_kernel): ask again after fiuncho_set_kernel or
 * fiuncho_autotune.  Returns 0 for invalid shapes.
 */
size_t fiuncho_workspace_bytes(const fiuncho_job *jobs, uint32_t n_jobs);

/*
 * fiuncho_scan_batch -- many independent searches in one persistent kernel
 * launch (the datasets may differ in size, class split and order).
 *   workspace   device memory of at least fiuncho_workspace_bytes(jobs, n_jobs),
 *               256-byte aligned, owned by the caller; must not be shared by
 *               calls that overlap in time
 *   hip_stream  hipStream_t to queue the work on (NULL = default stream)
 * Without FIUNCHO_DEVICE_PTRS, the inputs are host arrays, validated on the
 * host, and the call returns after the results are in the host arrays.
 * With FIUNCHO_DEVICE_PTRS, inputs and outputs live on the device, genotype and
 * phenotype values are validated by the kernels (an invalid job reports its
 * code through job.status and *n_out = 0), and the call only queues work.  The
 * first call with a given workspace and job set uploads a plan (lookup tables,
 * tile tables) synchronously; later calls with the same workspace and job set
 * queue kernels only, so they can be captured into a HIP graph and replayed.
 * The plan lives in the workspace: if anything else writes that memory, or it
 * is freed and allocated again, between two calls, pass FIUNCHO_UPLOAD_PLAN
 * on the next call.  Returns FIUNCHO_E_WORKSPACE if a plan upload is needed
 * while the stream is being captured.
 */
int fiuncho_scan_batch(const fiuncho_job *jobs, uint32_t n_jobs, uint32_t flags,
                       void *workspace, size_t ws_bytes, void *hip_stream);

/*
 * fiuncho_scan_batch_static -- fiuncho_scan_batch without a caller workspace
 * and without any device allocation, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  The workspace is a static array of
 * FIUNCHO_STATIC_SCRATCH_BYTES in the library's device code: each GPU the
 * library runs on holds one until the process ends, and every call on that
 * GPU shares it.  Calls that overlap in time on one GPU (on different
 * streams or threads) race on it and must not be made.
 *   jobs, n_jobs, flags, hip_stream  as for fiuncho_scan_batch (with
 *               FIUNCHO_DEVICE_PTRS the call only queues work; the first call
 *               for a job set uploads its plan synchronously)
 * Returns FIUNCHO_E_WORKSPACE, before any device work, when
 * fiuncho_workspace_bytes(jobs, n_jobs) (plus the host-input copies without
 * FIUNCHO_DEVICE_PTRS) exceeds FIUNCHO_STATIC_SCRATCH_BYTES.
 */
#define FIUNCHO_STATIC_SCRATCH_BYTES (64u << 20)
int fiuncho_scan_batch_static(const fiuncho_job *jobs, uint32_t n_jobs, uint32_t flags,
                              void *hip_stream);

/*
 * fiuncho_contingency -- contingency tables of explicit combinations
 * (section 3.2, Fig. 3).
 *   genotypes, phenotype  host arrays as in fiuncho_scan
 *   ranks      host array of n_ranks lexicographic ranks, each < C(snps, order)
 *   tables     host array of n_ranks * 3^order * 2 uint32, [rank][cell][class]
 * Synchronous.  The tables are counted from the same bit-packed genotype
 * tables as the search, by the kernel that rescores the search's kept
 * candidates (AND of the cell's rows, one population count per class and
 * cell), not by the search's counting kernels; those are checked through the
 * estimates they return with every hit (fiuncho_hit.est).
 */
int fiuncho_contingency(const uint8_t *genotypes, const uint8_t *phenotype,
                        uint32_t snps, uint32_t samples, int order,
                        const uint64_t *ranks, uint64_t n_ranks, uint32_t *tables);

/*
 * fiuncho_score -- mutual information (section 3.3, Eq. 1-3) of explicit
 * combinations, from the same device tables as the search.
 *   ranks  host array of n_ranks lexicographic ranks, each < C(snps, order)
 *   est    host float[n_ranks] or NULL: the plain single-precision evaluation
 *          the search filters with; |est - mi| is below a bound that
 *          depends only on order and samples
 *   mi32   host float[n_ranks] or NULL: compensated single precision, the
 *          value reported as fiuncho_hit.mi32
 *   mi     host double[n_ranks] or NULL: IEEE double, the value reported as
 *          fiuncho_hit.mi
 * Synchronous; validation and errors as in fiuncho_contingency.
 */
int fiuncho_score(const uint8_t *genotypes, const uint8_t *phenotype, uint32_t snps,
                  uint32_t samples, int order, const uint64_t *ranks, uint64_t n_ranks,
                  float *est, float *mi32, double *mi);

/*
 * fiuncho_shard_counts -- combinations each of `units` processing units gets
 * (host-only; no device work).
 *   scheme 0: the paper's static distribution (section 4.1, Fig. 4): the
 *             (order-1)-prefixes in ascending lexicographic order are dealt
 *             round-robin to the units, and a unit tests every combination
 *             that extends its prefixes;
 *   scheme 1: this library's shards (fiuncho_job.shard_index/shard_count):
 *             the work tiles of the search dealt in rotated blocks (the tiles
 *             depend on the kernel chosen for snps, samples and order).
 *   Errors: FIUNCHO_E_NULL (counts NULL), FIUNCHO_E_SHAPE (units 0, snps 0
 *   or an unknown scheme), FIUNCHO_E_ORDER, FIUNCHO_E_OVERFLOW as for a job.
 *   counts    host array of `units` entries
 * The relative imbalance of Eq. 4 (section 5.1) is
 * 100 * (max counts - C(snps,order)/units) / (C(snps,order)/units).
 */
int fiuncho_shard_counts(uint32_t snps, uint32_t samples, int order, uint32_t units, int scheme,
                         uint64_t *counts);

/*
 * Kernel choice.  Every job shape is searched by one of these counting
 * kernels; the choice is made per (order, bit length of snps, bit length of
 * ceil(samples / 64)) bucket: from a process-wide table filled by
 * fiuncho_set_kernel or fiuncho_autotune, else from a built-in rule measured
 * on MI355X.
 */
#define FIUNCHO_KERNEL_AUTO 0     /* no explicit choice (table entry cleared) */
#define FIUNCHO_KERNEL_POPCOUNT 1 /* AND + popcount of the prefix rows against rows
                                     g = 0, 1 of the last variant (any order) */
#define FIUNCHO_KERNEL_PAIRS 2    /* order 3: only the {0,1}^3 cells counted, the
                                     rest from stored pair tables */
#define FIUNCHO_KERNEL_MFMA 3     /* orders 2 and 3: one-hot int8 contraction on
                                     the matrix cores (order 2: variant x variant;
                                     order 3: prefix pair x variant, the other
                                     cells from pair tables) */
#define FIUNCHO_KERNEL_TRIPLES 4  /* order 4: only the {0,1}^4 cells counted, the
                                     rest from stored triple and pair tables
                                     (64 bytes of device memory per pair and
                                     variant; up to 16 GiB of tables) */
#define FIUNCHO_KERNEL_MFMA_FP4 5 /* orders 2 and 3: the FIUNCHO_KERNEL_MFMA
                                     contraction with FP4 (E2M1) 0/1 operands
                                     and FP32 accumulation (exact: counts stay
                                     below 2^24), 64 samples per instruction;
                                     orders 4 and 5: every genotype row of the
                                     prefix against rows 0, 1 of the last
                                     variant on the matrix cores (jobs of at
                                     most 20,447 samples; larger ones run on
                                     the popcount kernel) */
#define FIUNCHO_KERNEL_MFMA_FP4_TABLES 6 /* orders 4 and 5: the {0,1}^k cells
                                     on the matrix cores (FP4 operands,
                                     {0,1}^(k-1) rows of 4 or 2 prefixes per
                                     operand fragment), the rest by
                                     inclusion-exclusion from packed lower-
                                     order tables: triple and pair tables
                                     (32 bytes per pair and variant, up to
                                     16 GiB) and at order 5 quad tables (64
                                     bytes per 4-set, up to 48 GiB), built on
                                     the device per call;
                                     jobs of fewer than 16,384 samples (larger
                                     ones: order 4 on FIUNCHO_KERNEL_TRIPLES,
                                     order 5 on FIUNCHO_KERNEL_MFMA_FP4) */

/* The kernel a job of this shape would use now (a FIUNCHO_KERNEL_* value),
 * or FIUNCHO_E_ORDER. */
int fiuncho_get_kernel(uint32_t snps, uint32_t samples, int order);

/* Sets (or, with FIUNCHO_KERNEL_AUTO, clears) the table entry of the shape's
 * bucket, with waves_per_simd 0.  FIUNCHO_E_SHAPE if the kernel does not
 * handle the order. */
int fiuncho_set_kernel(uint32_t snps, uint32_t samples, int order, int kernel);

/*
 * The launch configuration of a shape's bucket: its counting kernel and the
 * most waves per SIMD (workgroups of 4 waves per compute unit) the kernel's
 * persistent launch keeps (0: as many as fit in registers and LDS; fewer
 * waves leave each more cache and LDS bandwidth).  A launch that counts jobs
 * of several buckets uses the largest of their limits (none if one has 0).
 *   fiuncho_get_config: the configuration a job of this shape would use now
 *     (FIUNCHO_E_NULL, FIUNCHO_E_ORDER).
 *   fiuncho_set_config: sets the bucket's table entry (kernel
 *     FIUNCHO_KERNEL_AUTO clears it); waves_per_simd in [0, 8], else
 *     FIUNCHO_E_SHAPE; FIUNCHO_E_SHAPE also if the kernel does not handle
 *     the order.
 */
int fiuncho_get_config(uint32_t snps, uint32_t samples, int order, int *kernel, int *waves_per_simd);
int fiuncho_set_config(uint32_t snps, uint32_t samples, int order, int kernel, int waves_per_simd);

/*
 * fiuncho_autotune -- times every kernel that handles this shape, each at full
 * occupancy and at 2 and 1 waves per SIMD, on a seeded synthetic dataset of
 * exactly this shape (balanced classes, top_n 16) on the current device,
 * `reps` timed runs each after one warm-up, records the fastest configuration
 * in the table for the shape's bucket (fiuncho_get_config reads it back) and
 * returns its kernel in *kernel.  Synchronous; allocates and frees its own
 * device memory.
 */
int fiuncho_autotune(uint32_t snps, uint32_t samples, int order, uint32_t reps, int *kernel);

/* Message of the last failed call on this thread ("" if none). */
const char *fiuncho_last_error(void);

/*
 * The input and output stages of the search (Fig. 1: the variants read from
 * a file, the saved combinations written to one).  The paper gives no file
 * format; these read and write plain ASCII text, on the host (no device is
 * needed):
 *   genotype file  one line per variant: the genotype (0, 1 or 2) of every
 *                  sample, in sample order, as digits, either contiguous or
 *                  separated by spaces, tabs or commas; empty lines and lines
 *                  whose first character is '#' are skipped; every variant
 *                  has the same number of samples
 *   phenotype file the class of every sample, 0 (control) or 1 (case), as
 *                  digits separated the same way, on any number of lines
 *   result file    a header line, then one line per hit, tab-separated: rank,
 *                  the order's variant indices, mi (17 significant digits),
 *                  mi32, rel_err, est
 * The library never retains a path or a buffer past the call.
 */

/*
 * fiuncho_read_genotypes -- reads a genotype file.  With genotypes NULL only
 * measures it: *snps and *samples receive its shape.  Otherwise writes the
 * [snps][samples] uint8 matrix (the layout fiuncho_scan takes) to genotypes,
 * which holds capacity bytes.
 * Errors: FIUNCHO_E_NULL (path, snps or samples NULL), FIUNCHO_E_IO (the file
 * cannot be read), FIUNCHO_E_SHAPE (no variant, variants of different
 * lengths, 2^24 samples or more, or capacity < snps * samples),
 * FIUNCHO_E_GENOTYPE (a character other than 0, 1, 2 or a separator; the
 * message names the line).
 */
int fiuncho_read_genotypes(const char *path, uint8_t *genotypes, size_t capacity, uint32_t *snps,
                           uint32_t *samples);

/*
 * fiuncho_read_phenotype -- reads a phenotype file into phenotype (capacity
 * bytes), or with phenotype NULL only counts its samples into *samples.
 * Errors: FIUNCHO_E_NULL (path or samples NULL), FIUNCHO_E_IO,
 * FIUNCHO_E_SHAPE (no sample, 2^24 samples or more, capacity too small),
 * FIUNCHO_E_PHENOTYPE (a character other than 0, 1 or a separator).
 */
int fiuncho_read_phenotype(const char *path, uint8_t *phenotype, size_t capacity, uint32_t *samples);

/*
 * fiuncho_write_hits -- writes n hits (as fiuncho_scan returns them, best
 * first) of the given order to a result file, replacing it.
 * Errors: FIUNCHO_E_NULL (path NULL, or hits NULL with n > 0),
 * FIUNCHO_E_ORDER (order outside [1, 8]), FIUNCHO_E_IO.
 */
int fiuncho_write_hits(const char *path, const fiuncho_hit *hits, uint32_t n, int order);

/* Per-phase device times (milliseconds), averaged over the fiuncho_scan_batch
 * calls made on this thread with profiling enabled since the last
 * fiuncho_get_profile; see fiuncho_set_profiling. */
typedef struct {
  float pack_ms;      /* class partition, bit packing (and pair / triple tables) */
  float pilot_ms;     /* pilot sample: scores of a sample of tiles, starting bound */
  float scan_ms;      /* popcount counting kernel + FP32 estimate + candidate filter */
  float mfma_ms;      /* matrix-core kernels (orders 2 and 3, int8 and FP4) + FP32
                         estimate + candidate filter */
  float select_ms;    /* candidate selection, FP64 rescoring, final order */
  float total_ms;     /* all of the above, first kernel start to last kernel end */
  uint32_t calls;        /* profiled calls averaged */
  uint32_t flags;        /* 4 = a rescored candidate's single-precision estimate was
                            farther from its FP64 MI than the stated bound (last
                            call, first job; never expected) */
  uint64_t combinations; /* combinations the last call tested: C(snps, order) per job,
                            a sharded job's share for a sharded job */
  uint64_t candidates;   /* candidates the scan appended (last call, first job) */
  uint32_t kept;         /* candidates rescored in double precision (last call, first job) */
  uint32_t kernels;      /* bit (1 << FIUNCHO_KERNEL_*) for each kernel the last call used */
} fiuncho_profile;

/* Enable (1) or disable (0) HIP-event timing of the phases of later
 * fiuncho_scan_batch calls on this thread (four events per call, recorded on
 * the call's stream). */
void fiuncho_set_profiling(int enable);

/* Collects (synchronising on their events) and clears the timings of the
 * profiled calls; FIUNCHO_E_NULL when there is none. */
int fiuncho_get_profile(fiuncho_profile *out);

#ifdef __cplusplus
}
#endif

#endif /* FIUNCHO_H */
