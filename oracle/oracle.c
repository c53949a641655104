/*
 * oracle.c -- plain, slow, obviously-correct CPU reference for the exhaustive
 * mutual-information epistasis scan of Fiuncho (Ponte-Fernandez, Gonzalez-
 * Dominguez, Martin; arXiv 2201.03331).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes or
 * calls this file; only the test-suite, the smoke check and the CPU-baseline leg
 * of the benchmark load it.  It shares no code, header, table or constant with
 * the HIP implementation.
 *
 * What it computes (paper section 3):
 *   - contingency table of a k-combination (section 3.2, Fig. 3): for every
 *     genotype cell x (3^k of them, built from the per-variant genotype rows of
 *     section 3.1 / Fig. 2) and class y, the number of samples in that cell and
 *     class.  Counted sample by sample: x = sum_i g[c_i][s] * 3^(k-1-i), i.e.
 *     the first variant of the combination is the most significant digit, which
 *     is the row order of Fig. 2 (a1 /\ b1, a1 /\ b2, ..., a3 /\ b3).
 *   - mutual information (section 3.3, Eq. 1-3): MI = H(X) + H(Y) - H(X,Y) with
 *     plug-in probabilities count/m, natural logarithm, 0 log 0 = 0.  Evaluated
 *     literally in IEEE double, in a fixed order (cells ascending, then
 *     classes ascending), as
 *        hx  = - sum_x p(x) log p(x),        p(x)   = (t[x][0]+t[x][1]) / m
 *        hy  = - sum_y p(y) log p(y),        p(y)   = m_y / m
 *        hxy = - sum_x sum_y p(x,y) log p(x,y), p(x,y) = t[x][y] / m
 *        mi  = (hx + hy) - hxy
 *     where every "- sum" is a left-to-right running subtraction starting at 0.
 *   - the search (Fig. 1, Algorithm 1 of section 4.2): every k-combination of
 *     the n variants in ascending lexicographic order, scored, and the S
 *     highest kept.  Ties are broken by lexicographic rank, smallest first, so
 *     the kept set is unique: order = (mi descending, rank ascending).
 *
 * Combinations are strictly increasing 0-based variant indices; the last
 * variant runs over every index above the previous one (section 4.2).  The
 * lexicographic rank of a combination is its position in that enumeration.
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fPIC -shared -pthread oracle.c -lm
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_MAX_ORDER 8

enum {
  ORACLE_OK = 0,
  ORACLE_BAD_ARG = -1,
  ORACLE_BAD_GENOTYPE = -3,
  ORACLE_BAD_PHENOTYPE = -4,
  ORACLE_BAD_ORDER = -5,
  ORACLE_BAD_TOPN = -6,
  ORACLE_OVERFLOW = -7,
  ORACLE_NOMEM = -10,
};

/* ---------------------------------------------------------------------------
 * Binomial coefficients and lexicographic ranks (section 4.1 counts the
 * C(n,k) combinations of each order; Tables 2-7 print them).
 * ------------------------------------------------------------------------- */

/* C(n, k) exactly, or UINT64_MAX when it does not fit in 64 bits. */
uint64_t oracle_binom(uint64_t n, uint64_t k) {
  if (k > n) return 0;
  if (k > n - k) k = n - k;
  unsigned __int128 r = 1;
  for (uint64_t i = 1; i <= k; ++i) {
    /* r * (n - k + i) / i is exact at every step (r = C(n-k+i-1, i-1)). */
    r = r * (unsigned __int128)(n - k + i);
    r = r / i;
    if (r > (unsigned __int128)UINT64_MAX) return UINT64_MAX;
  }
  return (uint64_t)r;
}

/* Position of the ascending combination c[0..k-1] of {0..n-1} in
 * lexicographic order: for each position i, every combination that agrees on
 * c[0..i-1] and has a smaller value v at position i comes first, and there are
 * C(n-1-v, k-1-i) of them for each such v. */
uint64_t oracle_rank(uint32_t n, int k, const uint32_t *c) {
  uint64_t r = 0;
  int64_t prev = -1;
  for (int i = 0; i < k; ++i) {
    for (int64_t v = prev + 1; v < (int64_t)c[i]; ++v)
      r += oracle_binom((uint64_t)(n - 1 - v), (uint64_t)(k - 1 - i));
    prev = c[i];
  }
  return r;
}

/* Inverse of oracle_rank: walk the same counts greedily. */
void oracle_unrank(uint32_t n, int k, uint64_t rank, uint32_t *c) {
  int64_t v = 0;
  for (int i = 0; i < k; ++i) {
    for (;;) {
      uint64_t below = oracle_binom((uint64_t)(n - 1 - v), (uint64_t)(k - 1 - i));
      if (rank < below) break;
      rank -= below;
      ++v;
    }
    c[i] = (uint32_t)v;
    ++v;
  }
}

/* Next combination in lexicographic order; returns 0 after the last one. */
static int next_combination(uint32_t n, int k, uint32_t *c) {
  int i = k - 1;
  while (i >= 0 && c[i] == n - (uint32_t)k + (uint32_t)i) --i;
  if (i < 0) return 0;
  ++c[i];
  for (int j = i + 1; j < k; ++j) c[j] = c[j - 1] + 1;
  return 1;
}

static uint32_t pow3(int k) {
  uint32_t p = 1;
  for (int i = 0; i < k; ++i) p *= 3;
  return p;
}

/* ---------------------------------------------------------------------------
 * Input validation (genotypes are 0/1/2, the phenotype is case/control).
 * ------------------------------------------------------------------------- */
int oracle_validate(const uint8_t *G, const uint8_t *y, uint32_t n, uint32_t m,
                    int k, uint32_t top_n) {
  if (!G || !y || n == 0 || m == 0) return ORACLE_BAD_ARG;
  for (uint64_t i = 0; i < (uint64_t)n * m; ++i)
    if (G[i] > 2) return ORACLE_BAD_GENOTYPE;
  for (uint32_t s = 0; s < m; ++s)
    if (y[s] > 1) return ORACLE_BAD_PHENOTYPE;
  if (k < 1 || k > ORACLE_MAX_ORDER || (uint32_t)k > n) return ORACLE_BAD_ORDER;
  if (top_n == 0) return ORACLE_BAD_TOPN;
  if (oracle_binom(n, (uint64_t)k) >= ((uint64_t)1 << 63)) return ORACLE_OVERFLOW;
  return ORACLE_OK;
}

/* ---------------------------------------------------------------------------
 * Contingency table (section 3.2): counted one sample at a time.
 * T has 3^k rows of two counts: T[2x + 0] controls, T[2x + 1] cases.
 * ------------------------------------------------------------------------- */
void oracle_table(const uint8_t *G, const uint8_t *y, uint32_t n, uint32_t m,
                  int k, const uint32_t *c, uint32_t *T) {
  (void)n;
  uint32_t cells = pow3(k);
  memset(T, 0, sizeof(uint32_t) * 2 * cells);
  for (uint32_t s = 0; s < m; ++s) {
    uint32_t x = 0;
    for (int i = 0; i < k; ++i) x = 3 * x + G[(uint64_t)c[i] * m + s];
    T[2 * x + y[s]] += 1;
  }
}

/* ---------------------------------------------------------------------------
 * Mutual information (section 3.3, Eq. 1-3), literal form described above.
 * plogp[t] must hold (t/m) * log(t/m) for t in [0, m], with plogp[0] = 0.
 * ------------------------------------------------------------------------- */
static double mi_from_table(const uint32_t *T, uint32_t cells, uint32_t m0,
                            uint32_t m1, const double *plogp) {
  double hx = 0.0, hy = 0.0, hxy = 0.0;
  for (uint32_t x = 0; x < cells; ++x) hx = hx - plogp[T[2 * x] + T[2 * x + 1]];
  hy = hy - plogp[m0];
  hy = hy - plogp[m1];
  for (uint32_t x = 0; x < cells; ++x) {
    hxy = hxy - plogp[T[2 * x]];
    hxy = hxy - plogp[T[2 * x + 1]];
  }
  return (hx + hy) - hxy;
}

static double *make_plogp(uint32_t m) {
  double *t = (double *)malloc(sizeof(double) * ((size_t)m + 1));
  if (!t) return NULL;
  t[0] = 0.0;
  for (uint32_t i = 1; i <= m; ++i) {
    double p = (double)i / (double)m;
    t[i] = p * log(p);
  }
  return t;
}

/* MI of one contingency table (3^k x 2 counts). */
double oracle_mi(const uint32_t *T, int k) {
  uint32_t cells = pow3(k), m0 = 0, m1 = 0;
  for (uint32_t x = 0; x < cells; ++x) {
    m0 += T[2 * x];
    m1 += T[2 * x + 1];
  }
  uint32_t m = m0 + m1;
  if (m == 0) return 0.0;
  double *pl = make_plogp(m);
  if (!pl) return NAN;
  double r = mi_from_table(T, cells, m0, m1, pl);
  free(pl);
  return r;
}

/* ---------------------------------------------------------------------------
 * Scoring of explicitly listed combinations (given by lexicographic rank).
 * mi_out[i] and, if tables_out is not NULL, tables_out[i * 2 * 3^k ...].
 * ------------------------------------------------------------------------- */
int oracle_score_ranks(const uint8_t *G, const uint8_t *y, uint32_t n, uint32_t m,
                       int k, const uint64_t *ranks, uint64_t count,
                       double *mi_out, uint32_t *tables_out) {
  int st = oracle_validate(G, y, n, m, k, 1);
  if (st != ORACLE_OK) return st;
  uint64_t total = oracle_binom(n, (uint64_t)k);
  uint32_t m0 = 0, m1 = 0;
  for (uint32_t s = 0; s < m; ++s) {
    if (y[s]) m1 += 1;
    else m0 += 1;
  }
  uint32_t cells = pow3(k);
  double *pl = make_plogp(m);
  uint32_t *T = (uint32_t *)malloc(sizeof(uint32_t) * 2 * cells);
  if (!pl || !T) {
    free(pl);
    free(T);
    return ORACLE_NOMEM;
  }
  uint32_t c[ORACLE_MAX_ORDER];
  for (uint64_t i = 0; i < count; ++i) {
    if (ranks[i] >= total) {
      free(pl);
      free(T);
      return ORACLE_BAD_ARG;
    }
    oracle_unrank(n, k, ranks[i], c);
    oracle_table(G, y, n, m, k, c, T);
    if (mi_out) mi_out[i] = mi_from_table(T, cells, m0, m1, pl);
    if (tables_out) memcpy(tables_out + i * 2 * cells, T, sizeof(uint32_t) * 2 * cells);
  }
  free(pl);
  free(T);
  return ORACLE_OK;
}

/* ---------------------------------------------------------------------------
 * The search (Fig. 1 / Algorithm 1): every combination of a contiguous range of
 * lexicographic ranks, each scored, the best top_n kept under the total order
 * (mi descending, rank ascending).  Threads take contiguous sub-ranges and keep
 * their own lists, which are merged under the same order at the end, so the
 * result does not depend on the thread count.
 * ------------------------------------------------------------------------- */
typedef struct {
  double mi;
  uint64_t rank;
} entry_t;

/* a comes before b in the output order */
static int better(const entry_t *a, const entry_t *b) {
  if (a->mi != b->mi) return a->mi > b->mi;
  return a->rank < b->rank;
}

/* list holds *len entries, best first, at most cap */
static void keep_best(entry_t *list, uint32_t *len, uint32_t cap, entry_t e) {
  if (*len == cap && !better(&e, &list[cap - 1])) return;
  uint32_t pos = (*len < cap) ? *len : cap - 1;
  while (pos > 0 && better(&e, &list[pos - 1])) {
    list[pos] = list[pos - 1];
    --pos;
  }
  list[pos] = e;
  if (*len < cap) ++*len;
}

typedef struct {
  const uint8_t *G, *y;
  uint32_t n, m, m0, m1, top_n;
  int k;
  uint64_t first, count;
  const double *plogp;
  entry_t *list;
  uint32_t len;
  int status;
} job_t;

static void *scan_worker(void *arg) {
  job_t *J = (job_t *)arg;
  J->len = 0;
  J->status = ORACLE_OK;
  if (J->count == 0) return NULL;
  const uint32_t m = J->m;
  const int k = J->k;
  const uint32_t cells = pow3(k);
  uint32_t *T = (uint32_t *)malloc(sizeof(uint32_t) * 2 * cells);
  /* per-sample cell index of the current (k-1)-prefix: the same per-sample
   * count, with the prefix digits carried over between combinations that
   * share them (section 4.1 reuses the prefix genotype table the same way) */
  uint32_t *pre = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)m);
  if (!T || !pre) {
    free(T);
    free(pre);
    J->status = ORACLE_NOMEM;
    return NULL;
  }
  uint32_t c[ORACLE_MAX_ORDER], pc[ORACLE_MAX_ORDER];
  oracle_unrank(J->n, k, J->first, c);
  int have_prefix = 0;
  uint64_t rank = J->first;
  for (uint64_t it = 0; it < J->count; ++it, ++rank) {
    int same = have_prefix;
    for (int i = 0; same && i < k - 1; ++i) same = (pc[i] == c[i]);
    if (!same) {
      for (uint32_t s = 0; s < m; ++s) {
        uint32_t x = 0;
        for (int i = 0; i < k - 1; ++i) x = 3 * x + J->G[(uint64_t)c[i] * m + s];
        pre[s] = x;
      }
      memcpy(pc, c, sizeof(uint32_t) * (size_t)k);
      have_prefix = 1;
    }
    memset(T, 0, sizeof(uint32_t) * 2 * cells);
    const uint8_t *gl = J->G + (uint64_t)c[k - 1] * m;
    for (uint32_t s = 0; s < m; ++s) T[2 * (3 * pre[s] + gl[s]) + J->y[s]] += 1;
    entry_t e;
    e.mi = mi_from_table(T, cells, J->m0, J->m1, J->plogp);
    e.rank = rank;
    keep_best(J->list, &J->len, J->top_n, e);
    if (it + 1 < J->count) next_combination(J->n, k, c);
  }
  free(T);
  free(pre);
  return NULL;
}

/* Scans ranks [first, first + count).  Writes min(top_n, count) results to
 * out_rank / out_mi (best first) and their number to *n_out.  nthreads <= 0
 * means one thread.  Returns ORACLE_OK or a negative code. */
int oracle_scan_range(const uint8_t *G, const uint8_t *y, uint32_t n, uint32_t m,
                      int k, uint32_t top_n, uint64_t first, uint64_t count,
                      int nthreads, uint64_t *out_rank, double *out_mi,
                      uint32_t *n_out) {
  if (n_out) *n_out = 0;
  int st = oracle_validate(G, y, n, m, k, top_n);
  if (st != ORACLE_OK) return st;
  if (!out_rank || !out_mi || !n_out) return ORACLE_BAD_ARG;
  uint64_t total = oracle_binom(n, (uint64_t)k);
  if (first > total || count > total - first) return ORACLE_BAD_ARG;
  if (nthreads <= 0) nthreads = 1;
  if ((uint64_t)nthreads > count && count > 0) nthreads = (int)count;
  if (count == 0) return ORACLE_OK;

  uint32_t m0 = 0, m1 = 0;
  for (uint32_t s = 0; s < m; ++s) {
    if (y[s]) m1 += 1;
    else m0 += 1;
  }
  double *pl = make_plogp(m);
  job_t *jobs = (job_t *)calloc((size_t)nthreads, sizeof(job_t));
  pthread_t *th = (pthread_t *)calloc((size_t)nthreads, sizeof(pthread_t));
  entry_t *lists = (entry_t *)malloc(sizeof(entry_t) * (size_t)top_n * (size_t)nthreads);
  if (!pl || !jobs || !th || !lists) {
    free(pl);
    free(jobs);
    free(th);
    free(lists);
    return ORACLE_NOMEM;
  }
  uint64_t per = count / (uint64_t)nthreads, extra = count % (uint64_t)nthreads;
  uint64_t at = first;
  for (int t = 0; t < nthreads; ++t) {
    job_t *J = &jobs[t];
    J->G = G;
    J->y = y;
    J->n = n;
    J->m = m;
    J->m0 = m0;
    J->m1 = m1;
    J->k = k;
    J->top_n = top_n;
    J->first = at;
    J->count = per + ((uint64_t)t < extra ? 1 : 0);
    J->plogp = pl;
    J->list = lists + (size_t)t * top_n;
    at += J->count;
  }
  int started = 0;
  for (int t = 0; t < nthreads; ++t) {
    if (pthread_create(&th[t], NULL, scan_worker, &jobs[t]) != 0) break;
    ++started;
  }
  for (int t = 0; t < started; ++t) pthread_join(th[t], NULL);
  for (int t = started; t < nthreads; ++t) scan_worker(&jobs[t]);

  entry_t *merged = (entry_t *)malloc(sizeof(entry_t) * (size_t)top_n);
  uint32_t len = 0;
  int status = ORACLE_OK;
  for (int t = 0; t < nthreads; ++t) {
    if (jobs[t].status != ORACLE_OK) status = jobs[t].status;
    for (uint32_t i = 0; i < jobs[t].len; ++i) keep_best(merged, &len, top_n, jobs[t].list[i]);
  }
  if (status == ORACLE_OK) {
    for (uint32_t i = 0; i < len; ++i) {
      out_rank[i] = merged[i].rank;
      out_mi[i] = merged[i].mi;
    }
    *n_out = len;
  }
  free(merged);
  free(pl);
  free(jobs);
  free(th);
  free(lists);
  return status;
}

/* Whole search: every combination of order k. */
int oracle_scan(const uint8_t *G, const uint8_t *y, uint32_t n, uint32_t m, int k,
                uint32_t top_n, int nthreads, uint64_t *out_rank, double *out_mi,
                uint32_t *n_out) {
  if (n_out) *n_out = 0;
  int st = oracle_validate(G, y, n, m, k, top_n);
  if (st != ORACLE_OK) return st;
  return oracle_scan_range(G, y, n, m, k, top_n, 0, oracle_binom(n, (uint64_t)k),
                           nthreads, out_rank, out_mi, n_out);
}
