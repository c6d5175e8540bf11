/*
 * Multi-threaded CPU baseline for the XCSR multigraph transpose -- test and
 * benchmark infrastructure only (the benchmark's CPU-baseline leg and the
 * tests that pin it against the single-threaded oracle in oracle.c).
 *
 * It is the scan-based parallel transpose the paper names among prior work
 * (Section 1, Wang et al.): the cells are cut into T contiguous chunks of
 * whole rows, each thread counts the columns of its own chunk, a vertical
 * scan over (column, thread) gives every thread its own write cursor per
 * column, and each thread then places its cells in input order. Chunks are in
 * input order and thread t's cursors for a column follow those of threads
 * t' < t, so equal-column cells keep their input order: the result is the
 * stable transpose, identical to the counting sort's. Payload sizes are
 * scanned into the transposed offsets, then every output cell's bytes are
 * copied, threads splitting the output cells.
 *
 * Inputs are assumed valid (the oracle validates); this code checks sizes
 * only. Offsets are 4- or 8-byte as in the library's ABI.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { MGS_OK = 0, MGS_EINVAL = -1, MGS_ENOMEM = -3 };

static inline int64_t rd(const void* a, int ow, int64_t i) {
  return ow == 4 ? (int64_t)((const int32_t*)a)[i] : ((const int64_t*)a)[i];
}
static inline void wr(void* a, int ow, int64_t i, int64_t v) {
  if (ow == 4) ((int32_t*)a)[i] = (int32_t)v; else ((int64_t*)a)[i] = v;
}

typedef struct {
  int64_t n_rows, n_cols, nnz;
  int ow, T;
  const void* row_ptr; const int32_t* col; const void* poff; const uint8_t* payload;
  void* t_row_ptr; int32_t* t_col; void* t_poff; uint8_t* t_payload; uint32_t* perm;
  int64_t* row_lo;   /* T+1 chunk row bounds                          */
  uint32_t* cnt;     /* T x n_cols: counts, then per-thread cursors    */
  int64_t* part;     /* T: partial sums of the column and size scans   */
  pthread_barrier_t bar;
  pthread_mutex_t mu;  /* start gate: workers wait until the thread count is final */
  pthread_cond_t cv;
  int go;              /* 1 = run, -1 = leave without work */
} Job;

typedef struct { Job* j; int t; } Arg;

static void range_of(int64_t n, int T, int t, int64_t* lo, int64_t* hi) {
  *lo = n * t / T;
  *hi = n * (t + 1) / T;
}

/* Exclusive scan of a[0..n) (width ow) in place by T threads; the total
 * goes to a[n] (written by the last thread). */
static void scan_exclusive(Job* j, int t, void* a, int64_t n) {
  int64_t lo, hi, s = 0;
  range_of(n, j->T, t, &lo, &hi);
  for (int64_t i = lo; i < hi; ++i) s += rd(a, j->ow, i);
  j->part[t] = s;
  pthread_barrier_wait(&j->bar);
  int64_t base = 0;
  for (int q = 0; q < t; ++q) base += j->part[q];
  for (int64_t i = lo; i < hi; ++i) {
    int64_t v = rd(a, j->ow, i);
    wr(a, j->ow, i, base);
    base += v;
  }
  if (t == j->T - 1) wr(a, j->ow, n, base);
  pthread_barrier_wait(&j->bar);
}

static void* worker(void* p) {
  Arg* g = (Arg*)p;
  Job* j = g->j;
  if (g->t) {
    pthread_mutex_lock(&j->mu);
    while (!j->go) pthread_cond_wait(&j->cv, &j->mu);
    const int go = j->go;
    pthread_mutex_unlock(&j->mu);
    if (go < 0) return NULL;
  }
  const int t = g->t, T = j->T, ow = j->ow;
  uint32_t* my = j->cnt + (size_t)t * (size_t)j->n_cols;
  const int64_t r0 = j->row_lo[t], r1 = j->row_lo[t + 1];
  const int64_t k0 = rd(j->row_ptr, ow, r0), k1 = rd(j->row_ptr, ow, r1);

  /* 1. per-thread column counts */
  memset(my, 0, (size_t)j->n_cols * sizeof(uint32_t));
  for (int64_t k = k0; k < k1; ++k) my[j->col[k]]++;
  pthread_barrier_wait(&j->bar);

  /* 2. vertical scan: per-thread cursors relative to the column start, and
   *    the column degrees into t_row_ptr */
  int64_t c0, c1;
  range_of(j->n_cols, T, t, &c0, &c1);
  for (int64_t c = c0; c < c1; ++c) {
    uint32_t s = 0;
    for (int q = 0; q < T; ++q) {
      uint32_t* e = j->cnt + (size_t)q * (size_t)j->n_cols + c;
      uint32_t v = *e;
      *e = s;
      s += v;
    }
    wr(j->t_row_ptr, ow, c, (int64_t)s);
  }
  pthread_barrier_wait(&j->bar);
  scan_exclusive(j, t, j->t_row_ptr, j->n_cols);

  /* 3. place the chunk's cells in input order; sizes go where the offsets
   *    will be */
  for (int64_t i = r0; i < r1; ++i) {
    const int64_t a = rd(j->row_ptr, ow, i), b = rd(j->row_ptr, ow, i + 1);
    for (int64_t k = a; k < b; ++k) {
      const int32_t c = j->col[k];
      const int64_t pos = rd(j->t_row_ptr, ow, c) + (int64_t)my[c]++;
      j->t_col[pos] = (int32_t)i;
      j->perm[pos] = (uint32_t)k;
      wr(j->t_poff, ow, pos, rd(j->poff, ow, k + 1) - rd(j->poff, ow, k));
    }
  }
  pthread_barrier_wait(&j->bar);
  scan_exclusive(j, t, j->t_poff, j->nnz);

  /* 4. payload bytes, output cells split evenly */
  int64_t p0, p1;
  range_of(j->nnz, T, t, &p0, &p1);
  for (int64_t p = p0; p < p1; ++p) {
    const int64_t k = j->perm[p];
    const int64_t src = rd(j->poff, ow, k), n = rd(j->poff, ow, k + 1) - src;
    if (n) memcpy(j->t_payload + rd(j->t_poff, ow, p), j->payload + src, (size_t)n);
  }
  return NULL;
}

int mgs_transpose(int64_t n_rows, int64_t n_cols, int32_t ow, const void* row_ptr,
                  const int32_t* col, const void* payload_off, const uint8_t* payload,
                  void* t_row_ptr, int32_t* t_col, void* t_payload_off, uint8_t* t_payload,
                  uint32_t* perm, int32_t threads) {
  if (n_rows < 0 || n_cols < 0 || (ow != 4 && ow != 8) || threads < 1 || threads > 1024 ||
      !row_ptr || !t_row_ptr || !t_payload_off)
    return MGS_EINVAL;
  Job j;
  memset(&j, 0, sizeof j);
  j.n_rows = n_rows; j.n_cols = n_cols; j.ow = ow;
  j.nnz = rd(row_ptr, ow, n_rows);
  if (j.nnz < 0 || j.nnz > (int64_t)UINT32_MAX) return MGS_EINVAL;
  j.T = threads;
  j.row_ptr = row_ptr; j.col = col; j.poff = payload_off; j.payload = payload;
  j.t_row_ptr = t_row_ptr; j.t_col = t_col; j.t_poff = t_payload_off; j.t_payload = t_payload;
  uint32_t* own_perm = NULL;
  if (!perm && j.nnz) {
    own_perm = (uint32_t*)malloc((size_t)j.nnz * sizeof(uint32_t));
    if (!own_perm) return MGS_ENOMEM;
  }
  j.perm = perm ? perm : own_perm;
  j.row_lo = (int64_t*)malloc(sizeof(int64_t) * (size_t)(threads + 1));
  j.part = (int64_t*)malloc(sizeof(int64_t) * (size_t)threads);
  j.cnt = (uint32_t*)malloc((size_t)threads * (size_t)(n_cols ? n_cols : 1) * sizeof(uint32_t));
  Arg* args = (Arg*)malloc(sizeof(Arg) * (size_t)threads);
  pthread_t* th = (pthread_t*)malloc(sizeof(pthread_t) * (size_t)threads);
  int st = MGS_OK, started = 0;
  if (!j.row_lo || !j.part || !j.cnt || !args || !th) { st = MGS_ENOMEM; goto out; }
  pthread_mutex_init(&j.mu, NULL);
  pthread_cond_init(&j.cv, NULL);
  /* start the helpers first; the work is split over however many started */
  for (int t = 1; t < threads; ++t) {
    args[t].j = &j; args[t].t = t;
    if (pthread_create(&th[t], NULL, worker, &args[t])) break;
    ++started;
  }
  j.T = started + 1;
  args[0].j = &j; args[0].t = 0;
  /* chunk t starts at the first row whose start is at or past t*nnz/T cells */
  j.row_lo[0] = 0;
  for (int t = 1; t < j.T; ++t) {
    const int64_t want = j.nnz * t / j.T;
    int64_t lo = j.row_lo[t - 1], hi = n_rows;
    while (lo < hi) {
      const int64_t mid = lo + (hi - lo) / 2;
      if (rd(row_ptr, ow, mid) < want) lo = mid + 1; else hi = mid;
    }
    j.row_lo[t] = lo;
  }
  j.row_lo[j.T] = n_rows;
  const int bar_ok = pthread_barrier_init(&j.bar, NULL, (unsigned)j.T) == 0;
  pthread_mutex_lock(&j.mu);
  j.go = bar_ok ? 1 : -1;
  pthread_cond_broadcast(&j.cv);
  pthread_mutex_unlock(&j.mu);
  if (bar_ok) worker(&args[0]); else st = MGS_ENOMEM;
  for (int t = 1; t <= started; ++t) pthread_join(th[t], NULL);
  if (bar_ok) pthread_barrier_destroy(&j.bar);
  pthread_cond_destroy(&j.cv);
  pthread_mutex_destroy(&j.mu);
out:
  free(th); free(args); free(j.cnt); free(j.part); free(j.row_lo); free(own_perm);
  return st;
}
