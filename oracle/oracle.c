/*
 * CPU ORACLE -- test infrastructure only.
 *
 * A plain, slow, single-threaded transpose of a row-distributed XCSR multigraph,
 * written from the paper's definitions so that a reader can check it by eye.
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg use
 * it; the GPU library never links, loads or calls it, and the two share no code.
 *
 * What it computes (Magalhaes & Schurmann, "Efficient Distributed Transposition
 * of Large-Scale Multigraphs and High-Cardinality Sparse Matrices"):
 *
 *  - Section 2, definition of the transpose: M^T_ij = M_ji, i.e. every edge
 *    {i, j, e} becomes {j, i, e} with its information e unchanged. In XCSR form
 *    (Section 2, the cell_counts extension) e is the cell's whole value list,
 *    carried here as an opaque byte string.
 *  - Multigraph cells: a row may hold several cells with the same column. They
 *    are kept, each with its own payload, in their original order (the output
 *    is ordered by column, then by original cell position; with canonical rows
 *    this is the reorder of received cells that ends Section 3 / Fig. 6).
 *  - Section 2, sparse transpose step 1 and Section 3 rank intervals: rank
 *    (partition) r owns rows [bounds[r], bounds[r+1]) with 0-based ranks; as the
 *    matrix is square and the vertex set is unchanged by the transpose, the
 *    same intervals split the output rows (= input columns).
 *  - Section 2, sparse transpose step 2: the dense R x R matrix of cells each
 *    rank sends to each rank, X[src][dst]; Section 3 / Fig. 6: the matching
 *    R x R matrix of value (byte) counts, B[src][dst]; their Alltoall transposes
 *    are the receive counts, and exclusive scans give Alltoallv displacements.
 *
 * The construction is Gustavson's counting-sort ("permuted") transposition,
 * which the paper cites among the prior sparse transposes: count the cells of
 * every column, take the exclusive prefix sum as the transposed row offsets,
 * then visit the input in row order and drop each cell into the next free slot
 * of its column. Visiting in input order is what keeps equal cells stable.
 *
 * Parity pins: brute-force sorting on tiny inputs, scipy's CSR->CSC on mid-size
 * ones, closed forms, involution and degree invariants, and a rank-by-rank
 * simulation of the paper's staged algorithm (see tests/).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

static int64_t ld_off(const void* a, int ow, int64_t i) {
  return ow == 4 ? (int64_t)((const int32_t*)a)[i] : ((const int64_t*)a)[i];
}
static void st_off(void* a, int ow, int64_t i, int64_t v) {
  if (ow == 4) ((int32_t*)a)[i] = (int32_t)v;
  else ((int64_t*)a)[i] = v;
}

/* Partition owning vertex v: the last r with bounds[r] <= v (upper_bound - 1). */
static int32_t owner(const int64_t* bounds, int32_t R, int64_t v) {
  int32_t lo = 0, hi = R; /* answer in [lo, hi) */
  while (hi - lo > 1) {
    int32_t mid = lo + (hi - lo) / 2;
    if (bounds[mid] <= v) lo = mid; else hi = mid;
  }
  return lo;
}

int mgo_validate(int64_t n_rows, int64_t n_cols, int32_t ow, const void* row_ptr,
                 const int32_t* col, const void* payload_off, int32_t R, const int64_t* bounds) {
  if (n_rows < 0 || n_cols < 0 || (ow != 4 && ow != 8)) return MGO_EINVAL;
  if (!row_ptr || !payload_off) return MGO_EINVAL;
  if (ld_off(row_ptr, ow, 0) != 0) return MGO_ERANGE;
  for (int64_t i = 0; i < n_rows; ++i)
    if (ld_off(row_ptr, ow, i + 1) < ld_off(row_ptr, ow, i)) return MGO_ERANGE;
  const int64_t nnz = ld_off(row_ptr, ow, n_rows);
  if (nnz > 0 && !col) return MGO_EINVAL;
  if (nnz >= ((int64_t)1 << 32)) return MGO_EUNSUPPORTED;
  for (int64_t k = 0; k < nnz; ++k)
    if (col[k] < 0 || (int64_t)col[k] >= n_cols) return MGO_ERANGE;
  if (ld_off(payload_off, ow, 0) != 0) return MGO_ERANGE;
  for (int64_t k = 0; k < nnz; ++k)
    if (ld_off(payload_off, ow, k + 1) < ld_off(payload_off, ow, k)) return MGO_ERANGE;
  if (R >= 1) {
    if (!bounds) return MGO_EINVAL;
    if (R > 1 && n_rows != n_cols) return MGO_EINVAL; /* square: output reuses the intervals */
    if (bounds[0] != 0 || bounds[R] != n_rows) return MGO_EINVAL;
    for (int32_t r = 0; r < R; ++r)
      if (bounds[r + 1] < bounds[r]) return MGO_EINVAL;
  }
  return MGO_OK;
}

int mgo_transpose(int64_t n_rows, int64_t n_cols, int32_t ow, const void* row_ptr,
                  const int32_t* col, const void* payload_off, const uint8_t* payload,
                  void* t_row_ptr, int32_t* t_col, void* t_payload_off, uint8_t* t_payload,
                  uint32_t* perm) {
  int st = mgo_validate(n_rows, n_cols, ow, row_ptr, col, payload_off, 0, NULL);
  if (st != MGO_OK) return st;
  const int64_t nnz = ld_off(row_ptr, ow, n_rows);

  /* 1. cells per column; exclusive scan = transposed row offsets. */
  int64_t* next = (int64_t*)calloc((size_t)n_cols + 1, sizeof(int64_t));
  if (!next) return MGO_ENOMEM;
  for (int64_t k = 0; k < nnz; ++k) next[col[k] + 1] += 1;
  for (int64_t c = 0; c < n_cols; ++c) next[c + 1] += next[c];
  for (int64_t c = 0; c <= n_cols; ++c) st_off(t_row_ptr, ow, c, next[c]);

  /* 2. visit rows in order, cells in order: cell k of row i goes to the next
   *    free slot of column col[k]; it becomes cell (col[k], i) of the transpose. */
  uint32_t* p_of = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)(nnz ? nnz : 1));
  if (!p_of) { free(next); return MGO_ENOMEM; }
  for (int64_t i = 0; i < n_rows; ++i) {
    for (int64_t k = ld_off(row_ptr, ow, i); k < ld_off(row_ptr, ow, i + 1); ++k) {
      int64_t p = next[col[k]]++;
      t_col[p] = (int32_t)i;
      p_of[p] = (uint32_t)k;
    }
  }

  /* 3. each cell's value list travels with it: sizes in output order, their
   *    exclusive scan, then one byte copy per cell. */
  int64_t acc = 0;
  for (int64_t p = 0; p < nnz; ++p) {
    const int64_t k = p_of[p];
    const int64_t src = ld_off(payload_off, ow, k);
    const int64_t sz = ld_off(payload_off, ow, k + 1) - src;
    st_off(t_payload_off, ow, p, acc);
    if (sz > 0) memcpy(t_payload + acc, payload + src, (size_t)sz);
    acc += sz;
  }
  st_off(t_payload_off, ow, nnz, acc);
  if (perm) for (int64_t p = 0; p < nnz; ++p) perm[p] = p_of[p];
  free(p_of);
  free(next);
  return MGO_OK;
}

int mgo_partition_counts(int64_t n_rows, int64_t n_cols, int32_t ow, const void* row_ptr,
                         const int32_t* col, const void* payload_off, int32_t R,
                         const int64_t* bounds, int64_t* xfer_cells, int64_t* xfer_bytes,
                         int64_t* part_cell_off, int64_t* part_byte_off, int64_t* sdispls,
                         int64_t* rdispls) {
  if (R < 1) return MGO_EINVAL;
  int st = mgo_validate(n_rows, n_cols, ow, row_ptr, col, payload_off, R, bounds);
  if (st != MGO_OK) return st;
  memset(xfer_cells, 0, sizeof(int64_t) * (size_t)R * (size_t)R);
  memset(xfer_bytes, 0, sizeof(int64_t) * (size_t)R * (size_t)R);
  /* Section 2 step 2: rank src counts what it sends to each rank dst (the owner
   * of the cell's column); Section 3 / Fig. 6: the same for value bytes. */
  for (int64_t i = 0; i < n_rows; ++i) {
    const int32_t src = owner(bounds, R, i);
    for (int64_t k = ld_off(row_ptr, ow, i); k < ld_off(row_ptr, ow, i + 1); ++k) {
      const int32_t dst = owner(bounds, R, col[k]);
      const int64_t sz = ld_off(payload_off, ow, k + 1) - ld_off(payload_off, ow, k);
      xfer_cells[(int64_t)src * R + dst] += 1;
      xfer_bytes[(int64_t)src * R + dst] += sz;
    }
  }
  /* Output partition s holds every cell received by rank s: its offset is the
   * sum over all earlier destinations of everything sent to them. */
  int64_t cells = 0, bytes = 0;
  for (int32_t s = 0; s < R; ++s) {
    if (part_cell_off) part_cell_off[s] = cells;
    if (part_byte_off) part_byte_off[s] = bytes;
    for (int32_t r = 0; r < R; ++r) {
      cells += xfer_cells[(int64_t)r * R + s];
      bytes += xfer_bytes[(int64_t)r * R + s];
    }
  }
  if (part_cell_off) part_cell_off[R] = cells;
  if (part_byte_off) part_byte_off[R] = bytes;
  /* Alltoallv displacements: send side scans a row of X along destinations;
   * receive side scans a column of X (a row of X^T) along sources. */
  if (sdispls)
    for (int32_t r = 0; r < R; ++r) {
      int64_t a = 0;
      for (int32_t s = 0; s < R; ++s) { sdispls[(int64_t)r * R + s] = a; a += xfer_cells[(int64_t)r * R + s]; }
    }
  if (rdispls)
    for (int32_t s = 0; s < R; ++s) {
      int64_t a = 0;
      for (int32_t r = 0; r < R; ++r) { rdispls[(int64_t)s * R + r] = a; a += xfer_cells[(int64_t)r * R + s]; }
    }
  return MGO_OK;
}

int mgo_transpose_columns(int64_t n_rows, int64_t n_cols, int32_t ow, const void* row_ptr,
                          const int32_t* col, const void* payload_off, const uint8_t* payload,
                          int64_t c_lo, int64_t c_hi, int64_t* t_row_ptr_slice,
                          int32_t* t_col_slice, int64_t* t_payload_off_slice,
                          uint8_t* t_payload_slice, uint32_t* perm_slice, int64_t* cells_out,
                          int64_t* bytes_out) {
  /* The transpose restricted to output rows (input columns) [c_lo, c_hi), with
   * offsets relative to the slice start. Same construction as mgo_transpose;
   * cells outside the range are skipped. Lets large outputs be checked slice by
   * slice without holding a second full copy. Pass NULL outputs to only size. */
  if (c_lo < 0 || c_hi < c_lo || c_hi > n_cols || n_rows < 0 || (ow != 4 && ow != 8))
    return MGO_EINVAL;
  const int64_t nnz = ld_off(row_ptr, ow, n_rows);
  const int64_t w = c_hi - c_lo;
  int64_t* next = (int64_t*)calloc((size_t)w + 1, sizeof(int64_t));
  int64_t* nbytes = (int64_t*)calloc((size_t)w + 1, sizeof(int64_t));
  if (!next || !nbytes) { free(next); free(nbytes); return MGO_ENOMEM; }
  for (int64_t k = 0; k < nnz; ++k) {
    const int64_t c = col[k];
    if (c < c_lo || c >= c_hi) continue;
    next[c - c_lo + 1] += 1;
    nbytes[c - c_lo + 1] += ld_off(payload_off, ow, k + 1) - ld_off(payload_off, ow, k);
  }
  for (int64_t c = 0; c < w; ++c) { next[c + 1] += next[c]; nbytes[c + 1] += nbytes[c]; }
  if (cells_out) *cells_out = next[w];
  if (bytes_out) *bytes_out = nbytes[w];
  if (t_row_ptr_slice)
    for (int64_t c = 0; c <= w; ++c) t_row_ptr_slice[c] = next[c];
  if (t_col_slice) {
    for (int64_t i = 0; i < n_rows; ++i) {
      for (int64_t k = ld_off(row_ptr, ow, i); k < ld_off(row_ptr, ow, i + 1); ++k) {
        const int64_t c = col[k];
        if (c < c_lo || c >= c_hi) continue;
        const int64_t p = next[c - c_lo]++;
        const int64_t src = ld_off(payload_off, ow, k);
        const int64_t sz = ld_off(payload_off, ow, k + 1) - src;
        const int64_t dst = nbytes[c - c_lo];
        nbytes[c - c_lo] += sz;
        t_col_slice[p] = (int32_t)i;
        if (perm_slice) perm_slice[p] = (uint32_t)k;
        if (t_payload_off_slice) t_payload_off_slice[p] = dst;
        if (t_payload_slice && sz > 0) memcpy(t_payload_slice + dst, payload + src, (size_t)sz);
      }
    }
  }
  free(next);
  free(nbytes);
  return MGO_OK;
}
