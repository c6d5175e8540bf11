/*
 * mgt -- transpose of row-distributed XCSR multigraphs on one MI355X (gfx950).
 *
 * C ABI of libmgt.so. Plain pointers and sizes only; every device buffer is
 * owned by the caller. All launches are asynchronous on the caller's stream.
 *
 * Terms (Magalhaes & Schurmann, arXiv 2012.06012):
 *  - XCSR (Section 2): CSR (row offsets row_ptr, column ids col) plus a value
 *    list per cell. Here a cell's value list is an opaque byte string:
 *    payload[payload_off[k] .. payload_off[k+1]) belongs to cell k. Cells may
 *    repeat a (row, col) pair: a multigraph keeps each edge as its own cell.
 *  - Transpose (Section 2): M^T_ij = M_ji; edge {i, j, e} becomes {j, i, e}.
 *    Output row j lists the input cells whose column is j, ordered by input row
 *    and, for repeated (row, col) cells, in their original order; each cell's
 *    payload moves with it. t_col holds the original row ids. Rows of the
 *    output are therefore always sorted by column; if the input's rows are
 *    sorted by column, transposing twice returns the input exactly (the
 *    paper's involution, Section 3).
 *  - Partitions (ranks, Section 2 step 1; Section 3 row intervals): partition r
 *    owns rows [part_bounds[r], part_bounds[r+1]) with 0-based r. A partitioned
 *    matrix is square and the output's rows (= input columns) are split by the
 *    same bounds. xfer_cells[r*R+s] counts the cells partition r sends to
 *    partition s (the owner of their column; Section 2 step 2), xfer_bytes the
 *    matching payload bytes (Section 3, value counts per recipient, Fig. 6).
 *
 * Sizes and limits: n_rows, n_cols < 2^31 (col ids are int32); nnz < 2^32;
 * payload offsets are 4- or 8-byte signed integers (offset_width), as are
 * row_ptr and the transposed offsets. A single cell's payload must be < 2^32
 * bytes, and any 16,384 consecutive cells must carry < 2^32 payload bytes
 * (checked on the device on every call: *d_status = MGT_EUNSUPPORTED).
 *
 * Errors: functions return an mgt_status. Host-detectable errors (bad
 * descriptor, NULL pointer, workspace too small, unsupported sizes) are
 * returned before anything is launched and leave the outputs untouched.
 * With MGT_VALIDATE, the device also checks the data (row_ptr and payload_off
 * start at 0, never decrease and end at nnz / payload_bytes; every col lies in
 * [0, n_cols)) and writes MGT_ERANGE to *d_status if it does not hold; the
 * remaining stages then skip their work and the outputs are undefined. Without
 * MGT_VALIDATE, invalid data is undefined behaviour. On success *d_status is
 * MGT_OK. d_status may be NULL.
 *
 * Thread safety: a plan's parameters are fixed at creation, and calls from
 * several threads may share a plan (the library serialises the host part of
 * calls on one plan: the descriptor upload through the plan's pinned staging
 * buffer). Calls whose device work may overlap need distinct workspaces.
 */
#ifndef MGT_H
#define MGT_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MGT_OK = 0,
  MGT_EINVAL = -1,       /* bad descriptor, pointer, bounds or argument          */
  MGT_ERANGE = -2,       /* data out of range (device-side check, MGT_VALIDATE)  */
  MGT_ENOMEM = -3,       /* workspace too small / host allocation failed         */
  MGT_EHIP = -4,         /* a HIP runtime call failed                            */
  MGT_EUNSUPPORTED = -5, /* sizes beyond the documented limits                   */
  MGT_ECANCELED = -6     /* batch item skipped because another item failed       */
} mgt_status;

enum {
  MGT_VALIDATE = 1u << 0,     /* device-side data checks, result in *d_status            */
  MGT_EMIT_PERM = 1u << 1,    /* callers will pass perm: perm[p] = input cell of output p */
  MGT_DEBUG_TIMING = 1u << 2, /* record per-stage times (mgt_plan_stage_times)           */
  MGT_FIXED_WIDTH = 1u << 3   /* every cell carries the same number of payload bytes     */
};

/*
 * Fixed-width cells (MGT_FIXED_WIDTH; the homogeneous-value variant of
 * Section 2 and the identical-cell-size case remarked on in Section 3): every
 * cell carries w = payload_bytes / nnz bytes, so cell k's payload is bytes
 * [k*w, (k+1)*w) on both sides and no offsets need to move. payload_bytes
 * must be a multiple of nnz (any value when nnz == 0), else MGT_EINVAL.
 * payload_off may then be NULL (it is never read); t_payload_off may be NULL
 * (it is then not written; when given it receives p*w as usual). For a batch
 * the flag is taken from each item's descriptor.
 */

typedef struct mgt_plan_s* mgt_plan_t;

/* Describes one matrix. For n_parts > 1 the matrix must be square. */
typedef struct {
  int64_t n_rows, n_cols;
  int64_t nnz;             /* = row_ptr[n_rows]                                    */
  int64_t payload_bytes;   /* = payload_off[nnz]                                   */
  int32_t offset_width;    /* 4 or 8: element size of row_ptr, payload_off and the
                              transposed offsets                                    */
  int32_t n_parts;         /* R >= 1 partitions (R <= 1024)                         */
  const int64_t* part_bounds; /* host, R+1 entries: 0 = b[0] <= b[1] <= ... <= b[R]
                              = n_rows; empty partitions allowed; may be NULL when
                              R == 1                                                */
  uint32_t flags;          /* MGT_VALIDATE | MGT_EMIT_PERM | MGT_DEBUG_TIMING |
                              MGT_FIXED_WIDTH                                       */
} mgt_desc;

/*
 * Creates a plan for matrices with this descriptor (sizes and partition bounds
 * are copied). Chooses the digit schedule and tile sizes and reports the
 * device workspace the transpose calls need. Host only; launches nothing.
 */
int mgt_plan(const mgt_desc* desc, mgt_plan_t* out, size_t* workspace_bytes);
int mgt_plan_destroy(mgt_plan_t plan);

/*
 * Plain transpose (Section 2 definition; the partition bounds of the plan, if
 * any, are ignored). Device pointers:
 *   inputs : row_ptr[n_rows+1], col[nnz], payload_off[nnz+1], payload[payload_bytes]
 *   outputs: t_row_ptr[n_cols+1], t_col[nnz], t_payload_off[nnz+1],
 *            t_payload[payload_bytes], perm[nnz] (only with MGT_EMIT_PERM, else NULL)
 * payload / t_payload may be NULL when payload_bytes == 0; with
 * MGT_FIXED_WIDTH payload_off and t_payload_off may be NULL. Outputs must not
 * overlap inputs. workspace: >= the size mgt_plan reported, 256-byte aligned.
 * A call without perm needs no cell index internally and may move less data
 * (the outputs are the same either way).
 */
int mgt_transpose(mgt_plan_t plan, const void* row_ptr, const int32_t* col,
                  const void* payload_off, const uint8_t* payload, void* t_row_ptr,
                  int32_t* t_col, void* t_payload_off, uint8_t* t_payload, uint32_t* perm,
                  void* workspace, size_t workspace_bytes, int32_t* d_status,
                  hipStream_t stream);

/*
 * Partitioned transpose: the paper's distributed transpose with the R ranks as
 * logical partitions of one device (Section 3: local transpose composed with
 * the view swap). Same inputs and outputs as mgt_transpose -- partition s of
 * the result is the slice [part_cell_off[s], part_cell_off[s+1]) of t_col /
 * t_payload_off (bytes [part_byte_off[s], part_byte_off[s+1]) of t_payload) and
 * t_row_ptr[part_bounds[s] .. part_bounds[s+1]] -- plus, in device memory:
 *   xfer_cells[R*R], xfer_bytes[R*R]  row-major [src][dst] (Section 2 step 2,
 *                                     Section 3 value counts)
 *   part_cell_off[R+1], part_byte_off[R+1]
 *   sdispls[R*R]  (may be NULL) send displacement of block src->dst inside
 *                 src's packed send order: exclusive scan of xfer_cells[src][.]
 *   rdispls[R*R]  (may be NULL) [dst][src]: receive displacement of block
 *                 src->dst inside partition dst: exclusive scan of
 *                 xfer_cells[.][dst] over src (Alltoallv displacements)
 */
int mgt_transpose_partitioned(mgt_plan_t plan, const void* row_ptr, const int32_t* col,
                              const void* payload_off, const uint8_t* payload, void* t_row_ptr,
                              int32_t* t_col, void* t_payload_off, uint8_t* t_payload,
                              uint32_t* perm, int64_t* xfer_cells, int64_t* xfer_bytes,
                              int64_t* part_cell_off, int64_t* part_byte_off, int64_t* sdispls,
                              int64_t* rdispls, void* workspace, size_t workspace_bytes,
                              int32_t* d_status, hipStream_t stream);

/*
 * Schedule of a single-matrix plan, for tuning (host only). The transpose is
 * a few stable partition passes over the column bits followed by a per-bucket
 * sort; by default the library picks the fewest passes, then the narrowest
 * finish buckets of about 4,096 cells, and tiles sized for the call.
 *   pass_bits   largest digit of a bits-mode pass, 1..8 (0: default)
 *   finish_bits column bits of a finish bucket, 0..10, exactly (-1: default)
 *   tile_cells  cells per tile: 2048, 4096, 8192 or 16384 (0: default)
 * The number of passes follows (fewest that cover the remaining bits). A
 * setting that would need more than four passes gives MGT_EUNSUPPORTED.
 * *workspace_bytes (may be NULL) receives the workspace the plan now needs:
 * later calls check against it. Results are the same for every schedule;
 * only the time differs. On a batch plan the setting applies to every item of
 * later submits (finish_bits capped by each item's column bits; an item whose
 * schedule would need more than four passes keeps the rule's), the tile size
 * to the whole batch, *workspace_bytes receives the plan's estimate again,
 * and mgt_batch_workspace gives a batch's exact need. View plans give
 * MGT_EINVAL.
 */
int mgt_plan_set_schedule(mgt_plan_t plan, int32_t pass_bits, int32_t finish_bits,
                          int32_t tile_cells, size_t* workspace_bytes);

/* The schedule a call on this single-matrix plan uses (host only): out[0] passes,
 * out[1..4] bits of each pass (partition passes: sub-bits below the
 * partition), out[5] finish bits, out[6] tile cells, out[7] 1 for a
 * partition-mode first pass. partitioned selects mgt_transpose_partitioned. */
int mgt_plan_schedule(mgt_plan_t plan, int32_t partitioned, int32_t* out);

/* ------------------------------------------------------------------ batches */

/*
 * The two halves of the distributed transpose on their own (Section 3:
 * Transpose = LocalTranspose . ViewSwap = ViewSwap . LocalTranspose), for a
 * matrix X (n_rows x n_cols) with R partitions given by part_bounds, which
 * split both axes (so R > 1 needs a square matrix). X is held in one of two
 * views (Fig. 1):
 *   MGT_ROW_VIEW     partition r holds X's rows [b_r, b_r+1): X's CSR,
 *                    row_ptr[n_rows + 1];
 *   MGT_COLUMN_VIEW  partition s holds X's columns [b_s, b_s+1) for every
 *                    row, as a CSR over all n_rows rows; the R partitions are
 *                    stored one after another, so row_ptr has R * n_rows + 1
 *                    entries and (virtual) row s * n_rows + i is row i of
 *                    partition s.
 * Column ids are X's own in both views. Cells keep their input order inside a
 * row.
 *   MGT_LOCAL_TRANSPOSE  every partition transposes its own block: a row view
 *       of X gives a column view of X^T (o_row_ptr[R * n_cols + 1]; partition
 *       r holds the transpose of X's rows in partition r); a column view of X
 *       gives a row view of X^T (o_row_ptr[n_cols + 1]). Output column ids are
 *       X's row ids.
 *   MGT_VIEW_SWAP  the same matrix in the other view: a row view of X gives a
 *       column view of X (o_row_ptr[R * n_rows + 1]); a column view gives a
 *       row view (o_row_ptr[n_rows + 1]). Output column ids are X's column ids.
 * Applying either twice returns X with each row's cells in column order when
 * they were (generally: grouped by their column's partition, for ViewSwap;
 * column-sorted, for LocalTranspose). Payload, perm, offset widths,
 * MGT_FIXED_WIDTH and the errors are as in mgt_transpose; with MGT_VALIDATE a
 * column outside [0, n_cols), or in column view outside its partition,
 * also gives MGT_ERANGE. Needs R * n_rows and R * n_cols below 2^31 where
 * they size a view, else MGT_EUNSUPPORTED.
 */
enum { MGT_LOCAL_TRANSPOSE = 0, MGT_VIEW_SWAP = 1 };
enum { MGT_ROW_VIEW = 0, MGT_COLUMN_VIEW = 1 };

/* Plan for one view operation on matrices described by desc (sizes of X, its
 * partitions, flags) given in view in_view. Host only. */
int mgt_view_plan(const mgt_desc* desc, int32_t op, int32_t in_view, mgt_plan_t* out,
                  size_t* workspace_bytes);

/* Runs the plan's view operation. Inputs as described for the plan's input
 * view; outputs o_row_ptr (size above), o_col[nnz], o_payload_off[nnz+1],
 * o_payload[payload_bytes], perm[nnz] (with MGT_EMIT_PERM). */
int mgt_view_transform(mgt_plan_t plan, const void* row_ptr, const int32_t* col,
                       const void* payload_off, const uint8_t* payload, void* o_row_ptr,
                       int32_t* o_col, void* o_payload_off, uint8_t* o_payload, uint32_t* perm,
                       void* workspace, size_t workspace_bytes, int32_t* d_status,
                       hipStream_t stream);

/* Capacity of a batch plan. Every submitted batch must fit all limits. */
typedef struct {
  int32_t max_items;
  int32_t offset_width;     /* shared by all items (4 or 8)                        */
  int64_t max_total_nnz;    /* sum of nnz over a batch                             */
  int64_t max_total_cols;   /* sum of n_cols                                       */
  int64_t max_total_rows;   /* sum of n_rows                                       */
  int64_t max_total_parts;  /* sum of n_parts                                      */
  int64_t max_item_nnz;     /* largest single item                                 */
  int64_t max_item_cols;
  uint32_t flags;           /* MGT_VALIDATE | MGT_EMIT_PERM                       */
} mgt_batch_limits;

/* One matrix of a batch: its descriptor (n_parts >= 1; partitioned outputs
 * are written when n_parts > 1) and its device buffers. */
typedef struct {
  mgt_desc desc;
  const void* row_ptr;
  const int32_t* col;
  const void* payload_off;
  const uint8_t* payload;
  void* t_row_ptr;
  int32_t* t_col;
  void* t_payload_off;
  uint8_t* t_payload;
  uint32_t* perm;           /* NULL unless MGT_EMIT_PERM                            */
  int64_t* xfer_cells;      /* n_parts > 1 only; else NULL                          */
  int64_t* xfer_bytes;
  int64_t* part_cell_off;
  int64_t* part_byte_off;
  int64_t* sdispls;         /* optional (NULL): as in mgt_transpose_partitioned     */
  int64_t* rdispls;
} mgt_item;

/* Creates a batch plan. *workspace_bytes receives an estimate for a batch at
 * the limits (payload bytes excluded); mgt_batch_workspace gives the exact
 * requirement of a particular batch. */
int mgt_batch_plan(const mgt_batch_limits* limits, mgt_plan_t* out, size_t* workspace_bytes);

/* Exact device workspace that mgt_batch_submit needs for these items. Host only. */
int mgt_batch_workspace(mgt_plan_t batch_plan, const mgt_item* items, int32_t n_items,
                        size_t* workspace_bytes);

/*
 * Transposes every item of the batch with one fixed sequence of stage kernels
 * whose grids cover all items at once (the item count does not change the
 * number of launches). Items may differ in size, payload width and partition
 * count. The descriptor table is copied to the device through the plan's
 * pinned staging buffer; the call returns once the copy is queued. d_status
 * (may be NULL) receives one status word per item. If `done` is not NULL it
 * is recorded on `stream` after the last stage.
 */
int mgt_batch_submit(mgt_plan_t batch_plan, const mgt_item* items, int32_t n_items,
                     void* workspace, size_t workspace_bytes, int32_t* d_status,
                     hipStream_t stream, hipEvent_t done);

/* ------------------------------------------------------------------ value lists */

/*
 * XCSR value lists (Section 2). The paper keeps one cell per (row, column)
 * pair whose value is a list of values, serialised as all values back to back
 * plus a count of values per cell (its cell_counts argument); a multigraph can
 * keep every edge as a cell of its own instead, so a pair with N edges is N
 * repeated cells. Both are CSRs over the same payload array here: the payload
 * bytes keep their order, so these calls neither read nor write them and the
 * caller keeps using its payload buffer. Every call is asynchronous on
 * `stream`; offset_width (4 or 8) is the width of every row-offset and
 * payload-offset array, in and out. Device pointers unless stated.
 *
 * mgt_coalesce: every run of consecutive cells of one row with the same
 *   column becomes one cell whose payload is the run's payloads in order.
 *   o_counts[j] (may be NULL) receives the run's length: the value count when
 *   every repeated cell holds one value. Rows sorted by column (every
 *   transpose output) give one cell per distinct (row, column) pair. Output
 *   capacity: o_row_ptr[n_rows + 1], o_col[nnz], o_payload_off[nnz + 1],
 *   o_counts[nnz]; the number m of output cells is written to *d_m (device
 *   int64; may be NULL) and entries past m are left alone. workspace: at least
 *   mgt_value_lists_workspace(nnz) bytes, 256-byte aligned.
 * mgt_expand: every cell whose payload is a list of value_bytes-wide values
 *   becomes one cell per value with the cell's row and column, in order:
 *   payload_bytes / value_bytes output cells (payload_bytes must be a
 *   multiple of value_bytes, else MGT_EINVAL). Outputs: o_row_ptr[n_rows + 1],
 *   o_col[payload_bytes / value_bytes], o_payload_off (may be NULL) receives
 *   q * value_bytes. If a payload offset is not a multiple of value_bytes,
 *   *d_status (may be NULL) is MGT_ERANGE and the outputs are undefined;
 *   otherwise MGT_OK.
 * mgt_counts_to_offsets: payload_off[k] = value_bytes * (counts[0] + ... +
 *   counts[k-1]) for k = 0..nnz, from the paper's per-cell value counts.
 *   Same workspace as mgt_coalesce.
 *
 * Sizes: nnz and the output cell count below 2^32, n_rows below 2^31, else
 * MGT_EUNSUPPORTED. Rows and offsets that break the CSR invariants give
 * undefined outputs but no out-of-bounds access.
 */
int mgt_value_lists_workspace(int64_t nnz, size_t* workspace_bytes);
int mgt_coalesce(int64_t n_rows, int64_t nnz, int32_t offset_width, const void* row_ptr,
                 const int32_t* col, const void* payload_off, void* o_row_ptr, int32_t* o_col,
                 void* o_payload_off, uint32_t* o_counts, int64_t* d_m, void* workspace,
                 size_t workspace_bytes, hipStream_t stream);
int mgt_expand(int64_t n_rows, int64_t nnz, int64_t payload_bytes, int32_t offset_width,
               int32_t value_bytes, const void* row_ptr, const int32_t* col,
               const void* payload_off, void* o_row_ptr, int32_t* o_col, void* o_payload_off,
               int32_t* d_status, hipStream_t stream);
int mgt_counts_to_offsets(int64_t nnz, const uint32_t* counts, int32_t value_bytes,
                          int32_t offset_width, void* payload_off, void* workspace,
                          size_t workspace_bytes, hipStream_t stream);

/* ------------------------------------------------------------------ unordered graphs */

/*
 * Unordered multigraphs stored as one triangle (Section 2: an unordered edge
 * {i, j, e} gives M_ij = M_ji = e, so the matrix is symmetric and its lower
 * triangle -- every cell with col <= row -- or its upper triangle -- col >=
 * row -- holds the whole graph). The triangle's own transpose (lower storage
 * to upper storage of the same graph and back) is mgt_transpose.
 *
 * mgt_symmetrize builds the full symmetric matrix S of a stored triangle:
 * every stored off-diagonal cell (i, j, e) appears in S as (i, j, e) and as
 * (j, i, e) with the same payload bytes; a stored diagonal cell (i, i, e)
 * appears once. Row i of S is, for MGT_LOWER, the stored cells of row i in
 * their stored order followed by the mirrored cells (i, r) in the order of
 * their source cells (source row r ascending, then stored order); for
 * MGT_UPPER the mirrored cells (sources in rows r < i) come first, then the
 * stored row. Rows stored in column order give rows of S in column order, and
 * the two storages of one graph give the same S.
 *   plan     a single-matrix plan (mgt_plan) of the stored triangle: square,
 *            without MGT_EMIT_PERM, MGT_FIXED_WIDTH or MGT_DEBUG_TIMING (else
 *            MGT_EINVAL); with MGT_VALIDATE a cell outside the triangle also
 *            gives *d_status = MGT_ERANGE.
 *   inputs   the triangle's row_ptr[n+1], col[nnz], payload_off[nnz+1],
 *            payload[payload_bytes] (device).
 *   outputs  s_row_ptr[n+1], s_col[2*nnz], s_payload_off[2*nnz+1],
 *            s_payload[2*payload_bytes] (device; capacities: S holds
 *            2*nnz - d cells and 2*payload_bytes - b bytes, d and b being the
 *            diagonal cells and their bytes; entries past those are left
 *            alone). d_sizes (device int64[2], may be NULL) receives S's cells
 *            and payload bytes.
 *   workspace  at least mgt_symmetrize_workspace bytes, 256-byte aligned.
 * A row of S must hold fewer than 2^32 payload bytes (else *d_status =
 * MGT_EUNSUPPORTED); with 4-byte offsets 2*nnz and 2*payload_bytes must stay
 * below 2^31 (else MGT_EUNSUPPORTED). Errors otherwise as for mgt_transpose.
 */
enum { MGT_LOWER = 0, MGT_UPPER = 1 };
int mgt_symmetrize_workspace(mgt_plan_t plan, size_t* workspace_bytes);
int mgt_symmetrize(mgt_plan_t plan, int32_t triangle, const void* row_ptr, const int32_t* col,
                   const void* payload_off, const uint8_t* payload, void* s_row_ptr,
                   int32_t* s_col, void* s_payload_off, uint8_t* s_payload, int64_t* d_sizes,
                   void* workspace, size_t workspace_bytes, int32_t* d_status,
                   hipStream_t stream);

/* ------------------------------------------------------------------ graphs */

/*
 * A transpose recorded once and replayed: for callers that transpose many
 * small matrices of a fixed shape into fixed buffers, where the host cost of
 * one call (descriptor upload, one launch per stage) outweighs the kernels.
 * The graph owns a pinned copy of the descriptor and every stage launch of
 * one mgt_transpose (partitioned == 0) or mgt_transpose_partitioned
 * (partitioned != 0) call with these exact pointers; arguments and errors are
 * those of that call (plans with MGT_DEBUG_TIMING, batch or view plans give
 * MGT_EINVAL). Nothing runs at creation. Each mgt_graph_launch runs the whole
 * call on `stream`, reading the inputs as they are at that time; the buffers
 * must stay allocated while the graph exists, and launches that overlap on
 * one workspace race. The plan may be destroyed after creation. Each replay
 * re-uploads the graph's descriptor copy (status words and first-pass tables
 * included) and clears counters with kernel stores (it records no memset).
 */
typedef struct mgt_graph_s* mgt_graph_t;

int mgt_graph_create(mgt_plan_t plan, int32_t partitioned, const void* row_ptr,
                     const int32_t* col, const void* payload_off, const uint8_t* payload,
                     void* t_row_ptr, int32_t* t_col, void* t_payload_off, uint8_t* t_payload,
                     uint32_t* perm, int64_t* xfer_cells, int64_t* xfer_bytes,
                     int64_t* part_cell_off, int64_t* part_byte_off, int64_t* sdispls,
                     int64_t* rdispls, void* workspace, size_t workspace_bytes,
                     int32_t* d_status, mgt_graph_t* out);
/* The same for one mgt_batch_submit call (a batch of n_items >= 1 items with
 * these exact buffers): every replay transposes all items with the batch's
 * fixed launch sequence. Arguments and errors as for mgt_batch_submit; plans
 * with MGT_DEBUG_TIMING give MGT_EINVAL. */
int mgt_batch_graph_create(mgt_plan_t batch_plan, const mgt_item* items, int32_t n_items,
                           void* workspace, size_t workspace_bytes, int32_t* d_status,
                           mgt_graph_t* out);
int mgt_graph_launch(mgt_graph_t graph, hipStream_t stream);
int mgt_graph_destroy(mgt_graph_t graph);

/* ------------------------------------------------------------------ no allocation */

/*
 * For callers that cannot allocate: code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation. The same transpose as
 * mgt_transpose (partitioned == 0) or mgt_transpose_partitioned (partitioned
 * != 0), with the same arguments, outputs and errors, except that there is no
 * workspace argument: every call uses the library's own device array of
 * MGT_NOALLOC_SCRATCH_BYTES bytes on the current device (each GPU the library
 * runs on holds its own until the process ends). The call allocates nothing
 * (no device or pinned memory, no events) and hands the plan's descriptor to
 * the device through kernel arguments.
 *   - A plan whose transpose needs more workspace than that (the size
 *     mgt_plan reported for this form) gives MGT_ENOMEM before anything is
 *     launched; plans with MGT_DEBUG_TIMING give MGT_EINVAL.
 *   - Every call on one GPU shares that GPU's array, and the array keeps the
 *     last call's contents (no call relies on it starting at zero). Calls whose
 *     device work may overlap on one GPU (several streams, several threads)
 *     race on it: order them on one stream, or use mgt_transpose with a
 *     workspace of its own.
 */
#define MGT_NOALLOC_SCRATCH_BYTES (64u << 20)
int mgt_transpose_noalloc(mgt_plan_t plan, int32_t partitioned, const void* row_ptr,
                          const int32_t* col, const void* payload_off, const uint8_t* payload,
                          void* t_row_ptr, int32_t* t_col, void* t_payload_off,
                          uint8_t* t_payload, uint32_t* perm, int64_t* xfer_cells,
                          int64_t* xfer_bytes, int64_t* part_cell_off, int64_t* part_byte_off,
                          int64_t* sdispls, int64_t* rdispls, int32_t* d_status,
                          hipStream_t stream);

/* ------------------------------------------------------------------ utilities */

/* Per-stage device times of the last call made with MGT_DEBUG_TIMING
 * (synchronises on the plan's events). names may be NULL. */
int mgt_plan_stage_times(mgt_plan_t plan, float* ms, const char** names, int32_t capacity,
                         int32_t* count);

/* Library version string. */
const char* mgt_version(void);

#ifdef __cplusplus
}
#endif
#endif /* MGT_H */
