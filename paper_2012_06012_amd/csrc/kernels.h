// Host-side launchers of the transpose stages (implemented in kernels.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/mgt.h"
#include "mgt_internal.h"

namespace mgt {

// Geometry shared by host and device.
constexpr int kBlock = 256;         // threads per workgroup (4 wave64)
constexpr int kSub = 2048;          // cells sorted in LDS at once
// Geometry of the records-only partition pass when its tiles hold at least
// kWideSub cells: twice the cells per LDS sort, so each digit's run of
// records is twice as long (kernels_wide.hip).
constexpr int kWideBlock = 512;
constexpr int kWideSub = 4096;
constexpr int kMaxPassBits = 8;     // digit bits of a bits-mode pass (fan-out 256)
constexpr int kMaxLastPassBits = 9; // the records-only pass in its 512-thread form (fan-out 512)
constexpr int kScanBlock = 4096;    // elements per scan workgroup

// Arguments of a partition pass (hist and scatter share them).
struct PassArgs {
  const ItemDev* items;
  const Seg* segs;
  uint32_t nseg;
  uint32_t pass;
  const uint64_t* tstart;     // nseg + 1
  const uint64_t* hstart;     // nseg + 1
  const uint2* ks_in;         // (key, size) records, pass >= 2
  const uint2* rk_in;         // (row, cell index) records, pass >= 2
  const uint8_t* pay_in;      // payload bytes, pass >= 2
  uint2* ks_out;
  uint2* rk_out;
  uint8_t* pay_out;           // unused when rso_out is set
  uint32_t* rso_out;          // last pass of two or more: per cell (row, cell index, byte
                              // offset of the payload in pay_in as two words) in place of
                              // rk_out; no payload is moved
  uint32_t* hcnt;             // [entry] cells of (segment, digit, tile)
  uint32_t* hbyt;             // [entry] payload bytes of (segment, digit, tile)
  uint32_t* ttot;             // [tile] payload bytes of the tile
  const uint64_t* ocnt;       // exclusive scan of hcnt (n + 1)
  const uint64_t* obyt;       // exclusive scan of hbyt (n + 1)
  const uint64_t* tsrc;       // exclusive scan of ttot (tiles + 1)
  int32_t* item_status;
  int32_t* abort_flag;
  uint64_t g8;                // grid size (multiple of 8)
  uint32_t tile_cells;        // multiple of kSub
  int32_t offset_width;
  int32_t has_val;            // first pass: the items carry vval (view operations)
  // Packed records: a call with exactly one records-only pass, made without
  // perm and not as a view operation, keeps (column | size << s, row) after
  // the first pass and (column | size << s, row, payload offset) after the
  // second, s being the item's column bits (ItemDev::pk_shift, <= 28),
  // provided every payload size is below 2^(32 - s) bytes; the first
  // histogram checks that and sets *no_pack otherwise.
  int32_t pk_on;
  int32_t* no_pack;           // zero at the start of the call (uploaded with the status words)
  int32_t pk_keys;            // with pk_on and no fixed-width item: the first histogram writes
                              // (column | size << s) per cell into rk_out, which the first pass
                              // reads instead of the columns and offsets
  int32_t pk_split;           // set by the launcher: a slim packed-only kernel runs beside this
                              // one and takes packed records (this one returns on them)
  int32_t slim0;              // first pass: packed records go to the slim first pass, in its
                              // bits-only form (1: every item split by column bits) or its
                              // partition form (2: some item split by partition, fan-out
                              // at most 512); 0: the plain kernel only
  int32_t rec12;              // the slim kernel writes 12-byte packed records (column | size,
                              // row, payload offset minus the finish bucket's first byte as a
                              // signed 32-bit word) unless *big_seg is set
  const int32_t* big_seg;
};

struct ChildArgs {
  const ItemDev* items;
  const Seg* segs;            // parents
  uint32_t nseg;
  uint32_t pass;              // pass whose output the children describe (0-based)
  const uint64_t* tstart;
  const uint64_t* hstart;
  const uint64_t* ocnt;
  const uint64_t* obyt;
  Seg* children;
  uint32_t* child_tiles;
  uint32_t* child_hsize;
  uint32_t tile_cells;
  const int32_t* abort_flag;
  int32_t* big_seg;           // non-null where the children are the last pass's input
                              // segments: set to 1 if one holds 2^31 payload bytes or more
};

struct FinishArgs {
  const ItemDev* items;
  uint32_t n_items;           // <= nbuckets: every item has at least one bucket
  const Seg* buckets;
  uint32_t nbuckets;
  const uint2* ks_in;
  const uint2* rk_in;
  const uint8_t* pay_in;      // payload level buffer (the one before the last pass if rso_in)
  const uint32_t* rso_in;     // (row, cell index, payload offset in pay_in) records of the
                              // last pass, read in place of rk_in, or null
  const int32_t* abort_flag;
  const int32_t* item_status;
  int32_t* d_status;          // the caller's status words (may be null), written with the tails
  int32_t offset_width;
  uint64_t g8;                // grid size (multiple of 8)
  int32_t pk_on;              // as in PassArgs
  const int32_t* no_pack;
  uint8_t* bucket_done;       // [nbuckets] gathering finish with packed records: 1 where
                              // k_finish_bucket wrote the bucket (k_finish skips it), else 0;
                              // null: k_finish takes every bucket
  uint32_t grid;              // k_finish_bucket: workgroups (one or two per CU)
  uint32_t bk_threads;        // k_finish_bucket: 1024 (buckets up to 9,216 cells, one
                              // workgroup per CU) or 512 (up to 4,608 cells, two per CU)
  uint32_t skip_done;         // k_finish_bucket: leave buckets already marked 1 alone (a
                              // 1,024-thread launch after a 512-thread one)
  int32_t rec12;              // packed records are 12 bytes (see PassArgs) unless *big_seg
  const int32_t* big_seg;
};

// Copies n bytes (a multiple of 4) from host memory to dst through kernel
// arguments, in chunks of kUploadChunk bytes: no staging buffer, no memcpy.
constexpr uint32_t kUploadChunk = 3072;
hipError_t launch_upload(void* dst, const void* src, size_t n, hipStream_t s);
hipError_t launch_validate(const ItemDev* items, uint32_t n_items, uint64_t max_len,
                           int32_t* item_status, int32_t* abort_flag, int32_t offset_width,
                           hipStream_t s);
// Exclusive scans of `narr` (1 or 2) u32 arrays of length *n (<= n_max) into
// u64 outputs of length n + 1 (out[n] = total).
hipError_t launch_scan(const uint32_t* in0, uint64_t* out0, const uint32_t* in1, uint64_t* out1,
                       const uint64_t* n_dev, uint64_t n_max, uint64_t* block_sums,
                       hipStream_t s);
// Per-cell sort key and carried value of a view operation (LocalTranspose or
// ViewSwap, Section 3) on one item whose bounds are already on the device.
struct ViewArgs {
  const ItemDev* items;       // item 0: row_ptr over the virtual rows, status slot
  const int64_t* bounds;      // device, n_parts + 1 partition bounds of X
  int32_t n_parts;
  const int32_t* col;         // the matrix's own column ids
  uint32_t* keys;             // out: sort key per cell (becomes the item's col)
  uint32_t* vals;             // out: value per cell (becomes the output column id)
  uint64_t nnz, n_virtual;    // cells; rows of the input CSR (n_rows, or R * n_rows)
  int64_t n_rows, n_cols;     // of the matrix X the views represent
  int32_t op;                 // 0 LocalTranspose, 1 ViewSwap
  int32_t column_view;        // input is in column view
  int32_t validate;
  int32_t offset_width;
  int32_t* item_status;
  int32_t* abort_flag;
};
hipError_t launch_view_keys(const ViewArgs& a, hipStream_t s);
hipError_t launch_pass_hist(const PassArgs& a, hipStream_t s);
hipError_t launch_pass_scatter(const PassArgs& a, hipStream_t s);
hipError_t launch_pass_scatter_wide(const PassArgs& a, hipStream_t s);  // records-only pass
hipError_t launch_pass0_slim(const PassArgs& a, hipStream_t s);         // packed first pass (slim)
hipError_t launch_children(const ChildArgs& a, hipStream_t s);
hipError_t launch_finish(const FinishArgs& a, hipStream_t s);
// Whole-bucket finish of a gathering call with packed records (runs before
// launch_finish, which then skips the buckets it wrote).
hipError_t launch_finish_bucket(const FinishArgs& a, hipStream_t s);
// mgt_symmetrize's stages after the transpose of the stored triangle
// (symmetric.hip). Every offset array has width ow.
struct SymArgs {
  uint64_t n, nnz;             // rows (= columns) and stored cells
  uint64_t pbytes;             // payload bytes of the triangle (and of its transpose)
  uint64_t cap_cells;          // capacity of s_col (2 nnz) and of s_payload (2 pbytes)
  uint64_t cap_bytes;
  int32_t ow, lower, validate;
  const void* row_ptr;         // the stored triangle
  const int32_t* col;
  const void* poff;
  const uint8_t* payload;
  const void* t_row_ptr;       // its transpose
  const int32_t* t_col;
  const void* t_poff;
  const uint8_t* t_payload;
  void* s_row_ptr;             // the full symmetric matrix
  int32_t* s_col;
  void* s_poff;
  uint8_t* s_payload;
  int64_t* d_sizes;            // cells and payload bytes of S (may be null)
  int32_t* d_status;           // the caller's status word (may be null)
  int32_t* st;                 // the call's status: the transpose's, then these stages'
  uint32_t* cnt;               // per row of S: cells, payload bytes
  uint32_t* byt;
  uint64_t* ocnt;              // their exclusive scans (n + 1 entries)
  uint64_t* obyt;
  uint64_t* scan;              // scratch of launch_scan for n entries
};
hipError_t launch_symmetrize(const SymArgs& a, hipStream_t s);

// The allocation-free transpose (runtime.cpp), called by mgt_transpose_noalloc.
int noalloc_call(mgt_plan_t p, int32_t partitioned, const void* row_ptr, const int32_t* col,
                 const void* payload_off, const uint8_t* payload, void* t_row_ptr, int32_t* t_col,
                 void* t_payload_off, uint8_t* t_payload, uint32_t* perm, int64_t* xfer_cells,
                 int64_t* xfer_bytes, int64_t* part_cell_off, int64_t* part_byte_off,
                 int64_t* sdispls, int64_t* rdispls, void* ws, size_t ws_bytes, int32_t* d_status,
                 hipStream_t stream);
// Scratch needed by launch_scan for n_max elements (bytes).
inline uint64_t scan_scratch_bytes(uint64_t n_max) {
  return 2 * 8 * ((n_max + kScanBlock - 1) / kScanBlock + 1) + 64;
}

}  // namespace mgt
