// Internal structures of libmgt (device tables and launch helpers).
//
// Pipeline (every stage is one launch whose grid covers all items of a call):
//
//   level 1..L  stable partition passes. Level 1 reads the caller's CSR arrays;
//               later levels read the previous level's packed records. A pass
//               splits each segment (a contiguous cell range covering a column
//               interval) into 2^bits children by the next digit of the column,
//               keeping input order inside every child. For a partitioned
//               matrix, level 1 splits by destination partition (the owner of
//               the column) and the top bits of the column inside it: this is
//               the pack-by-destination step, and writing each block straight
//               at its receive displacement stands in for the exchange.
//               Per pass: tile histograms -> flat exclusive scans -> child
//               segment table -> stable scatter of records and payload bytes.
//   finish      one workgroup per final bucket (a segment spanning at most
//               2^10 columns): column counts, transposed row offsets, and a
//               stable counting sort by column that writes the outputs and
//               copies every payload to its final place.
//
// Payload bytes move in every pass but the last. With two or more passes the
// last one moves records only and stores, per cell, where its payload sits in
// the previous level buffer (a byte offset); the finish then copies each
// payload from there. A finish bucket's cells all come from one segment of
// that level, whose bytes are a contiguous range, and the buckets run in
// column order, so those reads stay inside a few segments at a time.
//
// Positions: level buffers hold all items back to back; an item's cells
// keep, at every level, the range [cell_base, cell_base + nnz) and a segment's
// range is exactly where its cells sit in the final output. Byte ranges work
// the same way.
#pragma once
#include <stdint.h>

namespace mgt {

constexpr int kMaxLevels = 4;
constexpr int kMaxFanout = 1024;      // digits per partition pass (incl. partition mode)
constexpr int kMaxFinishBits = 10;    // columns per finish bucket <= 1024
constexpr int kMaxParts = 1024;

// One item (matrix) of a call, resident in the workspace.
struct ItemDev {
  const void* row_ptr;
  const int32_t* col;
  const void* poff;
  const uint8_t* payload;
  void* t_row_ptr;
  int32_t* t_col;
  void* t_poff;
  uint8_t* t_payload;
  uint32_t* perm;
  int64_t* xfer_cells;
  int64_t* xfer_bytes;
  int64_t* part_cell_off;
  int64_t* part_byte_off;
  int64_t* sdispls;
  int64_t* rdispls;
  const int64_t* bounds;      // device copy, n_parts + 1 entries
  const uint32_t* vval;       // per input cell: the value the output carries instead of the
                              // row id (view operations), or null
  int64_t n_rows, n_cols, nnz, payload_bytes;
  uint64_t cell_base;         // first cell of the item in the level buffers
  uint64_t byte_base;         // first payload byte of the item in the level buffers
  uint64_t tile_base;         // first level-1 tile of the item
  uint64_t hist_base;         // first level-1 histogram entry of the item
  uint64_t seg_base[kMaxLevels + 1];  // first segment of the item at each level (level index 0 = level 1)
  int32_t n_parts;
  int32_t n_levels;           // partition passes (>= 1)
  int32_t bits[kMaxLevels];   // digit bits per pass; in partition mode bits[0] = sub bits
  int32_t key_bits;           // column bits (plain) / bits of the widest partition
  int32_t part_mode;          // 1: pass 1 splits by destination partition
  int32_t status_index;       // where this item's status word lives
  int32_t fixed_w;            // payload bytes of every cell when all cells have the same
                              // width (offset arrays unused), else -1
  int32_t pk_shift;           // column bits of packed records, ceil(log2(n_cols)) (<= 28 when
                              // the call packs)
};

// A contiguous cell range that covers the column interval [key_lo, key_hi).
struct Seg {
  uint64_t cell0;   // first cell (level buffers; for pass 1, the item's cell_base)
  uint64_t byte0;   // first payload byte (level buffers)
  uint32_t len;     // cells
  uint32_t key_lo;
  uint32_t key_hi;
  uint32_t item;
  uint32_t shift;   // digit = (key - key_lo) >> shift, masked to `bits`
  uint32_t bits;    // fan-out 2^bits (partition mode: n_parts << bits)
  uint32_t mode;    // 0 bits mode, 1 partition mode
  uint32_t pad;
};
static_assert(sizeof(Seg) == 48, "Seg layout");

}  // namespace mgt
