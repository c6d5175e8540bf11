// Device stages of the XCSR multigraph transpose (gfx950).
//
// The transpose is a stable sort of the cells by column (Section 2 definition,
// M^T_ij = M_ji, with repeated cells kept in input order), carrying each cell's
// row id, index and payload bytes. It is done as a few stable partition passes
// over the column bits (most significant first) followed by a per-bucket
// counting sort in LDS; see mgt_internal.h for the data flow.
#include <hip/hip_runtime.h>

#include <cstring>

#include "../../include/mgt.h"
#include "kernels.h"
#include "prims.h"

// Workgroup geometry of this copy of the device code. The library holds two:
// 256 threads, 2,048-cell sub-chunks and 8-bit passes for every stage (this
// file), and 512 threads, 4,096-cell sub-chunks and up to 9-bit passes for the
// records-only pass alone (kernels_wide.hip, which includes this file in a
// namespace of its own).
#ifndef MGT_GEO_NS
#define MGT_GEO_NS geo256
#define MGT_GEO_BLOCK ::mgt::kBlock
#define MGT_GEO_SUB ::mgt::kSub
#define MGT_GEO_FANBITS ::mgt::kMaxPassBits
#endif

namespace mgt {
namespace MGT_GEO_NS {

constexpr int kBlock = MGT_GEO_BLOCK;      // threads per workgroup
constexpr int kSub = MGT_GEO_SUB;          // cells sorted in LDS at once
constexpr int kNW = kBlock / kWave;        // waves per workgroup
constexpr int kItems = kSub / kBlock;      // cells per lane per sub-chunk
constexpr int kWaveCells = kSub / kNW;     // cells of one wave per sub-chunk
constexpr int kFinishCols = 1 << kMaxFinishBits;
static_assert(kItems * kWave * kNW == kSub, "sub-chunk geometry");

// ----------------------------------------------------------------------------- helpers

__device__ __forceinline__ int64_t ld_off(const void* p, uint64_t i, int ow) {
  return ow == 4 ? (int64_t)gm((const int32_t*)p)[i] : gm((const int64_t*)p)[i];
}
// Low 32-bit word of offset i of an array of 2^lg-byte little-endian offsets
// (lg = 2 or 3). One load of the same type for both widths, so a run of them
// can be in flight at once; differences of low words are exact whenever the
// true difference is below 2^32.
__device__ __forceinline__ uint32_t ld_lo(const void* p, uint64_t i, int lg) {
  return *gm((const uint32_t*)((const uint8_t*)p + (i << lg)));
}
// Full offset i, read as two words without a branch on the width (for 4-byte
// offsets the second load re-reads word i, so it stays inside the array).
__device__ __forceinline__ uint64_t ld_full(const void* p, uint64_t i, int lg) {
  const uint8_t* a = (const uint8_t*)p + (i << lg);
  const uint32_t lo = *gm((const uint32_t*)a);
  const uint32_t hi = *gm((const uint32_t*)(a + (lg == 3 ? 4 : 0)));
  return (uint64_t)lo | ((uint64_t)(lg == 3 ? hi : 0u) << 32);
}
__device__ __forceinline__ void st_off(void* p, uint64_t i, int64_t v, int ow) {
  if (ow == 4) gm((int32_t*)p)[i] = (int32_t)v;
  else gm((int64_t*)p)[i] = v;
}

// Relaxed device-scope add on a 64-bit counter in global memory.
__device__ __forceinline__ void add_u64(uint64_t* p, uint64_t v) {
  __hip_atomic_fetch_add(gm((unsigned long long*)p), (unsigned long long)v, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
}

// Adds every active lane's cell (one cell of z bytes) to xc[key] and xb[key]
// with one atomic pair per distinct key in the wave: the lanes holding the
// leader's key are summed first. Sorted cells give a wave one or two keys.
// Called by whole waves (uniform control flow).
__device__ __forceinline__ void wave_add_xfer(bool active, uint32_t key, uint32_t z, uint64_t* xc,
                                              uint64_t* xb) {
  uint64_t left = ballot(active);
  while (left) {
    const int leader = __ffsll((unsigned long long)left) - 1;
    const uint32_t k = wave_bcast(key, leader);
    const bool mine = active && key == k;
    const uint64_t same = ballot(mine);
    const uint64_t incl = wave_incl_scan_u64(mine ? (uint64_t)z : 0ull);
    const uint64_t bytes = wave_bcast(incl, kWave - 1);
    if ((int)lane_id() == leader) {
      add_u64(&xc[k], (uint64_t)__popcll(same));
      add_u64(&xb[k], bytes);
    }
    left &= ~same;
  }
}

// Adds every active lane's cell (one cell of z bytes) to cnt[d] and byt[d] in
// LDS with one atomic pair per run of equal digits in consecutive lanes.
// Repeated cells (a column drawn many times in one row) otherwise send a whole
// wave's atomics to one address, where they execute one lane at a time. The
// lanes must hold consecutive cells, and a run's bytes stay below 2^32 (any
// 16,384 consecutive cells do). Called by whole waves (uniform control flow).
template <class TB>
__device__ __forceinline__ void hist_add_runs(bool act, uint32_t d, uint32_t z, uint32_t* cnt,
                                              TB* byt) {
  const uint32_t lane = lane_id();
  const uint32_t dk = act ? d : 0xFFFFFFFFu;
  const uint32_t prev = __shfl_up(dk, 1, kWave);    // lane 0 reads its own value
  const uint32_t next = __shfl_down(dk, 1, kWave);  // lane 63 reads its own value
  const bool head = lane == 0 || prev != dk;
  const bool tail = lane == kWave - 1 || next != dk;
  const uint64_t heads = ballot(head);
  const uint32_t zz = act ? z : 0u;
  const uint32_t incl = wave_incl_scan_u32(zz);
  const uint32_t excl = incl - zz;
  const int h = 63 - (int)__clzll(heads & ((2ull << lane) - 1ull));  // this lane's run head
  const uint32_t base = __shfl(excl, h, kWave);
  if (act && tail) {
    atomicAdd(&cnt[d], lane - (uint32_t)h + 1u);
    atomicAdd(&byt[d], (TB)(incl - base));
  }
}

__device__ __forceinline__ int ceil_log2(uint32_t x) { return x <= 1 ? 0 : 32 - __clz(x - 1); }

__device__ __forceinline__ uint32_t seg_fanout(const Seg& s, uint32_t R) {
  return s.mode ? (R << s.bits) : (1u << s.bits);
}

// Largest s with tstart[s] <= t (the segment that owns tile t), found by the
// whole workgroup: each round probes kBlock evenly spaced segments and keeps
// the last one <= t, so 2^16 segments take two dependent loads, not sixteen.
// Every thread must call it; all get the same answer.
__device__ __forceinline__ uint32_t coop_find_seg(const uint64_t* tstart, uint32_t nseg, uint64_t t) {
  uint32_t lo = 0, hi = nseg;  // tstart[lo] <= t, answer in [lo, hi)
  while (hi - lo > 1) {
    const uint32_t step = (hi - lo + kBlock - 1) / kBlock;
    const uint32_t p = lo + threadIdx.x * step;
    const bool ok = p < hi && tstart[p] <= t;
    int c = __syncthreads_count(ok);
    c = c < 1 ? 1 : c;
    lo = lo + (uint32_t)(c - 1) * step;
    hi = min(lo + step, hi);
  }
  return lo;
}

// Row owning cell k: the largest r in [lo, hi] with row_ptr[r] <= k.
__device__ __forceinline__ uint32_t row_of(const void* rp, int ow, uint64_t k, uint32_t lo,
                                           uint32_t hi) {
  uint32_t a = lo, b = hi + 1;
  while (b - a > 1) {
    const uint32_t mid = (a + b) >> 1;
    if ((uint64_t)ld_off(rp, mid, ow) <= k) a = mid;
    else b = mid;
  }
  return a;
}

// Partition owning vertex v: largest p with bounds[p] <= v (0-based ranks).
// The partition holding index v among the bounds lb: the largest p < R with
// lb[p] <= v, searched in [lo, hi) (lb[lo] <= v or lo = 0).
__device__ __forceinline__ uint32_t owner_in(const int32_t* lb, uint32_t lo, uint32_t hi, int64_t v) {
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (lb[mid] <= v) lo = mid;
    else hi = mid;
  }
  return lo;
}
__device__ __forceinline__ uint32_t owner_of(const int32_t* lb, uint32_t R, int64_t v) {
  return owner_in(lb, 0, R, v);
}

// Coarse owner table of a partitioned pass: ot[t] = owner of index t << osh
// for t = 0..kOwnerT, with n = lb[R] <= kOwnerT << osh. The owner of v lies
// in [ot[v >> osh], ot[(v >> osh) + 1]]: one or two partitions unless many
// small partitions share one table cell, instead of a search over all R.
constexpr int kOwnerT = 1024;
__device__ __forceinline__ int owner_shift(int64_t n) {
  int sh = 0;
  while (((int64_t)kOwnerT << sh) < n) ++sh;
  return sh;
}
__device__ __forceinline__ void fill_owner_table(const int32_t* lb, uint32_t R, int osh,
                                                 uint16_t* ot) {
  for (uint32_t t = threadIdx.x; t <= (uint32_t)kOwnerT; t += blockDim.x)
    ot[t] = (uint16_t)owner_in(lb, 0, R, (int64_t)t << osh);
}
__device__ __forceinline__ uint32_t owner_lut(const int32_t* lb, const uint16_t* ot, int osh,
                                              uint32_t R, int64_t v) {
  if (v < 0) return 0;
  const uint64_t t = (uint64_t)v >> osh;
  if (t >= (uint64_t)kOwnerT) return owner_in(lb, 0, R, v);  // beyond the bounds (invalid input)
  const uint32_t hi = min((uint32_t)ot[t + 1] + 1u, R);
  return owner_in(lb, ot[t], hi, v);
}

// Digit of a column inside a segment. Bits mode: the next `bits` bits of
// (key - key_lo) below `shift`. Partition mode (pass 1 of a partitioned
// matrix): the destination partition, then the top `bits` bits of the column
// inside it. Out-of-range keys (invalid input) are clamped into the fan-out.
__device__ __forceinline__ uint32_t digit_bits(uint32_t key, const Seg& s) {
  const uint32_t m = (1u << s.bits) - 1u;
  const uint32_t d = (key - s.key_lo) >> s.shift;
  return d > m ? m : d;
}
__device__ __forceinline__ uint32_t digit_of(uint32_t key, const Seg& s, const int32_t* lb,
                                             const uint16_t* ot, int osh, uint32_t R) {
  if (s.mode == 0) return digit_bits(key, s);
  const uint32_t m = (1u << s.bits) - 1u;
  const uint32_t p = owner_lut(lb, ot, osh, R, (int64_t)key);
  const int64_t rel = (int64_t)key - lb[p];
  uint32_t sub = rel < 0 ? 0u : (uint32_t)(rel >> s.shift);
  sub = sub > m ? m : sub;
  return (p << s.bits) | sub;
}

__device__ __forceinline__ void raise_status(int32_t* item_status, int32_t* abort_flag, int idx,
                                             int32_t code) {
  item_status[idx] = code;
  __hip_atomic_store(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ bool aborted(const int32_t* abort_flag) {
  return __hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
}
// Whether this call's records are packed: the host allows it (pk_on) and the
// first histogram found every payload size within 32 - pk_shift bits (it sets
// no_pack otherwise). Uniform over the grid.
__device__ __forceinline__ bool packed_records(int32_t pk_on, const int32_t* no_pack) {
  return pk_on && __hip_atomic_load(no_pack, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0;
}

// (the 512-thread copy of this file needs only the records-only scatter)
#ifndef MGT_WIDE
// ----------------------------------------------------------------------------- upload

// Bytes handed over as a kernel argument, copied word by word to dst.
struct UploadArgs {
  uint32_t* dst;
  uint32_t words;
  uint32_t pad;
  uint32_t data[kUploadChunk / 4];
};

__global__ __launch_bounds__(kBlock) void k_upload(UploadArgs a) {
  for (uint32_t i = threadIdx.x; i < a.words; i += kBlock) gm(a.dst)[i] = a.data[i];
}

// ----------------------------------------------------------------------------- init / validate

// Device-side data checks (MGT_VALIDATE): offsets start at 0, never decrease
// and end at nnz / payload_bytes; every column id lies in [0, n_cols); every
// cell's payload is smaller than 2^32 bytes.
__global__ __launch_bounds__(kBlock) void k_validate(const ItemDev* items, int32_t* item_status,
                                                     int32_t* abort_flag, int ow) {
  const ItemDev& it = items[blockIdx.y];
  const uint64_t n_rows = (uint64_t)it.n_rows, nnz = (uint64_t)it.nnz;
  const uint64_t span = (n_rows > nnz ? n_rows : nnz) + 1;
  bool bad = false;
  for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < span;
       i += (uint64_t)gridDim.x * kBlock) {
    if (i <= n_rows) {
      const int64_t r0 = ld_off(it.row_ptr, i, ow);
      if (i == 0 && r0 != 0) bad = true;
      if (i < n_rows && ld_off(it.row_ptr, i + 1, ow) < r0) bad = true;
      if (i == n_rows && r0 != it.nnz) bad = true;
    }
    if (i <= nnz) {
      if (it.fixed_w < 0) {  // fixed-width cells have no offsets to check
        const int64_t p0 = ld_off(it.poff, i, ow);
        if (i == 0 && p0 != 0) bad = true;
        if (i == nnz && p0 != it.payload_bytes) bad = true;
        if (i < nnz) {
          const int64_t d = ld_off(it.poff, i + 1, ow) - p0;
          if (d < 0 || d >= ((int64_t)1 << 32)) bad = true;
        }
      }
      if (i < nnz) {
        const int32_t c = it.col[i];
        if (c < 0 || (int64_t)c >= it.n_cols) bad = true;
      }
    }
  }
  if (bad) raise_status(item_status, abort_flag, it.status_index, MGT_ERANGE);
}

// ----------------------------------------------------------------------------- scans

// Exclusive scans (u32 in, u64 out, out[n] = total) by reduce / spine / down-sweep.
__global__ __launch_bounds__(kBlock) void k_scan_reduce(const uint32_t* in0, const uint32_t* in1,
                                                        const uint64_t* n_dev, uint64_t n_max,
                                                        uint64_t* bsum, uint64_t nb_cap) {
  __shared__ uint64_t red[kNW + 1];
  const uint64_t n = n_dev ? min(*n_dev, n_max) : n_max;
  const uint64_t lo = (uint64_t)blockIdx.x * kScanBlock;
  if (lo >= n) return;
  const uint64_t hi = min(n, lo + kScanBlock);
  uint64_t s0 = 0, s1 = 0;
  for (uint64_t i = lo + threadIdx.x; i < hi; i += kBlock) {
    s0 += in0[i];
    if (in1) s1 += in1[i];
  }
  uint64_t t0, t1;
  block_excl_scan<kNW>(s0, red, t0);
  block_excl_scan<kNW>(s1, red, t1);
  if (threadIdx.x == 0) {
    bsum[blockIdx.x] = t0;
    bsum[nb_cap + blockIdx.x] = t1;
  }
}

__global__ __launch_bounds__(1024) void k_scan_spine(const uint64_t* n_dev, uint64_t n_max,
                                                     uint64_t* bsum, uint64_t nb_cap,
                                                     uint64_t* out0, uint64_t* out1) {
  __shared__ uint64_t red[1024 / kWave + 1];
  const uint64_t n = n_dev ? min(*n_dev, n_max) : n_max;
  const uint64_t nb = (n + kScanBlock - 1) / kScanBlock;
  for (int arr = 0; arr < (out1 ? 2 : 1); ++arr) {
    uint64_t* b = bsum + (uint64_t)arr * nb_cap;
    uint64_t carry = 0;
    for (uint64_t base = 0; base < nb; base += 1024) {
      const uint64_t i = base + threadIdx.x;
      const uint64_t v = i < nb ? b[i] : 0;
      uint64_t tot;
      const uint64_t ex = block_excl_scan<1024 / kWave>(v, red, tot);
      if (i < nb) b[i] = carry + ex;
      carry += tot;
    }
    if (threadIdx.x == 0) (arr == 0 ? out0 : out1)[n] = carry;
  }
}

__global__ __launch_bounds__(kBlock) void k_scan_down(const uint32_t* in0, uint64_t* out0,
                                                      const uint32_t* in1, uint64_t* out1,
                                                      const uint64_t* n_dev, uint64_t n_max,
                                                      const uint64_t* bsum, uint64_t nb_cap) {
  __shared__ uint64_t red[kNW + 1];
  constexpr int kPer = kScanBlock / kBlock;
  const uint64_t n = n_dev ? min(*n_dev, n_max) : n_max;
  const uint64_t lo = (uint64_t)blockIdx.x * kScanBlock;
  if (lo >= n) return;
  for (int arr = 0; arr < (in1 ? 2 : 1); ++arr) {
    const uint32_t* in = arr ? in1 : in0;
    uint64_t* out = arr ? out1 : out0;
    const uint64_t base = bsum[(uint64_t)arr * nb_cap + blockIdx.x];
    const uint64_t t0 = lo + (uint64_t)threadIdx.x * kPer;
    uint32_t v[kPer];
    uint64_t s = 0;
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
      v[j] = (t0 + j < n) ? in[t0 + j] : 0u;
      s += v[j];
    }
    uint64_t tot;
    uint64_t ex = block_excl_scan<kNW>(s, red, tot) + base;
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
      if (t0 + j < n) out[t0 + j] = ex;
      ex += v[j];
    }
  }
}

// The three kernels above in one workgroup, for arrays of at most
// kSmallScan entries: the carry runs through the kScanBlock chunks in order,
// which costs less than two more launches while the array is this short.
constexpr uint64_t kSmallScan = 4 * (uint64_t)kScanBlock;

__global__ __launch_bounds__(1024) void k_scan_small(const uint32_t* in0, uint64_t* out0,
                                                     const uint32_t* in1, uint64_t* out1,
                                                     const uint64_t* n_dev, uint64_t n_max) {
  __shared__ uint64_t red[1024 / kWave + 1];
  constexpr int kPer = kScanBlock / 1024;
  const uint64_t n = n_dev ? min(*n_dev, n_max) : n_max;
  for (int arr = 0; arr < (out1 ? 2 : 1); ++arr) {
    const uint32_t* in = arr ? in1 : in0;
    uint64_t* out = arr ? out1 : out0;
    uint64_t carry = 0;
    for (uint64_t lo = 0; lo < n; lo += kScanBlock) {
      const uint64_t t0 = lo + (uint64_t)threadIdx.x * kPer;
      uint32_t v[kPer];
      uint64_t sum = 0;
#pragma unroll
      for (int j = 0; j < kPer; ++j) {
        v[j] = (in && t0 + j < n) ? in[t0 + j] : 0u;
        sum += v[j];
      }
      uint64_t tot;
      uint64_t ex = block_excl_scan<1024 / kWave>(sum, red, tot) + carry;
      if (in) {
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
          if (t0 + j < n) out[t0 + j] = ex;
          ex += v[j];
        }
      }
      carry += tot;
    }
    if (threadIdx.x == 0) out[n] = carry;
  }
}

// ----------------------------------------------------------------------------- pass: histogram

constexpr int kBatch = 8;  // independent loads in flight per lane

__global__ __launch_bounds__(kBlock) void k_pass_hist(PassArgs a) {
  __shared__ uint32_t s_cnt[kMaxFanout];
  __shared__ uint32_t s_byt[kMaxFanout];
  __shared__ int32_t s_lb[kMaxParts + 1];
  __shared__ uint16_t s_ot[kOwnerT + 1];
  __shared__ Seg s_seg;
  __shared__ uint32_t s_si;
  __shared__ uint64_t s_red[kNW + 1];
  if (aborted(a.abort_flag)) return;
  const uint64_t tile = xcd_tile(blockIdx.x, a.g8);
  if (tile >= a.tstart[a.nseg]) return;
  {
    const uint32_t si = coop_find_seg(a.tstart, a.nseg, tile);
    if (threadIdx.x == 0) {
      s_si = si;
      s_seg = a.segs[si];
    }
  }
  __syncthreads();
  const Seg sg = s_seg;
  const uint32_t si = s_si;
  const ItemDev* it = &a.items[sg.item];
  const uint32_t R = (uint32_t)it->n_parts;
  const uint32_t F = seg_fanout(sg, R);
  if (sg.mode)
    for (uint32_t i = threadIdx.x; i <= R; i += kBlock) s_lb[i] = (int32_t)gm(it->bounds)[i];
  for (uint32_t d = threadIdx.x; d < F; d += kBlock) {
    s_cnt[d] = 0;
    s_byt[d] = 0;
  }
  __syncthreads();
  int osh = 0;
  if (sg.mode) {  // block-uniform
    osh = owner_shift(s_lb[R]);
    fill_owner_table(s_lb, R, osh, s_ot);
    __syncthreads();
  }
  const uint64_t j = tile - a.tstart[si];
  if (a.pass == 0 && j == 0 && sg.mode && it->xfer_cells) {
    // the item's transfer matrices start at zero; the first pass's scatter
    // adds to them after this kernel
    const uint64_t rr = (uint64_t)R * R;
    for (uint64_t e = threadIdx.x; e < rr; e += kBlock) {
      it->xfer_cells[e] = 0;
      it->xfer_bytes[e] = 0;
    }
  }
  const uint64_t c_begin = j * a.tile_cells;
  const uint64_t c_end = min((uint64_t)sg.len, c_begin + a.tile_cells);
  const int ow = a.offset_width;
  uint64_t mybytes = 0;
  constexpr uint64_t kStride = (uint64_t)kBlock * kBatch;
  // sizes from 2^(32 - pk_shift) bytes on cannot be packed beside a column
  const int pk_shift = it->pk_shift;
  const uint64_t pk_lim = a.pk_on ? 1ull << (32 - pk_shift) : ~0ull;
  const uint32_t pk_mask = (uint32_t)((1ull << pk_shift) - 1u);
  // a packed call's first pass reads (column | size << pk_shift) from here: the
  // level buffer of (row, index) records that packed records leave unused
  uint32_t* const pk4 = (a.pk_on && a.pk_keys && a.pass == 0) ? (uint32_t*)a.rk_out : nullptr;
  bool too_wide = false;
  if (a.pass == 0) {
    const uint64_t kbase = sg.cell0 - it->cell_base;
    const int32_t* col = it->col;
    const void* poff = it->poff;
    const int lg = ow == 8 ? 3 : 2;
    const int32_t fw = it->fixed_w;
    // the tile's bytes exactly; below 2^32 they make every low-word size exact
    if (fw >= 0) {
      mybytes = threadIdx.x == 0 ? (c_end - c_begin) * (uint64_t)fw : 0;
      too_wide = (uint64_t)fw >= pk_lim;
    } else
      mybytes = threadIdx.x == 0 ? ld_full(poff, kbase + c_end, lg) - ld_full(poff, kbase + c_begin, lg) : 0;
    // (every loop below has the same trip count on all lanes: the run
    // aggregation works on whole waves)
    if (fw >= 0) {  // fixed-width cells: sizes are known, only the columns are read
      for (uint64_t c0 = c_begin; c0 < c_end; c0 += kStride) {
        const uint64_t c = c0 + threadIdx.x;
        uint32_t key[kBatch];
#pragma unroll
        for (int q = 0; q < kBatch; ++q)
          key[q] = (uint32_t)gm(col)[kbase + min(c + (uint64_t)q * kBlock, c_end - 1)];
#pragma unroll
        for (int q = 0; q < kBatch; ++q) {
          const bool act = c + (uint64_t)q * kBlock < c_end;
          const uint32_t d = act ? digit_of(key[q], sg, s_lb, s_ot, osh, R) : 0u;
          hist_add_runs(act, d, (uint32_t)fw, s_cnt, s_byt);
          if (pk4 && act) pk4[sg.cell0 + c + (uint64_t)q * kBlock] = (key[q] & pk_mask) | ((uint32_t)fw << pk_shift);
        }
      }
    } else
    for (uint64_t c0 = c_begin; c0 < c_end; c0 += kStride) {
      const uint64_t c = c0 + threadIdx.x;
      uint32_t key[kBatch], p0[kBatch], p1[kBatch];
#pragma unroll
      for (int q = 0; q < kBatch; ++q) {
        const uint64_t cc = min(c + (uint64_t)q * kBlock, c_end - 1);  // in bounds, no branch
        const uint64_t k = kbase + cc;
        key[q] = (uint32_t)gm(col)[k];
        p0[q] = ld_lo(poff, k, lg);
        p1[q] = ld_lo(poff, k + 1, lg);
      }
#pragma unroll
      for (int q = 0; q < kBatch; ++q) {
        const bool act = c + (uint64_t)q * kBlock < c_end;
        const uint32_t sz = p1[q] - p0[q];
        const uint32_t d = act ? digit_of(key[q], sg, s_lb, s_ot, osh, R) : 0u;
        hist_add_runs(act, d, sz, s_cnt, s_byt);
        too_wide |= act && (uint64_t)sz >= pk_lim;
        if (pk4 && act) pk4[sg.cell0 + c + (uint64_t)q * kBlock] = (key[q] & pk_mask) | (sz << pk_shift);
      }
    }
    if (a.pk_on && too_wide) gm(a.no_pack)[0] = 1;
  } else {
    // pass 1 reads the first pass's records, packed or not (uniform)
    const bool pk = packed_records(a.pk_on, a.no_pack);
    for (uint64_t c0 = c_begin; c0 < c_end; c0 += kStride) {
      const uint64_t c = c0 + threadIdx.x;
      uint2 ks[kBatch];
#pragma unroll
      for (int q = 0; q < kBatch; ++q) {
        const uint64_t cc = min(c + (uint64_t)q * kBlock, c_end - 1);
        ks[q] = a.ks_in[sg.cell0 + cc];
      }
#pragma unroll
      for (int q = 0; q < kBatch; ++q) {
        const bool act = c + (uint64_t)q * kBlock < c_end;
        const uint32_t key = pk ? ks[q].x & pk_mask : ks[q].x;
        const uint32_t sz = pk ? ks[q].x >> pk_shift : ks[q].y;
        const uint32_t d = act ? digit_of(key, sg, s_lb, s_ot, osh, R) : 0u;
        hist_add_runs(act, d, sz, s_cnt, s_byt);
        if (act) mybytes += sz;
      }
    }
  }
  uint64_t tot;
  block_excl_scan<kNW>(mybytes, s_red, tot);  // also orders the LDS histogram updates
  const uint64_t nt = a.tstart[si + 1] - a.tstart[si];
  const uint64_t hb = a.hstart[si];
  for (uint32_t d = threadIdx.x; d < F; d += kBlock) {
    a.hcnt[hb + (uint64_t)d * nt + j] = s_cnt[d];
    a.hbyt[hb + (uint64_t)d * nt + j] = s_byt[d];
  }
  if (threadIdx.x == 0) {
    a.ttot[tile] = (uint32_t)tot;
    if (tot >> 32) raise_status(a.item_status, a.abort_flag, it->status_index, MGT_EUNSUPPORTED);
  }
}

#endif  // MGT_WIDE

// ----------------------------------------------------------------------------- shared sub-chunk sort

// LDS state of one stable sub-chunk sort, for up to kFan digits. kBytes: the
// sorted byte prefix (bpre) is kept, for passes that place payload bytes.
// kSlim (packed records only): key holds the whole packed (column | size)
// word, and sizes, digits and cell indexes are not kept (the size and digit
// are recomputed from the key), which leaves 12 bytes per cell, 16 with the
// byte prefix.
template <int kFan, bool kBytes, bool kSlim = false>
struct SortLdsT {
  static constexpr bool has_bytes = kBytes;
  static constexpr bool slim = kSlim;
  uint32_t key[kSub];
  uint32_t sz[kSlim ? 1 : kSub];
  uint32_t row[kSub];
  uint32_t idx[kSlim ? 1 : kSub];
  uint32_t src[kSub];       // payload offset relative to the sub-chunk's first byte
  uint32_t bpre[kBytes ? kSub + 1 : 1];  // exclusive prefix of sz in sorted order; bpre[n] = total
  uint16_t dig[kSlim ? 1 : kSub];
  uint16_t wc[kFan * kNW];  // (digit, wave) counts, then their digit-major exclusive scan
};
using SortLds = SortLdsT<kMaxFanout, true>;
constexpr int kFanBits = 1 << MGT_GEO_FANBITS;  // fan-out of a bits-mode pass

// Ranks each lane's cells stably by digit (ballot multisplit per 64-cell
// round, counters per (digit, wave)), scans the counters digit-major and
// stores the cells in sorted order. Registers hold kItems cells per lane in
// wave order (cell i = wave*kWaveCells + r*64 + lane). Ends with a barrier.
// kIdx: the cell index travels (only perm needs it). szsh: in the slim form
// with a byte prefix, a cell's size is its key word shifted right by szsh.
template <bool kIdx = true, class LT>
__device__ __forceinline__ void sort_sub(LT& L, uint32_t F, int dbits, uint32_t n,
                                         const uint32_t (&key)[kItems], const uint32_t (&dg)[kItems],
                                         const uint32_t (&sz)[kItems], const uint32_t (&row)[kItems],
                                         const uint32_t (&idx)[kItems], const uint32_t (&src)[kItems],
                                         int szsh = 0) {
  const uint32_t w = threadIdx.x / kWave, lane = lane_id();
  const uint32_t E = F * kNW;
  for (uint32_t e = threadIdx.x; e < E; e += kBlock) L.wc[e] = 0;
  __syncthreads();
  uint32_t rank[kItems];
#pragma unroll
  for (int r = 0; r < kItems; ++r) {
    const uint32_t i = w * kWaveCells + r * kWave + lane;
    const bool act = i < n;
    const uint32_t d = act ? dg[r] : 0u;
    const uint64_t peers = match_peers(d, act, dbits);
    rank[r] = 0;
    if (act) {
      const uint32_t below = popc_below(peers);
      const uint32_t old = L.wc[d * kNW + w];
      if (below == 0) L.wc[d * kNW + w] = (uint16_t)(old + (uint32_t)__popcll(peers));
      rank[r] = old + below;
    }
  }
  __syncthreads();
  {
    const uint32_t per = (E + kBlock - 1) / kBlock;
    const uint32_t e0 = threadIdx.x * per;
    uint32_t s = 0;
    for (uint32_t e = e0; e < e0 + per && e < E; ++e) s += L.wc[e];
    __shared__ uint32_t red[kNW + 1];
    uint32_t tot;
    uint32_t ex = block_excl_scan<kNW>(s, red, tot);
    for (uint32_t e = e0; e < e0 + per && e < E; ++e) {
      const uint32_t v = L.wc[e];
      L.wc[e] = (uint16_t)ex;
      ex += v;
    }
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kItems; ++r) {
    const uint32_t i = w * kWaveCells + r * kWave + lane;
    if (i < n) {
      const uint32_t p = (uint32_t)L.wc[dg[r] * kNW + w] + rank[r];
      L.key[p] = key[r];
      if constexpr (!LT::slim) L.sz[p] = sz[r];
      L.row[p] = row[r];
      if constexpr (kIdx) L.idx[p] = idx[r];
      L.src[p] = src[r];
      if constexpr (!LT::slim) L.dig[p] = (uint16_t)dg[r];
    }
  }
  __syncthreads();
  if constexpr (LT::has_bytes) {
    constexpr int kPer = kSub / kBlock;
    const uint32_t p0 = threadIdx.x * kPer;
    uint32_t v[kPer];
    uint32_t s = 0;
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      if constexpr (LT::slim) v[q] = (p0 + q < n) ? L.key[p0 + q] >> szsh : 0u;
      else v[q] = (p0 + q < n) ? L.sz[p0 + q] : 0u;
      s += v[q];
    }
    __shared__ uint32_t red2[kNW + 1];
    uint32_t tot;
    uint32_t ex = block_excl_scan<kNW>(s, red2, tot);
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      if (p0 + q < n) L.bpre[p0 + q] = ex;
      ex += v[q];
    }
    if (threadIdx.x == 0) L.bpre[n] = tot;
    __syncthreads();
  }
}

// Exclusive prefix (in cell order i = wave*kWaveCells + r*64 + lane) of the
// per-cell sizes of a sub-chunk. Returns the sub-chunk total.
__device__ __forceinline__ uint32_t sub_src_prefix(const uint32_t (&sz)[kItems], uint32_t (&src)[kItems],
                                                   uint32_t* red) {
  const uint32_t w = threadIdx.x / kWave;
  uint32_t carry = 0;
#pragma unroll
  for (int r = 0; r < kItems; ++r) {
    const uint32_t inc = wave_incl_scan_u32(sz[r]) + carry;
    src[r] = inc - sz[r];
    carry = wave_bcast(inc, kWave - 1);
  }
  if (lane_id() == 0) red[w] = carry;
  __syncthreads();
  uint32_t wbase = 0, tot = 0;
  for (uint32_t q = 0; q < (uint32_t)kNW; ++q) {
    const uint32_t t = red[q];
    if (q < w) wbase += t;
    tot += t;
  }
#pragma unroll
  for (int r = 0; r < kItems; ++r) src[r] += wbase;
  __syncthreads();
  return tot;
}

// Row owning cell k of an item, found by the whole workgroup: each round
// probes kBlock evenly spaced row offsets and keeps the last one <= k.
__device__ __forceinline__ uint32_t coop_row_search(const void* rp, int ow, uint64_t n_rows,
                                                    uint64_t k) {
  uint64_t lo = 0, hi = n_rows;  // row_ptr[lo] <= k, answer in [lo, hi)
  while (hi - lo > 1) {
    const uint64_t step = (hi - lo + kBlock - 1) / kBlock;
    const uint64_t p = lo + (uint64_t)threadIdx.x * step;
    const bool ok = p < hi && (uint64_t)ld_off(rp, p, ow) <= k;
    int c = __syncthreads_count(ok);
    c = c < 1 ? 1 : c;
    lo = lo + (uint64_t)(c - 1) * step;
    hi = min(lo + step, hi);
  }
  return (uint32_t)lo;
}

// Rows of the cells [k0, k0 + n) of an item whose first cell lies in row r0:
// counts the rows starting at each position (empty rows included) and scans
// the counts, so row(k0 + i) = r0 + incl[i]. Uses `incl` (kSub entries of
// LDS). Returns the row of cell k0 + n. Every thread must call it.
// `pf` is row_ptr[r0 + 1 + threadIdx.x] (or ~0 past the last row), loaded
// ahead of time by the caller so the first batch does not wait for memory.
// Words of row_ptr[r0 + 1 + threadIdx.x] (index clamped to n_rows; callers
// test r < n_rows themselves), loaded without a branch on the offset width;
// combine with row_word().
struct RowPf {
  uint32_t lo, hi;
};
__device__ __forceinline__ RowPf prefetch_row(const void* rp, int lg, uint64_t n_rows, uint32_t r0) {
  const uint64_t r = min((uint64_t)r0 + 1 + threadIdx.x, n_rows);
  const uint8_t* b = (const uint8_t*)rp + (r << lg);
  return RowPf{*gm((const uint32_t*)b), *gm((const uint32_t*)(b + (lg == 3 ? 4 : 0)))};
}
__device__ __forceinline__ uint64_t row_word(RowPf p, int lg) {
  return (uint64_t)p.lo | ((uint64_t)(lg == 3 ? p.hi : 0u) << 32);
}

__device__ __forceinline__ uint32_t expand_rows(const void* rp, int ow, uint64_t n_rows, uint64_t k0,
                                                uint32_t n, uint32_t r0, uint64_t pf, uint32_t* incl,
                                                uint32_t* s_extra, uint32_t* red) {
  for (uint32_t i = threadIdx.x; i < (uint32_t)kSub; i += kBlock) incl[i] = 0;
  if (threadIdx.x == 0) *s_extra = 0;
  __syncthreads();
  const uint64_t kend = k0 + n;
  // the first kBlock rows come from the prefetched value, the rest (rows
  // shorter than kSub / kBlock cells on average) are loaded here
  bool more;
  {
    bool stop = (uint64_t)r0 + 1 + threadIdx.x >= n_rows;
    if (!stop) {
      if (pf >= k0 && pf < kend) atomicAdd(&incl[pf - k0], 1u);
      else if (pf == kend) atomicAdd(s_extra, 1u);
      stop = pf > kend;
    }
    more = !__syncthreads_or(stop);
  }
  for (uint64_t base = (uint64_t)r0 + 1 + kBlock; more; base += kBlock) {
    const uint64_t r = base + threadIdx.x;
    bool stop = r >= n_rows;
    if (!stop) {
      const uint64_t v = (uint64_t)ld_off(rp, r, ow);
      if (v >= k0 && v < kend) atomicAdd(&incl[v - k0], 1u);
      else if (v == kend) atomicAdd(s_extra, 1u);
      stop = v > kend;
    }
    more = !__syncthreads_or(stop);
  }
  // inclusive scan of the per-position row counts
  constexpr int kPer = kSub / kBlock;
  const uint32_t p0 = threadIdx.x * kPer;
  uint32_t v[kPer];
  uint32_t s = 0;
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    v[q] = incl[p0 + q];
    s += v[q];
  }
  uint32_t tot;
  uint32_t ex = block_excl_scan<kNW>(s, red, tot);
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    ex += v[q];
    incl[p0 + q] = ex;
  }
  __syncthreads();
  return r0 + tot + *s_extra;
}

// Payload copies of a lane's kItems cells, split in two so the caller can
// put other work (the record stores) between the loads and the stores. When
// every cell is dword aligned on both sides and at most 32 bytes, the words
// are loaded into registers up front (`fast`) as at most three pieces per
// cell (16, 16 or 8 + 4 bytes; dword-aligned multi-dword accesses are legal
// on gfx950), so a wave moves a cell in up to three instructions instead of
// up to eight. When every cell is at most 16 bytes at any alignment
// (`small`), the loads take the one or two 16-byte-aligned blocks that hold
// its bytes (an aligned block lies within one page, so reading all of it is
// safe), and the stores write exactly the cell's bytes: bytes up to the first
// dword boundary of the destination, the dwords after it (the source bytes
// shifted into place in registers), then the remaining bytes. Otherwise the
// cells are copied one by one in the store phase (up to 32 bytes the same
// way, in two halves).
constexpr int kPay = 4;  // cells per lane whose payload words are held at once

typedef uint32_t u32x4a __attribute__((ext_vector_type(4), aligned(4)));
typedef uint32_t v4u __attribute__((ext_vector_type(4)));  // 16-byte aligned record
typedef uint32_t u32x2a __attribute__((ext_vector_type(2), aligned(4)));
// A 12-byte packed record (a three-element vector type would be padded to 16).
struct alignas(4) Rec12 {
  uint32_t x, y, z;
};
static_assert(sizeof(Rec12) == 12, "12-byte record");
template <int N>
struct PayRegsT {
  u32x4a v[N][2];
  bool fast, small;
};

// The 4 bytes at byte b (0..3) of the 8-byte value hi:lo.
__device__ __forceinline__ uint32_t funnel_bytes(uint32_t hi, uint32_t lo, uint32_t b) {
  return (uint32_t)((((uint64_t)hi << 32) | lo) >> (8u * b));
}
// a_q for q in 0..4, without indexing registers by a lane value: a
// multiplexer on the bits of q, on values (a chain of equality tests, or
// selects between elements of one array, end up as loads from scratch memory).
__device__ __forceinline__ uint32_t mux5(uint32_t q, uint32_t a0, uint32_t a1, uint32_t a2,
                                         uint32_t a3, uint32_t a4) {
  const uint32_t a = (q & 1u) ? a1 : a0;
  const uint32_t b = (q & 1u) ? a3 : a2;
  const uint32_t c = (q & 2u) ? b : a;
  return (q & 4u) ? a4 : c;
}
// The dwords 0..5 of the window w0..w8 (w9 = 0) shifted down by q (0..4)
// dwords, then the five dwords starting b (0..3) bytes into that.
struct Shifted5 {
  uint32_t m0, m1, m2, m3, m4;
};
__device__ __forceinline__ Shifted5 shift_window(uint32_t q, uint32_t b, uint32_t w0, uint32_t w1,
                                                 uint32_t w2, uint32_t w3, uint32_t w4, uint32_t w5,
                                                 uint32_t w6, uint32_t w7, uint32_t w8) {
  const uint32_t t0 = mux5(q, w0, w1, w2, w3, w4), t1 = mux5(q, w1, w2, w3, w4, w5);
  const uint32_t t2 = mux5(q, w2, w3, w4, w5, w6), t3 = mux5(q, w3, w4, w5, w6, w7);
  const uint32_t t4 = mux5(q, w4, w5, w6, w7, w8), t5 = mux5(q, w5, w6, w7, w8, 0u);
  return Shifted5{funnel_bytes(t1, t0, b), funnel_bytes(t2, t1, b), funnel_bytes(t3, t2, b),
                  funnel_bytes(t4, t3, b), funnel_bytes(t5, t4, b)};
}

// Stores the n <= 16 bytes that start at byte o (0..15) of the 32-byte window
// v (the source's aligned blocks) to dst, touching no byte outside
// [dst, dst + n).
__device__ __forceinline__ void store_small(uint8_t* dst, const u32x4a (&v)[2], uint32_t o,
                                            uint32_t n) {
  const uint32_t w0 = v[0].x, w1 = v[0].y, w2 = v[0].z, w3 = v[0].w;
  const uint32_t w4 = v[1].x, w5 = v[1].y, w6 = v[1].z, w7 = v[1].w;
  GMEM uint8_t* const d = gm(dst);
  const uint32_t hd = min((4u - ((uint32_t)(uintptr_t)dst & 3u)) & 3u, n);  // bytes before a dword boundary
  const uint32_t qh = o >> 2;
  const uint32_t hv = funnel_bytes(mux5(qh, w1, w2, w3, w4, w5), mux5(qh, w0, w1, w2, w3, w4), o & 3u);
#pragma unroll
  for (int j = 0; j < 3; ++j)
    if ((uint32_t)j < hd) d[j] = (uint8_t)(hv >> (8 * j));
  const uint32_t x = o + hd;  // the dwords after the head
  const Shifted5 m = shift_window(x >> 2, x & 3u, w0, w1, w2, w3, w4, w5, w6, w7, 0u);
  const uint32_t nm = (n - hd) >> 2, nt = (n - hd) & 3u;
  GMEM uint32_t* const da = (GMEM uint32_t*)(d + hd);
  if (nm == 4u) {
    *(GMEM u32x4a*)da = u32x4a{m.m0, m.m1, m.m2, m.m3};
  } else {
    if (nm & 2u) *(GMEM u32x2a*)da = u32x2a{m.m0, m.m1};
    if (nm & 1u) da[nm & 2u] = (nm & 2u) ? m.m2 : m.m0;
  }
  const uint32_t tv = mux5(nm, m.m0, m.m1, m.m2, m.m3, m.m4);
  GMEM uint8_t* const dt = (GMEM uint8_t*)(da + nm);
#pragma unroll
  for (int j = 0; j < 3; ++j)
    if ((uint32_t)j < nt) dt[j] = (uint8_t)(tv >> (8 * j));
}
using PayRegs = PayRegsT<kPay>;

// Copies n <= 32 bytes of any alignment the same way, in two halves: the
// 16-byte-aligned blocks that hold the cell (up to three) are loaded first.
__device__ __forceinline__ void copy_medium(uint8_t* dst, const uint8_t* src, uint32_t n) {
  const uint32_t o = (uint32_t)(uintptr_t)src & 15u;
  const GMEM v4u* const b = (const GMEM v4u*)gm(src - o);  // 16-byte aligned
  u32x4a v[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    v[k] = u32x4a{0u, 0u, 0u, 0u};
    if (o + n > 16u * (uint32_t)k) {  // block k holds a byte of the cell
      const v4u x = b[k];
      v[k] = u32x4a{x.x, x.y, x.z, x.w};
    }
  }
  const u32x4a lo[2] = {v[0], v[1]}, hi[2] = {v[1], v[2]};
  store_small(dst, lo, o, n < 16u ? n : 16u);
  if (n > 16u) store_small(dst + 16, hi, o, n - 16u);
}

template <int N>
__device__ __forceinline__ void pay_load(PayRegsT<N>& P, uint8_t* const (&dst)[N],
                                         const uint8_t* const (&src)[N],
                                         const uint32_t (&sz)[N]) {
  bool fast = true, small = true;
#pragma unroll
  for (int r = 0; r < N; ++r) {
    fast &= sz[r] == 0u ||
            (sz[r] <= 32u && ((sz[r] | (uint32_t)(uintptr_t)src[r] | (uint32_t)(uintptr_t)dst[r]) & 3u) == 0);
    small &= sz[r] <= 16u;
  }
  P.fast = fast;
  P.small = !fast && small;
  if (P.small) {
#pragma unroll
    for (int r = 0; r < N; ++r) {
      const uint32_t z = sz[r];
      const uint32_t o = (uint32_t)(uintptr_t)src[r] & 15u;
      const GMEM v4u* const b = (const GMEM v4u*)gm(src[r] - o);  // 16-byte aligned
      P.v[r][0] = u32x4a{0u, 0u, 0u, 0u};
      P.v[r][1] = u32x4a{0u, 0u, 0u, 0u};
      if (z) {
        const v4u x = b[0];
        P.v[r][0] = u32x4a{x.x, x.y, x.z, x.w};
      }
      if (o + z > 16u) {
        const v4u y = b[1];
        P.v[r][1] = u32x4a{y.x, y.y, y.z, y.w};
      }
    }
  }
  if (fast) {
#pragma unroll
    for (int r = 0; r < N; ++r) {
      const GMEM uint8_t* s = gm(src[r]);
      const uint32_t z = sz[r];
      if (z >= 16u) P.v[r][0] = *(const GMEM u32x4a*)s;
      const uint32_t o1 = z >= 16u ? 16u : 0u, rem = z - o1;
      if (rem >= 16u) {
        P.v[r][1] = *(const GMEM u32x4a*)(s + 16);
      } else {
        if (rem >= 8u) P.v[r][1].xy = *(const GMEM u32x2a*)(s + o1);
        if (rem & 4u) P.v[r][1].z = *(const GMEM uint32_t*)(s + o1 + (rem & 8u));
      }
    }
  }
}

template <int N>
__device__ __forceinline__ void pay_store(const PayRegsT<N>& P, uint8_t* const (&dst)[N],
                                          const uint8_t* const (&src)[N],
                                          const uint32_t (&sz)[N]) {
  if (P.fast) {
#pragma unroll
    for (int r = 0; r < N; ++r) {
      GMEM uint8_t* d = gm(dst[r]);
      const uint32_t z = sz[r];
      if (z >= 16u) *(GMEM u32x4a*)d = P.v[r][0];
      const uint32_t o1 = z >= 16u ? 16u : 0u, rem = z - o1;
      if (rem >= 16u) {
        *(GMEM u32x4a*)(d + 16) = P.v[r][1];
      } else {
        if (rem >= 8u) *(GMEM u32x2a*)(d + o1) = P.v[r][1].xy;
        if (rem & 4u) *(GMEM uint32_t*)(d + o1 + (rem & 8u)) = P.v[r][1].z;
      }
    }
  } else if (P.small) {
#pragma unroll
    for (int r = 0; r < N; ++r)
      if (sz[r]) store_small(dst[r], P.v[r], (uint32_t)(uintptr_t)src[r] & 15u, sz[r]);
  } else {
#pragma unroll
    for (int r = 0; r < N; ++r) {
      if (sz[r] == 0u) continue;
      if (sz[r] <= 32u) copy_medium(dst[r], src[r], sz[r]);
      else copy_cell(dst[r], src[r], sz[r]);
    }
  }
}
// ----------------------------------------------------------------------------- pass: scatter

// Loads of one sub-chunk, kept in registers so the next sub-chunk can be in
// flight while the current one is sorted and written. Every load is issued
// unconditionally (indexes clamped into the range) and nothing is computed
// from a loaded value here, so the compiler has no reason to wait for one
// load before issuing the next.
//   pass 0:   a = column, c = low word of the payload offset; `pend` = low word
//             of the offset after the wave's last cell, `base` = full offset of
//             the sub-chunk's first cell
//   pass >=1: a = column, b = size, c = row, d = cell index, and (finish after
//             a records-only pass) e, f = low and high words of the payload offset
struct SubLoad {
  uint32_t a[kItems], b[kItems], c[kItems], d[kItems], e[kItems], f[kItems];
  uint32_t pend;
  uint32_t base_lo, base_hi;  // words of the first cell's offset (hi unused for 4-byte offsets)
};
// which SubLoad fields a kernel uses
constexpr int kFieldsPass0 = 1 | 4 | 32;
constexpr int kFieldsRec = 1 | 2 | 4 | 8;
constexpr int kFieldsRecSo = kFieldsRec | 16 | 64;

// Hands a prefetch to the next iteration. The empty asm statements read each
// value, so the wait for those loads lands here, inside the iteration that
// issued them, where the compiler counts the younger memory operations
// exactly; carried through the loop edge as pending loads, their first use
// would be given a conservative (full) wait instead.
__device__ __forceinline__ uint32_t settled(uint32_t v) {
  asm volatile("" : "+v"(v));
  return v;
}
template <int kFields>
__device__ __forceinline__ void settle(SubLoad& dst, const SubLoad& src) {
#pragma unroll
  for (int r = 0; r < kItems; ++r) {
    if (kFields & 1) dst.a[r] = settled(src.a[r]);
    if (kFields & 2) dst.b[r] = settled(src.b[r]);
    if (kFields & 4) dst.c[r] = settled(src.c[r]);
    if (kFields & 8) dst.d[r] = settled(src.d[r]);
    if (kFields & 16) dst.e[r] = settled(src.e[r]);
    if (kFields & 64) dst.f[r] = settled(src.f[r]);
  }
  if (kFields & 32) {
    dst.pend = settled(src.pend);
    dst.base_lo = settled(src.base_lo);
    dst.base_hi = settled(src.base_hi);
  }
}

// fw >= 0: fixed-width cells; their offsets are k * fw and nothing is loaded
// for them. val: per-cell carried values (view operations), into d.
__device__ __forceinline__ void load_sub_pass0(SubLoad& S, const int32_t* col, const void* poff,
                                               uint64_t kfirst, uint32_t n, int lg, int32_t fw,
                                               const uint32_t* val, uint32_t tid = threadIdx.x) {
  const uint32_t w = tid / kWave, lane = tid % kWave;
#pragma unroll
  for (int r = 0; r < kItems; ++r) {
    const uint32_t i = w * kWaveCells + r * kWave + lane;
    S.a[r] = (uint32_t)gm(col)[kfirst + min(i, n - 1)];
    if (val) S.d[r] = gm(val)[kfirst + min(i, n - 1)];
  }
  const uint64_t kend = kfirst + min(w * kWaveCells + kWaveCells, n);
  if (fw >= 0) {
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
      const uint32_t i = w * kWaveCells + r * kWave + lane;
      S.c[r] = (uint32_t)((kfirst + min(i, n)) * (uint64_t)fw);
    }
    S.pend = (uint32_t)(kend * (uint64_t)fw);
    const uint64_t b = kfirst * (uint64_t)fw;
    S.base_lo = (uint32_t)b;
    S.base_hi = (uint32_t)(b >> 32);
  } else {
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
      const uint32_t i = w * kWaveCells + r * kWave + lane;
      S.c[r] = ld_lo(poff, kfirst + min(i, n), lg);  // the offset array has one more entry
    }
    S.pend = ld_lo(poff, kend, lg);
    const uint8_t* b = (const uint8_t*)poff + (kfirst << lg);
    S.base_lo = *gm((const uint32_t*)b);
    S.base_hi = *gm((const uint32_t*)(b + (lg == 3 ? 4 : 0)));
  }
}

__device__ __forceinline__ void load_sub_rec(SubLoad& S, const uint2* ks, const uint2* rk,
                                             const uint32_t* rso, uint64_t pos0, uint32_t n,
                                             uint32_t tid = threadIdx.x) {
  const uint32_t w = tid / kWave, lane = tid % kWave;
#pragma unroll
  for (int r = 0; r < kItems; ++r) {
    const uint32_t i = min(w * kWaveCells + r * kWave + lane, n - 1);
    const uint2 x = ks[pos0 + i];
    S.a[r] = x.x; S.b[r] = x.y;
    if (rso) {  // (row, cell index, payload offset) records of a records-only pass
      const v4u y = gm((const v4u*)rso)[pos0 + i];
      S.c[r] = y.x; S.d[r] = y.y; S.e[r] = y.z; S.f[r] = y.w;
    } else {
      const uint2 y = rk[pos0 + i];
      S.c[r] = y.x; S.d[r] = y.y;
    }
  }
}

// Packed records (a single matrix with one records-only pass, no perm): after
// the first pass a cell is (column | size << pk_shift, row), after the second
// (column | size << pk_shift, row, payload offset as two words).
__device__ __forceinline__ void load_sub_pk8(SubLoad& S, const uint2* ks, uint64_t pos0, uint32_t n,
                                             uint32_t tid = threadIdx.x) {
  const uint32_t w = tid / kWave, lane = tid % kWave;
#pragma unroll
  for (int r = 0; r < kItems; ++r) {
    const uint32_t i = min(w * kWaveCells + r * kWave + lane, n - 1);
    const uint2 x = ks[pos0 + i];
    S.a[r] = x.x; S.c[r] = x.y;
  }
}
// rec12: 12-byte records whose third word is the payload offset minus the
// bucket's first byte `byte0`, as a signed 32-bit value.
__device__ __forceinline__ void load_sub_pk16(SubLoad& S, const uint32_t* rso, uint64_t pos0,
                                              uint32_t n, bool rec12, uint64_t byte0) {
  const uint32_t w = threadIdx.x / kWave, lane = lane_id();
  if (rec12) {
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
      const uint32_t i = min(w * kWaveCells + r * kWave + lane, n - 1);
      const GMEM Rec12* const y = gm((const Rec12*)rso) + pos0 + i;
      const uint64_t off = byte0 + (uint64_t)(int64_t)(int32_t)y->z;
      S.a[r] = y->x; S.c[r] = y->y; S.e[r] = (uint32_t)off; S.f[r] = (uint32_t)(off >> 32);
    }
  } else {
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
      const uint32_t i = min(w * kWaveCells + r * kWave + lane, n - 1);
      const v4u y = gm((const v4u*)rso)[pos0 + i];
      S.a[r] = y.x; S.c[r] = y.y; S.e[r] = y.z; S.f[r] = y.w;
    }
  }
}
constexpr int kFieldsPk8 = 1 | 4;
// First pass of a packed call: (column | size << pk_shift) per cell, written
// by the first histogram into the level buffer the first pass leaves unused
// (indexed like the level buffers), and the payload offset of the sub-chunk's
// first cell (item-local index kfirst) from the offsets or the fixed width.
__device__ __forceinline__ void load_sub_pk4(SubLoad& S, const uint32_t* pk4, const void* poff,
                                             uint64_t kfirst, uint64_t lfirst, uint32_t n, int lg,
                                             int32_t fw,
                                             uint32_t tid = threadIdx.x) {
  const uint32_t w = tid / kWave, lane = tid % kWave;
#pragma unroll
  for (int r = 0; r < kItems; ++r) {
    const uint32_t i = w * kWaveCells + r * kWave + lane;
    S.a[r] = gm(pk4)[lfirst + min(i, n - 1)];
  }
  S.pend = 0;
  if (fw >= 0) {
    const uint64_t b = kfirst * (uint64_t)fw;
    S.base_lo = (uint32_t)b;
    S.base_hi = (uint32_t)(b >> 32);
  } else {
    const uint8_t* b = (const uint8_t*)poff + (kfirst << lg);
    S.base_lo = *gm((const uint32_t*)b);
    S.base_hi = *gm((const uint32_t*)(b + (lg == 3 ? 4 : 0)));
  }
}
constexpr int kFieldsPk4 = 1 | 32;
constexpr int kFieldsPk16 = 1 | 4 | 16 | 64;

// Payload sizes of a pass-0 sub-chunk from the low offset words: each cell's
// size is the next cell's offset minus its own (the next cell is the next
// lane, or lane 0 of the next register, or the wave's `pend`).
__device__ __forceinline__ void sizes_from_offsets(const SubLoad& S, uint32_t (&sz)[kItems]) {
  const uint32_t lane = lane_id();
#pragma unroll
  for (int r = 0; r < kItems; ++r) {
    uint32_t nx = (uint32_t)__shfl_down((int)S.c[r], 1);
    const uint32_t wrap = r + 1 < kItems ? (uint32_t)__builtin_amdgcn_readlane((int)S.c[r + 1 < kItems ? r + 1 : r], 0)
                                         : S.pend;
    if (lane == kWave - 1) nx = wrap;
    sz[r] = nx - S.c[r];
  }
}

// kPk: packed records (see load_sub_pk8); only the first pass of a plain
// (not view) call and the records-only pass have a packed form.
template <bool kPass0, bool kDefer, bool kVal, bool kPk, bool kKeys, class Lds, bool kSlimParts = false>
__device__ __forceinline__ void scatter_body(const PassArgs& a, Lds& L, uint32_t* s_rc,
                                             uint64_t* s_rb, int32_t* s_lb, uint16_t* s_ot,
                                             Seg& s_seg, uint32_t& s_si, uint32_t& s_extra,
                                             uint32_t* s_red) {
  // the slim forms run only segments split by column bits, except the slim
  // first pass built for partitions (kSlimParts)
  constexpr bool kBitsOnly = Lds::slim && !kSlimParts;
  const uint64_t tile = xcd_tile(blockIdx.x, a.g8);
  if (tile >= a.tstart[a.nseg]) return;
  {
    const uint32_t si = coop_find_seg(a.tstart, a.nseg, tile);
    if (threadIdx.x == 0) {
      s_si = si;
      s_seg = a.segs[si];
    }
  }
  __syncthreads();
  const Seg sg = s_seg;
  const uint32_t si = s_si;
  const ItemDev* it = &a.items[sg.item];
  const uint32_t R = (uint32_t)it->n_parts;
  const uint32_t F = seg_fanout(sg, R);
  const int dbits = ceil_log2(F);
  const int ow = a.offset_width;
  const uint64_t j = tile - a.tstart[si];
  const uint64_t nt = a.tstart[si + 1] - a.tstart[si];
  const uint64_t hb = a.hstart[si];
  const uint64_t c_begin = j * a.tile_cells;
  const uint64_t c_end = min((uint64_t)sg.len, c_begin + a.tile_cells);
  constexpr bool pass0 = kPass0;
  constexpr bool kPk4 = kPass0 && kPk && kKeys;  // first pass reading the histogram's key words
  constexpr int kFields = kPass0 ? (kVal ? kFieldsPass0 | 8 : (kPk4 ? kFieldsPk4 : kFieldsPass0))
                                 : (kPk ? kFieldsPk8 : kFieldsRec);
  const uint32_t* const pk4 = (const uint32_t*)a.rk_out;  // first pass of a packed call
  const uint64_t kbase = sg.cell0 - it->cell_base;  // pass 0: item-local index of the segment
  const bool track_xfer = !kBitsOnly && pass0 && sg.mode && it->xfer_cells;
  // item fields used in the loop, read once
  const int32_t* const i_col = it->col;
  const void* const i_poff = it->poff;
  const void* const i_rp = it->row_ptr;
  const uint64_t i_nrows = (uint64_t)it->n_rows;
  const uint8_t* const i_pay = it->payload;
  const uint64_t i_pbytes = (uint64_t)it->payload_bytes;
  const int32_t i_fw = it->fixed_w;
  const int pk_shift = it->pk_shift;  // packed records: column bits
  const uint32_t pk_mask = (uint32_t)((1ull << pk_shift) - 1u);
  const int lg = ow == 8 ? 3 : 2;  // (4-byte offsets keep every payload below 2^31 bytes)
  const uint64_t seg_out = sg.cell0;  // a segment's children share its cell range

  if constexpr (kBitsOnly) {
    if (sg.mode) {  // (the launcher never gives it such a segment)
      if (threadIdx.x == 0) raise_status(a.item_status, a.abort_flag, it->status_index, MGT_EUNSUPPORTED);
      return;
    }
  } else if constexpr (kPass0) {
    if (sg.mode)
      for (uint32_t i = threadIdx.x; i <= R; i += kBlock) s_lb[i] = (int32_t)gm(it->bounds)[i];
  }
  // 12-byte packed records (slim records-only pass): each cell's payload
  // offset is stored relative to the first byte of the finish bucket it
  // lands in, digit d's child, kept in s_rb (block-uniform choice)
  const bool rec12 = Lds::slim && a.rec12 && *(volatile const int32_t*)a.big_seg == 0;
  for (uint32_t d = threadIdx.x; d < F; d += kBlock) {
    s_rc[d] = (uint32_t)(a.ocnt[hb + (uint64_t)d * nt + j] - seg_out);
    if constexpr (!kDefer) s_rb[d] = a.obyt[hb + (uint64_t)d * nt + j];
    else if constexpr (Lds::slim) s_rb[d] = a.obyt[hb + (uint64_t)d * nt];
  }
  uint32_t r0 = 0;
  RowPf rpf{0, 0}, rpf_next{0, 0};
  if constexpr (pass0 && !kVal) {
    r0 = coop_row_search(i_rp, ow, i_nrows, kbase + c_begin);
    rpf_next = prefetch_row(i_rp, lg, i_nrows, r0);
    rpf = RowPf{settled(rpf_next.lo), settled(rpf_next.hi)};
  }
  __syncthreads();
  int osh = 0;
  if constexpr (kPass0 && !kBitsOnly) {
    if (sg.mode) {  // block-uniform
      osh = owner_shift(s_lb[R]);
      fill_owner_table(s_lb, R, osh, s_ot);
      __syncthreads();
    }
  }
  uint64_t src_sub = pass0 ? 0 : a.tsrc[tile];  // level-buffer byte of the sub-chunk (pass >= 2)

  SubLoad cur, nxt;
  {
    const uint32_t n0 = (uint32_t)min((uint64_t)kSub, c_end - c_begin);
    if constexpr (kPk4) load_sub_pk4(nxt, pk4, i_poff, kbase + c_begin, sg.cell0 + c_begin, n0, lg,
                                             i_fw);
    else if constexpr (pass0) load_sub_pass0(nxt, i_col, i_poff, kbase + c_begin, n0, lg, i_fw,
                                        kVal ? it->vval : nullptr);
    else if constexpr (kPk) load_sub_pk8(nxt, a.ks_in, sg.cell0 + c_begin, n0);
    else load_sub_rec(nxt, a.ks_in, a.rk_in, nullptr, sg.cell0 + c_begin, n0);
    settle<kFields>(cur, nxt);  // the loop's first iteration then starts from settled registers too
  }
  for (uint64_t c0 = c_begin; c0 < c_end; c0 += kSub) {
    // the thread index, opaque to the compiler inside each iteration: the
    // per-cell indexes derived from it are recomputed here instead of being
    // hoisted out of the loop (and spilled)
    const uint32_t tid = settled((uint32_t)threadIdx.x);
    const uint32_t w = tid / kWave, lane = tid % kWave;
    const uint32_t n = (uint32_t)min((uint64_t)kSub, c_end - c0);
    const uint64_t c1 = c0 + kSub;
    uint32_t key[kItems], dg[kItems], sz[kItems], row[kItems], idx[kItems], src[kItems];
    uint64_t sub_base;
    uint32_t first_row = 0, last_row = 0;
    if constexpr (pass0) {
      const uint64_t kf = kbase + c0;
      sub_base = (uint64_t)cur.base_lo | ((uint64_t)(lg == 3 ? cur.base_hi : 0u) << 32);
      uint32_t r_next = 0;
      if constexpr (!kVal) {
        r_next = expand_rows(i_rp, ow, i_nrows, kf, n, r0, row_word(rpf, lg), L.bpre, &s_extra,
                             s_red);
        rpf_next = prefetch_row(i_rp, lg, i_nrows, r_next);  // next sub-chunk's rows
      }
      if constexpr (kPk4) {
#pragma unroll
        for (int r = 0; r < kItems; ++r) {
          const uint32_t i = w * kWaveCells + r * kWave + lane;
          sz[r] = i < n ? cur.a[r] >> pk_shift : 0u;
        }
        sub_src_prefix(sz, src, s_red);  // offsets within the sub-chunk, from the sizes
      } else {
        sizes_from_offsets(cur, sz);
      }
#pragma unroll
      for (int r = 0; r < kItems; ++r) {
        const uint32_t i = w * kWaveCells + r * kWave + lane;
        key[r] = kPk ? cur.a[r] & pk_mask : cur.a[r];
        if constexpr (!kPk4) src[r] = cur.c[r] - (uint32_t)sub_base;  // the sub-chunk spans under 2^32 bytes
        if constexpr (kVal) row[r] = cur.d[r];
        else row[r] = i < n ? r0 + L.bpre[i] : 0u;
        idx[r] = (uint32_t)(kf + i);
      }
      if constexpr (!kVal) {
        first_row = r0;
        last_row = r0 + L.bpre[n - 1];
        r0 = r_next;
        __syncthreads();  // rows consumed before sort_sub reuses the buffer
      }
    } else {
      sub_base = src_sub;
#pragma unroll
      for (int r = 0; r < kItems; ++r) {
        const uint32_t i = w * kWaveCells + r * kWave + lane;
        if constexpr (kPk) {
          key[r] = cur.a[r] & pk_mask; sz[r] = i < n ? cur.a[r] >> pk_shift : 0u;
          row[r] = cur.c[r]; idx[r] = 0u;
        } else {
          key[r] = cur.a[r]; sz[r] = i < n ? cur.b[r] : 0u; row[r] = cur.c[r]; idx[r] = cur.d[r];
        }
      }
      src_sub += sub_src_prefix(sz, src, s_red);
    }
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
      const uint32_t i = w * kWaveCells + r * kWave + lane;
      if constexpr (kBitsOnly) dg[r] = i < n ? digit_bits(key[r], sg) : 0u;
      else dg[r] = i < n ? digit_of(key[r], sg, s_lb, s_ot, osh, R) : 0u;
    }
    // Slim first pass split by column bits: a wave's cells are consecutive
    // input cells, so their payloads form one byte range of the input. One
    // dword of each of its 128-byte lines (up to 128 lines, 16 KB) is read
    // now, so that the payload gathers after the sort find the lines in the
    // caches instead of waiting on HBM. Each dword read lies in an aligned
    // line holding at least one byte of the range (the same page). The
    // values are consumed after the sort, where the wait is free.
    uint32_t touch[2] = {0u, 0u};
    if constexpr (kPass0 && kBitsOnly) {
      uint32_t whi = 0;  // end of the wave's range, relative to the sub-chunk
#pragma unroll
      for (int r = 0; r < kItems; ++r) {
        const uint32_t i = w * kWaveCells + r * kWave + lane;
        if (i < n) whi = max(whi, src[r] + sz[r]);
      }
#pragma unroll
      for (int o = kWave / 2; o >= 1; o >>= 1) whi = max(whi, (uint32_t)__shfl_xor((int)whi, o, kWave));
      const uint64_t b0 = sub_base + (uint32_t)__builtin_amdgcn_readfirstlane((int)src[0]);
      const uint64_t b1 = min(sub_base + whi, i_pbytes);
      if (w * kWaveCells < n && b0 < b1) {  // wave-uniform
        const uintptr_t p0 = (uintptr_t)(i_pay + b0) & ~(uintptr_t)127;
        const uintptr_t pe = (uintptr_t)(i_pay + b1);
#pragma unroll
        for (int k = 0; k < 2; ++k) {
          const uintptr_t q = p0 + ((uintptr_t)(k * kWave + lane) << 7);
          if (q < pe) touch[k] = *(const GMEM uint32_t*)q;
        }
      }
    }
    // The next sub-chunk's loads go out once this one's registers have been
    // read (the wait counter is in order, so a use of the current loads after
    // issuing these would wait for these too) and fly during the sort.
    if (c1 < c_end) {
      const uint32_t n1 = (uint32_t)min((uint64_t)kSub, c_end - c1);
      if constexpr (kPk4) load_sub_pk4(nxt, pk4, i_poff, kbase + c1, sg.cell0 + c1, n1, lg, i_fw, tid);
      else if constexpr (pass0) load_sub_pass0(nxt, i_col, i_poff, kbase + c1, n1, lg, i_fw,
                                          kVal ? it->vval : nullptr, tid);
      else if constexpr (kPk) load_sub_pk8(nxt, a.ks_in, sg.cell0 + c1, n1, tid);
      else load_sub_rec(nxt, a.ks_in, a.rk_in, nullptr, sg.cell0 + c1, n1, tid);
    }
    if constexpr (Lds::slim) {  // packed records: the whole (column | size) word
      static_assert(kPk, "the slim LDS form is for packed records");
      uint32_t kw[kItems];  // (a first pass reading columns packs the word here)
#pragma unroll
      for (int r = 0; r < kItems; ++r) kw[r] = (kDefer || kPk4) ? cur.a[r] : key[r] | (sz[r] << pk_shift);
      sort_sub<false>(L, F, dbits, n, kw, dg, sz, row, idx, src, pk_shift);
      if constexpr (kPass0 && kBitsOnly) asm volatile("" ::"v"(touch[0]), "v"(touch[1]));
    } else {
      sort_sub<!kPk>(L, F, dbits, n, key, dg, sz, row, idx, src);
    }

    const uint8_t* src_base = pass0 ? i_pay + sub_base : a.pay_in + sub_base;
    bool xfer_per_cell = false;
    uint32_t src_part = 0;
    if (track_xfer) {
      src_part = owner_of(s_lb, R, (int64_t)first_row);
      xfer_per_cell = owner_of(s_lb, R, (int64_t)last_row) != src_part;
    }
    if constexpr (kDefer) {
      // records only: each cell's payload stays where it is in the input
      // level buffer, and its byte offset there goes with the record
#pragma unroll
      for (int r = 0; r < kItems; ++r) {
        const uint32_t i = r * kBlock + tid;
        if (i < n) {
          uint32_t d;
          if constexpr (Lds::slim) d = digit_bits(L.key[i] & pk_mask, sg);
          else d = L.dig[i];
          const uint64_t cd = seg_out + s_rc[d] + (i - L.wc[d * kNW]);
          const uint64_t so = sub_base + L.src[i];
          v4u rec;
          if constexpr (Lds::slim) {
            if (rec12) {
              const uint32_t rel = (uint32_t)(so - s_rb[d]);  // |so - byte0| < 2^31
              GMEM Rec12* const q = gm((Rec12*)a.rso_out) + cd;
              q->x = L.key[i];
              q->y = L.row[i];
              q->z = rel;
              continue;
            }
            rec.x = L.key[i];
            rec.y = L.row[i];
          } else if constexpr (kPk) {
            rec.x = L.key[i] | (L.sz[i] << pk_shift);
            rec.y = L.row[i];
          } else {
            a.ks_out[cd] = make_uint2(L.key[i], L.sz[i]);
            rec.x = L.row[i];
            rec.y = L.idx[i];
          }
          rec.z = (uint32_t)so;
          rec.w = (uint32_t)(so >> 32);
          gm((v4u*)a.rso_out)[cd] = rec;
        }
      }
    }
    // write the sorted cells at their digit's running destination, kPayN
    // cells per lane at a time (two in the slim form, which has fewer
    // registers): payload loads first, then the records, then the payload
    // stores
    if constexpr (!kDefer) {
    constexpr int kPayN = Lds::slim ? 2 : kPay;
#pragma unroll
    for (int g = 0; g < kItems; g += kPayN) {
      uint8_t* pd[kPayN];
      const uint8_t* ps[kPayN];
      uint32_t pz[kPayN];
      uint64_t cdst[kPayN];
#pragma unroll
      for (int q = 0; q < kPayN; ++q) {
        const uint32_t i = (g + q) * kBlock + tid;
        pz[q] = 0;
        pd[q] = a.pay_out;
        ps[q] = src_base;
        cdst[q] = 0;
        if (i < n) {
          uint32_t d;
          if constexpr (Lds::slim) {  // size and digit from the (column | size) word
            const uint32_t kw = L.key[i];
            if constexpr (kBitsOnly) d = digit_bits(kw & pk_mask, sg);
            else d = digit_of(kw & pk_mask, sg, s_lb, s_ot, osh, R);
            pz[q] = kw >> pk_shift;
          } else {
            d = L.dig[i];
            pz[q] = L.sz[i];
          }
          const uint32_t ds = L.wc[d * kNW];
          cdst[q] = seg_out + s_rc[d] + (i - ds);
          pd[q] = a.pay_out + s_rb[d] + (L.bpre[i] - L.bpre[ds]);
          ps[q] = src_base + L.src[i];
        }
      }
      PayRegsT<kPayN> P;
      pay_load(P, pd, ps, pz);
#pragma unroll
      for (int q = 0; q < kPayN; ++q) {
        const uint32_t i = (g + q) * kBlock + tid;
        if (i < n) {
          const uint64_t cd = cdst[q];
          if constexpr (Lds::slim) {
            a.ks_out[cd] = make_uint2(L.key[i], L.row[i]);  // the whole (column | size) word
          } else if constexpr (kPk) {
            // a masked column keeps the size intact whatever the input holds
            a.ks_out[cd] = make_uint2((L.key[i] & pk_mask) | (pz[q] << pk_shift), L.row[i]);
          } else {
            a.ks_out[cd] = make_uint2(L.key[i], pz[q]);
            a.rk_out[cd] = make_uint2(L.row[i], L.idx[i]);
          }
        }
        if (!kBitsOnly && xfer_per_cell) {  // the sub-chunk spans source partitions (uniform)
          uint32_t key = 0;
          if (i < n) {
            const uint32_t sp = owner_lut(s_lb, s_ot, osh, R, (int64_t)L.row[i]);
            uint32_t di;
            if constexpr (Lds::slim) di = digit_of(L.key[i] & pk_mask, sg, s_lb, s_ot, osh, R);
            else di = L.dig[i];
            key = sp * R + (di >> sg.bits);
          }
          wave_add_xfer(i < n, key, pz[q], (uint64_t*)it->xfer_cells, (uint64_t*)it->xfer_bytes);
        }
      }
      pay_store(P, pd, ps, pz);
    }
    }
    if (track_xfer && !xfer_per_cell) {
      const uint32_t sub = 1u << sg.bits;
      for (uint32_t p = threadIdx.x; p < R; p += kBlock) {
        const uint32_t d0 = p << sg.bits, d1 = d0 + sub;
        const uint32_t i0 = L.wc[d0 * kNW];
        const uint32_t i1 = d1 < F ? L.wc[d1 * kNW] : n;
        if (i1 > i0) {
          add_u64((uint64_t*)&it->xfer_cells[(uint64_t)src_part * R + p], (uint64_t)(i1 - i0));
          add_u64((uint64_t*)&it->xfer_bytes[(uint64_t)src_part * R + p],
                  (uint64_t)(L.bpre[i1] - L.bpre[i0]));
        }
      }
    }
    __syncthreads();
    for (uint32_t d = threadIdx.x; d < F; d += kBlock) {
      const uint32_t i0 = L.wc[d * kNW];
      const uint32_t i1 = d + 1 < F ? L.wc[(d + 1) * kNW] : n;
      s_rc[d] += i1 - i0;
      if constexpr (!kDefer) s_rb[d] += L.bpre[i1] - L.bpre[i0];
    }
    __syncthreads();
    settle<kFields>(cur, nxt);
    if constexpr (pass0 && !kVal) rpf = RowPf{settled(rpf_next.lo), settled(rpf_next.hi)};
  }
}

// One instance per kind of pass, so the loop has no branch between the two
// load layouts: a branch there makes the compiler reconcile the registers of
// in-flight loads at the join, which waits for them. The packed and wide
// record forms are two loops of one kernel, chosen once per workgroup.
// The records-only pass keeps no byte prefix and no byte cursors, and only a
// bits-mode fan-out: under 53 KB of LDS and 168 VGPRs, so three workgroups fit
// on a CU instead of two.
// kVal (first pass only): every cell carries a value of its own (item vval)
// in place of its row id, so no rows are expanded.
// kSlim: packed records only, in the slim LDS form. The 512-thread
// records-only pass (about 58 KB, two workgroups per CU), or the 256-thread
// first pass of matrices split by column bits (about 38 KB with the byte
// prefix, three workgroups per CU instead of two: 161 VGPRs, two payload
// cells per lane in flight). It leaves a call whose records could not be
// packed to the plain kernel launched beside it, which in turn leaves packed
// calls to it (pk_split).
template <bool kPass0, bool kDefer, bool kVal, bool kSlim = false, bool kSlimParts = false,
          bool kSlimCols = false>
__global__ __launch_bounds__(kBlock, kSlim ? (kPass0 ? 768 / kBlock : 2048 / kBlock) : (kDefer ? 768 / kBlock : 2))
void k_pass_scatter(PassArgs a) {
  static_assert(!kSlim || (kPass0 != kDefer && !kVal), "slim: a packed first or records-only pass");
  static_assert(!(kSlimParts || kSlimCols) || (kSlim && kPass0), "forms of the slim first pass");
  // only the first pass may split by partition (its slim form up to a fan-out of 512)
  constexpr int kFan = kPass0 ? (kSlim ? (kSlimParts ? 2 << kMaxPassBits : 1 << kMaxPassBits) : kMaxFanout)
                              : kFanBits;
  constexpr bool kParts = kPass0 && (!kSlim || kSlimParts);
  __shared__ SortLdsT<kFan, !kDefer, kSlim> L;
  __shared__ uint32_t s_rc[kFan];                       // running destination cell per digit (segment relative)
  __shared__ uint64_t s_rb[kDefer && !kSlim ? 1 : kFan];  // running destination byte per digit
                                                          // (slim records-only: each child's first byte)
  __shared__ int32_t s_lb[kParts ? kMaxParts + 1 : 1];  // partition bounds (partition mode)
  __shared__ uint16_t s_ot[kParts ? kOwnerT + 1 : 1];   // their coarse owner table
  __shared__ Seg s_seg;
  __shared__ uint32_t s_si, s_extra;
  __shared__ uint32_t s_red[kNW + 1];
  if (aborted(a.abort_flag)) return;
  if constexpr (kSlim) {
    if (packed_records(a.pk_on, a.no_pack)) {
      if constexpr (kPass0)
        scatter_body<true, false, false, true, !kSlimCols, decltype(L), kSlimParts>(
            a, L, s_rc, s_rb, s_lb, s_ot, s_seg, s_si, s_extra, s_red);
      else
        scatter_body<false, true, false, true, false>(a, L, s_rc, s_rb, s_lb, s_ot, s_seg, s_si,
                                                      s_extra, s_red);
    }
    return;
  } else {
  if constexpr (!kVal && kPass0 != kDefer) {
    if (packed_records(a.pk_on, a.no_pack)) {
      if (a.pk_split) return;  // the slim kernel takes it
      if (kPass0 && a.pk_keys)
        scatter_body<kPass0, kDefer, kVal, true, true>(a, L, s_rc, s_rb, s_lb, s_ot, s_seg, s_si,
                                                       s_extra, s_red);
      else
        scatter_body<kPass0, kDefer, kVal, true, false>(a, L, s_rc, s_rb, s_lb, s_ot, s_seg, s_si,
                                                        s_extra, s_red);
      return;
    }
  }
  scatter_body<kPass0, kDefer, kVal, false, false>(a, L, s_rc, s_rb, s_lb, s_ot, s_seg, s_si,
                                                   s_extra, s_red);
  }
}

// (the 512-thread copy of this file needs only the records-only scatter)
#ifndef MGT_WIDE
// ----------------------------------------------------------------------------- view keys

// Sort key and carried value of every cell for LocalTranspose and ViewSwap
// (Section 3). Both are stable sorts of the cells by a key, so they run
// through the same passes as the transpose, with the key in place of the
// column and the value in place of the row id. X is the matrix the views
// represent (n_rows x n_cols, partitions V_p = [b_p, b_p+1)). A row-view input
// is X's CSR; a column-view input stores partition s (X restricted to the
// columns V_s) as a CSR over all rows, partition after partition (virtual row
// v = s * n_rows + i).
//   LocalTranspose, row view:    key = owner(i) * n_cols + j, value i
//   LocalTranspose, column view: key = j,                     value i
//   ViewSwap, row view:          key = owner(j) * n_rows + i, value j
//   ViewSwap, column view:       key = i,                     value j
// With validation, a column outside [0, n_cols) or, in column view, outside
// its partition's range sets MGT_ERANGE.
__global__ __launch_bounds__(kBlock) void k_view_keys(ViewArgs a) {
  __shared__ uint32_t incl[kSub];
  __shared__ int32_t s_lb[kMaxParts + 1];
  __shared__ uint16_t s_ot[kOwnerT + 1];
  __shared__ uint32_t s_extra;
  __shared__ uint32_t s_red[kNW + 1];
  if (aborted(a.abort_flag)) return;
  const ItemDev& it = a.items[0];
  const uint32_t R = (uint32_t)a.n_parts;
  for (uint32_t i = threadIdx.x; i <= R; i += kBlock) s_lb[i] = (int32_t)gm(a.bounds)[i];
  __syncthreads();
  const int osh = owner_shift(s_lb[R]);
  fill_owner_table(s_lb, R, osh, s_ot);
  __syncthreads();
  const uint64_t k0 = (uint64_t)blockIdx.x * kSub;
  if (k0 >= a.nnz) return;
  const uint32_t n = (uint32_t)min((uint64_t)kSub, a.nnz - k0);
  const int ow = a.offset_width, lg = ow == 8 ? 3 : 2;
  const uint32_t r0 = coop_row_search(it.row_ptr, ow, a.n_virtual, k0);
  const RowPf pf = prefetch_row(it.row_ptr, lg, a.n_virtual, r0);
  expand_rows(it.row_ptr, ow, a.n_virtual, k0, n, r0, row_word(pf, lg), incl, &s_extra, s_red);
  bool bad = false;
  for (uint32_t i = threadIdx.x; i < n; i += kBlock) {
    const uint64_t k = k0 + i;
    const uint64_t v = (uint64_t)r0 + incl[i];  // virtual row of cell k
    const int64_t j = gm(a.col)[k];
    uint64_t key, val;
    if (!a.column_view) {
      key = a.op == 0 ? (uint64_t)owner_lut(s_lb, s_ot, osh, R, (int64_t)v) * (uint64_t)a.n_cols + (uint64_t)j
                      : (uint64_t)owner_lut(s_lb, s_ot, osh, R, j) * (uint64_t)a.n_rows + v;
      val = a.op == 0 ? v : (uint64_t)j;
      if (a.validate && (j < 0 || j >= a.n_cols)) bad = true;
    } else {
      const uint64_t s = v / (uint64_t)a.n_rows, i_row = v - s * (uint64_t)a.n_rows;
      key = a.op == 0 ? (uint64_t)j : i_row;
      val = a.op == 0 ? i_row : (uint64_t)j;
      if (a.validate && (j < 0 || j >= a.n_cols || owner_lut(s_lb, s_ot, osh, R, j) != s)) bad = true;
    }
    gm(a.keys)[k] = (uint32_t)key;
    gm(a.vals)[k] = (uint32_t)val;
  }
  if (__syncthreads_or(bad)) {
    if (threadIdx.x == 0) raise_status(a.item_status, a.abort_flag, it.status_index, MGT_ERANGE);
  }
}

// ----------------------------------------------------------------------------- finish

// An item's tails, by one whole block: the caller's status word,
// t_row_ptr[n_cols] and t_payload_off[nnz], and for a partitioned item the
// partition offsets (column sums of X and B, scanned) and both displacement
// matrices (Section 2 step 2; Alltoallv displacements). Partitions are split
// in runs of `per` per thread, up to kMaxParts / kBlock.
constexpr int kTailPer = (kMaxParts + kBlock - 1) / kBlock;
__device__ void item_tails(const ItemDev& it, uint32_t i, const int32_t* item_status,
                           const int32_t* abort_flag, int ow, int32_t* d_status, uint64_t* red) {
  if (d_status && threadIdx.x == 0) {
    const int32_t st = item_status[i];
    d_status[i] = (st == MGT_OK && *abort_flag) ? MGT_ECANCELED : st;
  }
  if (aborted(abort_flag)) return;
  if (threadIdx.x == 0) {
    st_off(it.t_row_ptr, (uint64_t)it.n_cols, it.nnz, ow);
    if (it.t_poff) st_off(it.t_poff, (uint64_t)it.nnz, it.payload_bytes, ow);
  }
  if (!it.part_mode || !it.xfer_cells) return;
  const uint32_t R = (uint32_t)it.n_parts;
  const uint64_t rr = (uint64_t)R * R;
  if (it.nnz == 0) {  // no first-pass tile cleared the transfer matrices
    for (uint64_t e = threadIdx.x; e < rr; e += kBlock) {
      it.xfer_cells[e] = 0;
      it.xfer_bytes[e] = 0;
    }
    __syncthreads();
  }
  const uint32_t per = (R + kBlock - 1) / kBlock;  // <= kTailPer
  const uint32_t s0 = threadIdx.x * per;
  uint64_t cs[kTailPer], bs[kTailPer], cells = 0, bytes = 0;
#pragma unroll
  for (int k = 0; k < kTailPer; ++k) {  // cells / bytes received by partition s0 + k
    cs[k] = bs[k] = 0;
    const uint32_t s = s0 + (uint32_t)k;
    if ((uint32_t)k < per && s < R)
      for (uint32_t r = 0; r < R; ++r) {
        cs[k] += (uint64_t)it.xfer_cells[(uint64_t)r * R + s];
        bs[k] += (uint64_t)it.xfer_bytes[(uint64_t)r * R + s];
      }
    cells += cs[k];
    bytes += bs[k];
  }
  uint64_t tc, tb;
  uint64_t ec = block_excl_scan<kNW>(cells, red, tc);
  uint64_t eb = block_excl_scan<kNW>(bytes, red, tb);
#pragma unroll
  for (int k = 0; k < kTailPer; ++k) {
    const uint32_t s = s0 + (uint32_t)k;
    if ((uint32_t)k < per && s < R) {
      if (it.part_cell_off) it.part_cell_off[s] = (int64_t)ec;
      if (it.part_byte_off) it.part_byte_off[s] = (int64_t)eb;
    }
    ec += cs[k];
    eb += bs[k];
  }
  if (threadIdx.x == 0) {
    if (it.part_cell_off) it.part_cell_off[R] = (int64_t)tc;
    if (it.part_byte_off) it.part_byte_off[R] = (int64_t)tb;
  }
  for (uint32_t s = threadIdx.x; s < R; s += kBlock) {
    if (it.sdispls) {  // row s of X scanned along destinations
      int64_t acc = 0;
      for (uint32_t d = 0; d < R; ++d) {
        it.sdispls[(uint64_t)s * R + d] = acc;
        acc += it.xfer_cells[(uint64_t)s * R + d];
      }
    }
    if (it.rdispls) {  // column s of X scanned along sources
      int64_t acc = 0;
      for (uint32_t r = 0; r < R; ++r) {
        it.rdispls[(uint64_t)s * R + r] = acc;
        acc += it.xfer_cells[(uint64_t)r * R + s];
      }
    }
  }
}

// kGather: the last pass moved records only; each cell's payload is read
// from the previous level buffer at the bucket's src0 plus the cell's stored
// offset. Otherwise payloads follow the records in the same level buffer.
// kPk (gathering finish only): the last pass's records are packed (see
// load_sub_pk16); no cell index travels, so no perm is written.
template <bool kGather, bool kPk>
__device__ __forceinline__ void finish_body(const FinishArgs& a, SortLds& L, uint32_t* s_cc,
                                            uint64_t* s_cb, uint32_t* s_red, uint64_t* s_red64) {
  constexpr int kFields = kGather ? (kPk ? kFieldsPk16 : kFieldsRecSo) : kFieldsRec;
  const uint32_t* const so = kGather ? a.rso_in : nullptr;
  // packed records of 12 bytes (block-uniform; see PassArgs::rec12)
  const bool rec12 = kPk && a.rec12 && *(volatile const int32_t*)a.big_seg == 0;
  const uint64_t bk = kGather ? (uint64_t)blockIdx.x : xcd_tile(blockIdx.x, a.g8);
  if (bk >= a.nbuckets) return;
  const Seg sg = a.buckets[bk];
  const ItemDev* it = &a.items[sg.item];
  const int pk_shift = it->pk_shift;  // packed records: column bits
  const uint32_t pk_mask = (uint32_t)((1ull << pk_shift) - 1u);
  const int ow = a.offset_width;
  const uint32_t nc = sg.key_hi - sg.key_lo;
  if (nc == 0) return;
  const int dbits = ceil_log2(nc);
  const uint64_t out_cell0 = sg.cell0 - it->cell_base;
  const uint64_t out_byte0 = sg.byte0 - it->byte_base;
  const uint32_t len = sg.len;
  const bool multi = len > (uint32_t)kSub;
  const uint32_t w = threadIdx.x / kWave, lane = lane_id();
  void* t_row_ptr = it->t_row_ptr;
  uint8_t* const o_pay = it->t_payload;
  int32_t* const o_col = it->t_col;
  uint32_t* const o_perm = (uint32_t*)it->perm;
  void* const o_poff = it->t_poff;

  if (multi) {
    for (uint32_t c = threadIdx.x; c < nc; c += kBlock) {
      s_cc[c] = 0;
      s_cb[c] = 0;
    }
    __syncthreads();
    constexpr uint32_t kStride = kBlock * kBatch;
    for (uint32_t c0 = 0; c0 < len; c0 += kStride) {  // same trip count on all lanes
      const uint32_t c = c0 + threadIdx.x;
      uint2 ks[kBatch];
#pragma unroll
      for (int q = 0; q < kBatch; ++q) {
        const uint64_t e = sg.cell0 + min(c + q * kBlock, len - 1);
        if constexpr (kPk) {
          const uint32_t x = gm(so)[(rec12 ? 3u : 4u) * e];
          ks[q] = make_uint2(x & pk_mask, x >> pk_shift);
        } else {
          ks[q] = a.ks_in[e];
        }
      }
#pragma unroll
      for (int q = 0; q < kBatch; ++q) {
        const bool act = c + q * kBlock < len;
        uint32_t d = ks[q].x - sg.key_lo;
        d = d < nc ? d : nc - 1;
        hist_add_runs(act, d, ks[q].y, s_cc, (unsigned long long*)s_cb);
      }
    }
    __syncthreads();
    const uint32_t per = (nc + kBlock - 1) / kBlock;
    const uint32_t e0 = threadIdx.x * per;
    uint32_t s = 0;
    uint64_t sb = 0;
    for (uint32_t e = e0; e < e0 + per && e < nc; ++e) {
      s += s_cc[e];
      sb += s_cb[e];
    }
    uint32_t tot;
    uint64_t totb;
    uint32_t ex = block_excl_scan<kNW>(s, s_red, tot);
    uint64_t exb = block_excl_scan<kNW>(sb, s_red64, totb);
    for (uint32_t e = e0; e < e0 + per && e < nc; ++e) {
      const uint32_t v = s_cc[e];
      const uint64_t vb = s_cb[e];
      s_cc[e] = ex;
      s_cb[e] = exb;
      st_off(t_row_ptr, (uint64_t)sg.key_lo + e, (int64_t)(out_cell0 + ex), ow);
      ex += v;
      exb += vb;
    }
    __syncthreads();
  }

  uint64_t src_sub = sg.byte0;  // level-buffer byte of the current sub-chunk's first cell
  SubLoad cur, nxt;
  if (len) {
    if constexpr (kPk) load_sub_pk16(nxt, so, sg.cell0, min((uint32_t)kSub, len), rec12, sg.byte0);
    else load_sub_rec(nxt, a.ks_in, a.rk_in, so, sg.cell0, min((uint32_t)kSub, len));
    settle<kFields>(cur, nxt);
  }
  for (uint32_t c0 = 0; c0 < len || (c0 == 0 && !multi); c0 += kSub) {
    const uint32_t n = min((uint32_t)kSub, len - c0);
    const uint32_t c1 = c0 + kSub;
    uint32_t key[kItems], dg[kItems], sz[kItems], row[kItems], idx[kItems], src[kItems];
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
      const uint32_t i = w * kWaveCells + r * kWave + lane;
      if constexpr (kPk) {
        key[r] = cur.a[r] & pk_mask; sz[r] = i < n ? cur.a[r] >> pk_shift : 0u;
        row[r] = cur.c[r]; idx[r] = 0u;
      } else {
        key[r] = cur.a[r]; sz[r] = i < n ? cur.b[r] : 0u; row[r] = cur.c[r]; idx[r] = cur.d[r];
      }
      const uint32_t d = key[r] - sg.key_lo;
      dg[r] = i < n ? (d < nc ? d : nc - 1) : 0u;
    }
    uint32_t subtot = 0;
    if constexpr (kGather) {
      // the column is not needed after the sort here, so its LDS slot carries
      // the high word of the payload offset through it
#pragma unroll
      for (int r = 0; r < kItems; ++r) {
        src[r] = cur.e[r];
        key[r] = cur.f[r];
      }
    } else {
      subtot = sub_src_prefix(sz, src, s_red);
    }
    // next sub-chunk's loads, issued after this one's registers were read
    if (c1 < len) {
      if constexpr (kPk)
        load_sub_pk16(nxt, so, sg.cell0 + c1, min((uint32_t)kSub, len - c1), rec12, sg.byte0);
      else load_sub_rec(nxt, a.ks_in, a.rk_in, so, sg.cell0 + c1, min((uint32_t)kSub, len - c1));
    }
    sort_sub<!kPk>(L, nc, dbits, n, key, dg, sz, row, idx, src);
    if (!multi) {
      // one sub-chunk: its digit scan is the column layout of the whole bucket
      for (uint32_t c = threadIdx.x; c < nc; c += kBlock)
        st_off(t_row_ptr, (uint64_t)sg.key_lo + c, (int64_t)(out_cell0 + L.wc[c * kNW]), ow);
    }
    const uint8_t* src_base = a.pay_in + (kGather ? 0 : src_sub);
#pragma unroll
    for (int g = 0; g < kItems; g += kPay) {
      uint8_t* pd[kPay];
      const uint8_t* ps[kPay];
      uint32_t pz[kPay];
      uint64_t pp[kPay], pb[kPay];
#pragma unroll
      for (int q = 0; q < kPay; ++q) {
        const uint32_t i = (g + q) * kBlock + threadIdx.x;
        pz[q] = 0;
        pd[q] = o_pay;
        ps[q] = src_base;
        pp[q] = 0;
        pb[q] = 0;
        if (i < n) {
          if (multi) {
            const uint32_t d = L.dig[i];
            const uint32_t ds = L.wc[d * kNW];
            pp[q] = out_cell0 + s_cc[d] + (i - ds);
            pb[q] = out_byte0 + s_cb[d] + (L.bpre[i] - L.bpre[ds]);
          } else {
            pp[q] = out_cell0 + i;
            pb[q] = out_byte0 + L.bpre[i];
          }
          pz[q] = L.sz[i];
          pd[q] = o_pay + pb[q];
          ps[q] = src_base + (kGather ? ((uint64_t)L.key[i] << 32 | L.src[i]) : (uint64_t)L.src[i]);
        }
      }
      PayRegs P;
      pay_load(P, pd, ps, pz);
#pragma unroll
      for (int q = 0; q < kPay; ++q) {
        const uint32_t i = (g + q) * kBlock + threadIdx.x;
        if (i < n) {
          gm(o_col)[pp[q]] = (int32_t)L.row[i];
          if constexpr (!kPk)  // packed records carry no cell index (no perm)
            if (o_perm) gm(o_perm)[pp[q]] = L.idx[i];
          if (o_poff) st_off(o_poff, pp[q], (int64_t)pb[q], ow);
        }
      }
      pay_store(P, pd, ps, pz);
    }
    __syncthreads();
    if (multi) {
      for (uint32_t d = threadIdx.x; d < nc; d += kBlock) {
        const uint32_t i0 = L.wc[d * kNW];
        const uint32_t i1 = d + 1 < nc ? L.wc[(d + 1) * kNW] : n;
        s_cc[d] += i1 - i0;
        s_cb[d] += L.bpre[i1] - L.bpre[i0];
      }
      __syncthreads();
    }
    src_sub += subtot;
    settle<kFields>(cur, nxt);
    if (len == 0) break;
  }
}

template <bool kGather>
__global__ __launch_bounds__(kBlock, 2) void k_finish(FinishArgs a) {
  __shared__ SortLds L;
  __shared__ uint32_t s_cc[kFinishCols];  // per column: first output cell (bucket relative)
  __shared__ uint64_t s_cb[kFinishCols];  // per column: first output byte (bucket relative)
  __shared__ uint32_t s_red[kNW + 1];
  __shared__ uint64_t s_red64[kNW + 1];
  // Gathering finishes run their buckets in plain column order on all XCDs
  // at once: the buckets in flight then read from one or two source segments
  // (tens of MB, resident in the memory-side cache) instead of eight.
  // Block i < n_items also writes item i's tails. This comes first: after an
  // abort the bucket table below was never written, and only the status
  // words are.
  if (blockIdx.x < a.n_items)
    item_tails(a.items[blockIdx.x], blockIdx.x, a.item_status, a.abort_flag, a.offset_width,
               a.d_status, s_red64);
  if (aborted(a.abort_flag)) return;
  if constexpr (kGather) {
    if (packed_records(a.pk_on, a.no_pack)) {
      // buckets k_finish_bucket wrote are done
      if (a.bucket_done && blockIdx.x < a.nbuckets && a.bucket_done[blockIdx.x]) return;
      finish_body<kGather, true>(a, L, s_cc, s_cb, s_red, s_red64);
      return;
    }
  }
  finish_body<kGather, false>(a, L, s_cc, s_cb, s_red, s_red64);
}

// ----------------------------------------------------------------------------- whole-bucket finish

// A gathering finish with packed records (two passes, no perm) sorts a bucket
// of up to kBkCap cells in one piece: its records are read once, ranked by
// column with a ballot multisplit (each wave holds a contiguous run of
// kBkWaveCells cells, so wave order is cell order and the ranks are stable),
// placed in LDS in output order, and written out in that order. Consecutive
// output cells then go to consecutive addresses of t_col, t_payload_off and
// t_payload (whole lines); only the payload reads are scattered, inside one
// first-pass segment. A persistent grid walks the buckets in column order
// (all CUs on neighbouring buckets, so their payload sources share a segment
// held in the memory-side cache). A bucket it does not take (more cells than
// fit, payload sources spanning 2^32 bytes or more, 2^32 payload bytes or
// more) is marked 0 in bucket_done and left to k_finish, which skips those
// marked 1. A bucket of 2^7 columns of the large multigraph holds 8,192 cells
// on average and at most 8,834, under kBkCap.
constexpr int kBkPay = 2;  // cells per lane whose payload is in flight

// Two geometries: 1,024 threads (one workgroup per CU, ten cells per lane:
// buckets of up to 10,240 cells, 156 KB of LDS) and 512 threads (two
// workgroups per CU, nine cells per lane: up to 4,608 cells, 80 KB each).
// With two per CU, one workgroup's loads and LDS sort run while the other
// gathers, so the CU keeps L2 misses in flight through every phase. A tenth
// cell per lane would slow the 512-thread form, whose buckets stay under
// 4,608 cells anyway when it is chosen.
template <int kBkBlock>
struct BkGeo {
  static constexpr int kNW = kBkBlock / kWave;
  static constexpr int kItems = kBkBlock >= 1024 ? 10 : 9;  // cells per lane
  static constexpr int kCap = kBkBlock * kItems;            // cells of a bucket held at once
  static constexpr int kWaveCells = kItems * kWave;         // contiguous cells of one wave
};

template <int kBkBlock>
struct BucketLds {
  static constexpr int kBkNW = BkGeo<kBkBlock>::kNW, kBkCap = BkGeo<kBkBlock>::kCap;
  uint32_t row[kBkCap];              // output order: original row id
  uint32_t src[kBkCap];              // output order: payload offset above the bucket's lowest
  uint32_t bp[kBkCap + 1];           // output order: size, then its exclusive prefix
  uint16_t wc[kFinishCols * kBkNW];  // (column, wave) counts, then their column-major scan
  uint64_t lo[kBkNW], hi[kBkNW], tot[kBkNW];
  uint32_t red[kBkNW + 1];
  uint32_t next;                     // skip mode: the next bucket left by an earlier launch
};

__device__ __forceinline__ uint64_t wave_min_u64(uint64_t v) {
#pragma unroll
  for (int o = kWave / 2; o >= 1; o >>= 1) {
    const uint64_t u = __shfl_xor(v, o, kWave);
    v = u < v ? u : v;
  }
  return v;
}
__device__ __forceinline__ uint64_t wave_max_u64(uint64_t v) {
#pragma unroll
  for (int o = kWave / 2; o >= 1; o >>= 1) {
    const uint64_t u = __shfl_xor(v, o, kWave);
    v = u > v ? u : v;
  }
  return v;
}
__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
#pragma unroll
  for (int o = kWave / 2; o >= 1; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

// A bucket k_finish_bucket can hold (block-uniform).
template <int kBkBlock>
__device__ __forceinline__ bool bucket_loadable(const Seg& s) {
  return s.key_hi > s.key_lo && s.len > 0 && s.len <= (uint32_t)BkGeo<kBkBlock>::kCap;
}

// The bucket's packed records, wave w holding cells
// [w * kBkWaveCells, (w + 1) * kBkWaveCells) (clamped into the bucket), each
// as (column | size, row, payload offset low and high words). rec12: the
// records are 12 bytes, the offset stored relative to the bucket's first byte.
template <int kBkItems>
__device__ __forceinline__ void load_bucket(v4u (&r)[kBkItems], const uint32_t* rso, const Seg& s,
                                            uint32_t tid, bool rec12) {
  constexpr int kBkWaveCells = kBkItems * kWave;
  const uint32_t w = tid / kWave, lane = tid % kWave;
  if (rec12) {
#pragma unroll
    for (int q = 0; q < kBkItems; ++q) {
      const uint32_t i = min(w * kBkWaveCells + q * kWave + lane, s.len - 1);
      const GMEM Rec12* const t = gm((const Rec12*)rso) + s.cell0 + i;
      const uint64_t off = s.byte0 + (uint64_t)(int64_t)(int32_t)t->z;
      r[q] = v4u{t->x, t->y, (uint32_t)off, (uint32_t)(off >> 32)};
    }
  } else {
#pragma unroll
    for (int q = 0; q < kBkItems; ++q) {
      const uint32_t i = min(w * kBkWaveCells + q * kWave + lane, s.len - 1);
      r[q] = gm((const v4u*)rso)[s.cell0 + i];
    }
  }
}

template <int kBkItems>
__device__ __forceinline__ void zero_bucket(v4u (&r)[kBkItems]) {
#pragma unroll
  for (int q = 0; q < kBkItems; ++q) r[q] = v4u{0u, 0u, 0u, 0u};
}

template <int kBkBlock>
__global__ __launch_bounds__(kBkBlock, 4) void k_finish_bucket(FinishArgs a) {
  constexpr int kBkNW = BkGeo<kBkBlock>::kNW;
  constexpr int kBkItems = BkGeo<kBkBlock>::kItems;
  constexpr int kBkCap = BkGeo<kBkBlock>::kCap;
  constexpr int kBkWaveCells = BkGeo<kBkBlock>::kWaveCells;
  __shared__ BucketLds<kBkBlock> L;
  if (aborted(a.abort_flag) || !packed_records(a.pk_on, a.no_pack)) return;
  const bool rec12 = a.rec12 && *(volatile const int32_t*)a.big_seg == 0;  // block-uniform
  const uint32_t nb = a.nbuckets;
  uint32_t bk = blockIdx.x;
  if (bk >= nb) return;
  const int ow = a.offset_width;
  Seg sg = a.buckets[bk];
  for (; bk < nb; bk += gridDim.x) {
    if (a.skip_done) {
      // this workgroup's next bucket that an earlier launch left (its flags
      // read kBkBlock at a time), or none
      for (;;) {
        const uint32_t cand = bk + threadIdx.x * gridDim.x;
        const bool left = cand < nb && !a.bucket_done[cand];
        if (threadIdx.x == 0) L.next = ~0u;
        __syncthreads();
        if (left) atomicMin(&L.next, (uint32_t)threadIdx.x);
        __syncthreads();
        const uint32_t first = L.next;
        __syncthreads();
        const uint64_t nxt = first != ~0u ? (uint64_t)bk + (uint64_t)first * gridDim.x
                                          : (uint64_t)bk + (uint64_t)kBkBlock * gridDim.x;
        bk = nxt < nb ? (uint32_t)nxt : nb;
        if (first != ~0u || bk >= nb) break;
      }
      if (bk >= nb) break;
      sg = a.buckets[bk];
    }
    // the thread index, opaque to the compiler inside each iteration: the
    // per-cell indexes derived from it are recomputed here instead of being
    // hoisted out of the loop (and spilled)
    const uint32_t tid = settled((uint32_t)threadIdx.x);
    const uint32_t w = tid / kWave, lane = tid % kWave;
    const uint32_t bn = bk + gridDim.x;
    Seg sn = sg;
    if (bn < nb) sn = a.buckets[bn];
    v4u cur[kBkItems];
    if (bucket_loadable<kBkBlock>(sg)) load_bucket(cur, a.rso_in, sg, tid, rec12);
    else zero_bucket(cur);
    const ItemDev* it = &a.items[sg.item];
    const uint32_t nc = sg.key_hi - sg.key_lo;
    const uint32_t len = sg.len;
    const bool take = nc > 0 && len <= (uint32_t)kBkCap;  // block-uniform
    const uint64_t out_cell0 = sg.cell0 - it->cell_base;
    const uint64_t out_byte0 = sg.byte0 - it->byte_base;
    const int pk_shift = it->pk_shift;
    const uint32_t pk_mask = (uint32_t)((1ull << pk_shift) - 1u);
    bool fits = false;
    uint64_t blo = 0;
    if (take) {
      // digits, the lowest and highest payload byte and the total
      uint32_t dg[kBkItems], rank[kBkItems];
      uint64_t lo = ~0ull, hi = 0, tb = 0;
#pragma unroll
      for (int q = 0; q < kBkItems; ++q) {
        const uint32_t i = w * kBkWaveCells + q * kWave + lane;
        const uint32_t x = cur[q].x;
        const uint32_t sz = x >> pk_shift;
        const uint64_t off = (uint64_t)cur[q].z | ((uint64_t)cur[q].w << 32);
        uint32_t d = (x & pk_mask) - sg.key_lo;
        d = d < nc ? d : nc - 1;
        dg[q] = i < len ? d : 0u;
        if (i < len) {
          lo = off < lo ? off : lo;
          hi = off + sz > hi ? off + sz : hi;
          tb += sz;
        }
      }
      lo = wave_min_u64(lo);
      hi = wave_max_u64(hi);
      tb = wave_sum_u64(tb);
      if (lane == 0) {
        L.lo[w] = lo;
        L.hi[w] = hi;
        L.tot[w] = tb;
      }
      const uint32_t E = nc * kBkNW;
      for (uint32_t e = tid; e < E; e += kBkBlock) L.wc[e] = 0;
      __syncthreads();
      uint64_t bhi = 0, btot = 0;
      blo = ~0ull;
#pragma unroll
      for (int q = 0; q < kBkNW; ++q) {
        blo = L.lo[q] < blo ? L.lo[q] : blo;
        bhi = L.hi[q] > bhi ? L.hi[q] : bhi;
        btot += L.tot[q];
      }
      fits = len == 0 || (bhi - blo < (1ull << 32) && btot < (1ull << 32));
      if (len == 0) blo = 0;
      if (fits) {
        // stable ranks: per (column, wave) counters, each wave in cell order
        const int dbits = ceil_log2(nc);
#pragma unroll
        for (int q = 0; q < kBkItems; ++q) {
          const uint32_t i = w * kBkWaveCells + q * kWave + lane;
          const bool act = i < len;
          const uint64_t peers = match_peers(dg[q], act, dbits);
          rank[q] = 0;
          if (act) {
            const uint32_t below = popc_below(peers);
            const uint32_t old = L.wc[dg[q] * kBkNW + w];
            if (below == 0) L.wc[dg[q] * kBkNW + w] = (uint16_t)(old + (uint32_t)__popcll(peers));
            rank[q] = old + below;
          }
        }
        __syncthreads();
        {  // column-major exclusive scan of the counters: each column's first output cell
          const uint32_t per = (E + kBkBlock - 1) / kBkBlock;
          const uint32_t e0 = tid * per;
          uint32_t sum = 0;
          for (uint32_t e = e0; e < e0 + per && e < E; ++e) sum += L.wc[e];
          uint32_t tot;
          uint32_t ex = block_excl_scan<kBkNW>(sum, L.red, tot);
          for (uint32_t e = e0; e < e0 + per && e < E; ++e) {
            const uint32_t v = L.wc[e];
            L.wc[e] = (uint16_t)ex;
            ex += v;
          }
        }
        __syncthreads();
        for (uint32_t c = tid; c < nc; c += kBkBlock)
          st_off(it->t_row_ptr, (uint64_t)sg.key_lo + c, (int64_t)(out_cell0 + L.wc[c * kBkNW]), ow);
#pragma unroll
        for (int q = 0; q < kBkItems; ++q) {
          const uint32_t i = w * kBkWaveCells + q * kWave + lane;
          if (i < len) {
            const uint32_t p = (uint32_t)L.wc[dg[q] * kBkNW + w] + rank[q];
            const uint64_t off = (uint64_t)cur[q].z | ((uint64_t)cur[q].w << 32);
            L.row[p] = cur[q].y;
            L.src[p] = (uint32_t)(off - blo);
            L.bp[p] = cur[q].x >> pk_shift;
          }
        }
        __syncthreads();
      }
    }
    if (take && fits) {
      {  // sizes -> exclusive byte prefix in output order (kBkItems positions per lane)
        uint32_t v[kBkItems];
        uint32_t sum = 0;
#pragma unroll
        for (int q = 0; q < kBkItems; ++q) {
          const uint32_t p = tid * kBkItems + q;
          v[q] = p < len ? L.bp[p] : 0u;
          sum += v[q];
        }
        uint32_t tot;
        uint32_t ex = block_excl_scan<kBkNW>(sum, L.red, tot);
#pragma unroll
        for (int q = 0; q < kBkItems; ++q) {
          const uint32_t p = tid * kBkItems + q;
          if (p < len) L.bp[p] = ex;
          ex += v[q];
        }
        if (tid == 0) L.bp[len] = tot;
        __syncthreads();
      }
      // outputs in output order, kBkPay cells per lane with their payload
      // loads in flight before the stores
      uint8_t* const o_pay = it->t_payload;
      int32_t* const o_col = it->t_col;
      void* const o_poff = it->t_poff;
      const uint8_t* const src_base = a.pay_in + blo;
      // (kept rolled: with its three copy paths the body is too large to
      // unroll five times)
#pragma unroll 1
      for (int g = 0; g < kBkItems; g += kBkPay) {
        uint8_t* pd[kBkPay];
        const uint8_t* ps[kBkPay];
        uint32_t pz[kBkPay], pr[kBkPay], pb[kBkPay];
#pragma unroll
        for (int q = 0; q < kBkPay; ++q) {
          const uint32_t p = (uint32_t)(g + q) * kBkBlock + tid;
          pz[q] = 0;
          pr[q] = 0;
          pb[q] = 0;
          pd[q] = o_pay;
          ps[q] = src_base;
          if (p < len) {
            pb[q] = L.bp[p];
            pz[q] = L.bp[p + 1] - pb[q];
            pr[q] = L.row[p];
            pd[q] = o_pay + out_byte0 + pb[q];
            ps[q] = src_base + L.src[p];
          }
        }
        // Payloads of dword sizes up to 32 bytes at dword addresses (every cell
        // of the large workloads) take the staged path: each lane loads its
        // cell in whole 16-byte pieces (reading up to 12 bytes past it, inside
        // the level buffer's padding), the wave packs its 64 cells' bytes in
        // LDS in output order, and writes them back as 16 contiguous bytes
        // per lane. Payloads of up to 16 bytes at any alignment (`ustaged`)
        // pass through LDS too: each lane loads the 16-byte-aligned blocks
        // that hold its cell, shifts its bytes to their place in the wave's
        // run and ORs them into the zeroed stage, and the run is written back
        // 16 bytes per lane, with dword and byte stores at its two ends.
        // Other payloads are copied lane by lane.
        PayRegsT<kBkPay> P;
        bool staged = true, small = true;
#pragma unroll
        for (int q = 0; q < kBkPay; ++q) {
          staged &= pz[q] == 0u ||
                    (pz[q] <= 32u &&
                     ((pz[q] | (uint32_t)(uintptr_t)ps[q] | (uint32_t)(uintptr_t)pd[q]) & 3u) == 0);
          small &= pz[q] <= 16u;
        }
        staged = __all(staged);
        const bool ustaged = !staged && __all(small);
        if (staged) {
#pragma unroll
          for (int q = 0; q < kBkPay; ++q) {
            const GMEM uint8_t* sp = gm(ps[q]);
            if (pz[q]) P.v[q][0] = *(const GMEM u32x4a*)sp;
            if (pz[q] > 16u) P.v[q][1] = *(const GMEM u32x4a*)(sp + 16);
          }
        } else if (ustaged) {
#pragma unroll
          for (int q = 0; q < kBkPay; ++q) {
            const uint32_t o = (uint32_t)(uintptr_t)ps[q] & 15u;
            const GMEM v4u* const bk = (const GMEM v4u*)gm(ps[q] - o);  // 16-byte aligned
            P.v[q][0] = u32x4a{0u, 0u, 0u, 0u};
            P.v[q][1] = u32x4a{0u, 0u, 0u, 0u};
            if (pz[q]) {
              const v4u x = bk[0];
              P.v[q][0] = u32x4a{x.x, x.y, x.z, x.w};
            }
            if (o + pz[q] > 16u) {
              const v4u y = bk[1];
              P.v[q][1] = u32x4a{y.x, y.y, y.z, y.w};
            }
          }
        } else {
          pay_load(P, pd, ps, pz);
        }
#pragma unroll
        for (int q = 0; q < kBkPay; ++q) {
          const uint32_t p = (uint32_t)(g + q) * kBkBlock + tid;
          if (p < len) {
            gm(o_col)[out_cell0 + p] = (int32_t)pr[q];
            if (o_poff) st_off(o_poff, out_cell0 + p, (int64_t)(out_byte0 + pb[q]), ow);
          }
        }
        if (staged) {
          // the counters' LDS is free once the column scan is done: 2 KB per
          // wave holds 64 payloads of up to 32 bytes
          uint32_t* const stage = (uint32_t*)L.wc + w * (kWave * 8);
#pragma unroll
          for (int q = 0; q < kBkPay; ++q) {
            const uint32_t p = (uint32_t)(g + q) * kBkBlock + tid;
            const uint64_t act = ballot(p < len);  // a prefix of the wave's lanes
            if (act == 0) continue;                // wave-uniform
            const uint32_t last = 63u - (uint32_t)__clzll(act);
            const uint32_t b0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)pb[q]);
            const uint32_t rel = pb[q] - b0;
            const uint32_t tot =
                (uint32_t)__builtin_amdgcn_readlane((int)(rel + pz[q]), (int)last);
            const uint32_t nw = pz[q] >> 2;
            const uint32_t v[8] = {P.v[q][0].x, P.v[q][0].y, P.v[q][0].z, P.v[q][0].w,
                                   P.v[q][1].x, P.v[q][1].y, P.v[q][1].z, P.v[q][1].w};
#pragma unroll
            for (int j = 0; j < 8; ++j)
              if ((uint32_t)j < nw) stage[(rel >> 2) + j] = v[j];
            GMEM uint8_t* const dst = gm(o_pay + out_byte0 + b0);
            for (uint32_t o = lane * 16u; o < tot; o += kWave * 16u) {
              const uint32_t* sw = stage + (o >> 2);
              if (o + 16u <= tot) {
                *(GMEM u32x4a*)(dst + o) = u32x4a{sw[0], sw[1], sw[2], sw[3]};
              } else {
                for (uint32_t j = 0; j < ((tot - o) >> 2); ++j) ((GMEM uint32_t*)(dst + o))[j] = sw[j];
              }
            }
          }
        } else if (ustaged) {
          // stage dword 0 holds the dword-aligned address below the run's
          // first byte; a run of 64 cells of up to 16 bytes spans at most 257
          // of the wave's 512 stage dwords
          uint32_t* const stage = (uint32_t*)L.wc + w * (kWave * 8);
#pragma unroll
          for (int q = 0; q < kBkPay; ++q) {
            const uint32_t p = (uint32_t)(g + q) * kBkBlock + tid;
            const uint64_t act = ballot(p < len);  // a prefix of the wave's lanes
            if (act == 0) continue;                // wave-uniform
            const uint32_t last = 63u - (uint32_t)__clzll(act);
            const uint32_t b0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)pb[q]);
            const uint32_t rel = pb[q] - b0;
            const uint32_t tot =
                (uint32_t)__builtin_amdgcn_readlane((int)(rel + pz[q]), (int)last);
            uint8_t* const run = o_pay + out_byte0 + b0;
            const uint32_t sh = (uint32_t)(uintptr_t)run & 3u;
            const uint32_t end = sh + tot;  // stage bytes [sh, end) are the run's
            for (uint32_t e = lane; e < ((end + 3u) >> 2); e += kWave) stage[e] = 0u;
            const uint32_t z = pz[q];
            if (z) {
              const uint32_t sb = sh + rel, r = sb & 3u, d0 = sb >> 2;
              // the window with a zero dword in front, so the shift is >= 0
              const uint32_t x = ((uint32_t)(uintptr_t)ps[q] & 15u) + 4u - r;  // 1..19
              const Shifted5 m = shift_window(x >> 2, x & 3u, 0u, P.v[q][0].x, P.v[q][0].y,
                                              P.v[q][0].z, P.v[q][0].w, P.v[q][1].x, P.v[q][1].y,
                                              P.v[q][1].z, P.v[q][1].w);
              const uint32_t mv[5] = {m.m0, m.m1, m.m2, m.m3, m.m4};
              const uint32_t nd = (r + z + 3u) >> 2;
#pragma unroll
              for (int k = 0; k < 5; ++k) {
                if ((uint32_t)k < nd) {
                  const int lo = min(max((int)r - 4 * k, 0), 4);
                  const int hi = min(max((int)(r + z) - 4 * k, 0), 4);
                  const uint32_t mk = (hi >= 4 ? ~0u : (1u << (8 * hi)) - 1u) & ~((1u << (8 * lo)) - 1u);
                  __hip_atomic_fetch_or(&stage[d0 + k], mv[k] & mk, __ATOMIC_RELAXED,
                                        __HIP_MEMORY_SCOPE_WORKGROUP);
                }
              }
            }
            GMEM uint8_t* const base = gm(run - sh);  // dword aligned
            for (uint32_t o = lane * 16u; o < end; o += kWave * 16u) {
              const uint32_t* sw = stage + (o >> 2);
              if (o >= sh && o + 16u <= end) {
                *(GMEM u32x4a*)(base + o) = u32x4a{sw[0], sw[1], sw[2], sw[3]};
              } else {
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                  const uint32_t a0 = o + 4u * (uint32_t)j;
                  if (a0 >= sh && a0 + 4u <= end) {
                    *(GMEM uint32_t*)(base + a0) = sw[j];
                  } else {
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                      if (a0 + (uint32_t)i >= sh && a0 + (uint32_t)i < end)
                        base[a0 + (uint32_t)i] = (uint8_t)(sw[j] >> (8 * i));
                  }
                }
              }
            }
          }
        } else {
          pay_store(P, pd, ps, pz);
        }
      }
    }
    if (tid == 0) a.bucket_done[bk] = (take && fits) ? 1 : 0;
    __syncthreads();  // LDS is reused by the next bucket
    sg = sn;
  }
}

// ----------------------------------------------------------------------------- children

__global__ __launch_bounds__(kBlock) void k_children(ChildArgs a) {
  if (aborted(a.abort_flag)) return;
  const uint32_t si = blockIdx.x;
  const Seg sg = a.segs[si];
  const ItemDev* it = &a.items[sg.item];
  const uint32_t R = (uint32_t)it->n_parts;
  const uint32_t F = seg_fanout(sg, R);
  const uint64_t nt = a.tstart[si + 1] - a.tstart[si];
  const uint64_t hb = a.hstart[si];
  const uint32_t next = a.pass + 1;
  const uint32_t nbits = next < (uint32_t)it->n_levels ? (uint32_t)it->bits[next] : 0u;
  const uint64_t cbase = it->seg_base[next] + (uint64_t)(si - it->seg_base[a.pass]) * F;
  const uint32_t rb = sg.shift;  // bits spanned by one child's column range
  for (uint32_t d = threadIdx.x; d < F; d += kBlock) {
    uint64_t c0, c1, b0, b1;
    if (nt) {
      c0 = a.ocnt[hb + (uint64_t)d * nt];
      c1 = a.ocnt[hb + (uint64_t)(d + 1) * nt];
      b0 = a.obyt[hb + (uint64_t)d * nt];
      b1 = a.obyt[hb + (uint64_t)(d + 1) * nt];
    } else {
      c0 = c1 = sg.cell0;
      b0 = b1 = sg.byte0;
    }
    uint64_t lo, hi;
    if (sg.mode == 0) {
      lo = (uint64_t)sg.key_lo + ((uint64_t)d << sg.shift);
      hi = lo + (1ull << sg.shift);
      lo = lo < sg.key_hi ? lo : sg.key_hi;
      hi = hi < sg.key_hi ? hi : sg.key_hi;
    } else {
      const uint32_t p = d >> sg.bits, jj = d & ((1u << sg.bits) - 1u);
      const uint64_t blo = (uint64_t)it->bounds[p], bhi = (uint64_t)it->bounds[p + 1];
      lo = blo + ((uint64_t)jj << sg.shift);
      hi = lo + (1ull << sg.shift);
      lo = lo < bhi ? lo : bhi;
      hi = hi < bhi ? hi : bhi;
    }
    Seg ch;
    ch.cell0 = c0;
    ch.byte0 = b0;
    ch.len = (uint32_t)(c1 - c0);
    ch.key_lo = (uint32_t)lo;
    ch.key_hi = (uint32_t)hi;
    ch.item = sg.item;
    ch.bits = nbits;
    ch.shift = rb >= nbits ? rb - nbits : 0u;
    ch.mode = 0;
    ch.pad = 0;
    if (a.big_seg && b1 - b0 >= (1ull << 31)) *a.big_seg = 1;  // 12-byte records cannot reach
    a.children[cbase + d] = ch;
    if (a.child_tiles) {
      const uint32_t tiles = (uint32_t)((ch.len + a.tile_cells - 1) / a.tile_cells);
      a.child_tiles[cbase + d] = tiles;
      a.child_hsize[cbase + d] = tiles << nbits;
    }
  }
}

#endif  // MGT_WIDE


}  // namespace MGT_GEO_NS

// ----------------------------------------------------------------------------- launchers

namespace G = MGT_GEO_NS;

static inline dim3 grid1(uint64_t n) { return dim3((unsigned)n); }

#ifdef MGT_WIDE
hipError_t launch_pass_scatter_wide(const PassArgs& a, hipStream_t s) {
  if (a.g8) {
    PassArgs b = a;
    if (a.pk_on) {  // packed records in the slim form; the plain kernel takes the rest
      b.pk_split = 1;
      hipLaunchKernelGGL((G::k_pass_scatter<false, true, false, true>), grid1(a.g8), dim3(G::kBlock),
                         0, s, b);
    }
    hipLaunchKernelGGL((G::k_pass_scatter<false, true, false>), grid1(a.g8), dim3(G::kBlock), 0, s,
                       b);
  }
  return hipGetLastError();
}
#else
hipError_t launch_upload(void* dst, const void* src, size_t n, hipStream_t s) {
  const uint8_t* h = (const uint8_t*)src;
  for (size_t o = 0; o < n; o += kUploadChunk) {
    G::UploadArgs a;
    const size_t c = n - o < kUploadChunk ? n - o : kUploadChunk;
    a.dst = (uint32_t*)((uint8_t*)dst + o);
    a.words = (uint32_t)((c + 3) / 4);
    a.pad = 0;
    std::memcpy(a.data, h + o, c);
    hipLaunchKernelGGL(G::k_upload, dim3(1), dim3(G::kBlock), 0, s, a);
  }
  return hipGetLastError();
}

hipError_t launch_validate(const ItemDev* items, uint32_t n_items, uint64_t max_len,
                           int32_t* item_status, int32_t* abort_flag, int32_t ow, hipStream_t s) {
  uint64_t gx = (max_len + 1 + G::kBlock * 16 - 1) / (G::kBlock * 16);
  gx = gx < 1 ? 1 : (gx > 2048 ? 2048 : gx);
  hipLaunchKernelGGL(G::k_validate, dim3((unsigned)gx, n_items), dim3(G::kBlock), 0, s, items,
                     item_status, abort_flag, ow);
  return hipGetLastError();
}

hipError_t launch_scan(const uint32_t* in0, uint64_t* out0, const uint32_t* in1, uint64_t* out1,
                       const uint64_t* n_dev, uint64_t n_max, uint64_t* block_sums, hipStream_t s) {
  if (n_max <= G::kSmallScan) {
    hipLaunchKernelGGL(G::k_scan_small, dim3(1), dim3(1024), 0, s, in0, out0, in1, out1, n_dev,
                       n_max);
    return hipGetLastError();
  }
  const uint64_t nb = (n_max + kScanBlock - 1) / kScanBlock;
  const uint64_t cap = nb + 1;
  if (nb) {
    hipLaunchKernelGGL(G::k_scan_reduce, grid1(nb), dim3(G::kBlock), 0, s, in0, in1, n_dev, n_max,
                       block_sums, cap);
  }
  hipLaunchKernelGGL(G::k_scan_spine, dim3(1), dim3(1024), 0, s, n_dev, n_max, block_sums, cap, out0,
                     out1);
  if (nb) {
    hipLaunchKernelGGL(G::k_scan_down, grid1(nb), dim3(G::kBlock), 0, s, in0, out0, in1, out1, n_dev,
                       n_max, block_sums, cap);
  }
  return hipGetLastError();
}

hipError_t launch_pass_hist(const PassArgs& a, hipStream_t s) {
  if (a.g8) hipLaunchKernelGGL(G::k_pass_hist, grid1(a.g8), dim3(G::kBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_pass_scatter(const PassArgs& a, hipStream_t s) {
  if (a.g8) {
    if (a.pass == 0 && a.has_val)
      hipLaunchKernelGGL((G::k_pass_scatter<true, false, true>), grid1(a.g8), dim3(G::kBlock), 0, s, a);
    else if (a.pass == 0 && a.pk_on && a.slim0) {
      // packed records in the slim 512-thread form; the plain kernel takes the rest
      PassArgs b = a;
      b.pk_split = 1;
      hipError_t e = launch_pass0_slim(b, s);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL((G::k_pass_scatter<true, false, false>), grid1(a.g8), dim3(G::kBlock), 0, s, b);
    } else if (a.pass == 0)
      hipLaunchKernelGGL((G::k_pass_scatter<true, false, false>), grid1(a.g8), dim3(G::kBlock), 0, s, a);
    else if (a.rso_out && a.tile_cells >= (uint32_t)kWideSub)
      return launch_pass_scatter_wide(a, s);
    else if (a.rso_out)
      hipLaunchKernelGGL((G::k_pass_scatter<false, true, false>), grid1(a.g8), dim3(G::kBlock), 0, s, a);
    else
      hipLaunchKernelGGL((G::k_pass_scatter<false, false, false>), grid1(a.g8), dim3(G::kBlock), 0, s, a);
  }
  return hipGetLastError();
}

// The caller launches the plain first pass beside it with pk_split set.
// slim0 == 2: some item splits by partition (fan-out at most 512). Without
// the first histogram's key words (fixed-width items) the pass reads the
// columns and packs the words itself.
hipError_t launch_pass0_slim(const PassArgs& a, hipStream_t s) {
  if (!a.g8) return hipSuccess;
  const dim3 g = grid1(a.g8), b(G::kBlock);
  if (a.slim0 == 2 && a.pk_keys)
    hipLaunchKernelGGL((G::k_pass_scatter<true, false, false, true, true>), g, b, 0, s, a);
  else if (a.slim0 == 2)
    hipLaunchKernelGGL((G::k_pass_scatter<true, false, false, true, true, true>), g, b, 0, s, a);
  else if (a.pk_keys)
    hipLaunchKernelGGL((G::k_pass_scatter<true, false, false, true>), g, b, 0, s, a);
  else
    hipLaunchKernelGGL((G::k_pass_scatter<true, false, false, true, false, true>), g, b, 0, s, a);
  return hipGetLastError();
}

hipError_t launch_view_keys(const ViewArgs& a, hipStream_t s) {
  const uint64_t nb = (a.nnz + G::kSub - 1) / G::kSub;
  if (nb) hipLaunchKernelGGL(G::k_view_keys, grid1(nb), dim3(G::kBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_children(const ChildArgs& a, hipStream_t s) {
  if (a.nseg) hipLaunchKernelGGL(G::k_children, grid1(a.nseg), dim3(G::kBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_finish_bucket(const FinishArgs& a, hipStream_t s) {
  if (a.nbuckets && a.bucket_done && a.grid) {
    const dim3 g(a.grid < a.nbuckets ? a.grid : a.nbuckets);
    if (a.bk_threads == 512) hipLaunchKernelGGL(G::k_finish_bucket<512>, g, dim3(512), 0, s, a);
    else hipLaunchKernelGGL(G::k_finish_bucket<1024>, g, dim3(1024), 0, s, a);
  }
  return hipGetLastError();
}

hipError_t launch_finish(const FinishArgs& a, hipStream_t s) {
  if (a.nbuckets) {
    if (a.rso_in) hipLaunchKernelGGL(G::k_finish<true>, grid1(a.g8), dim3(G::kBlock), 0, s, a);
    else hipLaunchKernelGGL(G::k_finish<false>, grid1(a.g8), dim3(G::kBlock), 0, s, a);
  }
  return hipGetLastError();
}

#endif  // MGT_WIDE

}  // namespace mgt
