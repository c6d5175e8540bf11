// Conversions between repeated cells and XCSR value lists (Section 2: one cell
// per (row, column) pair whose value is a list of values, plus a count of
// values per cell). Both forms are CSRs over the same payload array: the
// payload bytes keep their order, so these kernels move only row offsets,
// column ids, payload offsets and counts.
//
// Inputs that break the CSR invariants cannot make these kernels access
// memory out of bounds: every offset read is clamped into [0, nnz] (or the
// payload size) before it indexes anything.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "../../include/mgt.h"
#include "kernels.h"
#include "prims.h"

namespace mgt {
namespace vl {

constexpr int kB = 256;

__device__ __forceinline__ uint64_t ld_o(const void* p, uint64_t i, int ow) {
  const int64_t v = ow == 4 ? (int64_t)gm((const int32_t*)p)[i] : gm((const int64_t*)p)[i];
  return v < 0 ? 0u : (uint64_t)v;
}
__device__ __forceinline__ void st_o(void* p, uint64_t i, uint64_t v, int ow) {
  if (ow == 4) gm((int32_t*)p)[i] = (int32_t)v;
  else gm((int64_t*)p)[i] = (int64_t)v;
}
__device__ __forceinline__ uint64_t gtid() { return (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; }
__device__ __forceinline__ uint64_t gstride() { return (uint64_t)gridDim.x * blockDim.x; }

// 1 where a cell starts a run of equal columns inside its row: the first
// cell, a column change (row starts are added by k_row_heads).
__global__ __launch_bounds__(kB) void k_heads(const int32_t* col, uint64_t nnz, uint32_t* h) {
  for (uint64_t k = gtid(); k < nnz; k += gstride())
    h[k] = (k == 0 || gm(col)[k] != gm(col)[k - 1]) ? 1u : 0u;
}

__global__ __launch_bounds__(kB) void k_row_heads(const void* rp, int ow, uint64_t n_rows,
                                                  uint64_t nnz, uint32_t* h) {
  for (uint64_t i = gtid(); i < n_rows; i += gstride()) {
    const uint64_t a = min(ld_o(rp, i, ow), nnz), b = min(ld_o(rp, i + 1, ow), nnz);
    if (a < b) h[a] = 1u;
  }
}

// Run heads to their output slot pos[k] (exclusive scan of the head flags;
// pos[nnz] = number of output cells m).
__global__ __launch_bounds__(kB) void k_emit(const int32_t* col, const void* poff, int ow,
                                             uint64_t nnz, const uint32_t* h, const uint64_t* pos,
                                             int32_t* o_col, void* o_poff, uint32_t* first,
                                             int64_t* d_m) {
  if (gtid() == 0) {
    const uint64_t m = min(pos[nnz], nnz);
    first[m] = (uint32_t)nnz;
    st_o(o_poff, m, ld_o(poff, nnz, ow), ow);
    if (d_m) *d_m = (int64_t)m;
  }
  for (uint64_t k = gtid(); k < nnz; k += gstride()) {
    if (!h[k]) continue;
    const uint64_t p = pos[k];
    gm(o_col)[p] = gm(col)[k];
    st_o(o_poff, p, ld_o(poff, k, ow), ow);
    first[p] = (uint32_t)k;
  }
}

// Output row offsets (heads before each row start) and run lengths.
__global__ __launch_bounds__(kB) void k_rows_counts(const void* rp, int ow, uint64_t n_rows,
                                                    uint64_t nnz, const uint64_t* pos,
                                                    const uint32_t* first, void* o_rp,
                                                    uint32_t* o_counts) {
  const uint64_t m = min(pos[nnz], nnz);
  const uint64_t n = max(nnz, n_rows + 1);
  for (uint64_t j = gtid(); j < n; j += gstride()) {
    if (j < m && o_counts) o_counts[j] = first[j + 1] - first[j];
    if (j <= n_rows) st_o(o_rp, j, pos[min(ld_o(rp, j, ow), nnz)], ow);
  }
}

// Expansion: row offsets in values, and the status word (MGT_OK; a later
// kernel overwrites it on a cell that is not a whole number of values).
__global__ __launch_bounds__(kB) void k_expand_rows(const void* rp, const void* poff, int ow,
                                                    uint64_t n_rows, uint64_t nnz, uint32_t w,
                                                    void* o_rp, int32_t* d_status) {
  if (gtid() == 0 && d_status) *d_status = MGT_OK;
  for (uint64_t i = gtid(); i <= n_rows; i += gstride())
    st_o(o_rp, i, ld_o(poff, min(ld_o(rp, i, ow), nnz), ow) / w, ow);
}

__global__ __launch_bounds__(kB) void k_expand_check(const void* poff, int ow, uint64_t nnz,
                                                     uint32_t w, int32_t* d_status) {
  bool bad = false;
  for (uint64_t k = gtid(); k <= nnz; k += gstride()) bad |= (ld_o(poff, k, ow) % w) != 0;
  if (bad && d_status) *d_status = MGT_ERANGE;
}

// One output cell per value: the cell holding byte q * w is the last cell
// whose payload offset is at most q * w.
__global__ __launch_bounds__(kB) void k_expand_cells(const int32_t* col, const void* poff, int ow,
                                                     uint64_t nnz, uint64_t nvals, uint32_t w,
                                                     int32_t* o_col, void* o_poff) {
  for (uint64_t q = gtid(); q < nvals; q += gstride()) {
    const uint64_t b = q * w;
    uint64_t lo = 0, hi = nnz;
    while (hi - lo > 1) {
      const uint64_t mid = (lo + hi) >> 1;
      if (ld_o(poff, mid, ow) <= b) lo = mid;
      else hi = mid;
    }
    gm(o_col)[q] = nnz ? gm(col)[lo] : 0;
    if (o_poff) st_o(o_poff, q, b, ow);
  }
  if (gtid() == 0 && o_poff) st_o(o_poff, nvals, nvals * w, ow);
}

__global__ __launch_bounds__(kB) void k_scale_offsets(const uint64_t* ex, uint64_t n, uint32_t w,
                                                      int ow, void* poff) {
  for (uint64_t k = gtid(); k <= n; k += gstride()) st_o(poff, k, ex[k] * w, ow);
}

inline dim3 grid_for(uint64_t n) {
  uint64_t g = (n + kB - 1) / kB;
  g = g < 1 ? 1 : (g > 16384 ? 16384 : g);
  return dim3((unsigned)g);
}

// Workspace layout: head flags (4 B per cell), their scan (8 B per cell + 1),
// run starts (4 B per cell + 1), scan scratch.
struct VlLayout {
  uint64_t o_h, o_pos, o_first, o_scan, bytes;
};
inline uint64_t up256(uint64_t x) { return (x + 255) & ~(uint64_t)255; }
inline VlLayout vl_layout(uint64_t nnz) {
  VlLayout y;
  y.o_h = 0;
  y.o_pos = up256(4 * nnz);
  y.o_first = y.o_pos + up256(8 * (nnz + 1));
  y.o_scan = y.o_first + up256(4 * (nnz + 1));
  y.bytes = y.o_scan + up256(scan_scratch_bytes(nnz + 1));
  return y;
}

}  // namespace vl
}  // namespace mgt

using namespace mgt;

#define MGT_VL_HIP(x)                              \
  do {                                             \
    if ((x) != hipSuccess) return MGT_EHIP;        \
  } while (0)

extern "C" {

int mgt_value_lists_workspace(int64_t nnz, size_t* workspace_bytes) {
  if (nnz < 0 || !workspace_bytes) return MGT_EINVAL;
  if ((uint64_t)nnz >= (1ull << 32)) return MGT_EUNSUPPORTED;
  *workspace_bytes = (size_t)vl::vl_layout((uint64_t)nnz).bytes;
  return MGT_OK;
}

int mgt_coalesce(int64_t n_rows, int64_t nnz, int32_t offset_width, const void* row_ptr,
                 const int32_t* col, const void* payload_off, void* o_row_ptr, int32_t* o_col,
                 void* o_payload_off, uint32_t* o_counts, int64_t* d_m, void* workspace,
                 size_t workspace_bytes, hipStream_t stream) {
  if (n_rows < 0 || nnz < 0 || (offset_width != 4 && offset_width != 8)) return MGT_EINVAL;
  if ((uint64_t)nnz >= (1ull << 32) || n_rows >= (1ll << 31)) return MGT_EUNSUPPORTED;
  if (!row_ptr || !payload_off || !o_row_ptr || !o_payload_off) return MGT_EINVAL;
  if (nnz > 0 && (!col || !o_col)) return MGT_EINVAL;
  if (!workspace || ((uintptr_t)workspace & 255u)) return MGT_EINVAL;
  const uint64_t n = (uint64_t)nnz, r = (uint64_t)n_rows;
  const vl::VlLayout y = vl::vl_layout(n);
  if (workspace_bytes < y.bytes) return MGT_ENOMEM;
  uint8_t* W = (uint8_t*)workspace;
  uint32_t* h = (uint32_t*)(W + y.o_h);
  uint64_t* pos = (uint64_t*)(W + y.o_pos);
  uint32_t* first = (uint32_t*)(W + y.o_first);
  uint64_t* scan = (uint64_t*)(W + y.o_scan);
  const int ow = offset_width;
  if (n) {
    hipLaunchKernelGGL(vl::k_heads, vl::grid_for(n), dim3(vl::kB), 0, stream, col, n, h);
    hipLaunchKernelGGL(vl::k_row_heads, vl::grid_for(r), dim3(vl::kB), 0, stream, row_ptr, ow, r,
                       n, h);
  }
  MGT_VL_HIP(hipGetLastError());
  MGT_VL_HIP(launch_scan(h, pos, nullptr, nullptr, nullptr, n, scan, stream));
  hipLaunchKernelGGL(vl::k_emit, vl::grid_for(n), dim3(vl::kB), 0, stream, col, payload_off, ow,
                     n, h, pos, o_col, o_payload_off, first, d_m);
  hipLaunchKernelGGL(vl::k_rows_counts, vl::grid_for(std::max(n, r + 1)), dim3(vl::kB), 0,
                     stream, row_ptr, ow, r, n, pos, first, o_row_ptr, o_counts);
  MGT_VL_HIP(hipGetLastError());
  return MGT_OK;
}

int mgt_expand(int64_t n_rows, int64_t nnz, int64_t payload_bytes, int32_t offset_width,
               int32_t value_bytes, const void* row_ptr, const int32_t* col,
               const void* payload_off, void* o_row_ptr, int32_t* o_col, void* o_payload_off,
               int32_t* d_status, hipStream_t stream) {
  if (n_rows < 0 || nnz < 0 || payload_bytes < 0 || value_bytes <= 0) return MGT_EINVAL;
  if (offset_width != 4 && offset_width != 8) return MGT_EINVAL;
  if (payload_bytes % value_bytes) return MGT_EINVAL;
  const uint64_t nvals = (uint64_t)(payload_bytes / value_bytes);
  if (nvals >= (1ull << 32) || (uint64_t)nnz >= (1ull << 32) || n_rows >= (1ll << 31))
    return MGT_EUNSUPPORTED;
  if (offset_width == 4 && payload_bytes >= (1ll << 31)) return MGT_EUNSUPPORTED;
  if (!row_ptr || !payload_off || !o_row_ptr) return MGT_EINVAL;
  if (nnz > 0 && !col) return MGT_EINVAL;
  if (nvals > 0 && (!o_col || nnz == 0)) return MGT_EINVAL;
  const uint64_t n = (uint64_t)nnz, r = (uint64_t)n_rows;
  const uint32_t w = (uint32_t)value_bytes;
  const int ow = offset_width;
  hipLaunchKernelGGL(vl::k_expand_rows, vl::grid_for(r + 1), dim3(vl::kB), 0, stream, row_ptr,
                     payload_off, ow, r, n, w, o_row_ptr, d_status);
  hipLaunchKernelGGL(vl::k_expand_check, vl::grid_for(n + 1), dim3(vl::kB), 0, stream,
                     payload_off, ow, n, w, d_status);
  hipLaunchKernelGGL(vl::k_expand_cells, vl::grid_for(nvals), dim3(vl::kB), 0, stream, col,
                     payload_off, ow, n, nvals, w, o_col, o_payload_off);
  MGT_VL_HIP(hipGetLastError());
  return MGT_OK;
}

int mgt_counts_to_offsets(int64_t nnz, const uint32_t* counts, int32_t value_bytes,
                          int32_t offset_width, void* payload_off, void* workspace,
                          size_t workspace_bytes, hipStream_t stream) {
  if (nnz < 0 || value_bytes <= 0 || (offset_width != 4 && offset_width != 8)) return MGT_EINVAL;
  if ((uint64_t)nnz >= (1ull << 32)) return MGT_EUNSUPPORTED;
  if (!payload_off || (nnz > 0 && !counts)) return MGT_EINVAL;
  if (!workspace || ((uintptr_t)workspace & 255u)) return MGT_EINVAL;
  const uint64_t n = (uint64_t)nnz;
  const vl::VlLayout y = vl::vl_layout(n);
  if (workspace_bytes < y.bytes) return MGT_ENOMEM;
  uint8_t* W = (uint8_t*)workspace;
  uint64_t* ex = (uint64_t*)(W + y.o_pos);
  uint64_t* scan = (uint64_t*)(W + y.o_scan);
  MGT_VL_HIP(launch_scan(counts, ex, nullptr, nullptr, nullptr, n, scan, stream));
  hipLaunchKernelGGL(vl::k_scale_offsets, vl::grid_for(n + 1), dim3(vl::kB), 0, stream, ex, n,
                     (uint32_t)value_bytes, offset_width, payload_off);
  MGT_VL_HIP(hipGetLastError());
  return MGT_OK;
}

}  // extern "C"
