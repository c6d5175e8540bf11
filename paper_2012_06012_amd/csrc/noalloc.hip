// The allocation-free transpose (mgt_transpose_noalloc): the library's own
// device array stands in for the caller's workspace, so a call allocates
// nothing. For callers that cannot allocate: code under HIP graph capture,
// tight serving loops, harnesses that forbid allocation.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/mgt.h"
#include "kernels.h"

namespace {

constexpr int kMaxDevices = 64;

// The workspace of every mgt_transpose_noalloc call on a device. Each GPU the
// library runs on holds its own copy until the process ends.
static __device__ __align__(256) uint8_t scratch[MGT_NOALLOC_SCRATCH_BYTES];

// Device address of this device's copy of `scratch`, looked up once per
// device with that device current (the array's name is only a host-side
// stand-in, not a device address).
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

int scratch_for_current_device(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return MGT_EHIP;
  if (dev < 0 || dev >= kMaxDevices) return MGT_EUNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return MGT_EHIP;
    g_ptr[dev] = ptr;
  }
  *out = g_ptr[dev];
  return MGT_OK;
}

}  // namespace

extern "C" int mgt_transpose_noalloc(mgt_plan_t plan, int32_t partitioned, const void* row_ptr,
                                     const int32_t* col, const void* payload_off,
                                     const uint8_t* payload, void* t_row_ptr, int32_t* t_col,
                                     void* t_payload_off, uint8_t* t_payload, uint32_t* perm,
                                     int64_t* xfer_cells, int64_t* xfer_bytes,
                                     int64_t* part_cell_off, int64_t* part_byte_off,
                                     int64_t* sdispls, int64_t* rdispls, int32_t* d_status,
                                     hipStream_t stream) {
  if (!plan) return MGT_EINVAL;
  void* ws = nullptr;
  const int st = scratch_for_current_device(&ws);
  if (st != MGT_OK) return st;
  return mgt::noalloc_call(plan, partitioned, row_ptr, col, payload_off, payload, t_row_ptr, t_col,
                           t_payload_off, t_payload, perm, xfer_cells, xfer_bytes, part_cell_off,
                           part_byte_off, sdispls, rdispls, ws, MGT_NOALLOC_SCRATCH_BYTES,
                           d_status, stream);
}
