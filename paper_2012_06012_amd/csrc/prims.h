// Wave64 / workgroup primitives for gfx950 (CDNA4): lane masks, DPP and
// shuffle scans, workgroup scans, and the ballot multisplit used to rank
// equal digits stably without atomics.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mgt {

constexpr int kWave = 64;

__device__ __forceinline__ uint32_t lane_id() {
  return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

// Number of set bits of m in lanes below the calling lane (v_mbcnt).
__device__ __forceinline__ uint32_t popc_below(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

// Inclusive wave scan of a 32-bit value with DPP: Hillis-Steele inside each
// 16-lane row (row_shr 1, 2, 4, 8, zero-filled at the row edge), then
// row_bcast15 / row_bcast31 carry the row totals into the rows above.
__device__ __forceinline__ uint32_t wave_incl_scan_u32(uint32_t v) {
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, false);  // row_shr:1
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, false);  // row_shr:2
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, false);  // row_shr:4
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, false);  // row_shr:8
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false);  // row_bcast:15
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false);  // row_bcast:31
  return v;
}

// Inclusive wave scan of a 64-bit value (cross-lane shuffles).
__device__ __forceinline__ uint64_t wave_incl_scan_u64(uint64_t v) {
  const uint32_t l = lane_id();
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    uint64_t u = __shfl_up(v, o, kWave);
    if (l >= (uint32_t)o) v += u;
  }
  return v;
}

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) { return wave_incl_scan_u32(v); }
__device__ __forceinline__ uint64_t wave_incl_scan(uint64_t v) { return wave_incl_scan_u64(v); }

template <class T>
__device__ __forceinline__ T wave_bcast(T v, int lane) { return __shfl(v, lane, kWave); }

// Exclusive scan over a workgroup of NW waves. `scratch` holds NW + 1 values.
// Every thread of the workgroup must call it. Returns the exclusive prefix;
// `total` receives the workgroup total.
template <int NW, class T>
__device__ __forceinline__ T block_excl_scan(T v, T* scratch, T& total) {
  const T inc = wave_incl_scan(v);
  const int w = threadIdx.x / kWave;
  if (lane_id() == kWave - 1) scratch[w] = inc;
  __syncthreads();
  if (threadIdx.x == 0) {
    T a = 0;
#pragma unroll
    for (int i = 0; i < NW; ++i) {
      T t = scratch[i];
      scratch[i] = a;
      a += t;
    }
    scratch[NW] = a;
  }
  __syncthreads();
  total = scratch[NW];
  const T r = inc - v + scratch[w];
  __syncthreads();
  return r;
}

// Lanes of the wave whose `digit` equals the calling lane's digit, among the
// lanes where `active` holds. `dbits` (wave-uniform) bounds the digit width.
__device__ __forceinline__ uint64_t match_peers(uint32_t digit, bool active, int dbits) {
  uint64_t m = ballot(active);
  for (int b = 0; b < dbits; ++b) {
    const bool bit = (digit >> b) & 1u;
    const uint64_t v = ballot(bit);
    m &= bit ? v : ~v;
  }
  return m;
}

// XCD-aware tile order: the hardware deals workgroups round robin over the 8
// XCDs, so this gives each XCD a contiguous run of tiles (neighbouring tiles
// then share that XCD's L2). `g8` is the grid size, a multiple of 8.
__device__ __forceinline__ uint64_t xcd_tile(uint64_t b, uint64_t g8) {
  return (b & 7u) * (g8 >> 3) + (b >> 3);
}

// Global-memory (address space 1) views of generic pointers. Accesses through
// them compile to global_* instructions, which only the vector-memory counter
// tracks; flat_* accesses are tracked by the LDS counter as well, so every
// wait for an LDS result would also wait for all outstanding HBM traffic.
#define GMEM __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ GMEM T* gm(T* p) { return (GMEM T*)p; }
template <typename T>
__device__ __forceinline__ const GMEM T* gm(const T* p) { return (const GMEM T*)p; }

// Copies one cell's payload (any width, any alignment). Every chunk issues
// all of its loads before its stores, so a lane waits for memory once per
// chunk instead of once per word. Source and destination sharing their
// alignment modulo 4 move as 4-byte words (up to 8 per chunk); otherwise as
// bytes (up to 16 per chunk).
__device__ __forceinline__ void copy_cell(uint8_t* __restrict__ dst_, const uint8_t* __restrict__ src_,
                                          uint32_t n) {
  GMEM uint8_t* dst = gm(dst_);
  const GMEM uint8_t* src = gm(src_);
  if ((((uintptr_t)dst_ ^ (uintptr_t)src_) & 3u) == 0) {
    uint32_t h = (4u - ((uintptr_t)dst_ & 3u)) & 3u;
    h = h < n ? h : n;
    uint8_t hb[3];
#pragma unroll
    for (int j = 0; j < 3; ++j)
      if ((uint32_t)j < h) hb[j] = src[j];
#pragma unroll
    for (int j = 0; j < 3; ++j)
      if ((uint32_t)j < h) dst[j] = hb[j];
    dst += h;
    src += h;
    n -= h;
    const GMEM uint32_t* s4 = (const GMEM uint32_t*)src;
    GMEM uint32_t* d4 = (GMEM uint32_t*)dst;
    uint32_t w = n >> 2;
    while (w) {
      const uint32_t m = w < 8u ? w : 8u;
      uint32_t v[8];
#pragma unroll
      for (int j = 0; j < 8; ++j)
        if ((uint32_t)j < m) v[j] = s4[j];
#pragma unroll
      for (int j = 0; j < 8; ++j)
        if ((uint32_t)j < m) d4[j] = v[j];
      s4 += m;
      d4 += m;
      w -= m;
    }
    const uint32_t t = n & 3u;
    const GMEM uint8_t* sb = (const GMEM uint8_t*)s4;
    GMEM uint8_t* db = (GMEM uint8_t*)d4;
    uint8_t tb[3];
#pragma unroll
    for (int j = 0; j < 3; ++j)
      if ((uint32_t)j < t) tb[j] = sb[j];
#pragma unroll
    for (int j = 0; j < 3; ++j)
      if ((uint32_t)j < t) db[j] = tb[j];
  } else {
    while (n) {
      const uint32_t m = n < 16u ? n : 16u;
      uint8_t v[16];
#pragma unroll
      for (int j = 0; j < 16; ++j)
        if ((uint32_t)j < m) v[j] = src[j];
#pragma unroll
      for (int j = 0; j < 16; ++j)
        if ((uint32_t)j < m) dst[j] = v[j];
      src += m;
      dst += m;
      n -= m;
    }
  }
}

}  // namespace mgt
