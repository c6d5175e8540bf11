// Host runtime of libmgt: descriptor checks, digit schedules, workspace
// layout and the launch sequence behind the C ABI declared in include/mgt.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/mgt.h"
#include "kernels.h"
#include "mgt_internal.h"

using namespace mgt;

namespace {

constexpr uint32_t kTileCells = 16384;    // cells per partition-pass tile (multiple of kSub)
constexpr uint64_t kTargetTiles = 1024;   // tiles a single-matrix pass aims for
constexpr uint64_t kTargetBuckets = 512;  // finish buckets a small single-matrix call aims for
constexpr int kMaxBitsPerPass = kMaxPassBits;  // fan-out 256 per bits-mode pass
constexpr uint32_t kMaxPartFanout = 512;  // largest preferred fan-out of the partition pass
// The partition pass aims for 256 digits (longer digit runs than 512) unless
// its segments would then average more than this much payload: the gathering
// finish streams a segment or two at a time through the 256 MB memory-side
// cache (large matrix with 64 partitions: 256; heterogeneous matrix with 30 GB
// of payload over 256 partitions: 512).
constexpr uint64_t kSegPayloadTarget = 48ull << 20;
constexpr int kMaxItems = 65535;
// Host bytes of one single-matrix descriptor upload built on the stack by the
// allocation-free call (item, status, flags, 1,025 partition bounds and the
// first-pass tables, each 256-byte aligned, fit with room to spare).
constexpr size_t kNoAllocUpload = 16384;
static_assert(kTileCells % kSub == 0, "tile geometry");

int ceil_log2_u64(uint64_t x) {
  int b = 0;
  while ((1ull << b) < x) ++b;
  return b;
}
int floor_log2_u64(uint64_t x) {
  int b = -1;
  while (x) { x >>= 1; ++b; }
  return b;
}
uint64_t align_up(uint64_t x, uint64_t a) { return (x + a - 1) / a * a; }

// Digit schedule of one matrix.
struct Sched {
  int n_levels = 1;
  int bits[kMaxLevels] = {0, 0, 0, 0};
  int key_bits = 0;
  int part_mode = 0;
  int finish_bits = 0;
};

// Schedule of a single-matrix plan set by the caller (mgt_plan_set_schedule,
// e.g. from an autotuner): a cap on the bits of a bits-mode pass, an exact
// finish width, a tile size; each unset field keeps the rule below.
struct Tune {
  int pass_bits = 0;     // 1..8, 0: the environment cap / default
  int finish_bits = -1;  // 0..10, -1: the rule's choice
  uint32_t tile = 0;     // 2048..16384 cells, 0: sized for the call
};

// Schedule caps from the environment: MGT_MAX_PASS_BITS (1..8) bounds the bits
// of a bits-mode pass and MGT_MAX_FINISH_BITS (0..10) the column bits of a
// finish bucket. Lower caps trade more passes for smaller fan-outs; tests use
// them to reach three- and four-pass schedules on small inputs.
int env_cap(const char* name, int lo, int hi, int dflt) {
  const char* e = std::getenv(name);
  if (e && *e) {
    const int v = std::atoi(e);
    if (v >= lo && v <= hi) return v;
  }
  return dflt;
}
int max_pass_bits() { return env_cap("MGT_MAX_PASS_BITS", 1, kMaxBitsPerPass, kMaxBitsPerPass); }
int max_finish_bits() { return env_cap("MGT_MAX_FINISH_BITS", 0, kMaxFinishBits, kMaxFinishBits); }

// Number of passes needed for `B` bits when the first pass may take
// `first_cap`, the last of two or more `last_cap` and every other one `mb`.
int passes_for(int B, int first_cap, int mb, int last_cap) {
  if (B <= first_cap) return 1;
  int L = 2, cap = first_cap + last_cap;
  while (cap < B) {
    ++L;
    cap += mb;
  }
  return L;
}

// spread: a single-matrix call, whose finish buckets shrink (down to kSub / 8
// cells) on small matrices so that about kTargetBuckets workgroups share the
// finish; a batch keeps 2 to 4 * kSub cells per bucket (the 1,024-thread
// whole-bucket finish holds up to 9,216), its items giving the parallelism. last_cap: the bits the last pass of two or more may take (its
// 512-thread form takes up to kMaxLastPassBits). level_budget > 0: the passes
// the call makes anyway (a batch pads every item to its largest pass count),
// so the finish width is the smallest one from the ideal up that needs no
// more passes than that, instead of the one that needs the fewest.
Sched make_sched_mb(int64_t n_cols, int64_t nnz, int64_t payload_bytes, int32_t R,
                    const int64_t* bounds, bool partitioned, int mb, int mf, bool spread,
                    int force_fb, int last_cap, int level_budget = 0) {
  Sched s;
  uint64_t width = (uint64_t)std::max<int64_t>(n_cols, 1);
  if (partitioned) {
    width = 1;
    for (int32_t r = 0; r < R; ++r) width = std::max<uint64_t>(width, (uint64_t)(bounds[r + 1] - bounds[r]));
    s.part_mode = 1;
  }
  const int K = ceil_log2_u64(width);
  s.key_bits = K;
  // Finish buckets of up to 2 * kSub cells (a batch: 4 * kSub): 2^fb columns
  // at nnz / n_cols cells each.
  int fb_ideal = 0;
  if (nnz > 0 && n_cols > 0) {
    const double per_col = (double)nnz / (double)n_cols;
    double target = (spread ? 2.0 : 4.0) * kSub;
    if (spread)
      target = std::min(target, std::max(kSub / 8.0, (double)nnz / (double)kTargetBuckets));
    fb_ideal = floor_log2_u64((uint64_t)std::max(1.0, target / per_col));
  } else {
    fb_ideal = mf;
  }
  fb_ideal = std::min(std::max(fb_ideal, 0), std::min(mf, K));
  const uint32_t part_fan =
      (uint64_t)std::max<int64_t>(payload_bytes, 0) / 256u > kSegPayloadTarget ? kMaxPartFanout : 256u;
  const int first_cap = partitioned
      ? std::min(mb, R <= (int32_t)part_fan ? floor_log2_u64(part_fan / (uint32_t)R) : 0)
      : mb;
  // Fewest passes first, then the smallest finish width that achieves them
  // (within a level budget: the smallest finish width that fits it).
  int best_fb = fb_ideal, best_L = 1 << 30;
  for (int fb = fb_ideal; fb <= std::min(mf, K); ++fb) {
    const int L = passes_for(K - fb, first_cap, mb, last_cap);
    if (level_budget > 0 && L <= level_budget) {
      best_L = L;
      best_fb = fb;
      break;
    }
    if (L < best_L) { best_L = L; best_fb = fb; }
  }
  if (K <= fb_ideal) { best_fb = K; best_L = 1; }
  if (force_fb >= 0) {  // a finish width set by the caller
    best_fb = std::min(force_fb, K);
    best_L = passes_for(K - best_fb, first_cap, mb, last_cap);
  }
  const int B = K - best_fb;
  s.finish_bits = best_fb;
  s.n_levels = best_L;
  int rest = B;
  s.bits[0] = std::min(B, first_cap);
  if (!partitioned && best_L > 1)  // spread evenly, within the caps
    s.bits[0] = std::min(first_cap, (B + best_L - 1) / best_L);
  rest -= s.bits[0];
  for (int l = 1; l < best_L; ++l) {
    const int left = best_L - l;
    const int cap = l == best_L - 1 ? last_cap : mb;
    s.bits[l] = l == best_L - 1 ? rest : std::min(cap, (rest + left - 1) / left);
    rest -= s.bits[l];
  }
  return s;
}

uint32_t tile_cells_for(uint64_t nnz);

// Column bits a finish bucket keeps when the last pass takes its extra bit.
constexpr int kWideFinishMinBits = 5;

// A single-matrix call whose tiles hold at least kWideSub cells runs its last
// pass (records only) in the 512-thread form, which takes up to
// kMaxLastPassBits bits when the pass cap is the full kMaxBitsPerPass.
// The schedule a setting gives (it may need more than kMaxLevels passes).
Sched make_sched_tuned(int64_t n_cols, int64_t nnz, int64_t payload_bytes, int32_t R,
                       const int64_t* bounds, bool partitioned, bool spread, const Tune* t,
                       int level_budget = 0) {
  const int mb = (t && t->pass_bits > 0) ? t->pass_bits : max_pass_bits();
  const int ff = (t && t->finish_bits >= 0) ? t->finish_bits : -1;
  const uint32_t tile = (t && t->tile) ? t->tile : tile_cells_for((uint64_t)std::max<int64_t>(nnz, 0));
  const bool wide = spread && tile >= (uint32_t)kWideSub;
  const int last_cap = (wide && mb >= kMaxBitsPerPass) ? kMaxLastPassBits : mb;
  Sched s = make_sched_mb(n_cols, nnz, payload_bytes, R, bounds, partitioned, mb, max_finish_bits(),
                          spread, ff, last_cap, level_budget);
  // A finish bucket of fewer than 2^kWideFinishMinBits columns carries the
  // spread of single column degrees: on skewed inputs many such buckets
  // outgrow the 512-thread finish. The extra last-pass bit is kept only when
  // the buckets it buys span that many columns.
  if (last_cap > mb && s.n_levels >= 2 && s.bits[s.n_levels - 1] > mb &&
      s.finish_bits < kWideFinishMinBits)
    s = make_sched_mb(n_cols, nnz, payload_bytes, R, bounds, partitioned, mb, max_finish_bits(),
                      spread, ff, mb, level_budget);
  return s;
}

Sched make_sched(int64_t n_cols, int64_t nnz, int64_t payload_bytes, int32_t R,
                 const int64_t* bounds, bool partitioned, bool spread, const Tune* t = nullptr,
                 int level_budget = 0) {
  Sched s = make_sched_tuned(n_cols, nnz, payload_bytes, R, bounds, partitioned, spread, t,
                             level_budget);
  if (s.n_levels > kMaxLevels) {
    const uint32_t tile = (t && t->tile) ? t->tile : tile_cells_for((uint64_t)std::max<int64_t>(nnz, 0));
    const bool wide = spread && tile >= (uint32_t)kWideSub;
    s = make_sched_mb(n_cols, nnz, payload_bytes, R, bounds, partitioned, kMaxBitsPerPass,
                      kMaxFinishBits, spread, -1, wide ? kMaxLastPassBits : kMaxBitsPerPass);
  }
  return s;
}

uint32_t fanout(const Sched& s, int l, int32_t R) {
  return (l == 0 && s.part_mode) ? ((uint32_t)R << s.bits[0]) : (1u << s.bits[l]);
}

// One matrix of a call, as the host sees it.
struct HostItem {
  mgt_desc d;
  Sched s;
  uint32_t tile = 0;  // cells per tile set by the caller (single-matrix calls), 0: sized here
  const int64_t* bounds;  // host
  ItemDev dev;
};

// The items of one call, as a view (no ownership): a vector's, or an array on
// the stack for calls that must not allocate.
struct Items {
  HostItem* p = nullptr;
  size_t n = 0;
  Items(std::vector<HostItem>& v) : p(v.data()), n(v.size()) {}
  Items(HostItem* a, size_t k) : p(a), n(k) {}
  HostItem& operator[](size_t i) const { return p[i]; }
  size_t size() const { return n; }
  bool empty() const { return n == 0; }
  HostItem* begin() const { return p; }
  HostItem* end() const { return p + n; }
};

// Workspace layout of one call.
struct Layout {
  uint32_t n_items = 0;
  int L = 1;
  uint64_t total_nnz = 0, total_bytes = 0, total_bounds = 0;
  uint64_t nseg[kMaxLevels + 1] = {};
  uint64_t tiles_max[kMaxLevels] = {};
  uint64_t hist_max = 0, tiles_all_max = 0, scan_max = 0;
  // offsets
  uint64_t o_items, o_status, o_abort, o_bounds;
  uint64_t o_segs[kMaxLevels + 1], o_tcnt[kMaxLevels], o_hsz[kMaxLevels], o_tstart[kMaxLevels],
      o_hstart[kMaxLevels];
  uint64_t o_hcnt, o_hbyt, o_ocnt, o_obyt, o_ttot, o_tsrc, o_scan;
  uint64_t o_ks[2], o_rk[2], o_pay[2], o_rso = 0;
  uint64_t o_bdone = 0;  // two or more passes: per finish bucket, written by k_finish_bucket
  // view operations: partition bounds of the matrix, per-cell keys and values
  uint64_t n_vbounds = 0, o_vbounds = 0, o_vkeys = 0, o_vvals = 0;
  uint64_t o_up_end = 0;  // the uploaded prefix: items, status, bounds, level-0 tables
  uint32_t tile_cells = kTileCells;
  uint64_t bytes = 0;
};

// Cells per partition-pass tile of a single-matrix call: the smallest power
// of two from kSub up that keeps the tile count near kTargetTiles, at most
// kTileCells. Small matrices thus spread over many workgroups instead of
// running a few long tiles one sub-chunk after another. Batches keep
// kTileCells (their items already give many tiles, and their workspace
// estimate must bound every batch within the limits).
uint32_t tile_cells_for(uint64_t nnz) {
  uint32_t t = kSub;
  while (t < kTileCells && (nnz + t - 1) / t > kTargetTiles) t *= 2;
  return t;
}

// n_vbounds > 0: a view operation on the single item, whose matrix has
// n_vbounds - 1 partitions.
Layout make_layout(Items items, uint64_t n_vbounds = 0) {
  Layout y;
  y.n_vbounds = n_vbounds;
  y.n_items = (uint32_t)items.size();
  if (items.size() == 1)
    y.tile_cells = items[0].tile ? items[0].tile : tile_cells_for((uint64_t)items[0].d.nnz);
  else if (!items.empty() && items[0].tile)
    y.tile_cells = items[0].tile;  // a batch plan's tile setting (the same for every item)
  const uint64_t tc = y.tile_cells;
  int L = 1;
  for (auto& it : items) L = std::max(L, it.s.n_levels);
  y.L = L;
  // pad every schedule to L passes (extra passes have 0 bits: copies)
  for (auto& it : items) {
    for (int l = it.s.n_levels; l < L; ++l) it.s.bits[l] = 0;
    it.s.n_levels = L;
  }
  uint64_t cell = 0, byte = 0, tiles0 = 0;
  for (auto& it : items) {
    it.dev.cell_base = cell;
    it.dev.byte_base = byte;
    cell += (uint64_t)it.d.nnz;
    byte += (uint64_t)it.d.payload_bytes;
    y.total_bounds += (uint64_t)it.d.n_parts + 1;
  }
  y.total_nnz = cell;
  y.total_bytes = byte;
  for (int l = 0; l <= L; ++l) y.nseg[l] = 0;
  for (auto& it : items) {
    uint64_t ns = 1;
    for (int l = 0; l <= L; ++l) {
      it.dev.seg_base[l] = y.nseg[l];
      y.nseg[l] += ns;
      if (l < L) ns *= fanout(it.s, l, it.d.n_parts);
    }
    const uint64_t t0 = ((uint64_t)it.d.nnz + tc - 1) / tc;
    it.dev.tile_base = tiles0;
    tiles0 += t0;
  }
  // per-pass tile and histogram bounds
  for (int l = 0; l < L; ++l) {
    uint64_t tiles = 0, hist = 0;
    for (auto& it : items) {
      uint64_t segs_item = 1;
      for (int q = 0; q < l; ++q) segs_item *= fanout(it.s, q, it.d.n_parts);
      const uint64_t t = ((uint64_t)it.d.nnz + tc - 1) / tc + (l ? segs_item : 0);
      tiles += t;
      hist += t * fanout(it.s, l, it.d.n_parts);
    }
    y.tiles_max[l] = tiles;
    y.tiles_all_max = std::max(y.tiles_all_max, tiles);
    y.hist_max = std::max(y.hist_max, hist);
  }
  y.scan_max = std::max<uint64_t>(y.hist_max, y.tiles_all_max);
  for (int l = 0; l <= L; ++l) y.scan_max = std::max(y.scan_max, y.nseg[l]);

  uint64_t o = 0;
  auto take = [&](uint64_t bytes) {
    const uint64_t at = o;
    o = align_up(o + bytes, 256);
    return at;
  };
  y.o_items = take(sizeof(ItemDev) * y.n_items);
  y.o_status = take(4ull * y.n_items);
  y.o_abort = take(64);
  y.o_bounds = take(8ull * y.total_bounds);
  if (n_vbounds) y.o_vbounds = take(8ull * n_vbounds);  // uploaded with the bounds
  // the level-0 tables (one segment per item) are filled on the host and
  // uploaded with the items
  y.o_segs[0] = take(sizeof(Seg) * y.nseg[0]);
  y.o_tcnt[0] = take(4ull * y.nseg[0]);
  y.o_hsz[0] = take(4ull * y.nseg[0]);
  y.o_tstart[0] = take(8ull * (y.nseg[0] + 1));
  y.o_hstart[0] = take(8ull * (y.nseg[0] + 1));
  y.o_up_end = o;
  for (int l = 1; l <= L; ++l) y.o_segs[l] = take(sizeof(Seg) * y.nseg[l]);
  for (int l = 1; l < L; ++l) {
    y.o_tcnt[l] = take(4ull * y.nseg[l]);
    y.o_hsz[l] = take(4ull * y.nseg[l]);
    y.o_tstart[l] = take(8ull * (y.nseg[l] + 1));
    y.o_hstart[l] = take(8ull * (y.nseg[l] + 1));
  }
  y.o_hcnt = take(4ull * y.hist_max);
  y.o_hbyt = take(4ull * y.hist_max);
  y.o_ocnt = take(8ull * (y.hist_max + 1));
  y.o_obyt = take(8ull * (y.hist_max + 1));
  y.o_ttot = take(4ull * y.tiles_all_max);
  y.o_tsrc = take(8ull * (y.tiles_all_max + 1));
  y.o_scan = take(scan_scratch_bytes(y.scan_max));
  // Records ping-pong between two level buffers. With two or more passes the
  // last one writes (row, cell index, payload offset) records of 16 bytes in
  // place of the 8-byte (row, cell index) ones, and no payload: a second
  // payload buffer, and a second (row, index) buffer, are needed only from
  // three passes on.
  const int nks = L >= 2 ? 2 : 1;
  const int nrk = L >= 3 ? 2 : 1;
  for (int b = 0; b < 2; ++b) {
    y.o_ks[b] = b < nks ? take(8ull * y.total_nnz) : y.o_ks[0];
    y.o_rk[b] = b < nrk ? take(8ull * y.total_nnz) : y.o_rk[0];
    y.o_pay[b] = b < nrk ? take(y.total_bytes + 16) : y.o_pay[0];
  }
  if (L >= 2) {
    y.o_rso = take(16ull * y.total_nnz);
    y.o_bdone = take(y.nseg[L]);
  }
  if (n_vbounds) {
    y.o_vkeys = take(4ull * y.total_nnz);
    y.o_vvals = take(4ull * y.total_nnz);
  }
  y.bytes = o + 256;
  return y;
}

int check_desc(const mgt_desc* d, bool need_bounds) {
  if (!d) return MGT_EINVAL;
  if (d->n_rows < 0 || d->n_cols < 0 || d->nnz < 0 || d->payload_bytes < 0) return MGT_EINVAL;
  if (d->offset_width != 4 && d->offset_width != 8) return MGT_EINVAL;
  if (d->n_rows >= (1ll << 31) || d->n_cols >= (1ll << 31)) return MGT_EUNSUPPORTED;
  if (d->nnz >= (1ll << 32)) return MGT_EUNSUPPORTED;
  if (d->offset_width == 4 && (d->nnz >= (1ll << 31) || d->payload_bytes >= (1ll << 31)))
    return MGT_EUNSUPPORTED;
  if (d->nnz > 0 && (d->n_rows == 0 || d->n_cols == 0)) return MGT_EINVAL;
  if ((d->flags & MGT_FIXED_WIDTH) && d->nnz > 0) {
    if (d->payload_bytes % d->nnz != 0) return MGT_EINVAL;
    if (d->payload_bytes / d->nnz >= (1ll << 31)) return MGT_EUNSUPPORTED;
  }
  if (d->n_parts < 1 || d->n_parts > kMaxParts) return MGT_EINVAL;
  if (d->n_parts > 1 || need_bounds) {
    if (!d->part_bounds) return MGT_EINVAL;
    if (d->n_parts > 1 && d->n_rows != d->n_cols) return MGT_EINVAL;
    if (d->part_bounds[0] != 0 || d->part_bounds[d->n_parts] != d->n_rows) return MGT_EINVAL;
    for (int32_t r = 0; r < d->n_parts; ++r)
      if (d->part_bounds[r + 1] < d->part_bounds[r]) return MGT_EINVAL;
  }
  return MGT_OK;
}

struct Timing {
  std::vector<hipEvent_t> ev;
  std::vector<const char*> names;
  int used = 0;
};

}  // namespace

struct mgt_plan_s {
  bool batch = false;
  mgt_desc desc{};
  std::vector<int64_t> bounds;
  mgt_batch_limits lim{};
  uint32_t flags = 0;
  // single-matrix plans: the two schedules and their workspace
  size_t ws_plain = 0, ws_part = 0;
  // upload staging (pinned) and its completion event
  void* staging = nullptr;
  size_t staging_bytes = 0;
  hipEvent_t upload_done = nullptr;
  bool upload_pending = false;
  Timing timing;
  // Serialises the host part of calls on this plan (staging buffer, upload
  // event, stage-timing events): calls from several threads may share it.
  std::mutex mu;
  Tune tune;  // single-matrix plans: schedule set by the caller
  // view-operation plans (mgt_view_plan): the operation, the input view, and
  // the descriptor the passes see (virtual rows, sort keys as columns)
  int32_t view_op = -1, column_view = 0;
  mgt_desc view_desc{};
  size_t ws_view = 0;
};

struct mgt_graph_s {
  hipGraphExec_t exec = nullptr;
  void* staging = nullptr;  // pinned upload buffer the graph's copy node reads
};

namespace {

int ensure_staging(mgt_plan_s* p, size_t bytes) {
  if (!p->upload_done &&
      hipEventCreateWithFlags(&p->upload_done, hipEventDisableTiming) != hipSuccess)
    return MGT_EHIP;
  if (p->upload_pending) {
    if (hipEventSynchronize(p->upload_done) != hipSuccess) return MGT_EHIP;
    p->upload_pending = false;
  }
  if (p->staging_bytes >= bytes) return MGT_OK;
  if (p->staging) (void)hipHostFree(p->staging);
  p->staging = nullptr;
  p->staging_bytes = 0;
  if (hipHostMalloc(&p->staging, bytes, hipHostMallocDefault) != hipSuccess) return MGT_ENOMEM;
  p->staging_bytes = bytes;
  return MGT_OK;
}

void time_mark(mgt_plan_s* p, hipStream_t s, const char* name) {
  if (!(p->flags & MGT_DEBUG_TIMING)) return;
  Timing& t = p->timing;
  if (t.used >= (int)t.ev.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return;
    t.ev.push_back(e);
    t.names.push_back(name);
  }
  t.names[t.used] = name;
  (void)hipEventRecord(t.ev[t.used], s);
  ++t.used;
}

// Compute units of the current device (read once per device).
// Mean cells per finish bucket up to which the whole-bucket finish runs first
// as two 512-thread workgroups per CU (capacity 4,608 cells), then as one
// 1,024-thread workgroup per CU for the buckets that left (up to 9,216).
constexpr uint64_t kBucketSmallMean = 4096;

uint32_t device_cus() {
  static uint32_t cus[64] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (!cus[dev]) {
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0)
      n = 256;
    cus[dev] = (uint32_t)n;
  }
  return cus[dev];
}

#define MGT_HIP(x)                          \
  do {                                      \
    if ((x) != hipSuccess) return MGT_EHIP; \
  } while (0)

// Runs the whole pipeline for `items` (already scheduled and laid out).
// A view operation's parameters (see k_view_keys).
struct ViewCall {
  const int32_t* col;       // the matrix's own column ids
  const int64_t* bounds;    // host, n_vbounds entries
  int64_t n_rows, n_cols;   // of the matrix X
  int32_t op, column_view;
};

// Bytes of the item table and bounds uploaded at the start of a call.
size_t upload_bytes(const Layout& y) { return y.o_up_end; }

// graph_staging: the call is being recorded into a graph that owns this
// pinned upload buffer (its contents are read at every replay); the plan's
// own staging buffer, completion event and stage timing are left alone.
// kernel_upload: the descriptor is built in this host buffer (at least
// upload_bytes(y) bytes, 16-byte aligned) and copied to the workspace by
// kernels taking it as arguments (launch_upload), so the call neither
// allocates nor touches the plan's pinned staging buffer.
int run(mgt_plan_s* p, Items items, const Layout& y, void* ws, int32_t* d_status,
        hipStream_t s, const ViewCall* vc = nullptr, void* graph_staging = nullptr,
        uint8_t* kernel_upload = nullptr) {
  uint8_t* W = (uint8_t*)ws;
  const int ow = items.empty() ? 8 : items[0].d.offset_width;
  const uint32_t n = y.n_items;
  // Every later pass fits the LDS of the kernel that will run it: 9 bits only
  // in a last pass run in the 512-thread form (tiles of kWideSub cells or more).
  const bool wide_last = y.L >= 2 && y.tile_cells >= (uint32_t)kWideSub;
  for (uint32_t i = 0; i < n; ++i)
    for (int l = 1; l < items[i].s.n_levels; ++l) {
      const int cap = (l == y.L - 1 && wide_last) ? kMaxLastPassBits : kMaxPassBits;
      if (items[i].s.bits[l] > cap) return MGT_EINVAL;
    }
  // Packed records (see PassArgs): one records-only pass, no perm, not a view
  // operation, at most 28 column bits in every item. The first histogram
  // falls back to the wide records if any payload size does not fit.
  int32_t pk_on = (n >= 1 && y.L == 2 && !vc && !env_cap("MGT_NO_PACK", 0, 1, 0)) ? 1 : 0;
  for (uint32_t i = 0; i < n && pk_on; ++i)
    if (items[i].dev.perm != nullptr ||
        ceil_log2_u64((uint64_t)std::max<int64_t>(items[i].d.n_cols, 1)) > 28)
      pk_on = 0;
  // 1. upload items + bounds through the pinned staging buffer
  const size_t up_bytes = upload_bytes(y);
  if (!graph_staging && !kernel_upload) {
    int st = ensure_staging(p, up_bytes);
    if (st != MGT_OK) return st;
  }
  uint8_t* H = kernel_upload ? kernel_upload : (uint8_t*)(graph_staging ? graph_staging : p->staging);
  int64_t* hb = (int64_t*)(H + y.o_bounds);
  uint64_t bo = 0;
  for (uint32_t i = 0; i < n; ++i) {
    HostItem& it = items[i];
    ItemDev& d = it.dev;
    d.n_rows = it.d.n_rows;
    d.n_cols = it.d.n_cols;
    d.nnz = it.d.nnz;
    d.payload_bytes = it.d.payload_bytes;
    d.n_parts = it.d.n_parts;
    d.n_levels = it.s.n_levels;
    for (int l = 0; l < kMaxLevels; ++l) d.bits[l] = it.s.bits[l];
    d.key_bits = it.s.key_bits;
    d.part_mode = it.s.part_mode;
    d.status_index = (int32_t)i;
    d.pk_shift = pk_on ? ceil_log2_u64((uint64_t)std::max<int64_t>(it.d.n_cols, 1)) : 0;
    d.fixed_w = (it.d.flags & MGT_FIXED_WIDTH)
                    ? (int32_t)(it.d.nnz > 0 ? it.d.payload_bytes / it.d.nnz : 0)
                    : -1;
    d.bounds = (const int64_t*)(W + y.o_bounds) + bo;
    for (int32_t r = 0; r <= it.d.n_parts; ++r)
      hb[bo + r] = (it.d.n_parts == 1 && !it.bounds) ? (r ? it.d.n_rows : 0) : it.bounds[r];
    bo += (uint64_t)it.d.n_parts + 1;
    std::memcpy(H + y.o_items + sizeof(ItemDev) * i, &d, sizeof(ItemDev));
  }
  if (vc) std::memcpy(H + y.o_vbounds, vc->bounds, 8ull * y.n_vbounds);
  // status words, the abort flag and the level-0 tables: each item is one
  // segment of columns [0, n_cols) split by its first digit, in tiles of
  // y.tile_cells cells
  {
    int32_t* h_status = (int32_t*)(H + y.o_status);
    std::memset(H + y.o_abort, 0, 64);
    uint32_t* h_tcnt = (uint32_t*)(H + y.o_tcnt[0]);
    uint32_t* h_hsz = (uint32_t*)(H + y.o_hsz[0]);
    uint64_t* h_tstart = (uint64_t*)(H + y.o_tstart[0]);
    uint64_t* h_hstart = (uint64_t*)(H + y.o_hstart[0]);
    uint64_t t_acc = 0, h_acc = 0;
    for (uint32_t i = 0; i < n; ++i) {
      const HostItem& it = items[i];
      h_status[i] = MGT_OK;
      Seg g;
      g.cell0 = it.dev.cell_base;
      g.byte0 = it.dev.byte_base;
      g.len = (uint32_t)it.d.nnz;
      g.key_lo = 0;
      g.key_hi = (uint32_t)it.d.n_cols;
      g.item = i;
      g.shift = (uint32_t)(it.s.key_bits - it.s.bits[0]);
      g.bits = (uint32_t)it.s.bits[0];
      g.mode = (uint32_t)it.s.part_mode;
      g.pad = 0;
      std::memcpy(H + y.o_segs[0] + sizeof(Seg) * i, &g, sizeof(Seg));
      const uint64_t tiles = ((uint64_t)it.d.nnz + y.tile_cells - 1) / y.tile_cells;
      const uint64_t hs = tiles * fanout(it.s, 0, it.d.n_parts);
      h_tcnt[i] = (uint32_t)tiles;
      h_hsz[i] = (uint32_t)hs;
      h_tstart[i] = t_acc;
      h_hstart[i] = h_acc;
      t_acc += tiles;
      h_acc += hs;
    }
    h_tstart[n] = t_acc;
    h_hstart[n] = h_acc;
  }
  time_mark(p, s, "start");
  if (kernel_upload) {
    MGT_HIP(launch_upload(W, H, up_bytes, s));
  } else {
    MGT_HIP(hipMemcpyAsync(W, H, up_bytes, hipMemcpyHostToDevice, s));
    if (!graph_staging) {
      MGT_HIP(hipEventRecord(p->upload_done, s));
      p->upload_pending = true;
    }
  }

  const ItemDev* d_items = (const ItemDev*)(W + y.o_items);
  int32_t* d_item_status = (int32_t*)(W + y.o_status);
  int32_t* d_abort = (int32_t*)(W + y.o_abort);
  auto segs = [&](int l) { return (Seg*)(W + y.o_segs[l]); };
  auto tcnt = [&](int l) { return (uint32_t*)(W + y.o_tcnt[l]); };
  auto hsz = [&](int l) { return (uint32_t*)(W + y.o_hsz[l]); };
  auto tstart = [&](int l) { return (uint64_t*)(W + y.o_tstart[l]); };
  auto hstart = [&](int l) { return (uint64_t*)(W + y.o_hstart[l]); };
  uint32_t* hcnt = (uint32_t*)(W + y.o_hcnt);
  uint32_t* hbyt = (uint32_t*)(W + y.o_hbyt);
  uint64_t* ocnt = (uint64_t*)(W + y.o_ocnt);
  uint64_t* obyt = (uint64_t*)(W + y.o_obyt);
  uint32_t* ttot = (uint32_t*)(W + y.o_ttot);
  uint64_t* tsrc = (uint64_t*)(W + y.o_tsrc);
  uint64_t* scan = (uint64_t*)(W + y.o_scan);

  if (vc) {
    ViewArgs v{};
    v.items = d_items;
    v.bounds = (const int64_t*)(W + y.o_vbounds);
    v.n_parts = (int32_t)(y.n_vbounds - 1);
    v.col = vc->col;
    v.keys = (uint32_t*)(W + y.o_vkeys);
    v.vals = (uint32_t*)(W + y.o_vvals);
    v.nnz = (uint64_t)items[0].d.nnz;
    v.n_virtual = (uint64_t)items[0].d.n_rows;
    v.n_rows = vc->n_rows;
    v.n_cols = vc->n_cols;
    v.op = vc->op;
    v.column_view = vc->column_view;
    v.validate = (p->flags & MGT_VALIDATE) ? 1 : 0;
    v.offset_width = ow;
    v.item_status = d_item_status;
    v.abort_flag = d_abort;
    MGT_HIP(launch_view_keys(v, s));
  }
  if (p->flags & MGT_VALIDATE) {
    uint64_t max_len = 0;
    for (auto& it : items) max_len = std::max<uint64_t>(max_len, (uint64_t)std::max(it.d.n_rows, it.d.nnz));
    MGT_HIP(launch_validate(d_items, n, max_len, d_item_status, d_abort, ow, s));
  }
  time_mark(p, s, "init");

  const int L = y.L;
  int32_t* d_no_pack = d_abort + 4;  // in the uploaded (zeroed) abort block
  int32_t* d_big_seg = d_abort + 5;  // likewise: a last-pass input segment of >= 2^31 bytes
  // 12-byte packed records where the slim records-only kernel runs
  const int32_t rec12 = (pk_on && wide_last) ? 1 : 0;
  // key words from the first histogram pay only where the first pass would
  // otherwise read payload offsets (fixed-width items read columns only)
  int32_t pk_keys = pk_on;
  for (uint32_t i = 0; i < n && pk_keys; ++i)
    if (items[i].d.flags & MGT_FIXED_WIDTH) pk_keys = 0;
  // The slim first pass takes packed records: its bits-only form when every
  // item's first pass splits by column bits, its partition form (fan-out up
  // to 512) when some item's first pass splits by partition.
  int32_t slim_form = n >= 1 ? 1 : 0;
  for (uint32_t i = 0; i < n && slim_form; ++i)
    if (items[i].s.part_mode)
      slim_form = fanout(items[i].s, 0, items[i].d.n_parts) <= 512u ? 2 : 0;
  for (int l = 0; l < L; ++l) {
    PassArgs a{};
    a.items = d_items;
    a.segs = segs(l);
    a.nseg = (uint32_t)y.nseg[l];
    a.pass = (uint32_t)l;
    a.tstart = tstart(l);
    a.hstart = hstart(l);
    const int bi = (l - 1) & 1, bo2 = l & 1;
    a.ks_in = l ? (const uint2*)(W + y.o_ks[bi]) : nullptr;
    a.rk_in = l ? (const uint2*)(W + y.o_rk[bi]) : nullptr;
    a.pay_in = l ? (const uint8_t*)(W + y.o_pay[bi]) : nullptr;
    a.ks_out = (uint2*)(W + y.o_ks[bo2]);
    a.rk_out = (uint2*)(W + y.o_rk[bo2]);
    a.pay_out = (uint8_t*)(W + y.o_pay[bo2]);
    a.rso_out = (L >= 2 && l == L - 1) ? (uint32_t*)(W + y.o_rso) : nullptr;
    if (a.rso_out) {
      a.pay_out = nullptr;
      a.rk_out = nullptr;
    }
    a.hcnt = hcnt;
    a.hbyt = hbyt;
    a.ttot = ttot;
    a.ocnt = ocnt;
    a.obyt = obyt;
    a.tsrc = tsrc;
    a.item_status = d_item_status;
    a.abort_flag = d_abort;
    a.g8 = align_up(y.tiles_max[l], 8);
    a.tile_cells = y.tile_cells;
    a.offset_width = ow;
    a.has_val = (vc && l == 0) ? 1 : 0;
    a.pk_on = pk_on;
    a.no_pack = d_no_pack;
    a.pk_keys = pk_keys;
    a.slim0 = (l == 0 && !vc) ? slim_form : 0;
    a.rec12 = (l == L - 1) ? rec12 : 0;
    a.big_seg = d_big_seg;
    MGT_HIP(launch_pass_hist(a, s));
    time_mark(p, s, "hist");
    const uint64_t nseg = y.nseg[l];
    MGT_HIP(launch_scan(hcnt, ocnt, hbyt, obyt, hstart(l) + nseg, y.hist_max, scan, s));
    if (l > 0) MGT_HIP(launch_scan(ttot, tsrc, nullptr, nullptr, tstart(l) + nseg, y.tiles_all_max, scan, s));
    ChildArgs c{};
    c.items = d_items;
    c.segs = segs(l);
    c.nseg = (uint32_t)nseg;
    c.pass = (uint32_t)l;
    c.tstart = tstart(l);
    c.hstart = hstart(l);
    c.ocnt = ocnt;
    c.obyt = obyt;
    c.children = segs(l + 1);
    c.child_tiles = (l + 1 < L) ? tcnt(l + 1) : nullptr;
    c.child_hsize = (l + 1 < L) ? hsz(l + 1) : nullptr;
    c.tile_cells = y.tile_cells;
    c.abort_flag = d_abort;
    c.big_seg = (rec12 && l + 2 == L) ? d_big_seg : nullptr;
    MGT_HIP(launch_children(c, s));
    if (l + 1 < L)
      MGT_HIP(launch_scan(tcnt(l + 1), tstart(l + 1), hsz(l + 1), hstart(l + 1), nullptr, y.nseg[l + 1], scan, s));
    time_mark(p, s, "scan");
    MGT_HIP(launch_pass_scatter(a, s));
    time_mark(p, s, "scatter");
  }
  FinishArgs f{};
  f.items = d_items;
  f.n_items = n;
  f.buckets = segs(L);
  f.nbuckets = (uint32_t)y.nseg[L];
  const int bl = (L - 1) & 1;
  f.ks_in = (const uint2*)(W + y.o_ks[bl]);
  f.rk_in = (const uint2*)(W + y.o_rk[bl]);
  f.pay_in = (const uint8_t*)(W + y.o_pay[L >= 2 ? (L - 2) & 1 : bl]);
  f.rso_in = L >= 2 ? (const uint32_t*)(W + y.o_rso) : nullptr;
  if (f.rso_in) f.rk_in = nullptr;
  f.abort_flag = d_abort;
  f.item_status = d_item_status;
  f.d_status = d_status;
  f.offset_width = ow;
  f.g8 = align_up(y.nseg[L], 8);
  f.pk_on = pk_on;
  f.no_pack = d_no_pack;
  f.rec12 = rec12;
  f.big_seg = d_big_seg;
  if (pk_on && f.rso_in) {
    // packed records: whole buckets first, the rest (and the tails) after.
    // Buckets of at most 4,096 cells on average go to the 512-thread form,
    // two workgroups per CU (MGT_BUCKET_THREADS=512 or 1024 forces one).
    f.bucket_done = W + y.o_bdone;
    const uint64_t nb = std::max<uint64_t>(y.nseg[L], 1);
    const bool small = y.total_nnz <= kBucketSmallMean * nb;
    const int forced = env_cap("MGT_BUCKET_THREADS", 512, 1024, 0);
    const bool run512 = forced ? forced == 512 : small;
    const bool run1024 = forced ? forced == 1024 : true;
    if (run512) {
      f.bk_threads = 512;
      f.skip_done = 0;
      f.grid = 2 * device_cus();
      MGT_HIP(launch_finish_bucket(f, s));
      time_mark(p, s, "finishs");
    }
    if (run1024) {  // after the 512-thread launch: the buckets it left, up to 9,216 cells
      f.bk_threads = 1024;
      f.skip_done = run512 ? 1 : 0;
      f.grid = device_cus();
      MGT_HIP(launch_finish_bucket(f, s));
      time_mark(p, s, "finishb");
    }
  }
  MGT_HIP(launch_finish(f, s));
  time_mark(p, s, "finish");

  return MGT_OK;
}

void fill_outputs(ItemDev& d, const void* row_ptr, const int32_t* col, const void* payload_off,
                  const uint8_t* payload, void* t_row_ptr, int32_t* t_col, void* t_payload_off,
                  uint8_t* t_payload, uint32_t* perm) {
  std::memset(&d, 0, sizeof(d));
  d.row_ptr = row_ptr;
  d.col = col;
  d.poff = payload_off;
  d.payload = payload;
  d.t_row_ptr = t_row_ptr;
  d.t_col = t_col;
  d.t_poff = t_payload_off;
  d.t_payload = t_payload;
  d.perm = perm;
}

int check_io(const mgt_desc& d, uint32_t flags, const void* row_ptr, const int32_t* col,
             const void* payload_off, const uint8_t* payload, const void* t_row_ptr,
             const int32_t* t_col, const void* t_payload_off, const uint8_t* t_payload,
             const uint32_t* perm) {
  const bool fixed = (d.flags & MGT_FIXED_WIDTH) != 0;
  if (!row_ptr || !t_row_ptr) return MGT_EINVAL;
  if (!fixed && (!payload_off || !t_payload_off)) return MGT_EINVAL;
  if (d.nnz > 0 && (!col || !t_col)) return MGT_EINVAL;
  if (d.payload_bytes > 0 && (!payload || !t_payload)) return MGT_EINVAL;
  const bool want_perm = (flags & MGT_EMIT_PERM) != 0;
  if (!want_perm && perm) return MGT_EINVAL;
  if (want_perm && !perm && d.nnz > 0) return MGT_EINVAL;
  return MGT_OK;
}

// Records one call into g: the pinned upload buffer and a private stream are
// made first (nothing is allocated while capturing), then the call is
// captured on that stream and instantiated.
int record_graph(mgt_plan_s* p, Items items, const Layout& y, void* ws,
                 int32_t* d_status, mgt_graph_s* g) {
  if (hipHostMalloc(&g->staging, upload_bytes(y), hipHostMallocDefault) != hipSuccess) {
    g->staging = nullptr;
    return MGT_ENOMEM;
  }
  hipStream_t s = nullptr;
  if (hipStreamCreate(&s) != hipSuccess) return MGT_EHIP;
  hipGraph_t graph = nullptr;
  int st = MGT_OK;
  if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) st = MGT_EHIP;
  if (st == MGT_OK) {
    st = run(p, items, y, ws, d_status, s, nullptr, g->staging);
    // the capture is ended whatever happened inside it
    if (hipStreamEndCapture(s, &graph) != hipSuccess && st == MGT_OK) st = MGT_EHIP;
  }
  if (st == MGT_OK && hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0) != hipSuccess) {
    g->exec = nullptr;
    st = MGT_EHIP;
  }
  if (graph) (void)hipGraphDestroy(graph);
  (void)hipStreamDestroy(s);
  return st;
}

// no_alloc: the call allocates nothing (no pinned staging, no events, no heap):
// plans with MGT_DEBUG_TIMING are refused and the descriptor goes up through
// kernel arguments.
int single_call(mgt_plan_s* p, bool partitioned, const void* row_ptr, const int32_t* col,
                const void* payload_off, const uint8_t* payload, void* t_row_ptr, int32_t* t_col,
                void* t_payload_off, uint8_t* t_payload, uint32_t* perm, int64_t* xc, int64_t* xb,
                int64_t* pco, int64_t* pbo, int64_t* sd, int64_t* rd, void* ws, size_t ws_bytes,
                int32_t* d_status, hipStream_t s, mgt_graph_s* graph = nullptr,
                bool no_alloc = false) {
  if (!p || p->batch || p->view_op >= 0) return MGT_EINVAL;
  if (no_alloc && (p->flags & MGT_DEBUG_TIMING)) return MGT_EINVAL;
  const mgt_desc& d = p->desc;
  int st = check_io(d, p->flags, row_ptr, col, payload_off, payload, t_row_ptr, t_col, t_payload_off,
                    t_payload, perm);
  if (st != MGT_OK) return st;
  if (partitioned && (!xc || !xb || !pco || !pbo)) return MGT_EINVAL;
  if (!ws || ((uintptr_t)ws & 255u)) return MGT_EINVAL;
  // The schedule is read under the plan's lock (mgt_plan_set_schedule may
  // change it from another thread) and the lock is held through the launches.
  std::lock_guard<std::mutex> lock(p->mu);
  HostItem items[1] = {};
  HostItem& it = items[0];
  it.d = d;
  it.bounds = p->bounds.empty() ? nullptr : p->bounds.data();
  it.s = make_sched(d.n_cols, d.nnz, d.payload_bytes, d.n_parts, it.bounds, partitioned, true,
                    &p->tune);
  it.tile = p->tune.tile;
  if (!partitioned) it.d.n_parts = 1;
  fill_outputs(it.dev, row_ptr, col, payload_off, payload, t_row_ptr, t_col, t_payload_off, t_payload,
               perm);
  if (partitioned) {
    it.dev.xfer_cells = xc;
    it.dev.xfer_bytes = xb;
    it.dev.part_cell_off = pco;
    it.dev.part_byte_off = pbo;
    it.dev.sdispls = sd;
    it.dev.rdispls = rd;
  }
  if (!partitioned) it.bounds = nullptr;
  Layout y = make_layout(Items(items, 1));
  if (ws_bytes < y.bytes) return MGT_ENOMEM;
  if (graph) return record_graph(p, Items(items, 1), y, ws, d_status, graph);
  p->timing.used = 0;
  if (no_alloc) {
    alignas(16) uint8_t up[kNoAllocUpload];
    if (upload_bytes(y) > sizeof(up)) return MGT_EUNSUPPORTED;
    return run(p, Items(items, 1), y, ws, d_status, s, nullptr, nullptr, up);
  }
  return run(p, Items(items, 1), y, ws, d_status, s);
}

size_t single_ws(const mgt_desc& d, const int64_t* bounds, bool partitioned, const Tune& t) {
  std::vector<HostItem> items(1);
  items[0].d = d;
  if (!partitioned) items[0].d.n_parts = 1;
  items[0].bounds = bounds;
  items[0].s =
      make_sched(d.n_cols, d.nnz, d.payload_bytes, d.n_parts, bounds, partitioned, true, &t);
  items[0].tile = t.tile;
  std::memset(&items[0].dev, 0, sizeof(ItemDev));
  return make_layout(items).bytes;
}

// Workspace estimate for a batch at the limits; mgt_batch_workspace gives the
// exact size of a given batch. Level buffers dominate: 2 x (16 B per cell +
// payload); payload is bounded by the caller, so it is not included here.
size_t batch_estimate(const mgt_batch_limits& lim) {
  const uint64_t cells = (uint64_t)lim.max_total_nnz;
  const uint64_t segs = 2ull * (uint64_t)lim.max_total_cols + cells / 512 + (uint64_t)lim.max_items;
  return (size_t)(2 * 16 * cells + 4 * segs * (sizeof(Seg) + 24) + 64ull * (cells / 16) + (1u << 20));
}

int batch_items(mgt_plan_s* p, const mgt_item* in, int32_t n, std::vector<HostItem>& items) {
  if (!p || !p->batch || n < 0 || (n > 0 && !in)) return MGT_EINVAL;
  if (n > p->lim.max_items || n > kMaxItems) return MGT_EUNSUPPORTED;
  Tune tune;  // the plan's schedule setting, read under its lock
  {
    std::lock_guard<std::mutex> lock(p->mu);
    tune = p->tune;
  }
  items.resize((size_t)n);
  int64_t tn = 0, tc = 0, tr = 0, tp = 0;
  for (int32_t i = 0; i < n; ++i) {
    const mgt_item& m = in[i];
    int st = check_desc(&m.desc, false);
    if (st != MGT_OK) return st;
    if (m.desc.offset_width != p->lim.offset_width) return MGT_EINVAL;
    st = check_io(m.desc, p->flags, m.row_ptr, m.col, m.payload_off, m.payload, m.t_row_ptr, m.t_col,
                  m.t_payload_off, m.t_payload, m.perm);
    if (st != MGT_OK) return st;
    const bool part = m.desc.n_parts > 1;
    if (part && (!m.xfer_cells || !m.xfer_bytes || !m.part_cell_off || !m.part_byte_off))
      return MGT_EINVAL;
    tn += m.desc.nnz;
    tc += m.desc.n_cols;
    tr += m.desc.n_rows;
    tp += m.desc.n_parts;
    if (m.desc.nnz > p->lim.max_item_nnz || m.desc.n_cols > p->lim.max_item_cols) return MGT_EUNSUPPORTED;
    HostItem& it = items[(size_t)i];
    it.d = m.desc;
    it.bounds = m.desc.part_bounds;
    it.s = make_sched(m.desc.n_cols, m.desc.nnz, m.desc.payload_bytes, m.desc.n_parts,
                      m.desc.part_bounds, part, false, &tune);
    it.tile = tune.tile;
    fill_outputs(it.dev, m.row_ptr, m.col, m.payload_off, m.payload, m.t_row_ptr, m.t_col,
                 m.t_payload_off, m.t_payload, m.perm);
    if (part) {
      it.dev.xfer_cells = m.xfer_cells;
      it.dev.xfer_bytes = m.xfer_bytes;
      it.dev.part_cell_off = m.part_cell_off;
      it.dev.part_byte_off = m.part_byte_off;
      it.dev.sdispls = m.sdispls;
      it.dev.rdispls = m.rdispls;
    }
  }
  if (tn > p->lim.max_total_nnz || tc > p->lim.max_total_cols || tr > p->lim.max_total_rows ||
      tp > p->lim.max_total_parts)
    return MGT_EUNSUPPORTED;
  // Every item makes as many passes as the item that needs the most (the
  // layout pads the others with 0-bit passes, which copy their records). An
  // item whose fewest passes come from a wider finish than its ideal takes
  // the padded passes' bits instead, keeping finish buckets near 4 * kSub
  // cells (wider ones outgrow the whole-bucket finish).
  int L = 1;
  for (const HostItem& it : items) L = std::max(L, it.s.n_levels);
  for (int32_t i = 0; i < n && L > 1; ++i) {
    HostItem& it = items[(size_t)i];
    if (it.s.n_levels >= L) continue;
    const mgt_desc& d = in[i].desc;
    const Sched s = make_sched(d.n_cols, d.nnz, d.payload_bytes, d.n_parts, d.part_bounds,
                               d.n_parts > 1, false, &tune, L);
    if (s.n_levels <= L) it.s = s;
  }
  return MGT_OK;
}

}  // namespace

namespace mgt {
// The allocation-free transpose behind mgt_transpose_noalloc (noalloc.hip),
// on a workspace the caller guarantees (the library's scratch array).
int noalloc_call(mgt_plan_s* p, int32_t partitioned, const void* row_ptr, const int32_t* col,
                 const void* payload_off, const uint8_t* payload, void* t_row_ptr, int32_t* t_col,
                 void* t_payload_off, uint8_t* t_payload, uint32_t* perm, int64_t* xfer_cells,
                 int64_t* xfer_bytes, int64_t* part_cell_off, int64_t* part_byte_off,
                 int64_t* sdispls, int64_t* rdispls, void* ws, size_t ws_bytes, int32_t* d_status,
                 hipStream_t stream) {
  if (partitioned && p && !p->batch && p->desc.n_parts > 1 && p->desc.n_rows != p->desc.n_cols)
    return MGT_EINVAL;
  return single_call(p, partitioned != 0, row_ptr, col, payload_off, payload, t_row_ptr, t_col,
                     t_payload_off, t_payload, perm, xfer_cells, xfer_bytes, part_cell_off,
                     part_byte_off, sdispls, rdispls, ws, ws_bytes, d_status, stream, nullptr,
                     true);
}
}  // namespace mgt

extern "C" {

const char* mgt_version(void) { return "mgt 0.1.0 (gfx950)"; }

int mgt_plan(const mgt_desc* desc, mgt_plan_t* out, size_t* workspace_bytes) {
  if (!out) return MGT_EINVAL;
  int st = check_desc(desc, false);
  if (st != MGT_OK) return st;
  if ((desc->flags & ~(uint32_t)(MGT_VALIDATE | MGT_EMIT_PERM | MGT_DEBUG_TIMING | MGT_FIXED_WIDTH)) != 0)
    return MGT_EINVAL;
  mgt_plan_s* p = new (std::nothrow) mgt_plan_s();
  if (!p) return MGT_ENOMEM;
  p->desc = *desc;
  p->flags = desc->flags;
  if (desc->part_bounds) p->bounds.assign(desc->part_bounds, desc->part_bounds + desc->n_parts + 1);
  else p->bounds = {0, desc->n_rows};
  p->desc.part_bounds = p->bounds.data();
  p->ws_plain = single_ws(p->desc, p->bounds.data(), false, p->tune);
  p->ws_part = single_ws(p->desc, p->bounds.data(), true, p->tune);
  *out = p;
  if (workspace_bytes) *workspace_bytes = std::max(p->ws_plain, p->ws_part);
  return MGT_OK;
}

int mgt_plan_destroy(mgt_plan_t p) {
  if (!p) return MGT_EINVAL;
  if (p->upload_pending) (void)hipEventSynchronize(p->upload_done);
  if (p->staging) (void)hipHostFree(p->staging);
  if (p->upload_done) (void)hipEventDestroy(p->upload_done);
  for (auto e : p->timing.ev) (void)hipEventDestroy(e);
  delete p;
  return MGT_OK;
}

int mgt_transpose(mgt_plan_t plan, const void* row_ptr, const int32_t* col, const void* payload_off,
                  const uint8_t* payload, void* t_row_ptr, int32_t* t_col, void* t_payload_off,
                  uint8_t* t_payload, uint32_t* perm, void* workspace, size_t workspace_bytes,
                  int32_t* d_status, hipStream_t stream) {
  return single_call(plan, false, row_ptr, col, payload_off, payload, t_row_ptr, t_col, t_payload_off,
                     t_payload, perm, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, workspace,
                     workspace_bytes, d_status, stream);
}

int mgt_transpose_partitioned(mgt_plan_t plan, const void* row_ptr, const int32_t* col,
                              const void* payload_off, const uint8_t* payload, void* t_row_ptr,
                              int32_t* t_col, void* t_payload_off, uint8_t* t_payload, uint32_t* perm,
                              int64_t* xfer_cells, int64_t* xfer_bytes, int64_t* part_cell_off,
                              int64_t* part_byte_off, int64_t* sdispls, int64_t* rdispls,
                              void* workspace, size_t workspace_bytes, int32_t* d_status,
                              hipStream_t stream) {
  if (plan && !plan->batch && plan->desc.n_parts > 1 && plan->desc.n_rows != plan->desc.n_cols)
    return MGT_EINVAL;
  return single_call(plan, true, row_ptr, col, payload_off, payload, t_row_ptr, t_col, t_payload_off,
                     t_payload, perm, xfer_cells, xfer_bytes, part_cell_off, part_byte_off, sdispls,
                     rdispls, workspace, workspace_bytes, d_status, stream);
}

int mgt_view_plan(const mgt_desc* desc, int32_t op, int32_t in_view, mgt_plan_t* out,
                  size_t* workspace_bytes) {
  if (!out) return MGT_EINVAL;
  if ((op != MGT_LOCAL_TRANSPOSE && op != MGT_VIEW_SWAP) ||
      (in_view != MGT_ROW_VIEW && in_view != MGT_COLUMN_VIEW))
    return MGT_EINVAL;
  int st = check_desc(desc, false);
  if (st != MGT_OK) return st;
  if ((desc->flags & ~(uint32_t)(MGT_VALIDATE | MGT_EMIT_PERM | MGT_DEBUG_TIMING | MGT_FIXED_WIDTH)) != 0)
    return MGT_EINVAL;
  const int64_t R = desc->n_parts;
  if (R > 1 && desc->n_rows != desc->n_cols) return MGT_EINVAL;
  if (desc->nnz > 0 && (desc->n_rows == 0 || desc->n_cols == 0)) return MGT_EINVAL;
  const int64_t n_virtual = in_view == MGT_COLUMN_VIEW ? R * desc->n_rows : desc->n_rows;
  int64_t n_key;
  if (op == MGT_LOCAL_TRANSPOSE) n_key = in_view == MGT_ROW_VIEW ? R * desc->n_cols : desc->n_cols;
  else n_key = in_view == MGT_ROW_VIEW ? R * desc->n_rows : desc->n_rows;
  if (n_virtual >= (1ll << 31) || n_key >= (1ll << 31)) return MGT_EUNSUPPORTED;
  mgt_plan_s* p = new (std::nothrow) mgt_plan_s();
  if (!p) return MGT_ENOMEM;
  p->desc = *desc;
  p->flags = desc->flags;
  if (desc->part_bounds) p->bounds.assign(desc->part_bounds, desc->part_bounds + R + 1);
  else p->bounds = {0, desc->n_rows};
  p->desc.part_bounds = p->bounds.data();
  p->view_op = op;
  p->column_view = in_view == MGT_COLUMN_VIEW;
  mgt_desc v = *desc;
  v.n_rows = n_virtual;
  v.n_cols = n_key;
  v.n_parts = 1;
  v.part_bounds = nullptr;
  p->view_desc = v;
  std::vector<HostItem> items(1);
  items[0].d = v;
  items[0].bounds = nullptr;
  items[0].s = make_sched(v.n_cols, v.nnz, v.payload_bytes, 1, nullptr, false, true);
  std::memset(&items[0].dev, 0, sizeof(ItemDev));
  p->ws_view = make_layout(items, (uint64_t)R + 1).bytes;
  *out = p;
  if (workspace_bytes) *workspace_bytes = p->ws_view;
  return MGT_OK;
}

int mgt_view_transform(mgt_plan_t p, const void* row_ptr, const int32_t* col,
                       const void* payload_off, const uint8_t* payload, void* o_row_ptr,
                       int32_t* o_col, void* o_payload_off, uint8_t* o_payload, uint32_t* perm,
                       void* workspace, size_t workspace_bytes, int32_t* d_status,
                       hipStream_t stream) {
  if (!p || p->batch || p->view_op < 0) return MGT_EINVAL;
  const mgt_desc& v = p->view_desc;
  int st = check_io(v, p->flags, row_ptr, col, payload_off, payload, o_row_ptr, o_col, o_payload_off,
                    o_payload, perm);
  if (st != MGT_OK) return st;
  if (!workspace || ((uintptr_t)workspace & 255u)) return MGT_EINVAL;
  std::vector<HostItem> items(1);
  HostItem& it = items[0];
  it.d = v;
  it.bounds = nullptr;
  it.s = make_sched(v.n_cols, v.nnz, v.payload_bytes, 1, nullptr, false, true);
  fill_outputs(it.dev, row_ptr, col, payload_off, payload, o_row_ptr, o_col, o_payload_off,
               o_payload, perm);
  Layout y = make_layout(items, p->bounds.size());
  if (workspace_bytes < y.bytes) return MGT_ENOMEM;
  uint8_t* W = (uint8_t*)workspace;
  it.dev.col = (const int32_t*)(W + y.o_vkeys);  // the passes sort by the keys ...
  it.dev.vval = (const uint32_t*)(W + y.o_vvals);  // ... and carry the values
  ViewCall vc{col, p->bounds.data(), p->desc.n_rows, p->desc.n_cols, p->view_op, p->column_view};
  std::lock_guard<std::mutex> lock(p->mu);
  p->timing.used = 0;
  return run(p, items, y, workspace, d_status, stream, &vc);
}

int mgt_graph_create(mgt_plan_t plan, int32_t partitioned, const void* row_ptr, const int32_t* col,
                     const void* payload_off, const uint8_t* payload, void* t_row_ptr,
                     int32_t* t_col, void* t_payload_off, uint8_t* t_payload, uint32_t* perm,
                     int64_t* xfer_cells, int64_t* xfer_bytes, int64_t* part_cell_off,
                     int64_t* part_byte_off, int64_t* sdispls, int64_t* rdispls, void* workspace,
                     size_t workspace_bytes, int32_t* d_status, mgt_graph_t* out) {
  if (!plan || !out || plan->batch || plan->view_op >= 0) return MGT_EINVAL;
  if (plan->flags & MGT_DEBUG_TIMING) return MGT_EINVAL;
  if (partitioned && plan->desc.n_parts > 1 && plan->desc.n_rows != plan->desc.n_cols)
    return MGT_EINVAL;
  mgt_graph_s* g = new (std::nothrow) mgt_graph_s();
  if (!g) return MGT_ENOMEM;
  int st = single_call(plan, partitioned != 0, row_ptr, col, payload_off, payload, t_row_ptr,
                       t_col, t_payload_off, t_payload, perm, xfer_cells, xfer_bytes,
                       part_cell_off, part_byte_off, sdispls, rdispls, workspace,
                       workspace_bytes, d_status, nullptr, g);
  if (st == MGT_OK && !g->exec) st = MGT_EINVAL;
  if (st != MGT_OK) {
    mgt_graph_destroy(g);
    return st;
  }
  *out = g;
  return MGT_OK;
}

int mgt_graph_launch(mgt_graph_t g, hipStream_t stream) {
  if (!g || !g->exec) return MGT_EINVAL;
  return hipGraphLaunch(g->exec, stream) == hipSuccess ? MGT_OK : MGT_EHIP;
}

int mgt_graph_destroy(mgt_graph_t g) {
  if (!g) return MGT_EINVAL;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->staging) (void)hipHostFree(g->staging);
  delete g;
  return MGT_OK;
}

int mgt_batch_plan(const mgt_batch_limits* lim, mgt_plan_t* out, size_t* workspace_bytes) {
  if (!lim || !out) return MGT_EINVAL;
  if (lim->max_items < 1 || lim->max_items > kMaxItems) return MGT_EUNSUPPORTED;
  if (lim->offset_width != 4 && lim->offset_width != 8) return MGT_EINVAL;
  if (lim->max_total_nnz < 0 || lim->max_total_cols < 0 || lim->max_total_rows < 0 ||
      lim->max_total_parts < 0 || lim->max_item_nnz < 0 || lim->max_item_cols < 0)
    return MGT_EINVAL;
  if ((lim->flags & ~(uint32_t)(MGT_VALIDATE | MGT_EMIT_PERM | MGT_DEBUG_TIMING)) != 0) return MGT_EINVAL;
  mgt_plan_s* p = new (std::nothrow) mgt_plan_s();
  if (!p) return MGT_ENOMEM;
  p->batch = true;
  p->lim = *lim;
  p->flags = lim->flags;
  *out = p;
  if (workspace_bytes) *workspace_bytes = batch_estimate(*lim);
  return MGT_OK;
}

int mgt_batch_workspace(mgt_plan_t plan, const mgt_item* items, int32_t n_items, size_t* bytes) {
  if (!bytes) return MGT_EINVAL;
  std::vector<HostItem> hi;
  int st = batch_items(plan, items, n_items, hi);
  if (st != MGT_OK) return st;
  *bytes = n_items ? make_layout(hi).bytes : 256;
  return MGT_OK;
}

int mgt_batch_submit(mgt_plan_t plan, const mgt_item* items, int32_t n_items, void* workspace,
                     size_t workspace_bytes, int32_t* d_status, hipStream_t stream, hipEvent_t done) {
  std::vector<HostItem> hi;
  int st = batch_items(plan, items, n_items, hi);
  if (st != MGT_OK) return st;
  if (n_items == 0) {
    if (done && hipEventRecord(done, stream) != hipSuccess) return MGT_EHIP;
    return MGT_OK;
  }
  if (!workspace || ((uintptr_t)workspace & 255u)) return MGT_EINVAL;
  Layout y = make_layout(hi);
  if (workspace_bytes < y.bytes) return MGT_ENOMEM;
  std::lock_guard<std::mutex> lock(plan->mu);
  plan->timing.used = 0;
  st = run(plan, hi, y, workspace, d_status, stream);
  if (st != MGT_OK) return st;
  if (done && hipEventRecord(done, stream) != hipSuccess) return MGT_EHIP;
  return MGT_OK;
}

int mgt_batch_graph_create(mgt_plan_t plan, const mgt_item* items, int32_t n_items,
                           void* workspace, size_t workspace_bytes, int32_t* d_status,
                           mgt_graph_t* out) {
  if (!out) return MGT_EINVAL;
  if (plan && (plan->flags & MGT_DEBUG_TIMING)) return MGT_EINVAL;
  std::vector<HostItem> hi;
  int st = batch_items(plan, items, n_items, hi);
  if (st != MGT_OK) return st;
  if (n_items == 0) return MGT_EINVAL;  // nothing to record
  if (!workspace || ((uintptr_t)workspace & 255u)) return MGT_EINVAL;
  Layout y = make_layout(hi);
  if (workspace_bytes < y.bytes) return MGT_ENOMEM;
  mgt_graph_s* g = new (std::nothrow) mgt_graph_s();
  if (!g) return MGT_ENOMEM;
  {
    std::lock_guard<std::mutex> lock(plan->mu);
    st = record_graph(plan, hi, y, workspace, d_status, g);
  }
  if (st == MGT_OK && !g->exec) st = MGT_EINVAL;
  if (st != MGT_OK) {
    mgt_graph_destroy(g);
    return st;
  }
  *out = g;
  return MGT_OK;
}

int mgt_plan_set_schedule(mgt_plan_t plan, int32_t pass_bits, int32_t finish_bits,
                          int32_t tile_cells, size_t* workspace_bytes) {
  if (!plan || plan->view_op >= 0) return MGT_EINVAL;
  if (pass_bits < 0 || pass_bits > kMaxBitsPerPass) return MGT_EINVAL;
  if (finish_bits < -1 || finish_bits > kMaxFinishBits) return MGT_EINVAL;
  if (tile_cells != 0 && tile_cells != 2048 && tile_cells != 4096 && tile_cells != 8192 &&
      tile_cells != 16384)
    return MGT_EINVAL;
  std::lock_guard<std::mutex> lock(plan->mu);
  Tune t;
  t.pass_bits = pass_bits;
  t.finish_bits = finish_bits;
  t.tile = (uint32_t)tile_cells;
  if (plan->batch) {
    // applied to every item of later submits (an item whose schedule would
    // need more than kMaxLevels passes keeps the rule's); the exact
    // workspace of a batch is mgt_batch_workspace's
    plan->tune = t;
    if (workspace_bytes) *workspace_bytes = batch_estimate(plan->lim);
    return MGT_OK;
  }
  const mgt_desc& d = plan->desc;
  for (int part = 0; part < 2; ++part) {  // a setting that needs over kMaxLevels passes is refused
    const Sched s = make_sched_tuned(d.n_cols, d.nnz, d.payload_bytes, d.n_parts,
                                     plan->bounds.data(), part != 0, true, &t);
    if (s.n_levels > kMaxLevels) return MGT_EUNSUPPORTED;
  }
  plan->tune = t;
  plan->ws_plain = single_ws(d, plan->bounds.data(), false, t);
  plan->ws_part = single_ws(d, plan->bounds.data(), true, t);
  if (workspace_bytes) *workspace_bytes = std::max(plan->ws_plain, plan->ws_part);
  return MGT_OK;
}

int mgt_plan_schedule(mgt_plan_t plan, int32_t partitioned, int32_t* out) {
  if (!plan || !out || plan->batch || plan->view_op >= 0) return MGT_EINVAL;
  std::lock_guard<std::mutex> lock(plan->mu);
  const mgt_desc& d = plan->desc;
  const Sched s = make_sched(d.n_cols, d.nnz, d.payload_bytes, d.n_parts, plan->bounds.data(),
                             partitioned != 0,
                             true, &plan->tune);  // as a call with these arguments makes it
  out[0] = s.n_levels;
  for (int l = 0; l < kMaxLevels; ++l) out[1 + l] = l < s.n_levels ? s.bits[l] : 0;
  out[5] = s.finish_bits;
  out[6] = (int32_t)(plan->tune.tile ? plan->tune.tile : tile_cells_for((uint64_t)d.nnz));
  out[7] = s.part_mode;
  return MGT_OK;
}

}  // extern "C"

namespace {

// Workspace of mgt_symmetrize: the transpose's own, then the transposed
// triangle and the per-row counts of S with their scans.
struct SymLayout {
  uint64_t o_t_row_ptr, o_t_col, o_t_poff, o_t_pay, o_cnt, o_byt, o_ocnt, o_obyt, o_scan, o_st;
  uint64_t bytes;
};

SymLayout sym_layout(const mgt_plan_s* p) {
  const mgt_desc& d = p->desc;
  const uint64_t n = (uint64_t)d.n_rows, nnz = (uint64_t)d.nnz, ow = (uint64_t)d.offset_width;
  SymLayout y{};
  uint64_t o = align_up(p->ws_plain, 256);
  auto take = [&](uint64_t bytes) {
    const uint64_t at = o;
    o = align_up(o + bytes, 256);
    return at;
  };
  y.o_t_row_ptr = take((n + 1) * ow);
  y.o_t_col = take(4 * nnz);
  y.o_t_poff = take((nnz + 1) * ow);
  y.o_t_pay = take((uint64_t)d.payload_bytes + 16);
  y.o_cnt = take(4 * n);
  y.o_byt = take(4 * n);
  y.o_ocnt = take(8 * (n + 1));
  y.o_obyt = take(8 * (n + 1));
  y.o_scan = take(scan_scratch_bytes(n));
  y.o_st = take(64);
  y.bytes = o;
  return y;
}

// A plan mgt_symmetrize takes: a square single-matrix plan without
// MGT_EMIT_PERM, MGT_FIXED_WIDTH or MGT_DEBUG_TIMING, whose doubled sizes fit
// its offsets.
int sym_check_plan(const mgt_plan_s* p) {
  if (!p || p->batch || p->view_op >= 0) return MGT_EINVAL;
  const mgt_desc& d = p->desc;
  if (d.n_rows != d.n_cols) return MGT_EINVAL;
  if (p->flags & (MGT_EMIT_PERM | MGT_FIXED_WIDTH | MGT_DEBUG_TIMING)) return MGT_EINVAL;
  if (2 * d.nnz >= (1ll << 32)) return MGT_EUNSUPPORTED;
  if (d.offset_width == 4 && (2 * d.nnz >= (1ll << 31) || 2 * d.payload_bytes >= (1ll << 31)))
    return MGT_EUNSUPPORTED;
  return MGT_OK;
}

}  // namespace

extern "C" {

int mgt_symmetrize_workspace(mgt_plan_t plan, size_t* workspace_bytes) {
  if (!workspace_bytes) return MGT_EINVAL;
  const int st = sym_check_plan(plan);
  if (st != MGT_OK) return st;
  std::lock_guard<std::mutex> lock(plan->mu);
  *workspace_bytes = (size_t)sym_layout(plan).bytes;
  return MGT_OK;
}

int mgt_symmetrize(mgt_plan_t plan, int32_t triangle, const void* row_ptr, const int32_t* col,
                   const void* payload_off, const uint8_t* payload, void* s_row_ptr, int32_t* s_col,
                   void* s_payload_off, uint8_t* s_payload, int64_t* d_sizes, void* workspace,
                   size_t workspace_bytes, int32_t* d_status, hipStream_t stream) {
  int st = sym_check_plan(plan);
  if (st != MGT_OK) return st;
  if (triangle != MGT_LOWER && triangle != MGT_UPPER) return MGT_EINVAL;
  const mgt_desc& d = plan->desc;
  if (!s_row_ptr || !s_payload_off || (d.nnz > 0 && (!s_col || !col)) ||
      (d.payload_bytes > 0 && (!s_payload || !payload)) || !row_ptr || !payload_off)
    return MGT_EINVAL;
  if (!workspace || ((uintptr_t)workspace & 255u)) return MGT_EINVAL;
  SymLayout y;
  {
    std::lock_guard<std::mutex> lock(plan->mu);
    y = sym_layout(plan);
  }
  if (workspace_bytes < y.bytes) return MGT_ENOMEM;
  uint8_t* W = (uint8_t*)workspace;
  SymArgs a{};
  a.n = (uint64_t)d.n_rows;
  a.nnz = (uint64_t)d.nnz;
  a.pbytes = (uint64_t)d.payload_bytes;
  a.cap_cells = 2 * a.nnz;
  a.cap_bytes = 2 * a.pbytes;
  a.ow = d.offset_width;
  a.lower = triangle == MGT_LOWER ? 1 : 0;
  a.validate = (plan->flags & MGT_VALIDATE) ? 1 : 0;
  a.row_ptr = row_ptr;
  a.col = col;
  a.poff = payload_off;
  a.payload = payload;
  a.t_row_ptr = W + y.o_t_row_ptr;
  a.t_col = (const int32_t*)(W + y.o_t_col);
  a.t_poff = W + y.o_t_poff;
  a.t_payload = W + y.o_t_pay;
  a.s_row_ptr = s_row_ptr;
  a.s_col = s_col;
  a.s_poff = s_payload_off;
  a.s_payload = s_payload;
  a.d_sizes = d_sizes;
  a.d_status = d_status;
  a.st = (int32_t*)(W + y.o_st);
  a.cnt = (uint32_t*)(W + y.o_cnt);
  a.byt = (uint32_t*)(W + y.o_byt);
  a.ocnt = (uint64_t*)(W + y.o_ocnt);
  a.obyt = (uint64_t*)(W + y.o_obyt);
  a.scan = (uint64_t*)(W + y.o_scan);
  // the stored triangle's transpose (its status word becomes the call's)
  st = single_call(plan, false, row_ptr, col, payload_off, payload, (void*)a.t_row_ptr,
                   (int32_t*)a.t_col, (void*)a.t_poff, (uint8_t*)a.t_payload, nullptr, nullptr,
                   nullptr, nullptr, nullptr, nullptr, nullptr, workspace, plan->ws_plain, a.st,
                   stream);
  if (st != MGT_OK) return st;
  return launch_symmetrize(a, stream) == hipSuccess ? MGT_OK : MGT_EHIP;
}

int mgt_plan_stage_times(mgt_plan_t plan, float* ms, const char** names, int32_t capacity,
                         int32_t* count) {
  if (!plan || !count) return MGT_EINVAL;
  std::lock_guard<std::mutex> lock(plan->mu);
  Timing& t = plan->timing;
  const int n = t.used > 1 ? t.used - 1 : 0;
  *count = n;
  if (n == 0) return MGT_OK;
  if (hipEventSynchronize(t.ev[t.used - 1]) != hipSuccess) return MGT_EHIP;
  for (int i = 0; i < n && i < capacity; ++i) {
    float v = 0.f;
    if (hipEventElapsedTime(&v, t.ev[i], t.ev[i + 1]) != hipSuccess) return MGT_EHIP;
    if (ms) ms[i] = v;
    if (names) names[i] = t.names[i + 1];
  }
  return MGT_OK;
}

}  // extern "C"
