// Seeded synthetic XCSR multigraph generators.
//
// This module produces inputs only: row offsets, column ids, per-cell payload
// offsets and payload bytes. It holds none of the transpose's arithmetic and is
// shared, as plain input data, by the CPU oracle and by the GPU library's tests
// and benchmarks.
//
// Randomness is counter based: every draw is SplitMix64's output function
// (Steele, Lea & Flood, "Fast splittable pseudorandom number generators",
// OOPSLA 2014) applied to key + (counter + 1) * golden-gamma, with a key derived
// from (seed, stream, index). Any row, cell or byte can therefore be generated
// independently, so rows are filled by several host threads and the result does
// not depend on the thread count.
//
// Workload shapes follow the paper's two benchmark families (Section 4: rows of
// very different sizes with multi-valued cells; a perfectly balanced matrix
// with a fixed number of cells per row) scaled to one device; see the config
// registry in gen.py for the recipes.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <thread>
#include <vector>

namespace {

inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}
constexpr uint64_t kGamma = 0x9e3779b97f4a7c15ULL;
inline uint64_t stream_key(uint64_t seed, uint64_t stream, uint64_t index) {
  return mix64(mix64(seed * kGamma + stream) ^ (index * 0xd1b54a32d192ed03ULL));
}
inline uint64_t draw(uint64_t key, uint64_t ctr) { return mix64(key + (ctr + 1) * kGamma); }
// Uniform integer in [0, m) by multiply-shift (no rejection; bias < m / 2^64).
inline uint64_t below(uint64_t u, uint64_t m) {
  return (uint64_t)(((unsigned __int128)u * (unsigned __int128)m) >> 64);
}
inline double unit(uint64_t u) { return (double)(u >> 11) * 0x1.0p-53; }
inline uint32_t float01_bits(uint64_t u) {
  // float32 in [0,1) with 24 random mantissa bits: m * 2^-24 is exact.
  float f = (float)(uint32_t)(u >> 40) * 0x1.0p-24f;
  uint32_t b;
  std::memcpy(&b, &f, 4);
  return b;
}

enum Stream : uint64_t {
  S_DEGREE = 1, S_COLS = 2, S_WIDTH = 3, S_PAYLOAD = 4, S_PARTW = 5, S_MATRIX = 6
};

}  // namespace

extern "C" {

// Degree laws.
enum { MGG_DEG_POISSON = 0, MGG_DEG_POWERLAW_BALANCED = 1, MGG_DEG_PART_WEIGHTED = 2,
       MGG_DEG_FIXED = 3, MGG_DEG_UNIFORM = 4 };
// Column laws.
enum { MGG_COL_UNIFORM = 0, MGG_COL_WINDOW = 1 };
// Multiplicity (run length of one drawn column) laws.
enum { MGG_MULT_GEOMETRIC = 0, MGG_MULT_UNIFORM = 1, MGG_MULT_ONE = 2 };
// Payload layouts.
enum { MGG_PAY_FLOATS_TAG = 0,   // U{w_lo..w_hi} float32 in [0,1) then int32 tag = cell index
       MGG_PAY_FLOATS = 1,       // U{w_lo..w_hi} float32 in [0,1)
       MGG_PAY_FLOATS_ROWCOL = 2,// w_lo float32 then int32 source row, int32 source col
       MGG_PAY_BYTES = 3,        // U{w_lo..w_hi} random bytes (any width, unaligned)
       MGG_PAY_TAG64 = 4 };      // exactly 8 bytes: (row << 32 | col) little endian, then w_lo..w_hi extra random bytes

typedef struct {
  int64_t n_rows, n_cols;
  uint64_t seed;
  int32_t deg_law;      // MGG_DEG_*
  double deg_mean;      // Poisson mean, or power-law exponent (alpha)
  int64_t deg_min, deg_max;  // power-law support / uniform support
  int64_t target_nnz;   // total cells for the balanced / weighted laws
  int32_t n_parts;      // partitions for the balanced / weighted laws (equal row blocks)
  int32_t col_law;      // MGG_COL_*
  int64_t window;       // half width of the locality window
  int32_t mult_law;     // MGG_MULT_*
  int32_t mult_max;     // for uniform multiplicity 1..mult_max
  int32_t sort_rows;    // 1: rows sorted by column (canonical)
  int32_t pay_law;      // MGG_PAY_*
  int32_t w_lo, w_hi;   // payload width parameters (floats or bytes)
  int32_t threads;      // 0: hardware concurrency (capped at 16)
} mgg_spec;

}  // extern "C"

namespace {

int n_threads(const mgg_spec* s) {
  int t = s->threads > 0 ? s->threads : (int)std::thread::hardware_concurrency();
  if (t < 1) t = 1;
  if (t > 16) t = 16;
  return t;
}

template <class F>
void parallel_for(int64_t n, int threads, F&& f) {
  if (n <= 0) return;
  if (threads <= 1 || n < 2) { f(0, n); return; }
  std::vector<std::thread> pool;
  int64_t chunk = (n + threads - 1) / threads;
  for (int t = 0; t < threads; ++t) {
    int64_t lo = t * chunk, hi = std::min(n, lo + chunk);
    if (lo >= hi) break;
    pool.emplace_back([=, &f] { f(lo, hi); });
  }
  for (auto& th : pool) th.join();
}

int64_t poisson(uint64_t key, double lambda) {
  // Knuth's multiplication method; one uniform per step, deterministic IEEE products.
  if (lambda <= 0) return 0;
  const double L = std::exp(-lambda);
  double p = 1.0;
  int64_t k = 0;
  for (;;) {
    p *= unit(draw(key, (uint64_t)k));
    if (p <= L) return k;
    ++k;
  }
}

int64_t powerlaw(uint64_t u, double alpha, int64_t dmin, int64_t dmax) {
  // Continuous Pareto(dmin, alpha-1) by inversion, floored and capped.
  double x = (double)dmin * std::pow(1.0 - unit(u), -1.0 / (alpha - 1.0));
  if (!(x < (double)dmax)) return dmax;
  int64_t d = (int64_t)x;
  return d < dmin ? dmin : d;
}

// Split `total` over `n` slots proportionally to w (integer floor), remainder +1 to the first slots.
void apportion(const std::vector<int64_t>& w, int64_t total, std::vector<int64_t>& out) {
  const int64_t n = (int64_t)w.size();
  unsigned __int128 W = 0;
  for (int64_t v : w) W += (unsigned __int128)v;
  out.assign(n, 0);
  if (W == 0) return;
  int64_t used = 0;
  for (int64_t i = 0; i < n; ++i) {
    out[i] = (int64_t)(((unsigned __int128)w[i] * (unsigned __int128)total) / W);
    used += out[i];
  }
  for (int64_t i = 0; used < total; i = (i + 1) % n, ++used) out[i] += 1;
}

}  // namespace

extern "C" {

// Fills row_ptr[0..n_rows] (int64) and returns nnz, or -1 on a bad spec.
int64_t mgg_degrees(const mgg_spec* s, int64_t* row_ptr) {
  const int64_t n = s->n_rows;
  if (n < 0 || !row_ptr) return -1;
  std::vector<int64_t> deg(n, 0);
  const int th = n_threads(s);
  switch (s->deg_law) {
    case MGG_DEG_POISSON:
      parallel_for(n, th, [&](int64_t lo, int64_t hi) {
        for (int64_t i = lo; i < hi; ++i) deg[i] = poisson(stream_key(s->seed, S_DEGREE, i), s->deg_mean);
      });
      break;
    case MGG_DEG_FIXED:
      for (int64_t i = 0; i < n; ++i) deg[i] = (int64_t)s->deg_mean;
      break;
    case MGG_DEG_UNIFORM:
      parallel_for(n, th, [&](int64_t lo, int64_t hi) {
        for (int64_t i = lo; i < hi; ++i)
          deg[i] = s->deg_min + (int64_t)below(draw(stream_key(s->seed, S_DEGREE, i), 0),
                                               (uint64_t)(s->deg_max - s->deg_min + 1));
      });
      break;
    case MGG_DEG_POWERLAW_BALANCED: {
      // Power-law draws, then each equal row block is rescaled to exactly target_nnz / n_parts cells.
      if (s->n_parts < 1 || n % s->n_parts || s->target_nnz % s->n_parts) return -1;
      parallel_for(n, th, [&](int64_t lo, int64_t hi) {
        for (int64_t i = lo; i < hi; ++i)
          deg[i] = powerlaw(draw(stream_key(s->seed, S_DEGREE, i), 0), s->deg_mean, s->deg_min, s->deg_max);
      });
      const int64_t rows_pp = n / s->n_parts, cells_pp = s->target_nnz / s->n_parts;
      parallel_for(s->n_parts, th, [&](int64_t lo, int64_t hi) {
        std::vector<int64_t> w, out;
        for (int64_t p = lo; p < hi; ++p) {
          w.assign(deg.begin() + p * rows_pp, deg.begin() + (p + 1) * rows_pp);
          apportion(w, cells_pp, out);
          std::copy(out.begin(), out.end(), deg.begin() + p * rows_pp);
        }
      });
      break;
    }
    case MGG_DEG_PART_WEIGHTED: {
      // Partition totals proportional to 10^u, u ~ U[0,1); rows of a partition share its total evenly.
      if (s->n_parts < 1 || n % s->n_parts) return -1;
      const int64_t P = s->n_parts, rows_pp = n / P;
      std::vector<int64_t> w(P), tot;
      for (int64_t p = 0; p < P; ++p) {
        double x = std::pow(10.0, unit(draw(stream_key(s->seed, S_PARTW, 0), (uint64_t)p)));
        w[p] = (int64_t)std::llround(x * 1048576.0);  // fixed-point weight
      }
      apportion(w, s->target_nnz, tot);
      for (int64_t p = 0; p < P; ++p) {
        int64_t base = tot[p] / rows_pp, rem = tot[p] % rows_pp;
        for (int64_t r = 0; r < rows_pp; ++r) deg[p * rows_pp + r] = base + (r < rem ? 1 : 0);
      }
      break;
    }
    default:
      return -1;
  }
  row_ptr[0] = 0;
  for (int64_t i = 0; i < n; ++i) row_ptr[i + 1] = row_ptr[i] + deg[i];
  return row_ptr[n];
}

// Fills col[row_ptr[i] .. row_ptr[i+1]) for each row: draw a column, repeat it
// (multiplicity law), truncate the last run at the row's degree; optionally sort.
int mgg_fill_cols(const mgg_spec* s, const int64_t* row_ptr, int32_t* col) {
  const int64_t n = s->n_rows, N = s->n_cols;
  if (N <= 0 && row_ptr[n] > 0) return -1;
  parallel_for(n, n_threads(s), [&](int64_t lo, int64_t hi) {
    for (int64_t i = lo; i < hi; ++i) {
      const uint64_t key = stream_key(s->seed, S_COLS, i);
      int64_t k = row_ptr[i];
      const int64_t end = row_ptr[i + 1];
      uint64_t ctr = 0;
      while (k < end) {
        int64_t c;
        uint64_t u = draw(key, ctr++);
        if (s->col_law == MGG_COL_WINDOW) {
          int64_t w = s->window;
          int64_t delta = (int64_t)below(u, (uint64_t)(2 * w + 1)) - w;
          c = ((i + delta) % N + N) % N;
        } else {
          c = (int64_t)below(u, (uint64_t)N);
        }
        int64_t m = 1;
        uint64_t v = draw(key, ctr++);
        if (s->mult_law == MGG_MULT_GEOMETRIC) m = v ? 1 + __builtin_ctzll(v) : 64;
        else if (s->mult_law == MGG_MULT_UNIFORM) m = 1 + (int64_t)below(v, (uint64_t)s->mult_max);
        for (int64_t j = 0; j < m && k < end; ++j) col[k++] = (int32_t)c;
      }
      if (s->sort_rows) std::sort(col + row_ptr[i], col + end);
    }
  });
  return 0;
}

static int64_t cell_width(const mgg_spec* s, uint64_t wkey, int64_t k) {
  switch (s->pay_law) {
    case MGG_PAY_FLOATS_TAG:
    case MGG_PAY_FLOATS: {
      int64_t f = s->w_lo + (int64_t)below(draw(wkey, (uint64_t)k), (uint64_t)(s->w_hi - s->w_lo + 1));
      return 4 * f + (s->pay_law == MGG_PAY_FLOATS_TAG ? 4 : 0);
    }
    case MGG_PAY_FLOATS_ROWCOL:
      return 4 * (int64_t)s->w_lo + 8;
    case MGG_PAY_BYTES:
      return s->w_lo + (int64_t)below(draw(wkey, (uint64_t)k), (uint64_t)(s->w_hi - s->w_lo + 1));
    case MGG_PAY_TAG64:
      return 8 + s->w_lo + (int64_t)below(draw(wkey, (uint64_t)k), (uint64_t)(s->w_hi - s->w_lo + 1));
  }
  return -1;
}

// Fills payload_off[0..nnz] (int64) and returns payload bytes.
int64_t mgg_widths(const mgg_spec* s, const int64_t* row_ptr, int64_t* poff) {
  const int64_t nnz = row_ptr[s->n_rows];
  const uint64_t wkey = stream_key(s->seed, S_WIDTH, 0);
  const int th = n_threads(s);
  // Two-pass parallel scan: block sums, then block-local prefix.
  const int64_t B = 1 << 16;
  const int64_t nb = nnz ? (nnz + B - 1) / B : 0;
  std::vector<int64_t> bsum(nb + 1, 0);
  parallel_for(nb, th, [&](int64_t lo, int64_t hi) {
    for (int64_t b = lo; b < hi; ++b) {
      int64_t acc = 0;
      for (int64_t k = b * B; k < std::min(nnz, (b + 1) * B); ++k) acc += cell_width(s, wkey, k);
      bsum[b + 1] = acc;
    }
  });
  for (int64_t b = 0; b < nb; ++b) bsum[b + 1] += bsum[b];
  parallel_for(nb, th, [&](int64_t lo, int64_t hi) {
    for (int64_t b = lo; b < hi; ++b) {
      int64_t acc = bsum[b];
      for (int64_t k = b * B; k < std::min(nnz, (b + 1) * B); ++k) {
        poff[k] = acc;
        acc += cell_width(s, wkey, k);
      }
    }
  });
  poff[nnz] = nb ? bsum[nb] : 0;
  return poff[nnz];
}

// Fills the payload bytes of every cell.
int mgg_fill_payload(const mgg_spec* s, const int64_t* row_ptr, const int32_t* col,
                     const int64_t* poff, uint8_t* payload) {
  const int64_t n = s->n_rows;
  parallel_for(n, n_threads(s), [&](int64_t lo, int64_t hi) {
    for (int64_t i = lo; i < hi; ++i) {
      for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
        const uint64_t key = stream_key(s->seed, S_PAYLOAD, (uint64_t)k);
        uint8_t* dst = payload + poff[k];
        const int64_t w = poff[k + 1] - poff[k];
        switch (s->pay_law) {
          case MGG_PAY_FLOATS_TAG:
          case MGG_PAY_FLOATS:
          case MGG_PAY_FLOATS_ROWCOL: {
            int64_t nf = (s->pay_law == MGG_PAY_FLOATS_ROWCOL) ? s->w_lo
                         : (s->pay_law == MGG_PAY_FLOATS_TAG ? (w - 4) / 4 : w / 4);
            for (int64_t f = 0; f < nf; ++f) {
              uint32_t b = float01_bits(draw(key, (uint64_t)f));
              std::memcpy(dst + 4 * f, &b, 4);
            }
            if (s->pay_law == MGG_PAY_FLOATS_TAG) {
              int32_t tag = (int32_t)k;
              std::memcpy(dst + 4 * nf, &tag, 4);
            } else if (s->pay_law == MGG_PAY_FLOATS_ROWCOL) {
              int32_t rc[2] = {(int32_t)i, col[k]};
              std::memcpy(dst + 4 * nf, rc, 8);
            }
            break;
          }
          case MGG_PAY_BYTES:
            for (int64_t j = 0; j < w; j += 8) {
              uint64_t u = draw(key, (uint64_t)(j / 8));
              std::memcpy(dst + j, &u, (size_t)std::min<int64_t>(8, w - j));
            }
            break;
          case MGG_PAY_TAG64: {
            uint64_t tag = ((uint64_t)(uint32_t)i << 32) | (uint32_t)col[k];
            std::memcpy(dst, &tag, 8);
            for (int64_t j = 8; j < w; j += 8) {
              uint64_t u = draw(key, (uint64_t)(j / 8));
              std::memcpy(dst + j, &u, (size_t)std::min<int64_t>(8, w - j));
            }
            break;
          }
        }
      }
    }
  });
  return 0;
}

// Raw counter-based draws, for workload-level parameters (matrix sizes, request mixes).
uint64_t mgg_draw(uint64_t seed, uint64_t stream, uint64_t index, uint64_t ctr) {
  return draw(stream_key(seed, S_MATRIX + stream, index), ctr);
}

}  // extern "C"
