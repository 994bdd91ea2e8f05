// Seeded synthetic sparse-matrix generators.
//
// These produce the inputs that both the CPU oracle and the GPU library are
// run on.  They hold none of the semiring product's arithmetic: they only
// draw patterns and values.  Every random number comes from a counter-based
// SplitMix64 stream (Steele, Lea and Flood, "Fast splittable pseudorandom
// number generators", OOPSLA 2014), keyed by (seed, stream tag, index), so the
// output is identical for any thread count.
//
// Generators:
//   * Erdos-Renyi rows: d distinct columns per row drawn uniformly without
//     replacement with Floyd's algorithm (Bentley and Floyd, CACM 1987).
//   * R-MAT (Chakrabarti, Zhan and Faloutsos, SDM 2004): m = ef * 2^s edges,
//     each placed by s rounds of quadrant choice with probabilities
//     (a, b, c, d); no noise, no vertex relabelling, self loops kept,
//     duplicate edges removed.
//   * value fills per stored entry, block-grid splits and row selections.
//
// All matrices are CSR with int64 row offsets and int32 column ids, columns
// sorted ascending and unique within a row.

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>
#include <omp.h>

namespace {

constexpr uint64_t kGolden = 0x9E3779B97F4A7C15ull;

inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Counter-based draw: the ctr-th output of the SplitMix64 sequence whose
// state starts at `key`.
inline uint64_t draw(uint64_t key, uint64_t ctr) { return mix64(key + (ctr + 1) * kGolden); }

inline uint64_t stream_key(uint64_t seed, uint64_t tag) { return mix64(mix64(seed) ^ (tag * 0xD1B54A32D192ED03ull)); }

// Uniform double in [0, 1) with 53 random bits.
inline double u53(uint64_t z) { return (double)(z >> 11) * 0x1.0p-53; }

// Uniform integer in [0, range) by Lemire's multiply-shift on the top 32 bits
// (range < 2^32).
inline uint64_t below(uint64_t z, uint64_t range) { return ((z >> 32) * range) >> 32; }

enum : uint64_t { TAG_ER = 1, TAG_RMAT = 2, TAG_VAL = 3, TAG_SEL = 4, TAG_BATCH = 5 };

}  // namespace

extern "C" {

// ---------------------------------------------------------------------------
// Erdos-Renyi pattern: nrows x ncols, exactly d distinct columns per row.
// rowptr has nrows+1 entries and is filled as i*d; col has nrows*d entries.
// Returns 0 on success, -1 on bad arguments (d > ncols).
int synth_er(int64_t nrows, int64_t ncols, int32_t d, uint64_t seed, int64_t* rowptr, int32_t* col) {
  if (d < 0 || d > ncols || ncols > INT32_MAX) return -1;
  const uint64_t key = stream_key(seed, TAG_ER);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < nrows; ++i) {
    int32_t* out = col + i * (int64_t)d;
    const uint64_t rk = mix64(key ^ mix64((uint64_t)i + 1));
    int32_t cnt = 0;
    // Floyd: for j = ncols-d .. ncols-1 pick t in [0, j]; take t unless
    // already taken, in which case take j.
    for (int64_t j = ncols - d; j < ncols; ++j) {
      int32_t t = (int32_t)below(draw(rk, (uint64_t)(j - (ncols - d))), (uint64_t)j + 1);
      bool seen = false;
      for (int32_t q = 0; q < cnt; ++q)
        if (out[q] == t) { seen = true; break; }
      out[cnt++] = seen ? (int32_t)j : t;
    }
    std::sort(out, out + d);
  }
  for (int64_t i = 0; i <= nrows; ++i) rowptr[i] = i * (int64_t)d;
  return 0;
}

// ---------------------------------------------------------------------------
// R-MAT edge list: m edges, each an (row, col) pair in [0, 2^scale)^2.
void synth_rmat_edges(int32_t scale, int64_t m, double a, double b, double c, uint64_t seed, int32_t* rows,
                      int32_t* cols) {
  const uint64_t key = stream_key(seed, TAG_RMAT);
  const double ab = a + b, abc = a + b + c;
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < m; ++e) {
    uint32_t r = 0, q = 0;
    for (int32_t l = 0; l < scale; ++l) {
      double u = u53(draw(key, (uint64_t)e * (uint64_t)scale + (uint64_t)l));
      uint32_t rb, cb;
      if (u < a) { rb = 0; cb = 0; }
      else if (u < ab) { rb = 0; cb = 1; }
      else if (u < abc) { rb = 1; cb = 0; }
      else { rb = 1; cb = 1; }
      r = (r << 1) | rb;
      q = (q << 1) | cb;
    }
    rows[e] = (int32_t)r;
    cols[e] = (int32_t)q;
  }
}

// Edge list -> CSR with sorted, de-duplicated rows.  Two calls: the first
// (col == nullptr) fills rowptr[nrows+1] and returns nnz; the second fills
// col (the arrays rows/cols are scratch and are reordered).
// Returns nnz or -1 on allocation failure.
int64_t synth_edges_to_csr(int64_t nrows, int64_t m, int32_t* rows, int32_t* cols, int64_t* rowptr,
                           int32_t* col) {
  // counting sort by row into a temporary
  std::vector<int64_t> start(nrows + 1, 0);
  {
    std::vector<std::atomic<int64_t>> cnt(nrows);
    for (int64_t i = 0; i < nrows; ++i) cnt[i].store(0, std::memory_order_relaxed);
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < m; ++e) cnt[rows[e]].fetch_add(1, std::memory_order_relaxed);
    for (int64_t i = 0; i < nrows; ++i) start[i + 1] = start[i] + cnt[i].load(std::memory_order_relaxed);
  }
  std::vector<int32_t> tmp(m);
  {
    std::vector<std::atomic<int64_t>> cur(nrows);
    for (int64_t i = 0; i < nrows; ++i) cur[i].store(start[i], std::memory_order_relaxed);
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < m; ++e) tmp[cur[rows[e]].fetch_add(1, std::memory_order_relaxed)] = cols[e];
  }
  std::vector<int64_t> uniq(nrows + 1, 0);
#pragma omp parallel for schedule(dynamic, 1024)
  for (int64_t i = 0; i < nrows; ++i) {
    int32_t* b = tmp.data() + start[i];
    int32_t* e = tmp.data() + start[i + 1];
    std::sort(b, e);
    uniq[i + 1] = std::unique(b, e) - b;
  }
  rowptr[0] = 0;
  for (int64_t i = 0; i < nrows; ++i) rowptr[i + 1] = rowptr[i] + uniq[i + 1];
  const int64_t nnz = rowptr[nrows];
  if (col) {
#pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t i = 0; i < nrows; ++i)
      std::memcpy(col + rowptr[i], tmp.data() + start[i], sizeof(int32_t) * (size_t)(rowptr[i + 1] - rowptr[i]));
  }
  return nnz;
}

// ---------------------------------------------------------------------------
// Values, one per stored entry, drawn from index-keyed streams.
//   kind 0: float64 uniform [lo, hi)       kind 1: float32 uniform [lo, hi)
//   kind 2: int64 uniform {lo .. hi}       kind 3: float64 N(0,1) (Box-Muller)
//   kind 4: float32 N(0,1) (the float64 draw rounded to nearest)
//   kind 5: uint8 all ones                 kind 6: uint8 Bernoulli(lo)
int synth_values(int32_t kind, int64_t n, double lo, double hi, uint64_t seed, void* out) {
  const uint64_t key = stream_key(seed, TAG_VAL);
  switch (kind) {
    case 0: {
      double* o = (double*)out;
#pragma omp parallel for schedule(static)
      for (int64_t e = 0; e < n; ++e) o[e] = lo + (hi - lo) * u53(draw(key, (uint64_t)e));
      return 0;
    }
    case 1: {
      float* o = (float*)out;
#pragma omp parallel for schedule(static)
      for (int64_t e = 0; e < n; ++e) {
        float v = (float)(lo + (hi - lo) * u53(draw(key, (uint64_t)e)));
        if (v >= (float)hi) v = std::nextafter((float)hi, (float)lo);  // keep [lo, hi)
        o[e] = v;
      }
      return 0;
    }
    case 2: {
      int64_t* o = (int64_t*)out;
      const uint64_t range = (uint64_t)((int64_t)hi - (int64_t)lo + 1);
#pragma omp parallel for schedule(static)
      for (int64_t e = 0; e < n; ++e) o[e] = (int64_t)lo + (int64_t)below(draw(key, (uint64_t)e), range);
      return 0;
    }
    case 3:
    case 4: {
#pragma omp parallel for schedule(static)
      for (int64_t e = 0; e < n; ++e) {
        double u1 = 1.0 - u53(draw(key, 2 * (uint64_t)e));  // (0, 1]
        double u2 = u53(draw(key, 2 * (uint64_t)e + 1));
        double z = std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2);
        if (kind == 3) ((double*)out)[e] = z;
        else ((float*)out)[e] = (float)z;
      }
      return 0;
    }
    case 5:
      std::memset(out, 1, (size_t)n);
      return 0;
    case 6: {
      uint8_t* o = (uint8_t*)out;
#pragma omp parallel for schedule(static)
      for (int64_t e = 0; e < n; ++e) o[e] = u53(draw(key, (uint64_t)e)) < lo ? 1 : 0;
      return 0;
    }
    default:
      return -1;
  }
}

// Uniform random selection of k distinct items from [0, n) (Floyd), sorted.
int synth_select(int64_t n, int64_t k, uint64_t seed, int64_t* out) {
  if (k < 0 || k > n) return -1;
  const uint64_t key = stream_key(seed, TAG_SEL);
  std::vector<int64_t> s;
  s.reserve((size_t)k);
  size_t cap = 16;
  while (cap < (size_t)k * 2 + 16) cap <<= 1;
  std::vector<int64_t> table(cap, -1);
  auto insert = [&](int64_t v) -> bool {
    size_t h = (size_t)mix64((uint64_t)v) & (cap - 1);
    while (table[h] != -1) {
      if (table[h] == v) return false;
      h = (h + 1) & (cap - 1);
    }
    table[h] = v;
    return true;
  };
  for (int64_t j = n - k; j < n; ++j) {
    int64_t t = (int64_t)(u53(draw(key, (uint64_t)(j - (n - k)))) * (double)(j + 1));
    if (t > j) t = j;
    if (insert(t)) s.push_back(t);
    else { insert(j); s.push_back(j); }
  }
  std::sort(s.begin(), s.end());
  std::memcpy(out, s.data(), sizeof(int64_t) * (size_t)k);
  return 0;
}

// Parameters of one instance of a batch of random ER products: n is
// floor(exp(U(ln nlo, ln nhi))) and d is uniform in {dlo .. dhi}.
void synth_batch_params(int32_t count, double nlo, double nhi, int32_t dlo, int32_t dhi, uint64_t seed, int64_t* n,
                        int32_t* d) {
  const uint64_t key = stream_key(seed, TAG_BATCH);
  const double l0 = std::log(nlo), l1 = std::log(nhi);
  for (int32_t b = 0; b < count; ++b) {
    double u = u53(draw(key, 2 * (uint64_t)b));
    int64_t nb = (int64_t)std::floor(std::exp(l0 + (l1 - l0) * u));
    if (nb < (int64_t)nlo) nb = (int64_t)nlo;
    n[b] = nb;
    d[b] = dlo + (int32_t)below(draw(key, 2 * (uint64_t)b + 1), (uint64_t)(dhi - dlo + 1));
  }
}

// ---------------------------------------------------------------------------
// Block-grid split.  The nrows x ncols matrix is cut into a gr x gc grid of
// blocks with row/column edges at multiples of (rb, cb); column ids become
// block-local.  Pass 1 (out_col == nullptr): fills blk_rowptr, a
// (gr*gc) x (rb+1) array of int64 block-local row offsets (rows beyond the
// matrix are empty).  Pass 2: given blk_base[gr*gc] (start of each block in
// the packed output) fills out_col and, when val_bytes > 0, out_val.
void synth_block_split(int64_t nrows, int64_t ncols, const int64_t* rowptr, const int32_t* col, const void* val,
                       int32_t val_bytes, int32_t gr, int32_t gc, int64_t rb, int64_t cb, int64_t* blk_rowptr,
                       const int64_t* blk_base, int32_t* out_col, void* out_val) {
  (void)ncols;
  const int64_t stride = rb + 1;
  if (!out_col) {
    std::memset(blk_rowptr, 0, sizeof(int64_t) * (size_t)(gr * gc) * (size_t)stride);
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < nrows; ++i) {
      const int64_t I = i / rb, li = i % rb;
      for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
        const int64_t J = col[e] / cb;
        blk_rowptr[(I * gc + J) * stride + li + 1]++;
      }
    }
#pragma omp parallel for schedule(static)
    for (int64_t b = 0; b < (int64_t)gr * gc; ++b) {
      int64_t* p = blk_rowptr + b * stride;
      for (int64_t r = 0; r < rb; ++r) p[r + 1] += p[r];
    }
    return;
  }
#pragma omp parallel for schedule(dynamic, 256)
  for (int64_t i = 0; i < nrows; ++i) {
    const int64_t I = i / rb, li = i % rb;
    int64_t pos[1024];  // gc <= 1024
    for (int32_t J = 0; J < gc; ++J) pos[J] = blk_base[I * gc + J] + blk_rowptr[(I * gc + J) * stride + li];
    for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
      const int64_t J = col[e] / cb;
      const int64_t o = pos[J]++;
      out_col[o] = (int32_t)(col[e] - J * cb);
      if (val_bytes > 0)
        std::memcpy((char*)out_val + o * val_bytes, (const char*)val + e * val_bytes, (size_t)val_bytes);
    }
  }
}

int synth_num_threads(void) { return omp_get_max_threads(); }

}  // extern "C"
