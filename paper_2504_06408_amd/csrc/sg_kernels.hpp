// Kernel templates of the semiring product and merge on gfx950.
//
// Pipeline for one product C = A (x).(+) B (the local multiply of a Sparse
// SUMMA stage, paper Sections 2.1 and 4.3):
//   analyze   p_i = sum_{k in A_i} nnz(B_k) products per row, row -> bin
//   bin       stable counting sort of rows into bins (lists per bin)
//   bounds    per B row, the offsets where each 16384-column tile starts
//   symbolic  nnz(C_i): wave sort (<= 64 products), LDS hash (<= 4096
//             products) or LDS bitmap over column tiles (dense rows); dense
//             rows also get per-tile output offsets
//   scan      C.rowptr = prefix sum of the counts
//   numeric   C_ij = (+)_k A_ik (x) B_kj: wave sort + segmented fold, LDS
//             hash + bitonic sort, or a dense LDS accumulator per
//             (row, column tile) task with bitmap compaction, which writes
//             rows sorted with no sort at all.
// The merge (Section 4.4) runs the same kernels with a different "source":
// the parts' rows instead of B rows selected by A's entries, and (x) replaced
// by taking the part's value.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sg_device.hpp"
#include "sg_semiring.hpp"

namespace sg {

// ---- bins and path parameters ----------------------------------------------
constexpr int kNB = 64;
constexpr int kBinEmpty = 0;
constexpr int kBinSmall = 1;
constexpr int kBinHash0 = 2;   // 2..8: hash table of 2^(7+b-2) slots
constexpr int kBinHashC0 = 9;  // 9..15: same, compensated float sums
constexpr int kBinDense0 = 16; // 16..63: dense rows, larger product counts first
constexpr int kHashLgMin = 7, kHashLgMax = 13;
constexpr int kSmallMax = 64;     // products of a wave-sorted row
constexpr int kHashCap = 4096;    // products (symbolic) / entries (numeric) of a hash row
constexpr int kTileLog = 14;      // dense column tile: 16384 columns
constexpr int kTile = 1 << kTileLog;
constexpr int kTileWords = kTile / 32;
constexpr int kSymTiles = 64;     // tiles per bitmap pass of the dense symbolic kernel (128 KB)

enum { kForceAuto = 0, kForceSmall = 1, kForceHash = 2, kForceDense = 3 };
enum { kCompNone = 0, kCompRule = 1, kCompAll = 2 };

struct Policy {
  int32_t numeric;  // 0: symbolic (hash size from products), 1: numeric (from entries)
  int32_t force;
  int64_t hash_max;  // rows with more products take the dense path
  int32_t comp_mode;
  int32_t comp_min_terms;
  int64_t comp_min_products;
  int32_t by_products;  // numeric hash bins sized from products (rows the merge kernel takes), not entries
};

SG_DEV int hash_bin(int64_t need, int lg_floor) {
  // smallest table 2^lg >= 2*need, at least 2^lg_floor
  int lg = ceil_log2_u64((uint64_t)(2 * need));
  lg = lg < lg_floor ? lg_floor : lg;
  return kBinHash0 + (lg - kHashLgMin);
}

SG_DEV bool is_dense(const Policy& pol, int64_t p) {
  if (p == 0) return false;
  if (pol.force == kForceDense) return true;
  if (pol.force == kForceSmall && p <= kSmallMax) return false;
  if (pol.force == kForceHash) return p > kHashCap;
  return p > pol.hash_max;
}

SG_DEV int bin_of(const Policy& pol, int64_t p, int64_t m, int64_t nterms) {
  if (p == 0) return kBinEmpty;
  if (is_dense(pol, p)) {
    int lg = ceil_log2_u64((uint64_t)p);
    lg = lg > 47 ? 47 : lg;
    return kNB - 1 - lg;  // 16..63
  }
  const bool small = (pol.force == kForceSmall || pol.force == kForceAuto) && p <= kSmallMax;
  if (small) return kBinSmall;
  if (!pol.numeric) return hash_bin(p, 8);
  const bool comp = pol.comp_mode == kCompAll ||
                    (pol.comp_mode == kCompRule && nterms > pol.comp_min_terms && p > pol.comp_min_products);
  const int64_t need = pol.by_products ? p : m;
  const int64_t mm = need < 1 ? 1 : (need > kHashCap ? kHashCap : need);
  return hash_bin(mm, kHashLgMin) + (comp ? (kBinHashC0 - kBinHash0) : 0);
}

// ---- sources -----------------------------------------------------------------

template <class T>
SG_DEV T shfl_any(T v, int src) {
  static_assert(sizeof(T) <= 8, "shfl_any");
  uint64_t u = 0;
  __builtin_memcpy(&u, &v, sizeof(T));
  const uint32_t lo = (uint32_t)__shfl((int)(uint32_t)u, src, kWave);
  uint32_t hi = 0;
  if (sizeof(T) > 4) hi = (uint32_t)__shfl((int)(uint32_t)(u >> 32), src, kWave);
  u = (uint64_t)lo | ((uint64_t)hi << 32);
  T o;
  __builtin_memcpy(&o, &u, sizeof(T));
  return o;
}

template <class T>
SG_DEV T shfl_down_any(T v, int d) {
  const int l = lane_id();
  return shfl_any(v, l + d < kWave ? l + d : l);
}

// Row i of A (x) B: one source per stored A_ik, segment = B's row k (or the
// part of it inside column tiles [t0, t1)).
template <class V, bool kVals>
struct SpgemmSrc {
  const int64_t* a_rowptr;
  const int32_t* a_col;
  const V* a_val;
  const int64_t* b_rowptr;
  const int32_t* b_col;
  const V* b_val;
  const int32_t* rp2;  // per B row: T+1 row-local offsets where tile t starts
  int32_t T;           // column tiles of B
  int64_t ncols;       // columns of B
  int64_t a0;
  int32_t t0, t1;
  static constexpr bool kParts = false;

  struct Item {
    V a;
  };

  SG_DEV int64_t bind(int64_t i, int32_t ta, int32_t tb) {
    a0 = a_rowptr[i];
    t0 = ta;
    t1 = tb;
    return a_rowptr[i + 1] - a0;
  }
  SG_DEV void load(int64_t j, Item& it, int64_t& start, int64_t& len) const {
    const int64_t e = a0 + j;
    const int32_t k = a_col[e];
    if constexpr (kVals) it.a = a_val[e];
    const int64_t b0 = b_rowptr[k];
    if (t0 == 0 && t1 == T) {
      start = b0;
      len = b_rowptr[k + 1] - b0;
    } else {
      const int32_t* r = rp2 + (int64_t)k * (T + 1);
      const int32_t s = r[t0];
      start = b0 + s;
      len = r[t1] - s;
    }
  }
  SG_DEV int32_t col(const Item&, int64_t idx) const { return b_col[idx]; }
  template <class Sr>
  SG_DEV typename Sr::Acc value(const Item& it, int64_t idx) const {
    return Sr::mul(it.a, b_val[idx]);
  }
  SG_DEV static Item shfl_item(const Item& it, int src) {
    Item o;
    o.a = shfl_any(it.a, src);
    return o;
  }
};

struct PartDesc {
  const int64_t* rowptr;
  const int32_t* col;
  const void* val;
  int64_t nnz;
};

SG_DEV int64_t lower_bound_col(const int32_t* col, int64_t lo, int64_t hi, int64_t x) {
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if ((int64_t)col[mid] < x) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// First position p in [a, b) with col[p] >= x (b if none), found by the 32
// lanes of a half-wavefront together: a 32-ary search, one load per lane and
// level (four dependent loads for rows of ~32k entries instead of ~15).
// Every lane of the half-wavefront gets the result.
SG_DEV int64_t halfwave_lower_bound(const int32_t* col, int64_t a, int64_t b, int64_t x) {
  const int hl = lane_id() & 31;
  const bool upper = lane_id() >= 32;
  while (b - a > 32) {
    const int64_t step = (b - a + 31) / 32;
    const int64_t p = a + hl * step;
    const unsigned long long m = __ballot(p < b && (int64_t)col[p] < x);
    const int c = __popc(upper ? (uint32_t)(m >> 32) : (uint32_t)m);
    if (c == 0) {
      b = a;
    } else {
      const int64_t nb = a + (int64_t)c * step;
      a = a + (int64_t)(c - 1) * step + 1;
      b = nb < b ? nb : b;
    }
  }
  const int64_t p = a + hl;
  const unsigned long long m = __ballot(p < b && (int64_t)col[p] < x);
  return a + __popc(upper ? (uint32_t)(m >> 32) : (uint32_t)m);
}

constexpr int kLdsParts = 64;  // merges of up to this many parts find their tile bounds together

// Row i of a merge: one source per part, segment = the part's row i.  For
// a task over column tiles [t0, t1) the segments are cut to the tiles' column
// range, by a binary search per part in load(), or from pre[2j], pre[2j+1]
// when the workgroup found them together beforehand (merge_bounds).
template <class V>
struct MergeSrc {
  const PartDesc* parts;
  int32_t nparts;
  int32_t T;
  int64_t ncols;
  int64_t row;
  int32_t t0, t1;
  const int64_t* pre = nullptr;
  static constexpr bool kParts = true;

  struct Item {
    const int32_t* col;
    const V* val;
  };

  SG_DEV int64_t bind(int64_t i, int32_t ta, int32_t tb) {
    row = i;
    t0 = ta;
    t1 = tb;
    pre = nullptr;
    return nparts;
  }
  SG_DEV void load(int64_t j, Item& it, int64_t& start, int64_t& len) const {
    const PartDesc P = parts[j];
    if (pre != nullptr) {
      it.col = P.col;
      it.val = (const V*)P.val;
      start = pre[2 * j];
      len = pre[2 * j + 1] - start;
      return;
    }
    int64_t s = P.rowptr[row], e = P.rowptr[row + 1];
    if (!(t0 == 0 && t1 == T)) {
      const int64_t lo = (int64_t)t0 << kTileLog;
      int64_t hi = (int64_t)t1 << kTileLog;
      hi = hi < ncols ? hi : ncols;
      s = lower_bound_col(P.col, s, e, lo);
      e = lower_bound_col(P.col, s, e, hi);
    }
    it.col = P.col;
    it.val = (const V*)P.val;
    start = s;
    len = e - s;
  }
  SG_DEV int32_t col(const Item& it, int64_t idx) const { return it.col[idx]; }
  template <class Sr>
  SG_DEV typename Sr::Acc value(const Item& it, int64_t idx) const {
    return Sr::lift(it.val[idx]);
  }
  // Segment bounds of every part for the bound tile range, one wavefront
  // per part (the lower bound in one half, the upper in the other), into
  // s_se[2j], s_se[2j+1]; then load() reads them.  All threads of the block
  // call it; it ends with a barrier.
  template <int BS>
  SG_DEV void merge_bounds(int64_t* s_se) {
    constexpr int NW = BS / kWave;
    const int64_t lo = (int64_t)t0 << kTileLog;
    int64_t hi = (int64_t)t1 << kTileLog;
    hi = hi < ncols ? hi : ncols;
    for (int j = wave_id(); j < nparts; j += NW) {
      const PartDesc P = parts[j];
      const int64_t s = P.rowptr[row], e = P.rowptr[row + 1];
      const int64_t r = halfwave_lower_bound(P.col, s, e, lane_id() < 32 ? lo : hi);
      if (lane_id() == 0) s_se[2 * j] = r;
      if (lane_id() == 32) s_se[2 * j + 1] = r;
    }
    block_sync();
    pre = s_se;
  }
  SG_DEV static Item shfl_item(const Item& it, int src) {
    Item o;
    o.col = shfl_any(it.col, src);
    o.val = shfl_any(it.val, src);
    return o;
  }
};

// Products each lane gathers before folding them into LDS (memory-level
// parallelism of the B-row gathers).
constexpr int kUnroll = 8;

template <class Acc>
struct ColVal {
  int32_t c;
  Acc v;
};

// ---- row sets ---------------------------------------------------------------------
//
// Kernels see a set of "global" rows r; Rows::get maps r to the source of the
// problem that owns it and the row's local index.  A single product or merge
// is OneRows (r is the local row); a batch concatenates the rows of all its
// products (TableRows) or merges (MergeTableRows) and finds the owner by a
// binary search over the problems' first rows.  Outputs are indexed by r.

template <class S>
struct OneRows {
  using Src = S;
  S src;
  int32_t Tmax;
  SG_DEV void get(int64_t r, S& s, int64_t& i) const {
    s = src;
    i = r;
  }
};

// One product of a batch (device table entry).
struct ProbDesc {
  const int64_t* a_rowptr;
  const int32_t* a_col;
  const void* a_val;
  const int64_t* b_rowptr;
  const int32_t* b_col;
  const void* b_val;
  const int32_t* rp2;
  int64_t ncols;
  int32_t T;
  int32_t pad;
};

// One merge of a batch: its parts' descriptors live in a parts table.
struct GroupDesc {
  const PartDesc* parts;
  int64_t ncols;
  int32_t nparts;
  int32_t T;
};

// Owner of global row r: the last problem q with rbase[q] <= r.
// owner_search looks among all n problems; owner_of only among those that
// begin inside r's block of 2^kOwnerShift rows (none, for a block inside one
// problem), from coarse[c], the owner of row min(c * 2^kOwnerShift, rows - 1),
// kept for every block c and one more.
constexpr int kOwnerShift = 8;
SG_DEV int owner_search(const int64_t* rbase, int32_t n, int64_t r) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (rbase[mid] <= r) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}
SG_DEV int owner_of(const int64_t* rbase, const int32_t* coarse, int64_t r) {
  const int64_t c = r >> kOwnerShift;
  int lo = coarse[c], hi = coarse[c + 1];
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (rbase[mid] <= r) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

template <class V, bool kVals>
struct TableRows {
  using Src = SpgemmSrc<V, kVals>;
  const ProbDesc* probs;
  const int64_t* rbase;   // first global row of each product, ascending
  const int32_t* coarse;  // owners of every 256th row (owner_of)
  int32_t nprob;
  int32_t Tmax;
  SG_DEV void get(int64_t r, Src& s, int64_t& i) const {
    const int q = owner_of(rbase, coarse, r);
    const ProbDesc& d = probs[q];
    s.a_rowptr = d.a_rowptr;
    s.a_col = d.a_col;
    s.a_val = (const V*)d.a_val;
    s.b_rowptr = d.b_rowptr;
    s.b_col = d.b_col;
    s.b_val = (const V*)d.b_val;
    s.rp2 = d.rp2;
    s.T = d.T;
    s.ncols = d.ncols;
    i = r - rbase[q];
  }
};

template <class V>
struct MergeTableRows {
  using Src = MergeSrc<V>;
  const GroupDesc* groups;
  const int64_t* rbase;
  const int32_t* coarse;
  int32_t ngroups;
  int32_t Tmax;
  SG_DEV void get(int64_t r, Src& s, int64_t& i) const {
    const int q = owner_of(rbase, coarse, r);
    const GroupDesc& g = groups[q];
    s.parts = g.parts;
    s.nparts = g.nparts;
    s.T = g.T;
    s.ncols = g.ncols;
    i = r - rbase[q];
  }
};

// ---- shared argument blocks ---------------------------------------------------

struct Bins {
  const int32_t* list;   // rows of all bins, bin after bin
  const int32_t* start;  // [kNB]
  const int32_t* count;  // [kNB]
  int32_t nd_cap;        // dense rows the per-tile offset array has room for
};

SG_DEV int32_t dense_rows(const Bins& bins) {
  const int32_t nd = bins.start[kNB - 1] + bins.count[kNB - 1] - bins.start[kBinDense0];
  return nd < bins.nd_cap ? nd : bins.nd_cap;
}

struct OutC {
  const int64_t* rowptr;
  int32_t* col;
  void* val;
};

// ---- analysis and binning ---------------------------------------------------------
// Each block of the analysis counts its rows per bin into a bin-major
// histogram, hist[b * gridDim.x + blockIdx.x].

template <class Rows, int BS>
__global__ __launch_bounds__(BS) void k_analyze(Rows rows, int64_t nrows, Policy pol, const int64_t* c_rowptr,
                                                  int64_t* p_out, int32_t* nt_out, uint8_t* bin_out, int32_t* hist,
                                                  int64_t* cnt_out) {
  using Src = typename Rows::Src;
  __shared__ int32_t s_hist[kNB];
  for (int b = threadIdx.x; b < kNB; b += BS) s_hist[b] = 0;
  block_sync();
  const int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x;
  const bool valid = i < nrows;
  Src s{};
  int64_t li = 0;
  if (valid) rows.get(i, s, li);
  const int64_t nsrc = valid ? s.bind(li, 0, s.T) : 0;
  int64_t p = 0;
  const bool heavy = nsrc > 32;
  if (!heavy) {
    // eight source loads in flight at a time (indices past the row's end
    // re-load its last source and are not counted)
    for (int64_t j0 = 0; j0 < nsrc; j0 += 8) {
      int64_t lens[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        typename Src::Item it;
        int64_t st;
        s.load(j0 + u < nsrc ? j0 + u : nsrc - 1, it, st, lens[u]);
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) p += j0 + u < nsrc ? lens[u] : 0;
    }
  }
  unsigned long long hmask = __ballot(heavy);
  while (hmask) {
    const int leader = __ffsll((long long)hmask) - 1;
    hmask &= hmask - 1;
    const int64_t ri = shfl(i, leader);
    Src t{};
    int64_t tl;
    rows.get(ri, t, tl);
    const int64_t n2 = t.bind(tl, 0, t.T);
    int64_t part = 0;
    // eight independent source loads per lane in flight (hub rows of power-law
    // graphs hold tens of thousands of entries)
    for (int64_t j0 = 0; j0 < n2; j0 += 8 * kWave) {
      // indices past the row's end re-load its last source, uncounted, so
      // the eight loads carry no branch
      int64_t lens[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int64_t j = j0 + u * kWave + lane_id();
        typename Src::Item it;
        int64_t st;
        t.load(j < n2 ? j : n2 - 1, it, st, lens[u]);
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) part += j0 + u * kWave + lane_id() < n2 ? lens[u] : 0;
    }
    part = wave_sum(part);
    if (lane_id() == leader) p = part;
  }
  if (valid) {
    p_out[i] = p;
    nt_out[i] = (int32_t)nsrc;
    const int64_t m = pol.numeric ? (c_rowptr[i + 1] - c_rowptr[i]) : 0;
    const int b = bin_of(pol, p, m, nsrc);
    bin_out[i] = (uint8_t)b;
    atomicAdd(&s_hist[b], 1);
    if (!pol.numeric && b == kBinEmpty) cnt_out[i] = 0;
  }
  block_sync();
  for (int b = threadIdx.x; b < kNB; b += BS) hist[(int64_t)b * gridDim.x + blockIdx.x] = s_hist[b];
}

// Numeric-pass binning from the product counts the symbolic pass already
// computed (no gathers): only C's row lengths and, for the compensation rule,
// the number of terms per row (also kept by the symbolic analysis) are read.
template <int BS>
__global__ __launch_bounds__(BS) void k_rebin(const int64_t* p_in, const int32_t* nt_in, const int64_t* c_rowptr,
                                              int64_t nrows, Policy pol, uint8_t* bin_out, int32_t* hist) {
  __shared__ int32_t s_hist[kNB];
  for (int b = threadIdx.x; b < kNB; b += BS) s_hist[b] = 0;
  block_sync();
  const int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (i < nrows) {
    const int64_t p = p_in[i];
    const int64_t m = c_rowptr[i + 1] - c_rowptr[i];
    const int b = bin_of(pol, p, m, nt_in[i]);
    bin_out[i] = (uint8_t)b;
    atomicAdd(&s_hist[b], 1);
  }
  block_sync();
  for (int b = threadIdx.x; b < kNB; b += BS) hist[(int64_t)b * gridDim.x + blockIdx.x] = s_hist[b];
}

// Stable scatter of row ids into their bins (ascending row order per bin).
template <int BS>
__global__ __launch_bounds__(BS) void k_bin_scatter(const uint8_t* bin_in, int64_t nrows, const int32_t* blk_off,
                                                      const int32_t* bin_start, int32_t* list) {
  constexpr int NW = BS / kWave;
  __shared__ int32_t s_cnt[NW][kNB];
  for (int x = threadIdx.x; x < NW * kNB; x += BS) (&s_cnt[0][0])[x] = 0;
  block_sync();
  const int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x;
  const bool valid = i < nrows;
  const int b = valid ? (int)bin_in[i] : 0;
  unsigned long long match = __ballot(valid);
#pragma unroll
  for (int bit = 0; bit < 6; ++bit) {
    const bool on = (b >> bit) & 1;
    const unsigned long long bb = __ballot(on);
    match &= on ? bb : ~bb;
  }
  const unsigned long long below = match & lanes_below();
  const int rank = __popcll(below);
  if (valid && below == 0) s_cnt[wave_id()][b] = __popcll(match);
  block_sync();
  if (valid) {
    int32_t pre = 0;
    for (int w = 0; w < wave_id(); ++w) pre += s_cnt[w][b];
    list[bin_start[b] + blk_off[(int64_t)b * gridDim.x + blockIdx.x] + pre + rank] = (int32_t)i;
  }
}

// ---- prefix sums over int64 (in place, inclusive) ----
constexpr int kScanBS = 1024, kScanPer = 8, kScanChunk = kScanBS * kScanPer;

template <class T>
__global__ void k_fill(T* p, int64_t n, T v) {
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += (int64_t)gridDim.x * blockDim.x)
    p[x] = v;
}

// ---- small rows: one wavefront per row, products held one per lane ---------------

// Gathers the (<= 64) products of the bound row into lanes: lane q gets
// product q (col, value); lanes beyond the row's product count get
// (INT32_MAX, identity).  Returns the product count.
template <class Sr, class Src, bool kVals>
SG_DEV int wave_gather_products(Src& s, int64_t nsrc, int32_t& key, typename Sr::Acc& acc) {
  using Item = typename Src::Item;
  const int l = lane_id();
  key = 0x7FFFFFFF;
  acc = Sr::ident();
  int base = 0;
  for (int64_t c0 = 0; c0 < nsrc; c0 += kWave) {
    const int64_t j = c0 + l;
    Item it{};
    int64_t start = 0, len = 0;
    if (j < nsrc) s.load(j, it, start, len);
    const int64_t incl = wave_incl_scan(len);
    const int64_t tot = shfl(incl, kWave - 1);
    int64_t rr = (int64_t)l - base;
    const bool mine = rr >= 0 && rr < tot;
    if (!mine) rr = 0;
    // owner: first lane whose inclusive offset exceeds rr
    int lo = 0, hi = kWave - 1;
#pragma unroll
    for (int step = 0; step < 6; ++step) {
      const int mid = (lo + hi) >> 1;
      const int64_t v = shfl(incl, mid);
      if (v > rr) hi = mid;
      else lo = mid + 1;
    }
    const int64_t o_start = shfl(start, lo);
    const int64_t o_excl = shfl(incl - len, lo);
    const Item o_item = Src::shfl_item(it, lo);
    if (mine) {
      const int64_t idx = o_start + (rr - o_excl);
      key = s.col(o_item, idx);
      if constexpr (kVals) acc = s.template value<Sr>(o_item, idx);
    }
    base += (int)tot;
  }
  return base;
}

template <class Rows>
__global__ __launch_bounds__(256) void k_sym_small(Rows rows, Bins bins, int bin, int64_t* cnt_out) {
  using Src = typename Rows::Src;
  const int n = bins.count[bin];
  const int32_t* L = bins.list + bins.start[bin];
  const int w0 = (int)(((int64_t)blockIdx.x * 256 + threadIdx.x) >> 6);
  const int nw = gridDim.x * 4;
  for (int r = w0; r < n; r += nw) {
    const int64_t i = L[r];
    Src s{};
    int64_t li;
    rows.get(i, s, li);
    const int64_t nsrc = s.bind(li, 0, s.T);
    int32_t key;
    uint8_t dummy;
    wave_gather_products<SrBool, Src, false>(s, nsrc, key, dummy);
    wave_bitonic_sort(key, dummy);
    const int32_t prev = __shfl_up(key, 1u, kWave);
    const bool head = key != 0x7FFFFFFF && (lane_id() == 0 || prev != key);
    const unsigned long long hm = __ballot(head);
    if (lane_id() == 0) cnt_out[i] = __popcll(hm);
  }
}

template <class Sr, class Rows>
__global__ __launch_bounds__(256) void k_num_small(Rows rows, Bins bins, int bin, OutC C, int32_t* err) {
  using Src = typename Rows::Src;
  using Acc = typename Sr::Acc;
  using V = typename Sr::V;
  const int n = bins.count[bin];
  const int32_t* L = bins.list + bins.start[bin];
  const int w0 = (int)(((int64_t)blockIdx.x * 256 + threadIdx.x) >> 6);
  const int nw = gridDim.x * 4;
  for (int r = w0; r < n; r += nw) {
    const int64_t i = L[r];
    Src s{};
    int64_t li;
    rows.get(i, s, li);
    const int64_t nsrc = s.bind(li, 0, s.T);
    int32_t key;
    Acc acc;
    wave_gather_products<Sr, Src, true>(s, nsrc, key, acc);
    wave_bitonic_sort(key, acc);
    // segmented fold of equal keys: after the loop the first lane of each run
    // holds the (+) of the whole run
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
      const int32_t ok = shfl_down_any(key, d);
      const Acc oa = shfl_down_any(acc, d);
      if (lane_id() + d < kWave && ok == key) acc = Sr::add(acc, oa);
    }
    const int32_t prev = __shfl_up(key, 1u, kWave);
    const bool head = key != 0x7FFFFFFF && (lane_id() == 0 || prev != key);
    const unsigned long long hm = __ballot(head);
    const int64_t o = C.rowptr[i];
    const int64_t m = C.rowptr[i + 1] - o;
    if (head) {
      const int pos = __popcll(hm & lanes_below());
      if (pos < m) {
        C.col[o + pos] = key;
        ((V*)C.val)[o + pos] = Sr::out(acc);
      }
    }
    if (lane_id() == 0 && __popcll(hm) != m) atomicOr(err, 1);
  }
}

// ---- hash rows: one workgroup per row, LDS open addressing --------------------------

template <class Rows, int LGS, int BS>
__global__ __launch_bounds__(BS) void k_sym_hash(Rows rows, Bins bins, int bin, int64_t* cnt_out) {
  using Src = typename Rows::Src;
  constexpr int S = 1 << LGS, NW = BS / kWave;
  using Item = typename Src::Item;
  __shared__ int32_t s_keys[S];
  __shared__ Item s_item[BS];
  __shared__ int64_t s_start[BS], s_off[BS], s_wave[NW];
  const int n = bins.count[bin];
  const int32_t* L = bins.list + bins.start[bin];
  for (int r = blockIdx.x; r < n; r += gridDim.x) {
    const int64_t i = L[r];
    for (int x = threadIdx.x; x < S; x += BS) s_keys[x] = kEmptyKey;
    block_sync();
    Src s{};
    int64_t li;
    rows.get(i, s, li);
    const int64_t nsrc = s.bind(li, 0, s.T);
    int64_t fresh_cnt = 0;
    auto fetch = [&](const Item& it, int64_t idx) { return s.col(it, idx); };
    auto apply = [&](int32_t c) {
      bool fresh;
      hash_insert(s_keys, LGS, c, &fresh);
      fresh_cnt += fresh ? 1 : 0;
    };
    for_each_product<BS, kUnroll>(s, nsrc, s_item, s_start, s_off, s_wave, fetch, apply);
    const int64_t tot = block_sum<NW, int64_t>(fresh_cnt, s_wave);
    if (threadIdx.x == 0) cnt_out[i] = tot;
  }
}

// Symbolic hash rows, one wavefront per row: each wavefront of the block
// counts the distinct columns of its own rows in its own LDS table of 2^LGS
// keys, with no workgroup barrier.  A row's sources are taken 64 at a time
// (one per lane: a wavefront scan of their segment lengths); the chunk's
// products are then spread over the lanes, kWaveU per lane per round, each
// lane finding its product's source by a binary search over the 64 segment
// offsets and issuing its round's gathers before inserting any column.
constexpr int kWaveU = 4;

template <class Rows, int LGS, int BS>
__global__ __launch_bounds__(BS) void k_sym_hash_wave(Rows rows, Bins bins, int bin, int64_t* cnt_out) {
  using Src = typename Rows::Src;
  using Item = typename Src::Item;
  constexpr int S = 1 << LGS, NW = BS / kWave;
  __shared__ int32_t s_keys[NW][S];
  __shared__ int64_t s_start[NW][kWave], s_off[NW][kWave];
  __shared__ Item s_item[NW][kWave];
  const int wv = wave_id(), l = lane_id();
  int32_t* keys = s_keys[wv];
  const int64_t* off = s_off[wv];
  const int n = bins.count[bin];
  const int32_t* L = bins.list + bins.start[bin];
  for (int r = blockIdx.x * NW + wv; r < n; r += gridDim.x * NW) {
    const int64_t i = L[r];
    for (int x = l; x < S; x += kWave) keys[x] = kEmptyKey;
    Src s{};
    int64_t li;
    rows.get(i, s, li);
    const int64_t nsrc = s.bind(li, 0, s.T);
    int32_t fresh = 0;
    for (int64_t j0 = 0; j0 < nsrc; j0 += kWave) {
      Item it{};
      int64_t st = 0, len = 0;
      if (j0 + l < nsrc) s.load(j0 + l, it, st, len);
      const int64_t inc = wave_incl_scan(len);
      const int64_t tot = lane_value(inc, kWave - 1);
      s_off[wv][l] = inc - len;
      s_start[wv][l] = st;
      s_item[wv][l] = it;
      wave_lds_sync();
      for (int64_t q0 = 0; q0 < tot; q0 += (int64_t)kWave * kWaveU) {
        int32_t c[kWaveU];
#pragma unroll
        for (int u = 0; u < kWaveU; ++u) {
          const int64_t q = q0 + u * kWave + l;
          c[u] = kEmptyKey;
          if (q < tot) {
            // the owner: the last source whose offset is at most q (sources
            // past the row's end have offset tot > q)
            int lo = 0;
#pragma unroll
            for (int step = kWave / 2; step > 0; step >>= 1)
              if (off[lo + step] <= q) lo += step;
            c[u] = s.col(s_item[wv][lo], s_start[wv][lo] + (q - off[lo]));
          }
        }
#pragma unroll
        for (int u = 0; u < kWaveU; ++u)
          if (c[u] != kEmptyKey) {
            bool fr;
            hash_insert(keys, LGS, c[u], &fr);
            fresh += fr ? 1 : 0;
          }
      }
      wave_lds_sync();
    }
    const int32_t cnt = wave_sum(fresh);
    if (l == 0) cnt_out[i] = cnt;
    wave_lds_sync();
  }
}

// Numeric rows of at most CAP entries over at most 32*WORDS columns, one
// wavefront per row, no workgroup barrier: pass 1 sets the row's columns in
// the wavefront's LDS bitmap, each lane turns the popcounts of its
// consecutive bitmap words into their ranks (one wavefront scan), pass 2
// folds every product into vals[rank(column)] and stores its column (16 bits:
// the columns lie below 65536) at the same rank -- the products are gathered
// again -- and the write-out copies columns and values in rank order: no
// hashing and no sort.
template <class Sr, class Rows, int WORDS, int CAP, int BS>
__global__ __launch_bounds__(BS) void k_num_wave_bitmap(Rows rows, Bins bins, int bin, OutC C, int32_t* err) {
  using Src = typename Rows::Src;
  using Item = typename Src::Item;
  using Acc = typename Sr::Acc;
  using V = typename Sr::V;
  constexpr int NW = BS / kWave;
  constexpr int kLaneWords = WORDS / kWave;
  static_assert(WORDS % kWave == 0 && CAP <= 65535, "whole words per lane, 16-bit ranks");
  __shared__ uint32_t s_bits[NW][WORDS];
  __shared__ uint16_t s_rank[NW][WORDS];
  __shared__ Acc s_val[NW][CAP];
  __shared__ uint16_t s_col[NW][CAP];
  __shared__ int64_t s_start[NW][kWave], s_off[NW][kWave];
  __shared__ Item s_item[NW][kWave];
  static_assert(32 * WORDS <= 65536, "16-bit columns");
  const int wv = wave_id(), l = lane_id();
  uint32_t* bits = s_bits[wv];
  uint16_t* rank = s_rank[wv];
  Acc* vals = s_val[wv];
  uint16_t* cols = s_col[wv];
  const int64_t* off = s_off[wv];
  for (int x = l; x < WORDS; x += kWave) bits[x] = 0u;
  const int n = bins.count[bin];
  const int32_t* L = bins.list + bins.start[bin];
  for (int r = blockIdx.x * NW + wv; r < n; r += gridDim.x * NW) {
    const int64_t i = L[r];
    const int64_t o = uniform64(C.rowptr[i]);
    const int32_t m = (int32_t)(C.rowptr[i + 1] - o);
    for (int x = l; x < m && x < CAP; x += kWave) vals[x] = Sr::ident();
    Src s{};
    int64_t li;
    rows.get(i, s, li);
    const int64_t nsrc = s.bind(li, 0, s.T);
    // the row's products, 64 sources at a time; f(col, value-index, item)
    auto products = [&](auto&& f) {
      for (int64_t j0 = 0; j0 < nsrc; j0 += kWave) {
        Item it{};
        int64_t st = 0, len = 0;
        if (j0 + l < nsrc) s.load(j0 + l, it, st, len);
        const int64_t inc = wave_incl_scan(len);
        const int64_t tot = lane_value(inc, kWave - 1);
        s_off[wv][l] = inc - len;
        s_start[wv][l] = st;
        s_item[wv][l] = it;
        wave_lds_sync();
        for (int64_t q0 = 0; q0 < tot; q0 += (int64_t)kWave * kWaveU) {
          int32_t c[kWaveU];
          int64_t idx[kWaveU];
          int own[kWaveU];
#pragma unroll
          for (int u = 0; u < kWaveU; ++u) {
            const int64_t q = q0 + u * kWave + l;
            c[u] = -1;
            idx[u] = 0;
            own[u] = 0;
            if (q < tot) {
              int lo = 0;
#pragma unroll
              for (int step = kWave / 2; step > 0; step >>= 1)
                if (off[lo + step] <= q) lo += step;
              own[u] = lo;
              idx[u] = s_start[wv][lo] + (q - off[lo]);
              c[u] = s.col(s_item[wv][lo], idx[u]);
            }
          }
#pragma unroll
          for (int u = 0; u < kWaveU; ++u)
            if (c[u] >= 0) f(c[u] & (32 * WORDS - 1), idx[u], s_item[wv][own[u]]);
        }
        wave_lds_sync();
      }
    };
    // pass 1: the column set
    products([&](int32_t c, int64_t, const Item&) { atomicOr(&bits[c >> 5], 1u << (c & 31)); });
    wave_lds_sync();
    // ranks: lane l owns words [l*lw, (l+1)*lw), lw covering the product's
    // own columns
    const int64_t ncw = (s.ncols + 31) >> 5;
    const int lw = ncw >= WORDS ? kLaneWords : (int)((ncw + kWave - 1) / kWave);
    const int w0 = l * lw;
    int32_t lt = 0;
    for (int k = 0; k < lw; ++k) lt += __popc(bits[w0 + k]);
    const int32_t linc = wave_incl_scan(lt);
    const int32_t total = lane_value(linc, kWave - 1);
    int32_t rk = linc - lt;
    for (int k = 0; k < lw; ++k) {
      rank[w0 + k] = (uint16_t)rk;
      rk += __popc(bits[w0 + k]);
    }
    if (l == 0 && total != m) atomicOr(err, 1);
    wave_lds_sync();
    // pass 2: fold every product into its compacted slot
    products([&](int32_t c, int64_t idx, const Item& it) {
      const int w = c >> 5;
      const int32_t rr = (int32_t)rank[w] + __popc(bits[w] & ((1u << (c & 31)) - 1u));
      if (rr < m && rr < CAP) {
        Sr::lds_acc(&vals[rr], s.template value<Sr>(it, idx));
        cols[rr] = (uint16_t)c;
      }
    });
    wave_lds_sync();
    // write-out in rank order; the row's words are cleared for the next row
    for (int x = l; x < m && x < CAP; x += kWave) {
      C.col[o + x] = (int32_t)cols[x];
      ((V*)C.val)[o + x] = Sr::out(vals[x]);
    }
    for (int k = 0; k < lw; ++k) bits[w0 + k] = 0u;
    wave_lds_sync();
  }
}

// Numeric rows of at most CAP entries over at most 32*WORDS columns, one
// workgroup per row: the same bitmap-and-rank scheme as k_num_wave_bitmap
// with the bitmap shared by the workgroup, so its LDS (bitmap, word ranks,
// CAP accumulators and columns, and the product iterator's arrays) leaves
// room for several rows per CU where a hash table with its sort buffer
// leaves one.  Thread t owns bitmap words [t*WORDS/BS, (t+1)*WORDS/BS):
// their popcounts and, after one block scan, their ranks.  Pass 2 also
// stores each entry's column (16 bits) at its rank, so the write-out copies
// both arrays.
template <class Sr, class Src, int WORDS, int CAP, int BS>
struct BitmapRowSmem {
  uint32_t bits[WORDS];
  uint16_t rank[WORDS];
  typename Sr::Acc val[CAP];
  uint16_t col[CAP];
  typename Src::Item item[BS];
  int64_t start[BS], off[BS], wave[BS / kWave];
  int64_t se[Src::kParts ? 2 * kLdsParts : 1];  // merge part bounds (merge_bounds)
};

// Products per lane per round of a workgroup-per-row fold over rows of about
// P products: small enough that every wavefront of the workgroup gets a
// block of the row, at most kUnroll.
constexpr int row_unroll(int P, int BS) { return P / BS < 1 ? 1 : (P / BS > kUnroll ? kUnroll : P / BS); }

// The part of local row li inside column tiles [t0, t1) (the whole row:
// 0, T), whose columns must lie below 32*WORDS past the range's first
// column; m entries written from o.  The bitmap is clear on entry and on
// exit.
template <class Sr, class Src, int WORDS, int CAP, int BS, bool kHold>
SG_DEV void bitmap_row_fold(BitmapRowSmem<Sr, Src, WORDS, CAP, BS>& sm, Src& s, int64_t li, int32_t t0, int32_t t1,
                            int64_t o, int32_t m, OutC C, int32_t* err) {
  using Item = typename Src::Item;
  using Acc = typename Sr::Acc;
  using V = typename Sr::V;
  constexpr int NW = BS / kWave;
  constexpr int kThreadWords = WORDS / BS;
  static_assert(WORDS % BS == 0 && CAP <= 65535, "whole words per thread, 16-bit ranks");
  static_assert(32 * WORDS <= 65536, "16-bit columns");
  constexpr int U = row_unroll(CAP, BS);
  const int w0 = (int)threadIdx.x * kThreadWords;
  for (int x = threadIdx.x; x < m && x < CAP; x += BS) sm.val[x] = Sr::ident();
  const int64_t nsrc = s.bind(li, t0, t1);
  if constexpr (Src::kParts) {
    if (s.nparts <= kLdsParts && !(t0 == 0 && t1 == s.T)) s.template merge_bounds<BS>(sm.se);
  }
  const int32_t c0 = t0 << kTileLog;  // columns relative to the range's first
  auto f1 = [&](const Item& it, int64_t idx) { return (s.col(it, idx) - c0) & (32 * WORDS - 1); };
  auto a1 = [&](int32_t c) { atomicOr(&sm.bits[c >> 5], 1u << (c & 31)); };
  auto f2 = [&](const Item& it, int64_t idx) {
    return ColVal<Acc>{(s.col(it, idx) - c0) & (32 * WORDS - 1), s.template value<Sr>(it, idx)};
  };
  // pass 1: the column set (columns masked to the bitmap); with kHold, a row
  // of one round keeps its products in registers for pass 2
  ColVal<Acc> pp[kHold ? U : 1];
  bool ok[kHold ? U : 1];
  bool held = false;
  if constexpr (kHold) {
    auto key = [](const ColVal<Acc>& p) { return p.c; };
    held = products_held<BS, U>(s, nsrc, sm.item, sm.start, sm.off, sm.wave, f2, key, f1, a1, pp, ok);
  } else {
    for_each_product<BS, U>(s, nsrc, sm.item, sm.start, sm.off, sm.wave, f1, a1);
  }
  int32_t lt = 0;
#pragma unroll
  for (int k = 0; k < kThreadWords; ++k) lt += __popc(sm.bits[w0 + k]);
  int32_t total;
  int32_t rk = block_excl_scan<NW, int32_t>(lt, (int32_t*)sm.wave, &total);
#pragma unroll
  for (int k = 0; k < kThreadWords; ++k) {
    sm.rank[w0 + k] = (uint16_t)rk;
    rk += __popc(sm.bits[w0 + k]);
  }
  if (threadIdx.x == 0 && total != m) atomicOr(err, 1);
  block_sync();
  // pass 2: fold every product into its compacted slot
  auto a2 = [&](const ColVal<Acc>& p) {
    const int w = p.c >> 5;
    const int32_t rr = (int32_t)sm.rank[w] + __popc(sm.bits[w] & ((1u << (p.c & 31)) - 1u));
    if (rr < m && rr < CAP) {
      Sr::lds_acc(&sm.val[rr], p.v);
      sm.col[rr] = (uint16_t)p.c;
    }
  };
  if (held) {
#pragma unroll
    for (int u = 0; u < (kHold ? U : 1); ++u)
      if (ok[u]) a2(pp[u]);
    block_sync();
  } else {
    for_each_product<BS, U>(s, nsrc, sm.item, sm.start, sm.off, sm.wave, f2, a2);
  }
  // write-out in rank order; the thread's words are cleared for the next row
  for (int x = threadIdx.x; x < m && x < CAP; x += BS) {
    C.col[o + x] = c0 + (int32_t)sm.col[x];
    ((V*)C.val)[o + x] = Sr::out(sm.val[x]);
  }
#pragma unroll
  for (int k = 0; k < kThreadWords; ++k) sm.bits[w0 + k] = 0u;
  block_sync();
}

template <class Sr, class Rows, int WORDS, int CAP, int BS>
__global__ __launch_bounds__(BS) void k_num_bitmap_row(Rows rows, Bins bins, int bin, OutC C, int32_t* err) {
  using Src = typename Rows::Src;
  __shared__ BitmapRowSmem<Sr, Src, WORDS, CAP, BS> sm;
  for (int x = threadIdx.x; x < WORDS; x += BS) sm.bits[x] = 0u;
  block_sync();
  const int n = bins.count[bin];
  const int32_t* L = bins.list + bins.start[bin];
  for (int r = blockIdx.x; r < n; r += gridDim.x) {
    const int64_t i = L[r];
    const int64_t o = C.rowptr[i];
    const int32_t m = (int32_t)(C.rowptr[i + 1] - o);
    Src s{};
    int64_t li;
    rows.get(i, s, li);
    // rows of up to 1024 products keep them in registers between the passes
    // (at 8 products per lane the registers would cost occupancy)
    bitmap_row_fold<Sr, Src, WORDS, CAP, BS, (row_unroll(CAP, BS) <= 4)>(sm, s, li, 0, s.T, o, m, C, err);
  }
}

// Numeric rows of at most CAP products over any B, one workgroup per row,
// with neither a hash table nor a sort: each source's segment of the row (a
// B row times its A value, or one part's row in a merge) is already sorted
// by column, so the row is the merge of its non-empty segments.  The
// products are staged in LDS in segment order (the runs); each round merges
// neighbouring runs pairwise along their merge paths (ties: the left run
// first, so equal columns stay in source order); after ceil(log2(runs))
// rounds equal columns are adjacent and the first element of each group
// folds the group with (+).  The groups' results are staged at their ranks in the free
// buffer and copied out coalesced.
// One round of the pairwise merge: the runs of this round are the round-0
// runs taken 2^sh at a time, run q covering [roff[q<<sh], roff[(q+1)<<sh])
// (clipped to the last), and runs 2p and 2p+1 are merged into the output
// range they cover together.  Thread t produces outputs [t*EPT, (t+1)*EPT):
// its pair by a binary search over the pairs, how many of the pair's first
// outputs come from the left run by a binary search along the pair's merge
// path (the left run's element goes first on equal columns, so the merge is
// stable), then EPT steps of a sequential merge, moving to the next pair
// where one ends.  Columns are below 2^31 - 1, which stands for "run empty".
template <class Acc, int EPT, bool kVals = true>
SG_DEV void merge_path_round(const int32_t* kin, const Acc* vin, int32_t* kout, Acc* vout, const uint16_t* roff,
                             int runs, int total, int sh) {
  const int x0 = (int)threadIdx.x * EPT;
  if (x0 >= total) return;
  const int sh1 = sh + 1;
  const int np = (runs + (1 << sh1) - 1) >> sh1;
  auto bound = [&](int r) { return (int)roff[r < runs ? r : runs]; };
  int p = 0;
  for (int step = 1 << (31 - __clz(np)); step > 0; step >>= 1) {
    const int t = p + step;
    if (t < np && (int)roff[t << sh1] <= x0) p = t;
  }
  int s = roff[p << sh1], mid = bound((2 * p + 1) << sh), e = bound((2 * p + 2) << sh);
  const int d = x0 - s;
  int lo = d > e - mid ? d - (e - mid) : 0, hi = d < mid - s ? d : mid - s;
  while (lo < hi) {
    const int m = (lo + hi) >> 1;
    if (kin[s + m] <= kin[mid + d - 1 - m]) lo = m + 1;
    else hi = m;
  }
  int a = s + lo, b = mid + (d - lo);
  constexpr int32_t kNone = 0x7FFFFFFF;
  int32_t ka = a < mid ? kin[a] : kNone, kb = b < e ? kin[b] : kNone;
#pragma unroll
  for (int k = 0; k < EPT; ++k) {
    const int x = x0 + k;
    if (x >= total) break;
    if (x == e) {  // the next pair starts here
      ++p;
      s = e;
      mid = bound((2 * p + 1) << sh);
      e = bound((2 * p + 2) << sh);
      a = s;
      b = mid;
      ka = a < mid ? kin[a] : kNone;
      kb = b < e ? kin[b] : kNone;
    }
    if (a < mid && (b >= e || ka <= kb)) {
      kout[x] = ka;
      if constexpr (kVals) vout[x] = vin[a];
      ++a;
      ka = a < mid ? kin[a] : kNone;
    } else {
      kout[x] = kb;
      if constexpr (kVals) vout[x] = vin[b];
      ++b;
      kb = b < e ? kin[b] : kNone;
    }
  }
}

template <class Sr, class Src, int CAP, int BS>
struct MergeRowSmem {
  static constexpr int kChunkBytes = BS * (16 + (int)sizeof(typename Src::Item));
  static constexpr int kBufBytes = CAP * (4 + (int)sizeof(typename Sr::Acc));
  int32_t key[CAP];
  typename Sr::Acc val[CAP];
  // the second (key, value) buffer of the rounds; while the products are
  // staged, the iterator's chunk arrays (start, off, item)
  alignas(16) char other[kBufBytes > kChunkBytes ? kBufBytes : kChunkBytes];
  uint16_t roff[CAP + 1];  // first element of each run (round 0)
  int64_t wave[BS / kWave];
};

template <class Sr, class Rows, int CAP, int BS>
__global__ __launch_bounds__(BS) void k_num_merge_row(Rows rows, Bins bins, int bin, OutC C, int32_t* err) {
  using Src = typename Rows::Src;
  using Item = typename Src::Item;
  using Acc = typename Sr::Acc;
  using V = typename Sr::V;
  constexpr int NW = BS / kWave;
  constexpr int EPT = (CAP + BS - 1) / BS;  // elements per thread
  constexpr int U = row_unroll(CAP, BS);
  static_assert(CAP <= 65535, "16-bit run offsets");
  __shared__ MergeRowSmem<Sr, Src, CAP, BS> sm;
  int64_t* const c_start = reinterpret_cast<int64_t*>(sm.other);
  int64_t* const c_off = c_start + BS;
  Item* const c_item = reinterpret_cast<Item*>(c_off + BS);
  const int n = bins.count[bin];
  const int32_t* L = bins.list + bins.start[bin];
  for (int r = blockIdx.x; r < n; r += gridDim.x) {
    const int64_t i = L[r];
    const int64_t o = C.rowptr[i];
    const int32_t m = (int32_t)(C.rowptr[i + 1] - o);
    Src s{};
    int64_t li;
    rows.get(i, s, li);
    const int64_t nsrc = s.bind(li, 0, s.T);
    auto fetch = [&](const Item& it, int64_t idx) {
      return ColVal<Acc>{s.col(it, idx), s.template value<Sr>(it, idx)};
    };
    // staging, one chunk of BS sources at a time: the products in segment
    // order and the first element of every non-empty segment
    int32_t total = 0, runs = 0;  // block-uniform
    bool over = false;
    for (int64_t c0 = 0; c0 < nsrc; c0 += BS) {
      int nc;
      const int64_t ct = product_chunk<BS>(s, nsrc, c0, c_item, c_start, c_off, sm.wave, &nc);
      if (ct > (int64_t)(CAP - total)) {
        over = true;
        break;
      }
      for (int k = threadIdx.x; k < nc; k += BS) sm.roff[runs + k] = (uint16_t)(total + c_off[k]);
      for (int64_t qb = (int64_t)wave_id() * kWave * U; qb < ct; qb += (int64_t)NW * kWave * U) {
        ColVal<Acc> p[U];
        bool ok[U];
        product_block<BS, U, Src>(c_item, c_start, c_off, nc, ct, qb, fetch, p, ok);
#pragma unroll
        for (int u = 0; u < U; ++u)
          if (ok[u]) {
            const int x = total + (int)(qb + u * kWave + lane_id());
            sm.key[x] = p[u].c;
            sm.val[x] = p[u].v;
          }
      }
      total += (int32_t)ct;
      runs += nc;
      block_sync();
    }
    if (over) {  // more products than the bin allows: the analysis disagrees
      if (threadIdx.x == 0) atomicOr(err, 1);
      continue;
    }
    if (threadIdx.x == 0) sm.roff[runs] = (uint16_t)total;
    block_sync();
    int32_t* kin = sm.key;
    Acc* vin = sm.val;
    int32_t* kout = reinterpret_cast<int32_t*>(sm.other);
    Acc* vout = reinterpret_cast<Acc*>(sm.other + CAP * 4);
    for (int sh = 0; (1 << sh) < runs; ++sh) {
      merge_path_round<Acc, EPT>(kin, vin, kout, vout, sm.roff, runs, total, sh);
      block_sync();
      int32_t* kt = kin;
      kin = kout;
      kout = kt;
      Acc* vt = vin;
      vin = vout;
      vout = vt;
    }
    // groups of equal columns: thread t holds elements [t*EPT, (t+1)*EPT)
    const int x0 = (int)threadIdx.x * EPT;
    int32_t heads = 0;
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
      const int x = x0 + k;
      if (x < total && (x == 0 || kin[x] != kin[x - 1])) ++heads;
    }
    int32_t nh;
    int32_t rk = block_excl_scan<NW, int32_t>(heads, (int32_t*)sm.wave, &nh);
    if (threadIdx.x == 0 && nh != m) atomicOr(err, 1);
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
      const int x = x0 + k;
      if (x < total && (x == 0 || kin[x] != kin[x - 1])) {
        const int32_t cx = kin[x];
        Acc a = vin[x];
        for (int y = x + 1; y < total && kin[y] == cx; ++y) a = Sr::add(a, vin[y]);
        kout[rk] = cx;
        vout[rk] = a;
        ++rk;
      }
    }
    block_sync();
    const int wr = nh < m ? nh : m;
    for (int x = threadIdx.x; x < wr; x += BS) {
      C.col[o + x] = kout[x];
      ((V*)C.val)[o + x] = Sr::out(vout[x]);
    }
    block_sync();
  }
}

// Symbolic count of rows of at most CAP products by the same merge of the
// row's sorted segments, columns only: the count is the number of groups of
// equal columns after the last round.
template <class Rows, int CAP, int BS>
__global__ __launch_bounds__(BS) void k_sym_merge_row(Rows rows, Bins bins, int bin, int64_t* cnt_out) {
  using Src = typename Rows::Src;
  using Item = typename Src::Item;
  constexpr int NW = BS / kWave;
  constexpr int EPT = (CAP + BS - 1) / BS;
  constexpr int U = row_unroll(CAP, BS);
  constexpr int kChunkBytes = BS * (16 + (int)sizeof(Item));
  static_assert(CAP <= 65535, "16-bit run offsets");
  __shared__ int32_t s_key[CAP];
  __shared__ __align__(16) char s_other[CAP * 4 > kChunkBytes ? CAP * 4 : kChunkBytes];
  __shared__ uint16_t s_roff[CAP + 1];
  __shared__ int64_t s_wave[NW];
  int64_t* const c_start = reinterpret_cast<int64_t*>(s_other);
  int64_t* const c_off = c_start + BS;
  Item* const c_item = reinterpret_cast<Item*>(c_off + BS);
  const int n = bins.count[bin];
  const int32_t* L = bins.list + bins.start[bin];
  for (int r = blockIdx.x; r < n; r += gridDim.x) {
    const int64_t i = L[r];
    Src s{};
    int64_t li;
    rows.get(i, s, li);
    const int64_t nsrc = s.bind(li, 0, s.T);
    auto fetch = [&](const Item& it, int64_t idx) { return s.col(it, idx); };
    int32_t total = 0, runs = 0;
    bool over = false;
    for (int64_t c0 = 0; c0 < nsrc; c0 += BS) {
      int nc;
      const int64_t ct = product_chunk<BS>(s, nsrc, c0, c_item, c_start, c_off, s_wave, &nc);
      if (ct > (int64_t)(CAP - total)) {
        over = true;
        break;
      }
      for (int k = threadIdx.x; k < nc; k += BS) s_roff[runs + k] = (uint16_t)(total + c_off[k]);
      for (int64_t qb = (int64_t)wave_id() * kWave * U; qb < ct; qb += (int64_t)NW * kWave * U) {
        int32_t p[U];
        bool ok[U];
        product_block<BS, U, Src>(c_item, c_start, c_off, nc, ct, qb, fetch, p, ok);
#pragma unroll
        for (int u = 0; u < U; ++u)
          if (ok[u]) s_key[total + (int)(qb + u * kWave + lane_id())] = p[u];
      }
      total += (int32_t)ct;
      runs += nc;
      block_sync();
    }
    if (over) {  // more products than the bin allows: count nothing, so the
                 // numeric pass flags the row
      if (threadIdx.x == 0) cnt_out[i] = 0;
      continue;
    }
    if (threadIdx.x == 0) s_roff[runs] = (uint16_t)total;
    block_sync();
    int32_t* kin = s_key;
    int32_t* kout = reinterpret_cast<int32_t*>(s_other);
    for (int sh = 0; (1 << sh) < runs; ++sh) {
      merge_path_round<int32_t, EPT, false>(kin, nullptr, kout, nullptr, s_roff, runs, total, sh);
      block_sync();
      int32_t* kt = kin;
      kin = kout;
      kout = kt;
    }
    int32_t heads = 0;
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
      const int x = (int)threadIdx.x * EPT + k;
      if (x < total && (x == 0 || kin[x] != kin[x - 1])) ++heads;
    }
    const int64_t tot = block_sum<NW, int64_t>((int64_t)heads, s_wave);
    if (threadIdx.x == 0) cnt_out[i] = tot;
  }
}

// Symbolic count of rows over at most 32*WORDS columns, one workgroup per
// row: the distinct columns are the set bits of an LDS bitmap.
template <class Rows, int WORDS, int BS, int U>
__global__ __launch_bounds__(BS) void k_sym_bitmap_row(Rows rows, Bins bins, int bin, int64_t* cnt_out) {
  using Src = typename Rows::Src;
  using Item = typename Src::Item;
  constexpr int NW = BS / kWave;
  constexpr int kThreadWords = WORDS / BS;
  static_assert(WORDS % BS == 0, "whole words per thread");
  __shared__ uint32_t s_bits[WORDS];
  __shared__ Item s_item[BS];
  __shared__ int64_t s_start[BS], s_off[BS], s_wave[NW];
  for (int x = threadIdx.x; x < WORDS; x += BS) s_bits[x] = 0u;
  block_sync();
  const int n = bins.count[bin];
  const int32_t* L = bins.list + bins.start[bin];
  const int w0 = (int)threadIdx.x * kThreadWords;
  for (int r = blockIdx.x; r < n; r += gridDim.x) {
    const int64_t i = L[r];
    Src s{};
    int64_t li;
    rows.get(i, s, li);
    const int64_t nsrc = s.bind(li, 0, s.T);
    auto f = [&](const Item& it, int64_t idx) { return s.col(it, idx) & (32 * WORDS - 1); };
    auto a = [&](int32_t c) { atomicOr(&s_bits[c >> 5], 1u << (c & 31)); };
    for_each_product<BS, U>(s, nsrc, s_item, s_start, s_off, s_wave, f, a);
    int64_t lt = 0;
#pragma unroll
    for (int k = 0; k < kThreadWords; ++k) {
      lt += __popc(s_bits[w0 + k]);
      s_bits[w0 + k] = 0u;
    }
    const int64_t tot = block_sum<NW, int64_t>(lt, s_wave);
    if (threadIdx.x == 0) cnt_out[i] = tot;
  }
}

// LDS of one hash task: a table of 2^LGS keys and accumulators, the sort
// buffer, the flattened iterator's per-source arrays and radix-sort counters.
template <class Sr, class Src, int LGS, int BS>
struct HashSmem {
  static constexpr int S = 1 << LGS, NW = BS / kWave;
  int32_t keys[S];
  typename Sr::Acc vals[S];
  uint64_t sort[S / 2];
  typename Src::Item item[BS];
  int64_t start[BS], off[BS], wave[NW];
  int32_t hist[(S >= 1024) ? NW * 256 : 1];
  int32_t wt[4];
  int32_t n;
  int64_t se[Src::kParts ? 2 * kLdsParts : 1];  // merge part bounds (merge_bounds)
};

// One hash task: the products of local row li restricted to column tiles
// [t0, t1) go into an LDS hash table (find-or-claim the column's slot, then
// an LDS atomic (+)); the occupied slots are compacted, sorted by column
// (radix sort above 256 entries, bitonic below) and written to
// C.col/C.val[o .. o+m).  Contains barriers; the whole workgroup calls it.
template <class Sr, class Src, int LGS, int BS>
SG_DEV void hash_task(HashSmem<Sr, Src, LGS, BS>& sm, Src& s, int64_t li, int32_t t0, int32_t t1, int64_t o,
                      int64_t m, OutC C, int32_t* err) {
  constexpr int S = 1 << LGS;
  using Item = typename Src::Item;
  using V = typename Sr::V;
  for (int x = threadIdx.x; x < S; x += BS) {
    sm.keys[x] = kEmptyKey;
    sm.vals[x] = Sr::ident();
  }
  if (threadIdx.x == 0) sm.n = 0;
  block_sync();
  const int64_t nsrc = s.bind(li, t0, t1);
  if constexpr (Src::kParts) {
    if (s.nparts <= kLdsParts && !(t0 == 0 && t1 == s.T)) s.template merge_bounds<BS>(sm.se);
  }
  auto fetch = [&](const Item& it, int64_t idx) {
    return ColVal<typename Sr::Acc>{s.col(it, idx), s.template value<Sr>(it, idx)};
  };
  auto apply = [&](const ColVal<typename Sr::Acc>& p) {
    bool fresh;
    const uint32_t slot = hash_insert(sm.keys, LGS, p.c, &fresh);
    if (slot != kHashFull) Sr::lds_acc(&sm.vals[slot], p.v);
    else atomicOr(err, 2);
  };
  for_each_product<BS, kUnroll>(s, nsrc, sm.item, sm.start, sm.off, sm.wave, fetch, apply);
  const int64_t key_base = (int64_t)t0 << kTileLog;
  for (int x = threadIdx.x; x < S; x += BS) {
    const int32_t k = sm.keys[x];
    if (k != kEmptyKey) {
      const int pos = atomicAdd(&sm.n, 1);
      if (pos < S / 2) sm.sort[pos] = ((uint64_t)(uint32_t)(k - key_base) << 32) | (uint32_t)x;
    }
  }
  block_sync();
  int cnt = sm.n;
  if (threadIdx.x == 0 && cnt != m) atomicOr(err, 1);
  cnt = cnt < S / 2 ? cnt : S / 2;
  const uint64_t* sorted = sm.sort;
  if (cnt > 256) {
    // radix sort on the bits of (column - key_base); the key table is free
    // now and serves as the second buffer
    int64_t hi = (int64_t)t1 << kTileLog;
    hi = hi < s.ncols ? hi : s.ncols;
    const int64_t width = hi - key_base;
    const int kbits = width > 1 ? 32 - __clz((int)(width - 1)) : 1;
    sorted = block_radix_sort_hi<BS, S / 2>(sm.sort, (uint64_t*)sm.keys, cnt, kbits, sm.hist, sm.wt);
  } else {
    int M = 1;
    while (M < cnt) M <<= 1;
    for (int x = cnt + threadIdx.x; x < M; x += BS) sm.sort[x] = ~0ull;
    block_sync();
    block_bitonic_sort<BS>(sm.sort, M);
  }
  const int64_t wr = cnt < m ? cnt : m;
  for (int x = threadIdx.x; x < wr; x += BS) {
    const uint64_t e = sorted[x];
    C.col[o + x] = (int32_t)((int64_t)(e >> 32) + key_base);
    ((V*)C.val)[o + x] = Sr::out(sm.vals[(uint32_t)e]);
  }
  block_sync();
}

template <class Sr, class Rows, int LGS, int BS>
__global__ __launch_bounds__(BS) void k_num_hash(Rows rows, Bins bins, int bin, OutC C, int32_t* err) {
  using Src = typename Rows::Src;
  __shared__ HashSmem<Sr, Src, LGS, BS> sm;
  const int n = bins.count[bin];
  const int32_t* L = bins.list + bins.start[bin];
  for (int r = blockIdx.x; r < n; r += gridDim.x) {
    const int64_t i = L[r];
    const int64_t o = C.rowptr[i];
    const int64_t m = C.rowptr[i + 1] - o;
    Src s{};
    int64_t li;
    rows.get(i, s, li);
    hash_task<Sr, Src, LGS, BS>(sm, s, li, 0, s.T, o, m, C, err);
  }
}

// ---- dense rows: column tiles ----------------------------------------------------------

// Symbolic: a bitmap over up to TILES tiles (64: 1M columns, 128 KB of LDS;
// 4 for narrow B, 8 KB, several workgroups per CU) per pass; per-tile
// popcounts give the row's count and its per-tile output offsets
// off2[h*(Tmax+1) + t] (t = 0..Tmax; entries past the row's own T repeat the
// total).
template <class Rows, int TILES, int BS>
__global__ __launch_bounds__(BS) void k_sym_dense(Rows rows, Bins bins, int64_t* cnt_out, int32_t* off2) {
  using Src = typename Rows::Src;
  constexpr int NW = BS / kWave;
  static_assert(TILES <= kWave, "one wavefront scans the tile counts");
  using Item = typename Src::Item;
  __shared__ uint32_t s_bm[TILES * kTileWords];
  __shared__ Item s_item[BS];
  __shared__ int64_t s_start[BS], s_off[BS], s_wave[NW];
  __shared__ int32_t s_tcnt[TILES];
  __shared__ int32_t s_run;
  const int32_t first = bins.start[kBinDense0];
  const int32_t nd = dense_rows(bins);
  const int32_t* L = bins.list + first;
  const int32_t Tmax = rows.Tmax;
  for (int h = blockIdx.x; h < nd; h += gridDim.x) {
    const int64_t i = L[h];
    Src s{};
    int64_t li;
    rows.get(i, s, li);
    const int32_t T = s.T;
    int32_t* o2 = off2 + (int64_t)h * (Tmax + 1);
    int32_t run = 0;
    for (int st = 0; st < T; st += TILES) {
      const int t1 = (st + TILES) < T ? (st + TILES) : T;
      const int64_t c0 = (int64_t)st << kTileLog;
      // whole tiles: columns are interleaved over a tile's words (column x
      // of a tile: word x mod 512, bit x / 512), since only per-tile counts
      // are needed; neighbouring columns then land in different words and
      // LDS banks
      const int nwords = (t1 - st) * kTileWords;
      for (int x = threadIdx.x; x < nwords; x += BS) s_bm[x] = 0u;
      block_sync();
      const int64_t nsrc = s.bind(li, st, t1);
      auto fetch = [&](const Item& it, int64_t idx) { return (int32_t)(s.col(it, idx) - c0); };
      auto apply = [&](int32_t c) {
        atomicOr(&s_bm[(c >> kTileLog) * kTileWords + (c & (kTileWords - 1))], 1u << ((c & (kTile - 1)) >> (kTileLog - 5)));
      };
      for_each_product<BS, kUnroll>(s, nsrc, s_item, s_start, s_off, s_wave, fetch, apply);
      // one wavefront per tile, lanes over its 512 words
      for (int tl = wave_id(); tl < t1 - st; tl += NW) {
        int32_t c = 0;
        for (int x = lane_id(); x < kTileWords; x += kWave) c += __popc(s_bm[tl * kTileWords + x]);
        c = wave_sum(c);
        if (lane_id() == 0) s_tcnt[tl] = c;
      }
      block_sync();
      if (wave_id() == 0) {
        const int ntl = t1 - st;
        const int32_t v = lane_id() < ntl ? s_tcnt[lane_id()] : 0;
        const int32_t inc = wave_incl_scan(v);
        if (lane_id() < ntl) o2[st + lane_id()] = run + inc - v;
        if (lane_id() == kWave - 1) s_run = run + inc;
      }
      block_sync();
      run = s_run;
    }
    for (int t = T + threadIdx.x; t <= Tmax; t += BS) o2[t] = run;
    if (threadIdx.x == 0) cnt_out[i] = run;
    block_sync();
  }
}

// ---- persistent work distribution -------------------------------------------
// Task lists are served through kQueues interleaved queues: task g belongs to
// queue g % kQueues, workgroup b serves queue b % kQueues (consecutive
// workgroups are dispatched round-robin over gfx950's 8 XCDs, so a queue's
// workgroups share one L2) and takes kGrab consecutive queue slots per atomic.
// Counter block layout (int32, zeroed before each use):
//   [0, 3)                      totals of the tile, range and slab task lists
//   [8, 14)                     entries of each list (three uint64)
//   kCtrQueue0 + (l*kQueues + q)*kCtrStride   queue q of list l (l = 3: slab symbolic)
constexpr int kQueues = 8;
constexpr int kGrab = 4;
constexpr int kCtrStride = 16;  // 64 bytes between counters
constexpr int kCtrEntries = 8;  // [8, 14): three uint64 sums of entries per task list (statistics)
constexpr int kCtrQueue0 = 64;
constexpr int kCtrLists = 4;
constexpr int kCtrInts = kCtrQueue0 + kCtrLists * kQueues * kCtrStride;
enum { kListTile = 0, kListRange = 1, kListSlab = 2, kListSymSlab = 3 };

SG_DEV int32_t* queue_ctr(int32_t* ctr, int list, int q) {
  return ctr + kCtrQueue0 + (list * kQueues + q) * kCtrStride;
}

// Calls task(g) for every task g < ntask of this workgroup's queue.  All
// threads of the block call it; task() must be block-uniform.
template <class F>
SG_DEV void for_each_queued(int32_t* ctr, int list, int64_t ntask, int64_t* s_slot, F&& task) {
  const int q = (int)(blockIdx.x % kQueues);
  int32_t* qc = queue_ctr(ctr, list, q);
  const int64_t nq = ntask > q ? (ntask - q + kQueues - 1) / kQueues : 0;
  while (true) {
    if (threadIdx.x == 0) *s_slot = atomicAdd(qc, kGrab);
    block_sync();
    const int64_t j0 = *s_slot;
    block_sync();
    if (j0 >= nq) break;
    const int64_t j1 = (j0 + kGrab) < nq ? (j0 + kGrab) : nq;
    for (int64_t j = j0; j < j1; ++j) task(q + j * kQueues);
  }
}

// for_each_queued for tasks that start from a record: the records of a
// grab's tasks are read together right after the grab (thread j reads the
// j-th with fetch(g)) and wait in s_rec (kGrab entries of LDS), so only a
// grab's first task waits for its record.  task(rec) as above.
template <class Rec, class Fetch, class F>
SG_DEV void for_each_queued_rec(int32_t* ctr, int list, int64_t ntask, int64_t* s_slot, Rec* s_rec, Fetch&& fetch,
                                F&& task) {
  const int q = (int)(blockIdx.x % kQueues);
  int32_t* qc = queue_ctr(ctr, list, q);
  const int64_t nq = ntask > q ? (ntask - q + kQueues - 1) / kQueues : 0;
  while (true) {
    if (threadIdx.x == 0) *s_slot = atomicAdd(qc, kGrab);
    block_sync();
    const int64_t j0 = *s_slot;
    if (j0 >= nq) break;  // uniform; s_slot is not written again
    const int64_t j1 = (j0 + kGrab) < nq ? (j0 + kGrab) : nq;
    if ((int64_t)threadIdx.x < j1 - j0) s_rec[threadIdx.x] = fetch(q + (j0 + (int64_t)threadIdx.x) * kQueues);
    block_sync();
    for (int64_t j = j0; j < j1; ++j) task(s_rec[j - j0]);
  }
}

// Numeric dense-row work is cut into tasks from the symbolic pass's per-tile
// counts.  With column slabs of G tiles (G > 0: single products), a slab
// holding at most slab_cap entries becomes one slab task (bitmap + rank
// accumulator over the slab).  Other tiles: a tile holding at least tile_min
// entries becomes a dense-tile task (dense LDS accumulator, written in column
// order with no sort); runs of sparser tiles inside one slab are grouped into
// range tasks of at most range_cap entries (LDS hash + radix sort).  One
// thread per dense row puts its tasks into per-bucket slots (bucket t of a
// list holds nd slots; tile and range tasks go to the bucket of their first
// tile, slab tasks to their slab); the task kernels walk the buckets in
// order, so all workgroups gather from one narrow column slice of B at a
// time and it stays cache resident.
//   book[l*Tmax + t]                    tasks in bucket t of list l (l = 0, 1, 2)
//   book[3*Tmax + l*(Tmax+1) + t]       bucket offsets of list l
//   ctr[l]                              task total of list l
struct Task {
  int32_t h, t0, t1;
};

__host__ __device__ inline int32_t* book_off(int32_t* book, int32_t Tmax, int list) {
  return book + 3 * Tmax + list * (Tmax + 1);
}
__host__ __device__ inline const int32_t* book_off(const int32_t* book, int32_t Tmax, int list) {
  return book + 3 * Tmax + list * (Tmax + 1);
}

// Bucket counters of up to kTaskAggBuckets tiles per list are aggregated in
// LDS per block (one global atomic per block and bucket instead of one per
// task: every dense row of the chip appends to the same few buckets).
constexpr int kTaskAggBuckets = 1024;
constexpr int kRangeSpanMax = 4;  // column tiles of a range task

template <int BS>
__global__ __launch_bounds__(BS) void k_dense_tasks(Bins bins, const int32_t* off2, int32_t Tmax, int32_t G,
                                                    int32_t slab_cap, int32_t tile_min, int32_t range_cap,
                                                    int32_t run_tiles, Task* tiles, Task* ranges, Task* slabs,
                                                    int32_t* book, int32_t* ctr) {
  __shared__ unsigned long long s_ent[3];
  __shared__ int32_t s_cnt[3 * kTaskAggBuckets], s_base[3 * kTaskAggBuckets];
  if (threadIdx.x < 3) s_ent[threadIdx.x] = 0ull;
  const bool agg = Tmax <= kTaskAggBuckets;  // uniform
  if (agg)
    for (int x = threadIdx.x; x < 3 * Tmax; x += BS) s_cnt[x] = 0;
  block_sync();
  unsigned long long ent[3] = {0ull, 0ull, 0ull};
  const int32_t nd = dense_rows(bins);
  int32_t* cnt_g[3] = {book, book + Tmax, book + 2 * Tmax};  // tile, range, slab buckets
  Task* lists[3] = {tiles, ranges, slabs};
  const int32_t span = G > 0 ? G : Tmax;
  // the tasks of dense row h, in a fixed order: emit(list, bucket, task)
  auto gen = [&](int32_t h, bool count, auto&& emit) {
    const int32_t* o2 = off2 + (int64_t)h * (Tmax + 1);
    for (int32_t ta = 0; ta < Tmax; ta += span) {
      const int32_t tb = (ta + span) < Tmax ? (ta + span) : Tmax;
      const int32_t ms = o2[tb] - o2[ta];
      if (ms == 0) continue;
      if (G > 0 && ms <= slab_cap) {
        emit(kListSlab, ta / G, Task{h, ta, tb});
        if (count) ent[kListSlab] += (unsigned long long)ms;
        continue;
      }
      int32_t r0 = -1, rlast = -1, racc = 0, run0 = -1;
      for (int t = ta; t < tb; ++t) {
        const int32_t c = o2[t + 1] - o2[t];
        if (c == 0) continue;
        if (c >= tile_min) {
          if (r0 >= 0) emit(kListRange, r0, Task{h, r0, rlast + 1});
          r0 = -1;
          racc = 0;
          emit(kListTile, t, Task{h, t, t + 1});
          if (count) ent[kListTile] += (unsigned long long)c;
          continue;
        }
        if (count) ent[kListRange] += (unsigned long long)c;
        if (run_tiles > 0) {
          // one run task per group of run_tiles tiles holding range tiles;
          // its kernel forms the ranges by the rules below
          const int32_t g0 = ta + (t - ta) / run_tiles * run_tiles;
          if (g0 != run0) {
            run0 = g0;
            emit(kListRange, g0, Task{h, g0, (g0 + run_tiles) < tb ? (g0 + run_tiles) : tb});
          }
          continue;
        }
        if (r0 >= 0 && (racc + c > range_cap || t + 1 - r0 > kRangeSpanMax)) {
          emit(kListRange, r0, Task{h, r0, rlast + 1});
          r0 = -1;
          racc = 0;
        }
        if (r0 < 0) r0 = t;
        rlast = t;
        racc += c;
      }
      if (r0 >= 0) emit(kListRange, r0, Task{h, r0, rlast + 1});
    }
  };
  if (!agg) {
    for (int h = blockIdx.x * BS + threadIdx.x; h < nd; h += gridDim.x * BS)
      gen(h, true, [&](int l, int32_t bk, const Task& tk) {
        lists[l][(int64_t)bk * nd + atomicAdd(&cnt_g[l][bk], 1)] = tk;
      });
  } else {
    for (int h0 = blockIdx.x * BS; h0 < nd; h0 += gridDim.x * BS) {
      const int h = h0 + (int)threadIdx.x;
      // count the block's tasks per bucket, reserve each bucket's range with
      // one global atomic, then generate the tasks again into their slots
      if (h < nd) gen(h, true, [&](int l, int32_t bk, const Task&) { atomicAdd(&s_cnt[l * Tmax + bk], 1); });
      block_sync();
      for (int x = threadIdx.x; x < 3 * Tmax; x += BS) {
        const int32_t c = s_cnt[x];
        s_base[x] = c > 0 ? atomicAdd(&cnt_g[x / Tmax][x % Tmax], c) : 0;
        s_cnt[x] = 0;
      }
      block_sync();
      if (h < nd)
        gen(h, false, [&](int l, int32_t bk, const Task& tk) {
          const int32_t k = l * Tmax + bk;
          lists[l][(int64_t)bk * nd + s_base[k] + atomicAdd(&s_cnt[k], 1)] = tk;
        });
      block_sync();
      for (int x = threadIdx.x; x < 3 * Tmax; x += BS) s_cnt[x] = 0;
      block_sync();
    }
  }
  // entries per task kind (statistics): block sums, one atomic each
  for (int l = 0; l < 3; ++l) {
    const unsigned long long v = wave_sum(ent[l]);
    if (lane_id() == 0 && v) atomicAdd(&s_ent[l], v);
  }
  block_sync();
  if (threadIdx.x < 3 && s_ent[threadIdx.x])
    atomicAdd((unsigned long long*)(ctr + kCtrEntries) + threadIdx.x, s_ent[threadIdx.x]);
}

// Exclusive scans of the three bucket-count arrays (one block) and the totals.
template <int BS>
__global__ __launch_bounds__(BS) void k_task_offsets(int32_t* book, int32_t Tmax, int32_t* ctr) {
  __shared__ int32_t s_wave[BS / kWave];
  for (int list = 0; list < 3; ++list) {
    const int32_t* cnt = book + list * Tmax;
    int32_t* off = book_off(book, Tmax, list);
    int32_t carry = 0;
    for (int t0 = 0; t0 < Tmax; t0 += BS) {
      const int t = t0 + threadIdx.x;
      const int32_t v = t < Tmax ? cnt[t] : 0;
      int32_t tot;
      const int32_t ex = block_excl_scan<BS / kWave, int32_t>(v, s_wave, &tot);
      if (t < Tmax) off[t] = carry + ex;
      carry += tot;
    }
    if (threadIdx.x == 0) {
      off[Tmax] = carry;
      ctr[list] = carry;
    }
  }
}

// Task g of a bucketed list: its bucket is the last t with off[t] <= g.
SG_DEV Task bucket_task(const Task* tasks, const int32_t* off, int32_t Tmax, int32_t nd, int32_t g) {
  int lo = 0, hi = Tmax - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= g) lo = mid;
    else hi = mid - 1;
  }
  return tasks[(int64_t)lo * nd + (g - off[lo])];
}

// Dense rows over at most 32*WORDS columns (blocks of a SUMMA grid, narrow
// products of a batch) with at most CAP entries: whole rows, one workgroup
// each, by the bitmap-and-rank fold of the narrow hash rows.  The tasks are
// the slab list of the dense task builder, run with one slab covering the
// whole row and CAP as its cap; fuller rows stay on the tile and range
// tasks.
template <class Sr, class Rows, int WORDS, int CAP, int BS>
__global__ __launch_bounds__(BS) void k_num_bitmap_dense(Rows rows, Bins bins, OutC C, const Task* tasks,
                                                         const int32_t* book, int32_t* ctr, int32_t* err) {
  using Src = typename Rows::Src;
  __shared__ BitmapRowSmem<Sr, Src, WORDS, CAP, BS> sm;
  __shared__ int64_t s_slot;
  for (int x = threadIdx.x; x < WORDS; x += BS) sm.bits[x] = 0u;
  block_sync();
  const int32_t* L = bins.list + bins.start[kBinDense0];
  const int32_t Tmax = rows.Tmax;
  const int32_t nd = dense_rows(bins);
  __shared__ Task s_rec[kGrab];
  auto fetch = [&](int64_t g) { return bucket_task(tasks, book_off(book, Tmax, kListSlab), Tmax, nd, (int32_t)g); };
  for_each_queued_rec(ctr, kListSlab, (int64_t)ctr[kListSlab], &s_slot, s_rec, fetch, [&](const Task& task) {
    const Task tk = task;
    const int64_t i = L[tk.h];
    const int64_t o = C.rowptr[i];
    const int32_t m = (int32_t)(C.rowptr[i + 1] - o);
    if (threadIdx.x == 0 && m > CAP) atomicOr(err, 1);
    Src s{};
    int64_t li;
    rows.get(i, s, li);
    bitmap_row_fold<Sr, Src, WORDS, CAP, BS, false>(sm, s, li, 0, s.T, o, m, C, err);
  });
}

// Range tasks (runs of sparse tiles, at most kRangeSpanMax tiles and CAP
// entries) by the same bitmap-and-rank fold over the range's columns,
// instead of a hash table and a sort.
template <class Sr, class Rows, int WORDS, int CAP, int BS>
__global__ __launch_bounds__(BS) void k_num_ranges_bitmap(Rows rows, Bins bins, OutC C, const int32_t* off2,
                                                          const Task* tasks, const int32_t* book, int32_t* ctr,
                                                          int32_t* err) {
  using Src = typename Rows::Src;
  static_assert(32 * WORDS >= kRangeSpanMax * kTile, "a range fits the bitmap");
  __shared__ BitmapRowSmem<Sr, Src, WORDS, CAP, BS> sm;
  __shared__ int64_t s_slot;
  for (int x = threadIdx.x; x < WORDS; x += BS) sm.bits[x] = 0u;
  block_sync();
  const int32_t* L = bins.list + bins.start[kBinDense0];
  const int32_t Tmax = rows.Tmax;
  const int32_t nd = dense_rows(bins);
  __shared__ Task s_rec[kGrab];
  auto fetch = [&](int64_t g) { return bucket_task(tasks, book_off(book, Tmax, kListRange), Tmax, nd, (int32_t)g); };
  for_each_queued_rec(ctr, kListRange, (int64_t)ctr[kListRange], &s_slot, s_rec, fetch, [&](const Task& task) {
    const Task tk = task;
    const int32_t* o2 = off2 + (int64_t)tk.h * (Tmax + 1);
    const int32_t lo = o2[tk.t0], hi = o2[tk.t1];
    const int64_t i = L[tk.h];
    if (threadIdx.x == 0 && (hi - lo > CAP || tk.t1 - tk.t0 > kRangeSpanMax)) atomicOr(err, 1);
    Src s{};
    int64_t li;
    rows.get(i, s, li);
    bitmap_row_fold<Sr, Src, WORDS, CAP, BS, (row_unroll(CAP, BS) <= 8)>(sm, s, li, tk.t0, tk.t1, C.rowptr[i] + lo,
                                                                         hi - lo, C, err);
  });
}

// Range runs of products: one task per (dense row, group of up to
// kRunTiles tiles) holding range tiles.  The row's sources (one per thread
// when they fit a chunk) load their B row, A value and B row start once;
// the task then forms the group's ranges by the task builder's rules and
// folds each on the column bitmap, where a source only reads its two tile
// offsets.  A per-range task reloaded every source.
constexpr int kRunTiles = 8;

template <class V>
struct RunSrc : SpgemmSrc<V, true> {
  using Base = SpgemmSrc<V, true>;
  bool cached = false;  // the calling thread holds its source below
  int32_t kk = 0;
  V av{};
  int64_t b0 = 0;
  SG_DEV void load(int64_t j, typename Base::Item& it, int64_t& start, int64_t& len) const {
    if (!cached) {
      Base::load(j, it, start, len);
      return;
    }
    it.a = av;
    const int32_t* r = this->rp2 + (int64_t)kk * (this->T + 1);
    const int32_t s0 = r[this->t0];
    start = b0 + s0;
    len = r[this->t1] - s0;
  }
};

template <class Sr, class Rows, int WORDS, int CAP, int BS>
__global__ __launch_bounds__(BS) void k_num_range_runs(Rows rows, Bins bins, OutC C, const int32_t* off2,
                                                       const Task* tasks, const int32_t* book, int32_t* ctr,
                                                       int32_t tile_min, int32_t* err) {
  using V = typename Sr::V;
  using Src = RunSrc<V>;
  static_assert(32 * WORDS >= kRangeSpanMax * kTile, "a range fits the bitmap");
  __shared__ BitmapRowSmem<Sr, Src, WORDS, CAP, BS> sm;
  __shared__ int64_t s_slot;
  for (int x = threadIdx.x; x < WORDS; x += BS) sm.bits[x] = 0u;
  block_sync();
  const int32_t* L = bins.list + bins.start[kBinDense0];
  const int32_t Tmax = rows.Tmax;
  const int32_t nd = dense_rows(bins);
  __shared__ Task s_rec[kGrab];
  auto fetch = [&](int64_t g) { return bucket_task(tasks, book_off(book, Tmax, kListRange), Tmax, nd, (int32_t)g); };
  for_each_queued_rec(ctr, kListRange, (int64_t)ctr[kListRange], &s_slot, s_rec, fetch, [&](const Task& task) {
    const Task tk = task;
    const int32_t* o2 = off2 + (int64_t)tk.h * (Tmax + 1);
    const int64_t i = L[tk.h];
    const int64_t obase = C.rowptr[i];
    Src s{};
    int64_t li;
    rows.get(i, s, li);
    const int64_t nsrc = s.bind(li, 0, s.T);
    if (nsrc <= BS) {
      s.cached = true;
      if ((int64_t)threadIdx.x < nsrc) {
        const int64_t e = s.a0 + threadIdx.x;
        s.kk = s.a_col[e];
        s.av = s.a_val[e];
        s.b0 = s.b_rowptr[s.kk];
      }
    }
    auto fold = [&](int32_t r0, int32_t r1) {
      const int32_t lo = o2[r0], hi = o2[r1];
      if (threadIdx.x == 0 && (hi - lo > CAP || r1 - r0 > kRangeSpanMax)) atomicOr(err, 1);
      bitmap_row_fold<Sr, Src, WORDS, CAP, BS, (row_unroll(CAP, BS) <= 8)>(sm, s, li, r0, r1, obase + lo, hi - lo,
                                                                           C, err);
    };
    int32_t r0 = -1, rlast = -1, racc = 0;
    for (int t = tk.t0; t < tk.t1; ++t) {
      const int32_t c = o2[t + 1] - o2[t];
      if (c == 0) continue;
      if (c >= tile_min) {  // a dense-tile task
        if (r0 >= 0) fold(r0, rlast + 1);
        r0 = -1;
        racc = 0;
        continue;
      }
      if (r0 >= 0 && (racc + c > CAP || t + 1 - r0 > kRangeSpanMax)) {
        fold(r0, rlast + 1);
        r0 = -1;
        racc = 0;
      }
      if (r0 < 0) r0 = t;
      rlast = t;
      racc += c;
    }
    if (r0 >= 0) fold(r0, rlast + 1);
  });
}

// Dense-tile tasks: persistent workgroups take tasks from a global counter; a
// tile's products are folded into a dense LDS accumulator of 16384 slots
// plus an occupancy bitmap; the bitmap is then compacted in column order
// straight into C, and the touched slots are reset to the identity.
template <class Sr, class Rows, int BS>
__global__ __launch_bounds__(BS) void k_num_tiles(Rows rows, Bins bins, OutC C, const int32_t* off2, const Task* tasks,
                                                  const int32_t* book, int32_t* ctr, int32_t* err) {
  using Src = typename Rows::Src;
  constexpr int NW = BS / kWave;
  static_assert(BS >= kTileWords, "one compaction word per thread");
  using Item = typename Src::Item;
  using Acc = typename Sr::Acc;
  using V = typename Sr::V;
  __shared__ Acc s_acc[kTile];
  __shared__ __align__(8) uint32_t s_bm[kTileWords];
  __shared__ Item s_item[BS];
  __shared__ int64_t s_start[BS], s_off[BS], s_wave[NW];
  __shared__ int32_t s_wcnt[NW];
  __shared__ int64_t s_slot;
  __shared__ int64_t s_se[Src::kParts ? 2 * kLdsParts : 1];
  for (int x = threadIdx.x; x < kTile; x += BS) s_acc[x] = Sr::ident();
  for (int x = threadIdx.x; x < kTileWords; x += BS) s_bm[x] = 0u;
  const int32_t* L = bins.list + bins.start[kBinDense0];
  const int32_t Tmax = rows.Tmax;
  const int32_t nd = dense_rows(bins);
  __shared__ Task s_rec[kGrab];
  auto fetch = [&](int64_t g) { return bucket_task(tasks, book_off(book, Tmax, kListTile), Tmax, nd, (int32_t)g); };
  for_each_queued_rec(ctr, kListTile, (int64_t)ctr[kListTile], &s_slot, s_rec, fetch, [&](const Task& task) {
    const Task tk = task;
    const int32_t* o2 = off2 + (int64_t)tk.h * (Tmax + 1);
    const int32_t lo = o2[tk.t0], hi = o2[tk.t1];
    const int64_t i = L[tk.h];
    const int64_t base = C.rowptr[i] + lo;
    const int64_t c0 = (int64_t)tk.t0 << kTileLog;
    Src s{};
    int64_t li;
    rows.get(i, s, li);
    const int64_t nsrc = s.bind(li, tk.t0, tk.t1);
    if constexpr (Src::kParts) {
      if (s.nparts <= kLdsParts && !(tk.t0 == 0 && tk.t1 == s.T)) s.template merge_bounds<BS>(s_se);
    }
    auto fetch = [&](const Item& it, int64_t idx) {
      return ColVal<Acc>{(int32_t)(s.col(it, idx) - c0), s.template value<Sr>(it, idx)};
    };
    auto apply = [&](const ColVal<Acc>& p) {
      Sr::lds_acc(&s_acc[p.c], p.v);
      atomicOr(&s_bm[p.c >> 5], 1u << (p.c & 31));
    };
    for_each_product<BS, kUnroll>(s, nsrc, s_item, s_start, s_off, s_wave, fetch, apply);
    // compaction: wavefront wv sweeps slots [wv*kSpanW, (wv+1)*kSpanW), 64
    // per step; a step's occupancy is two bitmap words (one broadcast read),
    // so its stores go to consecutive outputs; the wavefront's output base
    // is the popcount of the bitmap words before its span
    constexpr int kSpanW = kTile / NW, kSpanWords = kSpanW / 32;
    static_assert(kSpanWords <= kWave && kSpanW % (64 * 8) == 0, "a lane counts one word; whole groups of steps");
    const int wv = wave_id();
    const int sb = wv * kSpanW;
    const uint32_t wbits = lane_id() < kSpanWords ? s_bm[wv * kSpanWords + lane_id()] : 0u;
    const int32_t cnt = wave_sum((int32_t)__popc(wbits));
    if (lane_id() == 0) s_wcnt[wv] = cnt;
    block_sync();
    int32_t wbase = 0, tot = 0;
#pragma unroll
    for (int u = 0; u < NW; ++u) {
      const int32_t v = s_wcnt[u];
      wbase += u < wv ? v : 0;
      tot += v;
    }
    if (threadIdx.x == 0 && tot != hi - lo) atomicOr(err, 1);
    const uint32_t lim = (uint32_t)(hi - lo - wbase);
    char* colb = reinterpret_cast<char*>(C.col + uniform64(base + wbase));
    char* valb = reinterpret_cast<char*>((V*)C.val + uniform64(base + wbase));
    const unsigned long long* bm64 = reinterpret_cast<const unsigned long long*>(s_bm);
    uint32_t run = 0;
    for (int j0 = 0; j0 < kSpanW; j0 += 64 * 8) {
      Acc v[8];
      unsigned long long mk[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        v[k] = s_acc[sb + j0 + 64 * k + lane_id()];
        mk[k] = bm64[(sb + j0 + 64 * k) >> 6];
      }
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const int x = sb + j0 + 64 * k + lane_id();
        const bool occ = (mk[k] >> lane_id()) & 1ull;
        const uint32_t r =
            run + __builtin_amdgcn_mbcnt_hi((uint32_t)(mk[k] >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mk[k], 0u));
        if (occ) {
          if (r < lim) {
            *reinterpret_cast<int32_t*>(colb + r * (uint32_t)sizeof(int32_t)) = (int32_t)(c0 + x);
            *reinterpret_cast<V*>(valb + r * (uint32_t)sizeof(V)) = Sr::out(v[k]);
          }
          s_acc[x] = Sr::ident();
        }
        run += (uint32_t)__popcll(mk[k]);
      }
    }
    if (lane_id() < kSpanWords) s_bm[wv * kSpanWords + lane_id()] = 0u;
    block_sync();
  });
}

// Range tasks: persistent workgroups, one hash task per range of tiles.
template <class Sr, class Rows, int LGS, int BS>
__global__ __launch_bounds__(BS) void k_num_ranges(Rows rows, Bins bins, OutC C, const int32_t* off2,
                                                   const Task* tasks, const int32_t* book, int32_t* ctr,
                                                   int32_t* err) {
  using Src = typename Rows::Src;
  __shared__ HashSmem<Sr, Src, LGS, BS> sm;
  __shared__ int64_t s_slot;
  const int32_t* L = bins.list + bins.start[kBinDense0];
  const int32_t Tmax = rows.Tmax;
  const int32_t nd = dense_rows(bins);
  __shared__ Task s_rec[kGrab];
  auto fetch = [&](int64_t g) { return bucket_task(tasks, book_off(book, Tmax, kListRange), Tmax, nd, (int32_t)g); };
  for_each_queued_rec(ctr, kListRange, (int64_t)ctr[kListRange], &s_slot, s_rec, fetch, [&](const Task& task) {
    const Task tk = task;
    const int32_t* o2 = off2 + (int64_t)tk.h * (Tmax + 1);
    const int32_t lo = o2[tk.t0], hi = o2[tk.t1];
    const int64_t i = L[tk.h];
    Src s{};
    int64_t li;
    rows.get(i, s, li);
    hash_task<Sr, Src, LGS, BS>(sm, s, li, tk.t0, tk.t1, C.rowptr[i] + lo, hi - lo, C, err);
  });
}

}  // namespace sg
