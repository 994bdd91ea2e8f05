// Column-slab path for the dense rows of a single product C = A (x).(+) B.
//
// B's columns are cut into slabs of 2^ls columns (one to eight 16384-column
// tiles).  A partition of B keeps, for slab s and B row k, the entries of
// B_k inside the slab contiguous:  pcol/pval[prow[s*nb + k] .. prow[s*nb + k + 1]),
// and rpt[(s*nb + k)*(G+1) + t] holds where tile t of the slab starts inside
// that segment.  A dense row's work is one task per (row, slab); every task
// finds each source's segment with one read of prow, and the tasks run in
// slab-major order, so at any moment the whole chip gathers from one slab
// of B.
//
//   symbolic  per task an LDS bitmap of the slab (16 KB at 2^17 columns);
//             per-tile popcounts become the row's per-tile output counts
//   numeric   bitmap + rank accumulator over a window of the slab: pass 1
//             sets the window's bitmap, a scan turns it into per-word ranks,
//             pass 2 folds every product into the compacted slot
//             rank(column) of an LDS value array, and the bitmap walk writes
//             the window's entries in column order (no sort, no probing).
//             A slab whose entries fit the value array is one window; a
//             larger one is cut into runs of whole tiles that fit, and a
//             single tile holding more than the array is done in rank chunks
//             (pass 2 repeated, each pass keeping one range of ranks).  The
//             task's sources are read once and kept in LDS for all passes.
#pragma once

#include "sg_kernels.hpp"

namespace sg {

constexpr int kSlabLogMin = kTileLog;  // a slab is 1..8 column tiles
constexpr int kSlabLogMax = 17;
constexpr int kSlabWordsMax = 1 << (kSlabLogMax - 5);
constexpr int kSlabTilesMax = 1 << (kSlabLogMax - kTileLog);

// Per dense row (position h in the dense list): its A row.
struct DenseRow {
  int64_t a0;    // first entry of the row in A
  int32_t nsrc;  // stored entries of the row
  int32_t i;     // row id
};

template <int BS>
__global__ __launch_bounds__(BS) void k_dense_rows(Bins bins, const int64_t* a_rowptr, DenseRow* dr) {
  const int32_t* L = bins.list + bins.start[kBinDense0];
  const int64_t nd = dense_rows(bins);
  for (int64_t h = (int64_t)blockIdx.x * BS + threadIdx.x; h < nd; h += (int64_t)gridDim.x * BS) {
    const int32_t i = L[h];
    const int64_t a0 = a_rowptr[i];
    dr[h] = DenseRow{a0, (int32_t)(a_rowptr[i + 1] - a0), i};
  }
}

// Per B row (one wavefront each): the slab bounds bnd[k*(S+1) + s] (row-local
// offset where slab s starts; s = S: the row length) and, per slab, the tile
// offsets rpt[(s*nb + k)*(G+1) + t] relative to the slab's start (t = G: the
// slab's length; tiles past the last column tile repeat it).
template <int BS>
__global__ __launch_bounds__(BS) void k_slab_bounds(const int64_t* rowptr, const int32_t* col, int64_t nb, int32_t T,
                                                    int32_t G, int32_t S, int32_t* bnd, int32_t* rpt) {
  const int64_t w0 = ((int64_t)blockIdx.x * BS + threadIdx.x) >> 6;
  const int64_t nw = ((int64_t)gridDim.x * BS) >> 6;
  const int per = G + 1;
  const int nx = S * per + S + 1;
  for (int64_t k = w0; k < nb; k += nw) {
    const int64_t b = rowptr[k], e = rowptr[k + 1];
    auto pos = [&](int t) -> int32_t {
      if (t <= 0) return 0;
      if (t >= T) return (int32_t)(e - b);
      return (int32_t)(lower_bound_col(col, b, e, (int64_t)t << kTileLog) - b);
    };
    for (int x = lane_id(); x < nx; x += kWave) {
      if (x < S * per) {
        const int s = x / per, t = x - s * per;
        const int tg = s * G + t < T ? s * G + t : T;
        rpt[((int64_t)s * nb + k) * per + t] = pos(tg) - pos(s * G);
      } else {
        const int s = x - S * per;
        bnd[k * (S + 1) + s] = pos(s * G < T ? s * G : T);
      }
    }
  }
}

// ---- B partition by column slab ------------------------------------------------
// Per-slab segment lengths of every B row from the slab bounds bnd (S+1
// row-local offsets per row), written one past their slot so that an
// inclusive scan of prow[1 ..] gives the segment starts.
template <int BS>
__global__ __launch_bounds__(BS) void k_slab_counts(const int32_t* bnd, int64_t nb, int32_t S, int64_t* prow) {
  const int64_t n = (int64_t)S * nb;
  for (int64_t x = (int64_t)blockIdx.x * BS + threadIdx.x; x < n; x += (int64_t)gridDim.x * BS) {
    const int64_t s = x / nb, k = x - s * nb;
    const int32_t* r = bnd + k * (S + 1);
    prow[1 + x] = (int64_t)(r[s + 1] - r[s]);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) prow[0] = 0;
}

// One wavefront per B row scatters its entries into their slab segments.
// Entries that do not fall where the bounds say (unsorted or out-of-range
// columns) are dropped and flagged instead of written out of place.
template <class V, bool kCols, bool kVals>
__global__ __launch_bounds__(256) void k_slab_scatter(const int64_t* rowptr, const int32_t* col, const V* val,
                                                      int64_t nb, int32_t ls, int32_t S, const int32_t* bnd,
                                                      const int64_t* prow, int32_t* pcol, V* pval, int32_t* err) {
  const int64_t w0 = ((int64_t)blockIdx.x * 256 + threadIdx.x) >> 6;
  const int64_t nw = ((int64_t)gridDim.x * 256) >> 6;
  for (int64_t k = w0; k < nb; k += nw) {
    const int64_t s0 = rowptr[k], e = rowptr[k + 1];
    const int32_t* r = bnd + k * (S + 1);
    for (int64_t j = s0 + lane_id(); j < e; j += kWave) {
      const int32_t c = col[j];
      const int32_t s = c >> ls;
      bool ok = c >= 0 && s < S;
      int64_t dst = 0;
      if (ok) {
        const int64_t o = (j - s0) - r[s];
        ok = o >= 0 && o < (int64_t)(r[s + 1] - r[s]);
        dst = prow[(int64_t)s * nb + k] + o;
      }
      if (!ok) {
        atomicOr(err, 1);
        continue;
      }
      if constexpr (kCols) pcol[dst] = c;
      if constexpr (kVals) pval[dst] = val[j];
    }
  }
}

// One wavefront per dense row: raw per-tile counts -> exclusive offsets,
// entry T = the row's count, which also goes to cnt_out.
template <int BS>
__global__ __launch_bounds__(BS) void k_off2_finish(Bins bins, const DenseRow* dr, int32_t* off2, int32_t T,
                                                    int64_t* cnt_out) {
  const int64_t nd = dense_rows(bins);
  const int64_t w0 = ((int64_t)blockIdx.x * BS + threadIdx.x) >> 6;
  const int64_t nw = ((int64_t)gridDim.x * BS) >> 6;
  for (int64_t h = w0; h < nd; h += nw) {
    int32_t* o2 = off2 + h * (T + 1);
    int32_t run = 0;
    for (int t0 = 0; t0 < T; t0 += kWave) {
      const int t = t0 + lane_id();
      const int32_t v = t < T ? o2[t] : 0;
      const int32_t inc = wave_incl_scan(v);
      if (t < T) o2[t] = run + inc - v;
      run += shfl(inc, kWave - 1);
    }
    if (lane_id() == 0) {
      o2[T] = run;
      cnt_out[dr[h].i] = run;
    }
  }
}

// ---- tasks ------------------------------------------------------------------------
// A task is one (dense row, slab) with everything its kernel needs up front
// (no dependent lookups before the sources).
struct SlabTask {
  int32_t h, s;   // position in the dense list, slab
  int64_t out;    // C position of the slab's first entry (numeric)
  int64_t a0;     // first A entry of the row
  int32_t nsrc;   // A entries of the row
  int32_t m;      // C entries in the slab (numeric)
};

// Entries of a light task's LDS value array (32 KB of accumulators).
template <class Sr>
constexpr int slab_cap() {
  return 32768 / (int)sizeof(typename Sr::Acc);
}

// Column tiles per window of a heavy task's dense accumulator (128 KB or
// less of accumulators).
template <class Sr>
constexpr int heavy_tiles() {
  return sizeof(typename Sr::Acc) >= 8 ? 1 : (sizeof(typename Sr::Acc) >= 4 ? 2 : 4);
}

// One thread per dense row.  A slab with at most `cap` entries becomes a
// light task (list kListSlab), a fuller one a heavy task (list kListTile);
// both lists hold per-slab buckets of nd slots (book[l*T + s] counts bucket
// s of list l).  Entries per list are summed for the statistics.
template <int BS>
__global__ __launch_bounds__(BS) void k_slab_tasks(Bins bins, const DenseRow* dr, const int32_t* off2, int32_t T,
                                                   int32_t G, int32_t cap, const int64_t* c_rowptr,
                                                   SlabTask* light, SlabTask* heavy, int32_t* book, int32_t* ctr) {
  __shared__ unsigned long long s_ent[2];
  if (threadIdx.x < 2) s_ent[threadIdx.x] = 0ull;
  __syncthreads();
  const int64_t nd = dense_rows(bins);
  int32_t* cnt_l = book + kListSlab * T;
  int32_t* cnt_h = book + kListTile * T;
  unsigned long long el = 0ull, eh = 0ull;
  for (int64_t h = (int64_t)blockIdx.x * BS + threadIdx.x; h < nd; h += (int64_t)gridDim.x * BS) {
    const DenseRow d = dr[h];
    const int32_t* o2 = off2 + h * (T + 1);
    const int64_t base = c_rowptr[d.i];
    int32_t s = 0;
    for (int32_t ta = 0; ta < T; ta += G, ++s) {
      const int32_t tb = ta + G < T ? ta + G : T;
      const int32_t lo = o2[ta], m = o2[tb] - lo;
      if (m <= 0) continue;
      const SlabTask tk{(int32_t)h, s, base + lo, d.a0, d.nsrc, m};
      if (m <= cap) {
        light[(int64_t)s * nd + atomicAdd(&cnt_l[s], 1)] = tk;
        el += (unsigned long long)m;
      } else {
        heavy[(int64_t)s * nd + atomicAdd(&cnt_h[s], 1)] = tk;
        eh += (unsigned long long)m;
      }
    }
  }
  el = wave_sum(el);
  eh = wave_sum(eh);
  if (lane_id() == 0 && el) atomicAdd(&s_ent[0], el);
  if (lane_id() == 0 && eh) atomicAdd(&s_ent[1], eh);
  __syncthreads();
  unsigned long long* ent = (unsigned long long*)(ctr + kCtrEntries);
  if (threadIdx.x == 0 && s_ent[0]) atomicAdd(ent + kListSlab, s_ent[0]);
  if (threadIdx.x == 1 && s_ent[1]) atomicAdd(ent + kListTile, s_ent[1]);
}

template <class V>
struct SlabB {
  const int64_t* prow;
  const int32_t* pcol;
  const V* pval;
  const int32_t* rpt;
  int64_t nb;
  int32_t G, T;
};

constexpr int kBoffCache = 256;  // slab-bucket offsets kept in LDS

// LDS of a slab task: its sources (A entry's value and column, the slab
// segment's start and length) and the current window's per-source offsets.
template <class V, int BS>
struct SlabLds {
  V a[BS];
  int32_t k[BS], slen[BS], wo[BS];
  int64_t sst[BS], off[BS], wave[BS / kWave];
  int32_t tc[kSlabTilesMax + 1];
  int32_t boff[kBoffCache + 1];
  int64_t slot;
};

// Task g of a slab-bucketed list: its bucket is the last s with boff[s] <= g.
template <class V, int BS>
SG_DEV SlabTask slab_task(const SlabTask* tasks, const int32_t* boff, const SlabLds<V, BS>& L, bool bcache,
                          int32_t S, int32_t nd, int64_t g) {
  int lo = 0, hi = S - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if ((bcache ? L.boff[mid] : boff[mid]) <= g) lo = mid;
    else hi = mid - 1;
  }
  return tasks[(int64_t)lo * nd + (g - (bcache ? L.boff[lo] : boff[lo]))];
}

// The next task of a workgroup, fetched in three dependent stages (record,
// A entries, slab segments) that ride along with the current task's own
// memory waits; commit() moves the sources into LDS when the task starts.
// Only tasks whose sources fit one workgroup chunk are prefetched.
template <class V, bool kVals, int BS>
struct SlabNext {
  SlabTask tk;
  int32_t k;
  V a;
  int64_t sst;
  int32_t slen;
  bool has;
  SG_DEV bool mine() const { return has && tk.nsrc <= BS && (int)threadIdx.x < tk.nsrc; }
  SG_DEV void sources(const int32_t* a_col, const V* a_val) {
    if (!mine()) return;
    const int64_t e = tk.a0 + threadIdx.x;
    k = a_col[e];
    if constexpr (kVals) a = a_val[e];
  }
  SG_DEV void segments(const SlabB<V>& b) {
    if (!mine()) return;
    const int64_t* pr = b.prow + (int64_t)tk.s * b.nb + k;
    sst = pr[0];
    slen = (int32_t)(pr[1] - sst);
  }
  SG_DEV void commit(SlabLds<V, BS>& L) const {
    if (!mine()) return;
    L.k[threadIdx.x] = k;
    if constexpr (kVals) L.a[threadIdx.x] = a;
    L.sst[threadIdx.x] = sst;
    L.slen[threadIdx.x] = slen;
  }
};

// Sources [c0, c0 + nc) of task tk into LDS (one per thread).
template <class V, bool kVals, int BS>
SG_DEV void slab_load_sources(const SlabB<V>& b, const int32_t* a_col, const V* a_val, const SlabTask& tk,
                              int64_t c0, int nc, SlabLds<V, BS>& L) {
  if ((int)threadIdx.x < nc) {
    const int64_t e = tk.a0 + c0 + threadIdx.x;
    const int32_t k = a_col[e];
    L.k[threadIdx.x] = k;
    if constexpr (kVals) L.a[threadIdx.x] = a_val[e];
    const int64_t* pr = b.prow + (int64_t)tk.s * b.nb + k;
    const int64_t st = pr[0];
    L.sst[threadIdx.x] = st;
    L.slen[threadIdx.x] = (int32_t)(pr[1] - st);
  }
}

// Every product of window [t0, t1) (tiles, inside the task's slab whose first
// tile is ts0) of task tk: fetch(owner, index into pcol/pval) returns a
// product and apply(product, valid) folds it into LDS; apply is called by
// every lane, with valid false where a lane has no product.  With `one` the
// task's sources are already in LDS; otherwise they are loaded chunk by
// chunk.  Sources' window segments come from rpt unless the window is the
// whole slab.  Lanes take consecutive products (coalesced gathers), kUnroll
// loads in flight each.
template <int BS, class V, bool kVals, class Fetch, class Apply>
SG_DEV void slab_window(const SlabB<V>& b, const int32_t* a_col, const V* a_val, const SlabTask& tk, int ts0,
                        int t0, int t1, bool whole, bool one, SlabLds<V, BS>& L, Fetch& fetch, Apply& apply) {
  constexpr int NW = BS / kWave;
  constexpr int64_t kBlock = (int64_t)kWave * kUnroll;
  using P = decltype(fetch(0, (int64_t)0));
  const int wv = wave_id();
  for (int64_t c0 = 0; c0 < tk.nsrc; c0 += BS) {
    const int nc = (int)((tk.nsrc - c0) < BS ? (tk.nsrc - c0) : BS);
    if (!one) {
      __syncthreads();
      slab_load_sources<V, kVals, BS>(b, a_col, a_val, tk, c0, nc, L);
      __syncthreads();
    }
    int64_t len = 0;
    int32_t wo = 0;
    if ((int)threadIdx.x < nc) {
      if (whole) {
        len = L.slen[threadIdx.x];
      } else {
        const int32_t* r = b.rpt + ((int64_t)tk.s * b.nb + L.k[threadIdx.x]) * (b.G + 1);
        wo = r[t0 - ts0];
        len = r[t1 - ts0] - wo;
      }
    }
    int64_t total;
    const int64_t off = block_excl_scan<NW, int64_t>(len, L.wave, &total);
    L.off[threadIdx.x] = off;
    L.wo[threadIdx.x] = wo;
    __syncthreads();
    for (int64_t qb = (int64_t)wv * kBlock; qb < total; qb += (int64_t)NW * kBlock) {
      const int64_t qe = (qb + kBlock - 1) < (total - 1) ? (qb + kBlock - 1) : (total - 1);
      int a = 0, bb = nc - 1;
      while (a < bb) {
        const int mid = (a + bb + 1) >> 1;
        if (L.off[mid] <= qb) a = mid;
        else bb = mid - 1;
      }
      int e = a, f = nc - 1;
      while (e < f) {
        const int mid = (e + f + 1) >> 1;
        if (L.off[mid] <= qe) e = mid;
        else f = mid - 1;
      }
      P pp[kUnroll];
      bool ok[kUnroll];
      int ow = a;
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        const int64_t q = qb + u * kWave + lane_id();
        ok[u] = q < total;
        if (ok[u]) {
          int h2 = e;
          while (ow < h2) {
            const int mid = (ow + h2 + 1) >> 1;
            if (L.off[mid] <= q) ow = mid;
            else h2 = mid - 1;
          }
          pp[u] = fetch(ow, L.sst[ow] + L.wo[ow] + (q - L.off[ow]));
        }
      }
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) apply(pp[u], ok[u]);
    }
    __syncthreads();
  }
}

// ---- symbolic --------------------------------------------------------------------
// Task g = (slab s = g / nd, dense row h = g % nd), tasks in slab-major order,
// workgroup b takes tasks b, b + grid, ... (the next one prefetched).  The
// per-tile popcounts of the slab's bitmap are written raw to
// off2[h*(T+1) + t]; k_off2_finish turns them into per-row offsets.
template <int BS>
__global__ __launch_bounds__(BS) void k_sym_slab(SlabB<uint8_t> b, const DenseRow* dr, const int32_t* a_col,
                                                 Bins bins, int32_t S, int32_t* off2) {
  constexpr int NW = BS / kWave;
  __shared__ uint32_t s_bm[kSlabWordsMax];
  __shared__ SlabLds<uint8_t, BS> L;
  const int T = b.T, G = b.G;
  const int nwords = G * kTileWords;
  for (int x = threadIdx.x; x < nwords; x += BS) s_bm[x] = 0u;
  const int64_t nd = dense_rows(bins);
  const int64_t ntask = nd * S;
  const uint32_t cmax = (uint32_t)nwords * 32u;
  auto record = [&](int64_t g, SlabNext<uint8_t, false, BS>& nx) {
    nx.has = g < ntask;
    if (!nx.has) return;
    const int32_t s = (int32_t)(g / nd);
    const int64_t h = g - (int64_t)s * nd;
    const DenseRow d = dr[h];
    nx.tk = SlabTask{(int32_t)h, s, 0, d.a0, d.nsrc, 0};
  };
  SlabNext<uint8_t, false, BS> nx;
  record(blockIdx.x, nx);
  nx.sources(a_col, nullptr);
  nx.segments(b);
  for (int64_t g = blockIdx.x; g < ntask; g += gridDim.x) {
    const SlabTask tk = nx.tk;
    nx.commit(L);
    __syncthreads();
    const bool one = tk.nsrc <= BS;
    record(g + gridDim.x, nx);
    const int ts0 = tk.s * G;
    const int64_t c0 = (int64_t)ts0 << kTileLog;
    auto fetch = [&](int, int64_t idx) { return (int32_t)(b.pcol[idx] - c0); };
    auto apply = [&](int32_t c, bool ok) { wave_or_bits(s_bm, c, ok && (uint32_t)c < cmax); };
    slab_window<BS, uint8_t, false>(b, a_col, nullptr, tk, ts0, ts0, ts0 + G, true, one, L, fetch, apply);
    nx.sources(a_col, nullptr);
    int32_t* o2 = off2 + (int64_t)tk.h * (T + 1);
    for (int tl = wave_id(); tl < G; tl += NW) {
      int32_t c = 0;
      for (int x = lane_id(); x < kTileWords; x += kWave) {
        const int wx = tl * kTileWords + x;
        c += __popc(s_bm[wx]);
        s_bm[wx] = 0u;
      }
      c = wave_sum(c);
      const int t = ts0 + tl;
      if (lane_id() == 0 && t < T) o2[t] = c;
    }
    nx.segments(b);
    __syncthreads();
  }
}

// ---- numeric ---------------------------------------------------------------------
// Light tasks (at most CAP entries in the slab): one window, bitmap + rank.
// Workgroup b takes tasks b, b + grid, ... of the slab-major list, the next
// one prefetched.
template <class Sr, class V, int BS, int CAP>
__global__ __launch_bounds__(BS) void k_num_slab(SlabB<V> b, const int32_t* a_col, const V* a_val, OutC C,
                                                 const SlabTask* tasks, const int32_t* boff, int32_t S, int32_t nd,
                                                 const int32_t* ctr, int32_t* err) {
  constexpr int NW = BS / kWave;
  static_assert(NW * kWave <= kTileWords, "each wavefront owns a multiple of 64 words of a window");
  static_assert(CAP <= 65535, "ranks are 16-bit");
  using Acc = typename Sr::Acc;
  __shared__ uint32_t s_bits[kSlabWordsMax];
  __shared__ uint16_t s_rank[kSlabWordsMax];
  __shared__ Acc s_val[CAP];
  __shared__ SlabLds<V, BS> L;
  __shared__ int32_t s_wt[NW];
  const int T = b.T, G = b.G;
  for (int x = threadIdx.x; x < kSlabWordsMax; x += BS) s_bits[x] = 0u;
  const bool bcache = S < kBoffCache;
  if (bcache)
    for (int x = threadIdx.x; x <= S; x += BS) L.boff[x] = boff[x];
  __syncthreads();
  const int64_t ntask = ctr[kListSlab];
  const int wv = wave_id();
  auto record = [&](int64_t g, SlabNext<V, true, BS>& nx) {
    nx.has = g < ntask;
    if (nx.has) nx.tk = slab_task<V, BS>(tasks, boff, L, bcache, S, nd, g);
  };
  SlabNext<V, true, BS> nx;
  record(blockIdx.x, nx);
  nx.sources(a_col, a_val);
  nx.segments(b);
  for (int64_t g = blockIdx.x; g < ntask; g += gridDim.x) {
    const SlabTask tk = nx.tk;
    nx.commit(L);
    __syncthreads();
    record(g + gridDim.x, nx);
    const int ts0 = tk.s * G, ts1 = ts0 + G < T ? ts0 + G : T;
    const int32_t m = tk.m < CAP ? tk.m : CAP;
    if (threadIdx.x == 0 && tk.m > CAP) atomicOr(err, 1);
    const bool one = tk.nsrc <= BS;
    const int64_t cw0 = (int64_t)ts0 << kTileLog;
    const int nwords = (ts1 - ts0) * kTileWords;
    const int wpw = nwords / NW;
    const uint32_t cmax = (uint32_t)nwords * 32u;
    // pass 1: the slab's column set
    auto f1 = [&](int, int64_t idx) { return (int32_t)(b.pcol[idx] - cw0); };
    auto a1 = [&](int32_t c, bool ok) { wave_or_bits(s_bits, c, ok && (uint32_t)c < cmax); };
    slab_window<BS, V, true>(b, a_col, a_val, tk, ts0, ts0, ts1, true, one, L, f1, a1);
    nx.sources(a_col, a_val);
    // ranks: wavefront wv owns words [wv*wpw, (wv+1)*wpw), lanes consecutive
    int32_t run = 0;
    for (int it = 0; it < wpw; it += kWave) {
      const int w = wv * wpw + it + lane_id();
      const int32_t pc = __popc(s_bits[w]);
      const int32_t inc = wave_incl_scan(pc);
      s_rank[w] = (uint16_t)(run + inc - pc);
      run += shfl(inc, kWave - 1);
    }
    if (lane_id() == 0) s_wt[wv] = run;
    for (int x = threadIdx.x; x < m; x += BS) s_val[x] = Sr::ident();
    __syncthreads();
    int32_t wbase = 0, tot = 0;
#pragma unroll
    for (int u = 0; u < NW; ++u) {
      const int32_t v = s_wt[u];
      wbase += u < wv ? v : 0;
      tot += v;
    }
    if (threadIdx.x == 0 && tot != tk.m) atomicOr(err, 1);
    if (wbase)
      for (int it = 0; it < wpw; it += kWave) {
        const int w = wv * wpw + it + lane_id();
        s_rank[w] = (uint16_t)(s_rank[w] + wbase);
      }
    __syncthreads();
    // pass 2: fold every product into its compacted slot
    auto f2 = [&](int ow, int64_t idx) {
      return ColVal<Acc>{(int32_t)(b.pcol[idx] - cw0), Sr::mul(L.a[ow], b.pval[idx])};
    };
    auto a2 = [&](const ColVal<Acc>& p, bool ok) {
      if (!ok || (uint32_t)p.c >= cmax) return;
      const int w = p.c >> 5;
      const int32_t r = (int32_t)s_rank[w] + __popc(s_bits[w] & ((1u << (p.c & 31)) - 1u));
      if (r < m) Sr::lds_acc(&s_val[r], p.v);
    };
    slab_window<BS, V, true>(b, a_col, a_val, tk, ts0, ts0, ts1, true, one, L, f2, a2);
    nx.segments(b);
    // column-ordered write-out; clears the bitmap for the next task
    for (int it = 0; it < wpw; it += kWave) {
      const int w = wv * wpw + it + lane_id();
      uint32_t bits = s_bits[w];
      int32_t r = s_rank[w];
      while (bits) {
        const int bt = __ffs((int)bits) - 1;
        bits &= bits - 1u;
        if (r < m) {
          C.col[tk.out + r] = (int32_t)(cw0 + w * 32 + bt);
          ((V*)C.val)[tk.out + r] = Sr::out(s_val[r]);
        }
        ++r;
      }
      s_bits[w] = 0u;
    }
    __syncthreads();
  }
}

// Heavy tasks: the task's sources are read once; the slab is swept in
// windows of WD column tiles, each folded in a single pass into a dense LDS
// accumulator with an occupancy bitmap, then compacted in column order
// (touched slots are reset to the identity as they are written out).  Tasks
// vary widely in size, so workgroups take them from the interleaved queues.
template <class Sr, class V, int BS, int WD>
__global__ __launch_bounds__(BS) void k_num_slab_heavy(SlabB<V> b, const int32_t* a_col, const V* a_val,
                                                       const int32_t* off2, OutC C, const SlabTask* tasks,
                                                       const int32_t* boff, int32_t S, int32_t nd, int32_t* ctr,
                                                       int32_t* err) {
  constexpr int NW = BS / kWave;
  constexpr int kW = WD * kTile;
  constexpr int kWW = WD * kTileWords;
  using Acc = typename Sr::Acc;
  __shared__ Acc s_acc[kW];
  __shared__ uint32_t s_bm[kWW];
  __shared__ SlabLds<V, BS> L;
  __shared__ int32_t s_wave32[NW];
  const int T = b.T, G = b.G;
  for (int x = threadIdx.x; x < kW; x += BS) s_acc[x] = Sr::ident();
  for (int x = threadIdx.x; x < kWW; x += BS) s_bm[x] = 0u;
  const bool bcache = S < kBoffCache;
  if (bcache)
    for (int x = threadIdx.x; x <= S; x += BS) L.boff[x] = boff[x];
  __syncthreads();
  for_each_queued(ctr, kListTile, (int64_t)ctr[kListTile], &L.slot, [&](int64_t g) {
    const SlabTask tk = slab_task<V, BS>(tasks, boff, L, bcache, S, nd, g);
    const int ts0 = tk.s * G, ts1 = ts0 + G < T ? ts0 + G : T;
    if ((int)threadIdx.x <= ts1 - ts0) {
      const int32_t* o2 = off2 + (int64_t)tk.h * (T + 1);
      L.tc[threadIdx.x] = o2[ts0 + threadIdx.x] - o2[ts0];
    }
    const bool one = tk.nsrc <= BS;
    if (one) slab_load_sources<V, true, BS>(b, a_col, a_val, tk, 0, tk.nsrc, L);
    __syncthreads();
    for (int t0 = ts0; t0 < ts1; t0 += WD) {
      const int t1 = t0 + WD < ts1 ? t0 + WD : ts1;
      const int32_t rel0 = L.tc[t0 - ts0], mw = L.tc[t1 - ts0] - rel0;
      if (mw <= 0) continue;
      const int64_t cw0 = (int64_t)t0 << kTileLog;
      const int nwords = (t1 - t0) * kTileWords;
      auto f = [&](int ow, int64_t idx) {
        return ColVal<Acc>{(int32_t)(b.pcol[idx] - cw0), Sr::mul(L.a[ow], b.pval[idx])};
      };
      auto ap = [&](const ColVal<Acc>& p, bool ok) {
        const bool in = ok && (uint32_t)p.c < (uint32_t)kW;
        if (in) Sr::lds_acc(&s_acc[p.c], p.v);
        wave_or_bits(s_bm, p.c, in);
      };
      slab_window<BS, V, true>(b, a_col, a_val, tk, ts0, t0, t1, t0 == ts0 && t1 == ts1, one, L, f, ap);
      // compaction: round w0 takes words [w0, w0 + BS), consecutive threads
      // on consecutive words
      int32_t carry = 0;
      for (int w0 = 0; w0 < nwords; w0 += BS) {
        const int w = w0 + threadIdx.x;
        uint32_t bits = w < nwords ? s_bm[w] : 0u;
        int32_t tot;
        int32_t r = carry + block_excl_scan<NW, int32_t>(__popc(bits), s_wave32, &tot);
        while (bits) {
          const int bt = __ffs((int)bits) - 1;
          bits &= bits - 1u;
          const int c = w * 32 + bt;
          if (r < mw) {
            C.col[tk.out + rel0 + r] = (int32_t)(cw0 + c);
            ((V*)C.val)[tk.out + rel0 + r] = Sr::out(s_acc[c]);
          }
          s_acc[c] = Sr::ident();
          ++r;
        }
        if (w < nwords) s_bm[w] = 0u;
        carry += tot;
      }
      if (threadIdx.x == 0 && carry != mw) atomicOr(err, 1);
      __syncthreads();
    }
  });
}

}  // namespace sg
