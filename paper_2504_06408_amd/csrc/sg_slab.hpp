// Column-slab path for the dense rows of a single product C = A (x).(+) B.
//
// B's columns are cut into slabs of 2^ls columns (one to eight 16384-column
// tiles).  A partition of B keeps, for slab s and B row k, the entries of
// B_k inside the slab contiguous:  pbit/pcv[prow[s*nb + k] .. prow[s*nb + k + 1])
// (pbit: column ids for the symbolic pass; pcv: column and value pairs for
// the numeric pass),
// and rpt[(s*nb + k)*(G+1) + t] holds where tile t of the slab starts inside
// that segment.  A dense row's work is one task per (row, slab); every task
// finds each source's segment with one read of prow, and the tasks run in
// slab-major order, so at any moment the whole chip gathers from one slab
// of B.
//
//   symbolic  per task an LDS bitmap of the slab (16 KB at 2^17 columns);
//             per-tile popcounts become the row's per-tile output counts
//   numeric   a slab holding at most a light task's capacity of entries is
//             one light task: pass 1 sets the slab's bitmap, a scan turns it
//             into per-word ranks, pass 2 folds every product into the
//             compacted slot rank(column) of an LDS value array and stores
//             its column there too, and both arrays are copied out in column
//             order (no sort, no probing).  A fuller slab is one heavy task:
//             the row's sources are read once, then each tile is folded into
//             a dense LDS accumulator of kTile slots and compacted in column
//             order by a sweep whose wavefronts take their output offsets
//             from the symbolic pass's span counts; a sparse tile uses the
//             light scheme in LDS borrowed from the accumulator instead
//             (products in registers when they fit a round and the tile has
//             no span counts, else staged in that LDS when products plus
//             entries fit it).
#pragma once

#include "sg_kernels.hpp"

namespace sg {

constexpr int kSlabLogMin = kTileLog;  // a slab is 1..8 column tiles
constexpr int kSlabLogMax = 17;
constexpr int kSlabWordsMax = 1 << (kSlabLogMax - 5);
constexpr int kSlabTilesMax = 1 << (kSlabLogMax - kTileLog);

// Span counts: for every (dense row, tile) whose entry count reaches
// kSpanMin, the symbolic slab pass also records the entries in each of the
// tile's kSpans spans of kTile / kSpans columns (uint16 each, 16 bytes per
// tile), so that the heavy numeric kernel, whose wavefronts each compact one
// span, knows every wavefront's output offset without counting first.  They
// follow the per-row tile offsets (nd * (T + 1) int32) in the same buffer.
constexpr int kSpans = 8;
constexpr int32_t kSpanMin = 1024;
static_assert(kTile / kSpans == 4 * kTileWords, "a span is four bits of every word of the interleaved bitmap");
inline size_t span_offset(int64_t nd, int32_t T) { return ((size_t)nd * (size_t)(T + 1) * 4 + 15) & ~(size_t)15; }
inline size_t off2_span_bytes(int64_t nd, int32_t T) {
  return span_offset(nd, T) + (size_t)nd * (size_t)T * kSpans * sizeof(uint16_t);
}

// One entry of the numeric partition of B: column id and value side by side,
// so a product is one load (8 bytes, or 16 for 8-byte values).
template <class V>
struct alignas(sizeof(V) >= 8 ? 16 : 8) ColV {
  int32_t c;
  V v;
};

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
    const int64_t n = e - b;
    // a row of at most 63 entries (almost every row) is held one column tile
    // per lane; lane t finds pos(t), the entries below tile t, by a search
    // over the lanes' tiles (non-decreasing along the lanes: the row is sorted)
    int32_t mypos = 0;
    // (a full wavefront of entries would need a 65th answer; lanes hold tiles
    // below 64 only)
    const bool inlanes = n < kWave && T <= kWave;
    if (inlanes) {
      const int l = lane_id();
      const int32_t tl = l < n ? (col[b + l] >> kTileLog) : INT32_MAX;
      int lo = 0;  // first lane whose tile is >= t (n if none)
#pragma unroll
      for (int step = kWave / 2; step > 0; step >>= 1) {
        const int32_t v = __shfl(tl, lo + step - 1, kWave);
        if (v < l) lo += step;
      }
      mypos = lo < (int)n ? lo : (int32_t)n;
    }
    auto pos = [&](int t) -> int32_t {
      int32_t sh = 0;
      if (inlanes) sh = __shfl(mypos, t & (kWave - 1), kWave);  // the whole wavefront takes part
      if (t <= 0) return 0;
      if (t >= T) return (int32_t)n;
      if (inlanes) return t < kWave ? sh : (int32_t)n;
      return (int32_t)(lower_bound_col(col, b, e, (int64_t)t << kTileLog) - b);
    };
    // every lane runs every round (the lane shuffles of pos read all lanes)
    for (int x0 = 0; x0 < nx; x0 += kWave) {
      const int x = x0 + lane_id();
      int t1, t0;
      if (x < S * per) {
        const int s = x / per, t = x - s * per;
        t1 = s * G + t < T ? s * G + t : T;
        t0 = s * G;
      } else {
        const int s = x < nx ? x - S * per : S;
        t1 = s * G < T ? s * G : T;
        t0 = 0;
      }
      const int32_t p1 = pos(t1), p0 = pos(t0);
      if (x < S * per) {
        const int s = x / per, t = x - s * per;
        rpt[((int64_t)s * nb + k) * per + t] = p1 - p0;
      } else if (x < nx) {
        bnd[k * (S + 1) + (x - S * per)] = p1;
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

// Scatter of B's entries into their slab segments.  Each lane takes one B
// row (wavefront w: rows 64w .. 64w+63); rows with more than kScatterLane
// entries are then walked by the whole wavefront, one after another.  Entries
// go kScatterU at a time per lane: their columns, then their slab bounds and
// segment starts, are loaded together before any is stored.  With kCols the
// column ids go to pbit and, if perm is given, each entry's destination to
// perm (so later value scatters need no bounds); with kVals the values go to
// pval.  Entries that do not fall where the bounds say (unsorted or
// out-of-range columns) are dropped and flagged instead of written out of
// place.
constexpr int kScatterLane = 32;
constexpr int kScatterU = 8;

// Position of column c in the symbolic bitmap of its slab (slabs of 2^ls
// columns): a tile's columns are interleaved over its kTileWords words
// (column x of the tile: word x mod kTileWords, bit x / kTileWords), and the
// code is word*128 + bit, so that code >> 5 is the word's byte offset and the
// code's low 5 bits are the bit.  Any c gives a word below kSlabWordsMax.
SG_DEV int32_t slab_bit_code(int32_t c, int32_t ls) {
  const int32_t r = c & ((1 << ls) - 1);
  const int32_t word = ((r >> kTileLog) * kTileWords) | (r & (kTileWords - 1));
  return (word << 7) | ((r & (kTile - 1)) / kTileWords);
}

// Entries jb + u*step (u < kScatterU, those below e) of row k starting at s0,
// whose row-local slab bounds are r[0..S].
template <class V, bool kCols, bool kVals>
SG_DEV void slab_scatter_entries(const int32_t* col, const V* val, int64_t nb, int32_t ls, int32_t S,
                                 const int32_t* r, const int64_t* prow, int64_t k, int64_t s0, int64_t e, int64_t jb,
                                 int step, int32_t* pbit, ColV<V>* pcv, int32_t* perm, int32_t* err) {
  int32_t c[kScatterU];
  V v[kScatterU];
#pragma unroll
  for (int u = 0; u < kScatterU; ++u) {
    const int64_t j = jb + (int64_t)u * step < e ? jb + (int64_t)u * step : e - 1;
    c[u] = col[j];
    if constexpr (kVals) v[u] = val[j];
  }
  int32_t lo[kScatterU], hi[kScatterU];
  int64_t pb[kScatterU];
#pragma unroll
  for (int u = 0; u < kScatterU; ++u) {
    int32_t sl = c[u] >> ls;
    sl = sl < 0 ? 0 : (sl >= S ? S - 1 : sl);
    lo[u] = r[sl];
    hi[u] = r[sl + 1];
    pb[u] = prow[(int64_t)sl * nb + k];
  }
#pragma unroll
  for (int u = 0; u < kScatterU; ++u) {
    const int64_t j = jb + (int64_t)u * step;
    if (j >= e) break;
    const int64_t o = (j - s0) - lo[u];
    const bool ok = c[u] >= 0 && (c[u] >> ls) < S && o >= 0 && o < (int64_t)(hi[u] - lo[u]);
    if (!ok) {
      atomicOr(err, 1);
      if (perm) perm[j] = -1;
      continue;
    }
    const int64_t dst = pb[u] + o;
    if constexpr (kCols) {
      pbit[dst] = slab_bit_code(c[u], ls);
      if (perm) perm[j] = (int32_t)dst;
    }
    if constexpr (kVals) pcv[dst] = ColV<V>{c[u], v[u]};
  }
}

template <class V, bool kCols, bool kVals>
__global__ __launch_bounds__(256) void k_slab_scatter(const int64_t* rowptr, const int32_t* col, const V* val,
                                                      int64_t nb, int32_t ls, int32_t S, const int32_t* bnd,
                                                      const int64_t* prow, int32_t* pbit, ColV<V>* pcv, int32_t* perm,
                                                      int32_t* err) {
  const int64_t nwaves = ((int64_t)gridDim.x * 256) >> 6;
  for (int64_t k0 = (((int64_t)blockIdx.x * 256 + threadIdx.x) >> 6) * kWave; k0 < nb; k0 += nwaves * kWave) {
    const int64_t k = k0 + lane_id();
    int64_t s0 = 0, e = 0;
    if (k < nb) {
      s0 = rowptr[k];
      e = rowptr[k + 1];
    }
    const bool longrow = e - s0 > kScatterLane;
    if (!longrow)
      for (int64_t jb = s0; jb < e; jb += kScatterU)
        slab_scatter_entries<V, kCols, kVals>(col, val, nb, ls, S, bnd + k * (S + 1), prow, k, s0, e, jb, 1, pbit,
                                              pcv, perm, err);
    unsigned long long m = __ballot(longrow);
    while (m) {
      const int l = __ffsll((long long)m) - 1;
      m &= m - 1ull;
      const int64_t kk = k0 + l;
      const int64_t ss = shfl_any(s0, l), ee = shfl_any(e, l);
      for (int64_t jb = ss + lane_id(); jb < ee; jb += (int64_t)kWave * kScatterU)
        slab_scatter_entries<V, kCols, kVals>(col, val, nb, ls, S, bnd + kk * (S + 1), prow, kk, ss, ee, jb, kWave,
                                              pbit, pcv, perm, err);
    }
  }
}

// Numeric partition through the destinations recorded by the column
// scatter (one thread per B entry).
template <class V>
__global__ __launch_bounds__(256) void k_slab_perm_cv(const int32_t* col, const V* val, const int32_t* perm, int64_t n,
                                                      ColV<V>* pcv) {
  for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < n; j += (int64_t)gridDim.x * 256) {
    const int32_t d = perm[j];
    if (d >= 0) pcv[d] = ColV<V>{col[j], val[j]};
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
// A numeric task is one (dense row, slab) with everything its kernel needs
// up front.  (t0, t1: the slab's column tiles.)
struct SlabTask {
  int32_t h, s;    // position in the dense list, slab
  int32_t t0, t1;  // tiles of the slab
  int64_t out;     // C position of the slab's first entry
  int64_t a0;      // first A entry of the row
  int32_t nsrc;    // A entries of the row
  int32_t m;       // C entries in the slab
};

// Entries of a light task's LDS arrays: besides its accumulator a light
// task keeps each entry's column (its low 16 bits) at its rank, so the
// write-out is two coalesced copies instead of a walk over the bitmap; the
// value and column arrays share 42 KB of LDS.
constexpr int light_cap_of(int acc_bytes) { return (43008 / (acc_bytes + 2)) & ~63; }

template <class Sr>
constexpr int slab_cap() {
  return light_cap_of((int)sizeof(typename Sr::Acc));
}

constexpr int kTaskSlabsLds = 512;  // slabs whose bucket counters a block keeps in LDS

// One thread per dense row: every non-empty slab of the row becomes a light
// task (at most `cap` entries: bitmap + rank in LDS) or a heavy one (a dense
// LDS accumulator per tile).  Both lists hold per-slab buckets of nd slots
// (book[l*T + s] counts bucket s of list l; nd = bins.nd_cap), so walking
// them in order is slab-major.  A block counts its tasks per (list, slab) in LDS, reserves
// each range with one global atomic, then writes the tasks.  Entries per
// list are summed for the statistics.
template <int BS>
__global__ __launch_bounds__(BS) void k_slab_tasks(Bins bins, const DenseRow* dr, const int32_t* off2, int32_t T,
                                                   int32_t G, int32_t S, int32_t cap, const int64_t* c_rowptr,
                                                   SlabTask* light, SlabTask* heavy, int32_t* book, int32_t* ctr) {
  __shared__ int32_t s_cnt[2][kTaskSlabsLds];
  __shared__ int32_t s_base[2][kTaskSlabsLds];
  __shared__ unsigned long long s_ent[2];
  const bool lds = S <= kTaskSlabsLds;
  if (threadIdx.x < 2) s_ent[threadIdx.x] = 0ull;
  block_sync();
  const int64_t nd = dense_rows(bins);
  const int64_t stride = bins.nd_cap;  // slots per bucket
  int32_t* cnt_g[2] = {book + kListSlab * T, book + kListTile * T};
  unsigned long long ent[2] = {0ull, 0ull};
  for (int64_t h0 = (int64_t)blockIdx.x * BS; h0 < nd; h0 += (int64_t)gridDim.x * BS) {
    const int64_t h = h0 + threadIdx.x;
    const bool mine = h < nd;
    const int32_t* o2 = off2 + (mine ? h : 0) * (T + 1);
    if (lds) {
      for (int x = threadIdx.x; x < 2 * S; x += BS) s_cnt[x / S][x % S] = 0;
      block_sync();
      if (mine)
        for (int32_t sl = 0, ta = 0; ta < T; ta += G, ++sl) {
          const int32_t tb = ta + G < T ? ta + G : T;
          const int32_t m = o2[tb] - o2[ta];
          if (m > 0) atomicAdd(&s_cnt[m <= cap ? 0 : 1][sl], 1);
        }
      block_sync();
      for (int x = threadIdx.x; x < 2 * S; x += BS) {
        const int l = x / S, sl = x % S;
        const int32_t c = s_cnt[l][sl];
        s_base[l][sl] = c ? atomicAdd(&cnt_g[l][sl], c) : 0;
        s_cnt[l][sl] = 0;
      }
      block_sync();
    }
    if (mine) {
      const DenseRow d = dr[h];
      const int64_t base = c_rowptr[d.i];
      for (int32_t sl = 0, ta = 0; ta < T; ta += G, ++sl) {
        const int32_t tb = ta + G < T ? ta + G : T;
        const int32_t lo = o2[ta], m = o2[tb] - lo;
        if (m <= 0) continue;
        const int l = m <= cap ? 0 : 1;
        const int32_t slot = lds ? s_base[l][sl] + atomicAdd(&s_cnt[l][sl], 1) : atomicAdd(&cnt_g[l][sl], 1);
        (l == 0 ? light : heavy)[(int64_t)sl * stride + slot] =
            SlabTask{(int32_t)h, sl, ta, tb, base + lo, d.a0, d.nsrc, m};
        ent[l] += (unsigned long long)m;
      }
    }
    if (lds) block_sync();
  }
  for (int l = 0; l < 2; ++l) {
    const unsigned long long v = wave_sum(ent[l]);
    if (lane_id() == 0 && v) atomicAdd(&s_ent[l], v);
  }
  block_sync();
  unsigned long long* eg = (unsigned long long*)(ctr + kCtrEntries);
  if (threadIdx.x == 0 && s_ent[0]) atomicAdd(eg + kListSlab, s_ent[0]);
  if (threadIdx.x == 1 && s_ent[1]) atomicAdd(eg + kListTile, s_ent[1]);
}

template <class V>
struct SlabB {
  const int64_t* prow;
  const int32_t* pbit;  // symbolic bitmap codes (slab_bit_code) of the entries
  const ColV<V>* pcv;
  const int32_t* rpt;
  int64_t nb;
  int32_t G, T;
};

constexpr int kBoffCache = 256;  // bucket offsets kept in LDS

// LDS of one chunk of a task's sources whose window segment is not empty
// (slots): the A value, the exclusive prefix of the segment lengths (off,
// the chunk index of the slot's first product) and the segment's start in
// the partition minus off (st), so product q of slot j sits at st[j] + q.
constexpr int kRoundRowsMax = 8;  // rows of 64 products in one gather round

template <class V, int BS>
struct SrcLds {
  V a[BS];
  int64_t st[BS], off[BS], wave[BS / kWave];
  int32_t boff[kBoffCache + 1];
  alignas(16) uint32_t rb[BS / kWave][2 * kRoundRowsMax];  // per wavefront: slot starts inside its round
  int64_t slot;
};

// Task g of a bucketed list: its bucket is the last t with boff[t] <= g.
template <class V, int BS>
SG_DEV SlabTask bucket_slab_task(const SlabTask* tasks, const int32_t* boff, const SrcLds<V, BS>& L, bool bcache,
                                 int32_t nb, int32_t nd, int64_t g) {
  int lo = 0, hi = nb - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if ((bcache ? L.boff[mid] : boff[mid]) <= g) lo = mid;
    else hi = mid - 1;
  }
  return tasks[(int64_t)lo * nd + (g - (bcache ? L.boff[lo] : boff[lo]))];
}

// Block scan of the sources' segment lengths (one source per thread) that
// keeps only the sources with a non-empty segment: such a source goes to
// slot pos = number of non-empty sources before it, with its first
// product's index off and the partition index of product q of the slot,
// minus q (st - off), and (kVals) its A value.  Slot offsets strictly
// increase, so the owner of product q is the last slot whose offset is at
// most q.  Lengths and flags share one 64-bit scan (flags in the low 16
// bits).  Returns the product count; *n receives the slot count.
template <class V, bool kVals, int BS>
SG_DEV int64_t src_compact(SrcLds<V, BS>& L, int64_t st, int64_t len, V av, int* n) {
  static_assert(BS < (1 << 16), "slot counts fit the low 16 bits");
  const int64_t pk = (len << 16) | (len > 0 ? 1 : 0);
  int64_t tot;
  const int64_t ex = block_excl_scan<BS / kWave, int64_t>(pk, L.wave, &tot);
  if (len > 0) {
    const int pos = (int)(ex & 0xffff);
    L.off[pos] = ex >> 16;
    L.st[pos] = st - (ex >> 16);
    if constexpr (kVals) L.a[pos] = av;
  }
  block_sync();
  *n = (int)(tot & 0xffff);
  return tot >> 16;
}

// The segment of B row k inside tiles [s*G + tr0, s*G + tr1) of slab s
// (whole: the full slab segment, from prow alone; otherwise prow + the tile
// offsets rpt): its start in the partition and its length.
template <class V>
SG_DEV void src_segment(const SlabB<V>& b, int32_t k, int32_t s, int32_t tr0, int32_t tr1, bool whole, int64_t* st,
                        int64_t* len) {
  const int64_t* pr = b.prow + (int64_t)s * b.nb + k;
  *st = pr[0];
  if (whole) {
    *len = pr[1] - *st;
  } else {
    const int32_t* r = b.rpt + ((int64_t)s * b.nb + k) * (b.G + 1);
    const int32_t w0 = r[tr0];
    *st += w0;
    *len = r[tr1] - w0;
  }
}

// Sources [c0, c0 + nc) of the row starting at A entry a0, restricted to
// tiles [s*G + tr0, s*G + tr1) of slab s, one per thread, compacted into
// slots.  Returns the chunk's product count; *n the slots.
template <class V, bool kVals, int BS>
SG_DEV int64_t slab_chunk(const SlabB<V>& b, const int32_t* a_col, const V* a_val, int64_t a0, int32_t s,
                          int32_t tr0, int32_t tr1, bool whole, int64_t c0, int nc, SrcLds<V, BS>& L, int* n) {
  int64_t st = 0, len = 0;
  V av{};
  if ((int)threadIdx.x < nc) {
    const int64_t e = a0 + c0 + threadIdx.x;
    const int32_t k = a_col[e];
    if constexpr (kVals) av = a_val[e];
    src_segment(b, k, s, tr0, tr1, whole, &st, &len);
  }
  return src_compact<V, kVals, BS>(L, st, len, av, n);
}

// Partition elements are loaded as one integer of their size; pin_loaded
// makes the whole integer live at that point, so that the compiler cannot
// split the load and defer its value half behind a branch on the column.
template <int N> struct RawBits;
template <> struct RawBits<4> { using T = unsigned int; };
template <> struct RawBits<8> { using T = unsigned long long; };
template <> struct RawBits<16> { typedef unsigned int T __attribute__((ext_vector_type(4))); };

template <class T>
SG_DEV void pin_loaded(T& v) {
  asm volatile("" : "+v"(v));
}

// One block of 64*U consecutive products [qb, qb + 64*U) of a chunk's nc
// slots: lane l takes q = qb + u*64 + l (u < U), so every load instruction
// is coalesced.  Owners come without per-lane searches: the owner a of qb by
// a 64-ary search (one LDS read per lane and level), then every later slot
// that starts inside the block marks its start in the wavefront's 64*U-bit
// mask, and q's owner is a plus the starts at or below q - qb.  The round
// then issues its U loads of src together and fetch(slot, loaded element)
// makes each product.  ok[u] tells which pp[u] hold one.
template <int BS, int U, class V, bool kNarrow, class R, class Fetch, class P>
SG_DEV void slab_round(SrcLds<V, BS>& L, int nc, int64_t total, int64_t qb, const R* src, Fetch& fetch, P* pp,
                       bool* ok) {
  static_assert(U <= kRoundRowsMax, "round mask rows");
  static_assert(BS <= kWave * (kWave - 1), "two search levels cover the slots");
  constexpr int64_t kBlock = (int64_t)kWave * U;
  if (qb >= total) {
#pragma unroll
    for (int u = 0; u < U; ++u) ok[u] = false;
    return;
  }
  const int lane = lane_id();
  const int64_t qe = (qb + kBlock - 1) < (total - 1) ? (qb + kBlock - 1) : (total - 1);
  int a;
  {
    // an odd stride spreads the 8-byte offsets the lanes read over all LDS
    // banks (an even one puts 32 lanes on 32 / gcd banks)
    const int stride = ((nc + kWave - 1) / kWave) | 1;
    const int i1 = lane * stride;
    const int c1 = __popcll(__ballot(i1 < nc && L.off[i1] <= qb));
    const int b2 = (c1 - 1) * stride, i2 = b2 + lane;
    a = b2 + __popcll(__ballot(lane < stride && i2 < nc && L.off[i2] <= qb)) - 1;
  }
  uint32_t* rb = L.rb[wave_id()];
  if (lane < 2 * U) rb[lane] = 0u;
  __builtin_amdgcn_wave_barrier();
  for (int j0 = a + 1; j0 < nc; j0 += kWave) {
    const int j = j0 + lane;
    const int64_t o = j < nc ? L.off[j] : qe + 1;
    const bool in = o <= qe;
    if (in) {
      // a slot starting at position p (1 <= p < 64*U) marks bit p - 1
      const int p = (int)(o - qb) - 1;
      atomicOr(&rb[p >> 5], 1u << (p & 31));
    }
    if (__ballot(in) != ~0ull) break;
  }
  __builtin_amdgcn_wave_barrier();
  // the mask rows, two per 16-byte read
  static_assert(U % 2 == 0, "mask rows read in pairs");
  unsigned long long w[U];
  const uint4* rb4 = reinterpret_cast<const uint4*>(rb);
#pragma unroll
  for (int u = 0; u < U; u += 2) {
    const uint4 q = rb4[u / 2];
    w[u] = (unsigned long long)q.x | ((unsigned long long)q.y << 32);
    w[u + 1] = (unsigned long long)q.z | ((unsigned long long)q.w << 32);
  }
  // products of the block: lane's row u holds product qb + u*64 + lane,
  // owned by slot a plus the starts marked at bits below its position (the
  // bits below the lane in its row: mbcnt); lanes past the chunk's end take
  // its last product, so every index is valid and needs no branch
  const int lim = (total - qb) < kBlock ? (int)(total - qb) : (int)kBlock;
  int own[U];
  int cnt = a;
#pragma unroll
  for (int u = 0; u < U; ++u) {
    ok[u] = u * kWave + lane < lim;
    own[u] = cnt + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(w[u] >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)w[u], 0u));
    cnt += __popcll(w[u]);
  }
  using Bits = typename RawBits<sizeof(R)>::T;
  Bits raw[U];
  if constexpr (kNarrow) {
    // the caller guarantees that src spans less than 4 GiB: a product's byte
    // offset from src is then exact in 32-bit arithmetic (the partition
    // index st + q is exact modulo 2^32), and each load is the uniform base
    // plus one 32-bit offset
    const char* base = reinterpret_cast<const char*>(src);
    const uint32_t q0 = (uint32_t)qb;
    uint32_t off[U];
#pragma unroll
    for (int u = 0; u < U; ++u) off[u] = (uint32_t)L.st[own[u]];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int x = u * kWave + lane < lim - 1 ? u * kWave + lane : lim - 1;  // ok[u] ? position : last
      off[u] = (off[u] + q0 + (uint32_t)x) * (uint32_t)sizeof(R);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) raw[u] = *reinterpret_cast<const Bits*>(base + off[u]);
  } else {
    int64_t idx[U];
#pragma unroll
    for (int u = 0; u < U; ++u) idx[u] = L.st[own[u]];
#pragma unroll
    for (int u = 0; u < U; ++u) idx[u] += qb + (ok[u] ? u * kWave + lane : lim - 1);
    const Bits* bsrc = reinterpret_cast<const Bits*>(src);
#pragma unroll
    for (int u = 0; u < U; ++u) raw[u] = bsrc[idx[u]];
  }
#pragma unroll
  for (int u = 0; u < U; ++u) pin_loaded(raw[u]);
#pragma unroll
  for (int u = 0; u < U; ++u) pp[u] = fetch(own[u], __builtin_bit_cast(R, raw[u]));
}

// Flattened walk over the chunk's `total` products: wavefront w takes the
// blocks w, w + NW, ... and folds each product with apply(product).  With
// kRepeat, applying a product twice equals applying it once (a bitmap or, a
// minimum), so lanes past the chunk's end apply the last product again
// instead of branching.  Those repeats all hit one LDS word, and atomics on
// one address serialize: worth it only where LDS is not the limit.
template <int BS, int U, class V, bool kRepeat, bool kNarrow, class R, class Fetch, class Apply>
SG_DEV void slab_iterate(SrcLds<V, BS>& L, int nc, int64_t total, const R* src, Fetch& fetch, Apply& apply) {
  constexpr int NW = BS / kWave;
  constexpr int64_t kBlock = (int64_t)kWave * U;
  using P = decltype(fetch(0, src[0]));
  for (int64_t qb = (int64_t)wave_id() * kBlock; qb < total; qb += (int64_t)NW * kBlock) {
    P pp[U];
    bool ok[U];
    slab_round<BS, U, V, kNarrow>(L, nc, total, qb, src, fetch, pp, ok);
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (kRepeat || ok[u]) apply(pp[u]);
  }
}

// All products of a window of task (a0, nsrc, s, tr0, tr1): chunk by chunk
// unless the caller already loaded the single chunk (`loaded`: nl slots,
// total products).  The columns and A values of chunk c+1 are loaded while
// chunk c is gathered, so a chunk waits for its segment bounds only.
template <int BS, int U, class V, bool kVals, bool kRepeat, bool kNarrow, class R, class Fetch, class Apply>
SG_DEV void slab_products(const SlabB<V>& b, const int32_t* a_col, const V* a_val, int64_t a0, int32_t nsrc,
                          int32_t s, int32_t tr0, int32_t tr1, bool whole, bool loaded, int nl, int64_t total,
                          SrcLds<V, BS>& L, const R* src, Fetch& fetch, Apply& apply) {
  if (loaded) {
    slab_iterate<BS, U, V, kRepeat, kNarrow>(L, nl, total, src, fetch, apply);
    return;
  }
  const int64_t tid = threadIdx.x;
  int32_t kn = 0;
  V avn{};
  if (tid < nsrc) {
    kn = a_col[a0 + tid];
    if constexpr (kVals) avn = a_val[a0 + tid];
  }
  for (int64_t c0 = 0; c0 < nsrc; c0 += BS) {
    int64_t st = 0, len = 0;
    const V av = avn;
    if (c0 + tid < nsrc) src_segment(b, kn, s, tr0, tr1, whole, &st, &len);
    if (c0 + BS + tid < nsrc) {
      kn = a_col[a0 + c0 + BS + tid];
      if constexpr (kVals) avn = a_val[a0 + c0 + BS + tid];
    }
    block_sync();
    int ns;
    const int64_t tc = src_compact<V, kVals, BS>(L, st, len, av, &ns);
    slab_iterate<BS, U, V, kRepeat, kNarrow>(L, ns, tc, src, fetch, apply);
  }
}

// Products per lane per gather round in the slab kernels (one round covers
// 64*kSlabU products per wavefront).
constexpr int kSlabU = 8;

// ---- symbolic --------------------------------------------------------------------
// Task g = (slab s = g / nd, dense row h = g % nd), slab-major, from the
// interleaved queues.  The per-tile popcounts of the slab's bitmap are written
// raw to off2[h*(T+1) + t]; k_off2_finish turns them into per-row offsets.
// kNarrow: the bitmap-code array spans less than 4 GiB (32-bit gathers).
template <int BS, bool kNarrow>
__global__ __launch_bounds__(BS, 7) void k_sym_slab(SlabB<uint8_t> b, const DenseRow* dr, const int32_t* a_col,
                                                 Bins bins, int32_t S, int32_t* off2, uint4* spn, int32_t* ctr) {
  constexpr int NW = BS / kWave;
  constexpr int kTilesPerWave = (kSlabTilesMax + NW - 1) / NW;
  static_assert(kTileWords == kWave * 8, "a lane counts 8 words of a tile");
  __shared__ __align__(16) uint32_t s_bm[kSlabWordsMax];
  __shared__ SrcLds<uint8_t, BS> L;
  const int T = b.T, G = b.G;
  const int nwords = G * kTileWords;
  for (int x = threadIdx.x; x < nwords; x += BS) s_bm[x] = 0u;
  const int64_t nd = dense_rows(bins);
  struct SymTask {
    DenseRow d;
    int64_t h;
    int32_t s;
  };
  __shared__ SymTask s_rec[kGrab];
  auto fetch = [&](int64_t g) {
    const int32_t sl = (int32_t)(g / nd);
    const int64_t hh = g - (int64_t)sl * nd;
    return SymTask{dr[hh], hh, sl};
  };
  for_each_queued_rec(ctr, kListSymSlab, nd * S, &L.slot, s_rec, fetch, [&](const SymTask& task) {
    const int32_t s = task.s;
    const int64_t h = task.h;
    const DenseRow d = task.d;
    const int ts0 = s * G;
    // the partition holds each entry's bitmap code (slab_bit_code): only
    // each tile's count of distinct columns is needed, and with a tile's
    // columns interleaved over its words, neighbouring columns, which the
    // lanes of a round mostly hold, land in different words and LDS banks
    auto fetch = [&](int, int32_t code) { return code; };
    auto apply = [&](int32_t code) {
      atomicOr(reinterpret_cast<uint32_t*>(reinterpret_cast<char*>(s_bm) + (code >> 5)), 1u << (code & 31));
    };
    slab_products<BS, kSlabU, uint8_t, false, false, kNarrow>(b, a_col, nullptr, d.a0, d.nsrc, s, 0, G, true, false, 0,
                                                              0, L, b.pbit, fetch, apply);
    block_sync();
    // per-tile counts: wavefront w takes tiles w, w + NW, ..., lane l the
    // words [4l, 4l + 4) and [256 + 4l, 256 + 4l + 4) of each (two 16-byte
    // reads, consecutive over the lanes); all reads are issued before the
    // first count, and the words are cleared for the next task
    int32_t* o2 = off2 + h * (T + 1);
    uint4* bm4 = reinterpret_cast<uint4*>(s_bm);
    uint4 q[kTilesPerWave][2];
#pragma unroll
    for (int i = 0; i < kTilesPerWave; ++i) {
      const int tl = wave_id() + i * NW;
      if (tl < G) {
        q[i][0] = bm4[tl * (kTileWords / 4) + lane_id()];
        q[i][1] = bm4[tl * (kTileWords / 4) + kWave + lane_id()];
      }
    }
#pragma unroll
    for (int i = 0; i < kTilesPerWave; ++i) {
      const int tl = wave_id() + i * NW;
      if (tl < G) {
        const int32_t c = wave_sum((int32_t)(__popc(q[i][0].x) + __popc(q[i][0].y) + __popc(q[i][0].z) +
                                             __popc(q[i][0].w) + __popc(q[i][1].x) + __popc(q[i][1].y) +
                                             __popc(q[i][1].z) + __popc(q[i][1].w)));
        const int t = ts0 + tl;
        if (spn != nullptr && c >= kSpanMin && t < T) {
          // span k holds bits [4k, 4k + 4) of every word: nibble popcounts
          // (SWAR), summed per lane in bytes (at most 32), widened to 16-bit
          // fields for the wavefront sums (at most 2048)
          uint32_t ev = 0u, od = 0u;
          const uint32_t wds[8] = {q[i][0].x, q[i][0].y, q[i][0].z, q[i][0].w,
                                   q[i][1].x, q[i][1].y, q[i][1].z, q[i][1].w};
#pragma unroll
          for (int k = 0; k < 8; ++k) {
            uint32_t x = wds[k] - ((wds[k] >> 1) & 0x55555555u);
            x = (x & 0x33333333u) + ((x >> 2) & 0x33333333u);
            ev += x & 0x0F0F0F0Fu;
            od += (x >> 4) & 0x0F0F0F0Fu;
          }
          const uint32_t s04 = (uint32_t)wave_sum((int32_t)(ev & 0x00FF00FFu));         // spans 0 | 4
          const uint32_t s26 = (uint32_t)wave_sum((int32_t)((ev >> 8) & 0x00FF00FFu));  // spans 2 | 6
          const uint32_t s15 = (uint32_t)wave_sum((int32_t)(od & 0x00FF00FFu));         // spans 1 | 5
          const uint32_t s37 = (uint32_t)wave_sum((int32_t)((od >> 8) & 0x00FF00FFu));  // spans 3 | 7
          if (lane_id() == 0)
            spn[h * T + t] = uint4{(s04 & 0xFFFFu) | (s15 << 16), (s26 & 0xFFFFu) | (s37 << 16),
                                   (s04 >> 16) | (s15 & 0xFFFF0000u), (s26 >> 16) | (s37 & 0xFFFF0000u)};
        }
        const uint4 z{0u, 0u, 0u, 0u};
        bm4[tl * (kTileWords / 4) + lane_id()] = z;
        bm4[tl * (kTileWords / 4) + kWave + lane_id()] = z;
        if (lane_id() == 0 && t < T) o2[t] = c;
      }
    }
  });
}

// ---- numeric ---------------------------------------------------------------------
// Light windows (at most CAP entries): bitmap + rank, two passes over the
// products (sources loaded once when one chunk holds them).
template <class Sr, class V, int BS, int CAP, bool kNarrow>
__global__ __launch_bounds__(BS, 4) void k_num_slab(SlabB<V> b, const int32_t* a_col, const V* a_val, OutC C,
                                                 const SlabTask* tasks, const int32_t* boff, int32_t nd,
                                                 int32_t* ctr, int32_t* err) {
  constexpr int NW = BS / kWave;
  static_assert(kTileWords % (NW * kWave) == 0, "each wavefront owns a multiple of 64 words of a window");
  static_assert(kSlabWordsMax <= kSlabTilesMax * kWave * NW, "a lane owns at most kSlabTilesMax words");
  static_assert(CAP <= 65535, "ranks are 16-bit");
  using Acc = typename Sr::Acc;
  __shared__ uint32_t s_bits[kSlabWordsMax];
  __shared__ uint16_t s_rank[kSlabWordsMax];
  __shared__ Acc s_val[CAP];
  __shared__ uint16_t s_col[CAP];
  __shared__ SrcLds<V, BS> L;
  __shared__ int32_t s_wt[NW];
  const int T = b.T, G = b.G;
  for (int x = threadIdx.x; x < kSlabWordsMax; x += BS) s_bits[x] = 0u;
  const bool bcache = T < kBoffCache;
  if (bcache)
    for (int x = threadIdx.x; x <= T; x += BS) L.boff[x] = boff[x];
  block_sync();
  const int wv = wave_id();
  __shared__ SlabTask s_rec[kGrab];
  auto fetch = [&](int64_t g) { return bucket_slab_task<V, BS>(tasks, boff, L, bcache, T, nd, g); };
  for_each_queued_rec(ctr, kListSlab, (int64_t)ctr[kListSlab], &L.slot, s_rec, fetch, [&](const SlabTask& task) {
    const SlabTask tk = task;
    const int ts0 = tk.s * G, ts1 = ts0 + G < T ? ts0 + G : T;
    const bool whole = tk.t0 == ts0 && tk.t1 == ts1;
    const int32_t tr0 = tk.t0 - ts0, tr1 = tk.t1 - ts0;
    const int32_t m = tk.m < CAP ? tk.m : CAP;
    if (threadIdx.x == 0 && tk.m > CAP) atomicOr(err, 1);
    const int64_t cw0 = (int64_t)tk.t0 << kTileLog;
    const int nwords = (tk.t1 - tk.t0) * kTileWords;
    const int wpw = nwords / NW;
    const bool one = tk.nsrc <= BS;
    int64_t total = 0;
    int nl = 0;
    block_sync();
    if (one) total = slab_chunk<V, true, BS>(b, a_col, a_val, tk.a0, tk.s, tr0, tr1, whole, 0, tk.nsrc, L, &nl);
    // With one round of products per wavefront the products stay in
    // registers for pass 2; otherwise pass 2 gathers them again.
    const bool held = one && total <= (int64_t)NW * kWave * kSlabU;
    // a window column c lies below nwords*32; the word index is masked to
    // the bitmap all the same, so that no partition content can reach
    // beyond it
    auto f1 = [&](int, const ColV<V>& e) { return (int32_t)(e.c - cw0); };
    auto a1 = [&](int32_t c) { atomicOr(&s_bits[(c >> 5) & (kSlabWordsMax - 1)], 1u << (c & 31)); };
    auto f2 = [&](int ow, const ColV<V>& e) { return ColVal<Acc>{(int32_t)(e.c - cw0), Sr::mul(L.a[ow], e.v)}; };
    auto a2 = [&](const ColVal<Acc>& p) {
      const int w = (p.c >> 5) & (kSlabWordsMax - 1);
      const int32_t r = (int32_t)s_rank[w] + __popc(s_bits[w] & ((1u << (p.c & 31)) - 1u));
      if (r < m) {
        Sr::lds_acc(&s_val[r], p.v);
        s_col[r] = (uint16_t)p.c;
      }
    };
    ColVal<Acc> pp[kSlabU];
    bool ok[kSlabU];
    // a held round that is not empty repeats its last product in the lanes
    // past the end, which idempotent folds may apply again
    const bool hround = (int64_t)wv * kWave * kSlabU < total;
    // pass 1: the window's column set
    if (held) {
      slab_round<BS, kSlabU, V, kNarrow>(L, nl, total, (int64_t)wv * kWave * kSlabU, b.pcv, f2, pp, ok);
      if (hround)
#pragma unroll
        for (int u = 0; u < kSlabU; ++u) a1(pp[u].c);
    } else {
      slab_products<BS, kSlabU, V, true, true, kNarrow>(b, a_col, a_val, tk.a0, tk.nsrc, tk.s, tr0, tr1, whole, one, nl,
                                                        total, L, b.pcv, f1, a1);
    }
    block_sync();
    // ranks: wavefront wv owns words [wv*wpw, (wv+1)*wpw), lane l the kpl
    // consecutive words from wv*wpw + l*kpl; word popcounts stay in
    // registers between the count and the rank pass
    const int kpl = wpw / kWave;
    const int w0 = wv * wpw + lane_id() * kpl;
    int32_t pcw[kSlabTilesMax];
    int32_t lt = 0;
#pragma unroll
    for (int i = 0; i < kSlabTilesMax; ++i) {
      pcw[i] = i < kpl ? __popc(s_bits[w0 + i]) : 0;
      lt += pcw[i];
    }
    const int32_t linc = wave_incl_scan(lt);
    if (lane_id() == kWave - 1) s_wt[wv] = linc;
    for (int x = threadIdx.x; x < m; x += BS) s_val[x] = Sr::ident();
    block_sync();
    int32_t wbase = 0, tot = 0;
#pragma unroll
    for (int u = 0; u < NW; ++u) {
      const int32_t v = s_wt[u];
      wbase += u < wv ? v : 0;
      tot += v;
    }
    if (threadIdx.x == 0 && tot != tk.m) atomicOr(err, 1);
    int32_t rk = wbase + linc - lt;
#pragma unroll
    for (int i = 0; i < kSlabTilesMax; ++i)
      if (i < kpl) {
        s_rank[w0 + i] = (uint16_t)rk;
        rk += pcw[i];
      }
    block_sync();
    // pass 2: fold every product into its compacted slot
    if (held) {
#pragma unroll
      for (int u = 0; u < kSlabU; ++u)
        if (Sr::kIdempotent ? hround : ok[u]) a2(pp[u]);
    } else {
      slab_products<BS, kSlabU, V, true, Sr::kIdempotent, kNarrow>(b, a_col, a_val, tk.a0, tk.nsrc, tk.s, tr0, tr1,
                                                                   whole, one, nl, total, L, b.pcv, f2, a2);
    }
    block_sync();
    // write-out: columns and values in rank order, both coalesced (lanes
    // store at 32-bit offsets from the task's uniform output base); window
    // columns are below 2^17, and bit 16 is set exactly for the ranks from
    // that of word 2048 on; the bitmap is cleared for the next task
    const int64_t o0 = uniform64(tk.out);
    char* colb = reinterpret_cast<char*>(C.col + o0);
    char* valb = reinterpret_cast<char*>((V*)C.val + o0);
    const uint32_t split = nwords > 2048 ? (uint32_t)s_rank[2048] : (uint32_t)m;
    for (uint32_t x = threadIdx.x; x < (uint32_t)m; x += BS) {
      const int32_t c = (int32_t)s_col[x] | (x >= split ? 65536 : 0);
      *reinterpret_cast<int32_t*>(colb + x * (uint32_t)sizeof(int32_t)) = (int32_t)cw0 + c;
      *reinterpret_cast<V*>(valb + x * (uint32_t)sizeof(V)) = Sr::out(s_val[x]);
    }
    for (int it = 0; it < wpw; it += kWave) s_bits[wv * wpw + it + lane_id()] = 0u;
  });
}

// Products plus entries of a heavy task's tile that take the staged path:
// at most 8192, and no more than the accumulator's LDS holds next to the
// tile's bitmap and word ranks (a product or an entry takes its
// accumulator and a 16-bit column).
template <class Acc>
constexpr int stage_max() {
  constexpr int fit = (kTile * (int)sizeof(Acc) - kTileWords * 6 - 8) / ((int)sizeof(Acc) + 2);
  return fit < 8192 ? fit : 8192;
}

// Heavy tasks (a slab holding more entries than a light task's value
// array): the row's sources are loaded once (A value, column, slab segment
// start), then each non-empty tile of the slab is folded in one pass into a
// dense 16384-slot LDS accumulator and compacted in column order, or, when
// sparse, ranked on a bitmap of its columns (see the staged path below);
// when the row's sources fit one chunk (one per thread), their tile offsets
// stay in registers for every tile.  Slots are reset to the
// identity as they are compacted; for semirings whose identity no product
// reaches (kValueMarks) occupancy is read off the accumulator, otherwise an
// occupancy bitmap is kept.  8-byte accumulators fill 128 KB of LDS: one
// workgroup per CU.  Wavefront w compacts span w of the tile; where the
// symbolic pass recorded the tile's span counts they give each wavefront its
// output offset, otherwise the wavefronts count their spans first.
template <class Sr, class V, int BS, bool kNarrow>
__global__ __launch_bounds__(BS, sizeof(typename Sr::Acc) > 4 ? 2 : 4) void k_num_slab_heavy(
    SlabB<V> b, const int32_t* a_col, const V* a_val, const int32_t* off2, const uint4* spn, OutC C,
    const SlabTask* tasks, const int32_t* boff, int32_t nd, int32_t* ctr, int32_t* err) {
  constexpr int NW = BS / kWave;
  constexpr int kSpan = kTile / NW;  // accumulator slots compacted per wavefront
  static_assert(kSpan % kWave == 0, "whole steps of 64 slots per wavefront");
  static_assert(NW == kSpans, "one symbolic span per wavefront");
  using Acc = typename Sr::Acc;
  __shared__ Acc s_acc[kTile];
  __shared__ uint32_t s_bm[Sr::kValueMarks ? 1 : kTileWords];
  __shared__ SrcLds<V, BS> L;
  __shared__ int32_t s_wave32[NW];
  __shared__ int32_t s_tc[kSlabTilesMax + 1];
  const int T = b.T, G = b.G;
  const int wv = wave_id();
  for (int x = threadIdx.x; x < kTile; x += BS) s_acc[x] = Sr::ident();
  if constexpr (!Sr::kValueMarks)
    for (int x = threadIdx.x; x < kTileWords; x += BS) s_bm[x] = 0u;
  const bool bcache = T < kBoffCache;
  if (bcache)
    for (int x = threadIdx.x; x <= T; x += BS) L.boff[x] = boff[x];
  block_sync();
  // accumulator slots [0, dirty) were used by a staged tile and hold no
  // identity; the next tile that folds into the dense accumulator resets them
  int32_t dirty = 0;
  __shared__ SlabTask s_rec[kGrab];
  auto fetch = [&](int64_t g) { return bucket_slab_task<V, BS>(tasks, boff, L, bcache, T, nd, g); };
  for_each_queued_rec(ctr, kListTile, (int64_t)ctr[kListTile], &L.slot, s_rec, fetch, [&](const SlabTask& task) {
    const SlabTask tk = task;
    const int ts0 = tk.t0, ts1 = tk.t1;
    block_sync();
    if ((int)threadIdx.x <= ts1 - ts0) {
      const int32_t* o2 = off2 + (int64_t)tk.h * (T + 1);
      s_tc[threadIdx.x] = o2[ts0 + threadIdx.x] - o2[ts0];
    }
    // the row's sources: one per thread when one chunk holds them all, with
    // the A value and the source's tile offsets kept in registers for every
    // tile; each tile compacts its non-empty segments into slots
    const bool one = tk.nsrc <= BS;
    int64_t sst = 0;
    V av{};
    int32_t rec[kSlabTilesMax + 1];
#pragma unroll
    for (int q = 0; q <= kSlabTilesMax; ++q) rec[q] = 0;
    if (one && (int)threadIdx.x < tk.nsrc) {
      const int64_t e = tk.a0 + threadIdx.x;
      const int32_t k = a_col[e];
      av = a_val[e];
      sst = b.prow[(int64_t)tk.s * b.nb + k];
      const int32_t* r = b.rpt + ((int64_t)tk.s * b.nb + k) * (G + 1);
#pragma unroll
      for (int q = 0; q <= kSlabTilesMax; ++q)
        if (q <= G) rec[q] = r[q];
    }
    block_sync();
    for (int t = ts0; t < ts1; ++t) {
      const int32_t rel = s_tc[t - ts0], mt = s_tc[t + 1 - ts0] - rel;
      if (mt <= 0) continue;
      const bool spans = spn != nullptr && mt >= kSpanMin;
      uint4 sp{0u, 0u, 0u, 0u};
      if (spans) sp = spn[(int64_t)tk.h * T + t];
      const int32_t cw0 = t << kTileLog;
      // the tile's products: column within the tile (tiles are aligned, so
      // the low bits; masking also bounds any partition content)
      auto f = [&](int ow, const ColV<V>& e) { return ColVal<Acc>{e.c & (kTile - 1), Sr::mul(L.a[ow], e.v)}; };
      auto ap = [&](const ColVal<Acc>& p) {
        Sr::lds_acc(&s_acc[p.c], p.v);
        if constexpr (!Sr::kValueMarks) atomicOr(&s_bm[p.c >> 5], 1u << (p.c & 31));
      };
      if (one) {
        int64_t len = 0, st = 0;
        if ((int)threadIdx.x < tk.nsrc) {
          int32_t w0 = 0, w1 = 0;
#pragma unroll
          for (int q = 0; q < kSlabTilesMax; ++q)
            if (q == t - ts0) {
              w0 = rec[q];
              w1 = rec[q + 1];
            }
          st = sst + w0;
          len = w1 - w0;
        }
        int nl;
        const int64_t total = src_compact<V, true, BS>(L, st, len, av, &nl);
        constexpr int kWinU = 2;  // products held per lane (registers: the kernel sits at 128)
        if (mt < kSpanMin && total <= (int64_t)NW * kWave * kWinU) {
          // a sparse tile (no span counts) whose products fit one round: the
          // light tasks' scheme instead of two sweeps of all kTile slots --
          // products held in registers, a bitmap of the tile's columns and
          // word ranks, values and 16-bit columns at their ranks, copied out
          // in order; its LDS is borrowed from the head of the accumulator
          // and reset to the identity afterwards
          uint32_t* w_bits = reinterpret_cast<uint32_t*>(s_acc);
          uint16_t* w_rank = reinterpret_cast<uint16_t*>(w_bits + kTileWords);
          Acc* w_val = reinterpret_cast<Acc*>(w_rank + kTileWords);
          uint16_t* w_col = reinterpret_cast<uint16_t*>(w_val + kSpanMin);
          constexpr int kWinSlots =
              (int)((kTileWords * 6 + kSpanMin * (sizeof(Acc) + 2) + sizeof(Acc) - 1) / sizeof(Acc));
          static_assert(kWinSlots <= kTile, "the window fits the accumulator");
          w_bits[threadIdx.x] = 0u;
          for (int x = threadIdx.x; x < mt; x += BS) w_val[x] = Sr::ident();
          block_sync();
          static_assert(BS == kTileWords, "one bitmap word per thread");
          ColVal<Acc> pp[kWinU];
          bool ok[kWinU];
          slab_round<BS, kWinU, V, kNarrow>(L, nl, total, (int64_t)wv * kWave * kWinU, b.pcv, f, pp, ok);
#pragma unroll
          for (int u = 0; u < kWinU; ++u)
            if (ok[u]) atomicOr(&w_bits[pp[u].c >> 5], 1u << (pp[u].c & 31));
          block_sync();
          const uint32_t wb = w_bits[threadIdx.x];
          int32_t tot;
          const int32_t ex = block_excl_scan<NW, int32_t>(__popc(wb), s_wave32, &tot);
          w_rank[threadIdx.x] = (uint16_t)ex;
          if (threadIdx.x == 0 && tot != mt) atomicOr(err, 1);
          block_sync();
#pragma unroll
          for (int u = 0; u < kWinU; ++u)
            if (ok[u]) {
              const int w = pp[u].c >> 5;
              const int32_t r = (int32_t)w_rank[w] + __popc(w_bits[w] & ((1u << (pp[u].c & 31)) - 1u));
              if (r < mt) {
                Sr::lds_acc(&w_val[r], pp[u].v);
                w_col[r] = (uint16_t)pp[u].c;
              }
            }
          block_sync();
          const int64_t o0 = uniform64(tk.out + rel);
          char* colb = reinterpret_cast<char*>(C.col + o0);
          char* valb = reinterpret_cast<char*>((V*)C.val + o0);
          for (uint32_t x = threadIdx.x; x < (uint32_t)mt; x += BS) {
            *reinterpret_cast<int32_t*>(colb + x * (uint32_t)sizeof(int32_t)) = cw0 + (int32_t)w_col[x];
            *reinterpret_cast<V*>(valb + x * (uint32_t)sizeof(V)) = Sr::out(w_val[x]);
          }
          block_sync();
          dirty = dirty > kWinSlots ? dirty : kWinSlots;
          continue;
        }
        if (total + mt <= stage_max<Acc>()) {
          // a sparse tile whose products fit LDS next to its entries: the
          // products are staged in LDS (16-bit column, value) while the
          // tile's column bitmap is set, the bitmap's word ranks give each
          // product its entry, and the entries are copied out in order --
          // no sweep of all kTile slots.  The LDS is the accumulator's.
          char* base = reinterpret_cast<char*>(s_acc);
          uint32_t* g_bits = reinterpret_cast<uint32_t*>(base);
          uint16_t* g_rank = reinterpret_cast<uint16_t*>(base + kTileWords * 4);
          Acc* g_val = reinterpret_cast<Acc*>(base + kTileWords * 6);
          uint16_t* g_col = reinterpret_cast<uint16_t*>(g_val + mt);
          const int pv0 = (kTileWords * 6 + mt * (int)(sizeof(Acc) + 2) + 7) & ~7;
          Acc* g_pv = reinterpret_cast<Acc*>(base + pv0);
          uint16_t* g_pc = reinterpret_cast<uint16_t*>(g_pv + total);
          static_assert(BS == kTileWords, "one bitmap word per thread");
          g_bits[threadIdx.x] = 0u;
          for (int x = threadIdx.x; x < mt; x += BS) g_val[x] = Sr::ident();
          block_sync();
          constexpr int64_t kBlock = (int64_t)kWave * kSlabU;
          for (int64_t qb = (int64_t)wv * kBlock; qb < total; qb += (int64_t)NW * kBlock) {
            ColVal<Acc> pp[kSlabU];
            bool ok[kSlabU];
            slab_round<BS, kSlabU, V, kNarrow>(L, nl, total, qb, b.pcv, f, pp, ok);
#pragma unroll
            for (int u = 0; u < kSlabU; ++u)
              if (ok[u]) {
                const int q = (int)qb + u * kWave + lane_id();
                g_pc[q] = (uint16_t)pp[u].c;
                g_pv[q] = pp[u].v;
                atomicOr(&g_bits[pp[u].c >> 5], 1u << (pp[u].c & 31));
              }
          }
          block_sync();
          const uint32_t wb = g_bits[threadIdx.x];
          int32_t tot;
          const int32_t ex = block_excl_scan<NW, int32_t>(__popc(wb), s_wave32, &tot);
          g_rank[threadIdx.x] = (uint16_t)ex;
          if (threadIdx.x == 0 && tot != mt) atomicOr(err, 1);
          block_sync();
          for (int q = threadIdx.x; q < (int)total; q += BS) {
            const int c = g_pc[q];
            const int w = c >> 5;
            const int32_t r = (int32_t)g_rank[w] + __popc(g_bits[w] & ((1u << (c & 31)) - 1u));
            if (r < mt) {
              Sr::lds_acc(&g_val[r], g_pv[q]);
              g_col[r] = (uint16_t)c;
            }
          }
          block_sync();
          const int64_t o0 = uniform64(tk.out + rel);
          char* colb = reinterpret_cast<char*>(C.col + o0);
          char* valb = reinterpret_cast<char*>((V*)C.val + o0);
          for (uint32_t x = threadIdx.x; x < (uint32_t)mt; x += BS) {
            *reinterpret_cast<int32_t*>(colb + x * (uint32_t)sizeof(int32_t)) = cw0 + (int32_t)g_col[x];
            *reinterpret_cast<V*>(valb + x * (uint32_t)sizeof(V)) = Sr::out(g_val[x]);
          }
          block_sync();
          const int32_t used = (pv0 + (int)total * (int)(sizeof(Acc) + 2) + (int)sizeof(Acc) - 1) / (int)sizeof(Acc);
          dirty = dirty > used ? dirty : used;
          continue;
        }
        if (dirty) {
          for (int x = threadIdx.x; x < dirty; x += BS) s_acc[x] = Sr::ident();
          dirty = 0;
          block_sync();
        }
        slab_iterate<BS, kSlabU, V, false, kNarrow>(L, nl, total, b.pcv, f, ap);
      } else {
        if (dirty) {
          for (int x = threadIdx.x; x < dirty; x += BS) s_acc[x] = Sr::ident();
          dirty = 0;
          block_sync();
        }
        slab_products<BS, kSlabU, V, true, false, kNarrow>(b, a_col, a_val, tk.a0, tk.nsrc, tk.s, t - ts0, t + 1 - ts0,
                                                           false, false, 0, 0, L, b.pcv, f, ap);
      }
      block_sync();
      // compaction: wavefront wv owns slots [wv*kSpan, (wv+1)*kSpan) and
      // reads 64 consecutive slots per step (no bank conflicts); a ballot of
      // the occupied slots gives each lane its output rank, so the stores of
      // a step are contiguous.  Slots are reset as they are read.
      const int sb = wv * kSpan;
      int32_t cnt = 0, base = 0, tot = 0;
      if (spans) {
        const uint32_t pk[4] = {sp.x, sp.y, sp.z, sp.w};  // span 2i | span 2i+1 << 16
#pragma unroll
        for (int u = 0; u < NW; ++u) {
          const int32_t v = (int32_t)((pk[u >> 1] >> (16 * (u & 1))) & 0xFFFFu);
          base += u < wv ? v : 0;
          cnt = u == wv ? v : cnt;
          tot += v;
        }
      } else {
        if constexpr (Sr::kValueMarks) {
#pragma unroll 8
          for (int j = 0; j < kSpan; j += kWave)
            cnt += __popcll(__ballot(s_acc[sb + j + lane_id()] != Sr::ident()));
        } else {
          static_assert(kSpan == 32 * kWave, "one bitmap word per lane");
          cnt = wave_sum((int32_t)__popc(s_bm[(sb >> 5) + lane_id()]));
        }
        if (lane_id() == 0) s_wave32[wv] = cnt;
        block_sync();
#pragma unroll
        for (int u = 0; u < NW; ++u) {
          const int32_t v = s_wave32[u];
          base += u < wv ? v : 0;
          tot += v;
        }
      }
      // output pointers of the wavefront's first entry: lanes store at 32-bit
      // offsets from a uniform base
      const int64_t o0 = uniform64(tk.out + rel + base);
      char* colb = reinterpret_cast<char*>(C.col + o0);
      char* valb = reinterpret_cast<char*>((V*)C.val + o0);
      const uint32_t lim = (uint32_t)(mt - base);
      uint32_t run = 0;
      // kBatch steps per group: their slots are read before any is reset
      constexpr int kBatch = 8;
      static_assert(kSpan % (kBatch * kWave) == 0, "whole groups of steps");
      for (int j0 = 0; j0 < kSpan; j0 += kBatch * kWave) {
        Acc v[kBatch];
#pragma unroll
        for (int k = 0; k < kBatch; ++k) v[k] = s_acc[sb + j0 + k * kWave + lane_id()];
#pragma unroll
        for (int k = 0; k < kBatch; ++k) {
          const int x = sb + j0 + k * kWave + lane_id();
          bool occ;
          if constexpr (Sr::kValueMarks) occ = v[k] != Sr::ident();
          else occ = (s_bm[x >> 5] >> (x & 31)) & 1u;
          const unsigned long long mk = __ballot(occ);
          const uint32_t r =
              run + __builtin_amdgcn_mbcnt_hi((uint32_t)(mk >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mk, 0u));
          if (occ && r < lim) {
            *reinterpret_cast<int32_t*>(colb + r * (uint32_t)sizeof(int32_t)) = (int32_t)(cw0 + x);
            *reinterpret_cast<V*>(valb + r * (uint32_t)sizeof(V)) = Sr::out(v[k]);
          }
          s_acc[x] = Sr::ident();
          run += (uint32_t)__popcll(mk);
        }
      }
      if constexpr (!Sr::kValueMarks) s_bm[(sb >> 5) + lane_id()] = 0u;
      // the symbolic and numeric passes must agree on every span
      if (lane_id() == 0 && run != (uint32_t)cnt) atomicOr(err, 1);
      if (threadIdx.x == 0 && tot != mt) atomicOr(err, 1);
      block_sync();
    }
  });
}

}  // namespace sg
