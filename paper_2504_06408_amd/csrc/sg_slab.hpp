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

// Row i of A (x) B restricted to one slab (structure only): one source per
// stored A_ik, its segment = the slab part of B_k in the partition.
struct SlabSrc {
  const DenseRow* drow;
  const int32_t* a_col;
  const int64_t* prow;
  const int32_t* pcol;
  int64_t nb;
  int64_t a0;
  int64_t sb;

  struct Item {
    uint8_t unused;
  };

  SG_DEV int64_t bind(int64_t h, int32_t s) {
    const DenseRow d = drow[h];
    a0 = d.a0;
    sb = (int64_t)s * nb;
    return d.nsrc;
  }
  SG_DEV void load(int64_t j, Item&, int64_t& start, int64_t& len) const {
    const int32_t k = a_col[a0 + j];
    const int64_t* r = prow + sb + k;
    start = r[0];
    len = r[1] - start;
  }
  SG_DEV int32_t col(const Item&, int64_t idx) const { return pcol[idx]; }
};

// ---- symbolic --------------------------------------------------------------------
// Task g = (slab s, dense row h) with s = g / nd: per-tile popcounts of the
// slab's bitmap are written raw to off2[h*(T+1) + t]; k_off2_finish turns
// them into per-row offsets.
template <int BS>
__global__ __launch_bounds__(BS) void k_sym_slab(SlabSrc src0, Bins bins, int32_t S, int32_t ls, int32_t T,
                                                 int32_t* off2, int32_t* ctr) {
  constexpr int NW = BS / kWave;
  using Item = SlabSrc::Item;
  __shared__ uint32_t s_bm[kSlabWordsMax];
  __shared__ Item s_item[BS];
  __shared__ int64_t s_start[BS], s_off[BS], s_wave[NW];
  __shared__ int64_t s_slot;
  const int nwords = 1 << (ls - 5);
  const int G = 1 << (ls - kTileLog);
  for (int x = threadIdx.x; x < nwords; x += BS) s_bm[x] = 0u;
  const int64_t nd = dense_rows(bins);
  const uint32_t cmax = (uint32_t)nwords * 32u;
  for_each_queued(ctr, kListSymSlab, nd * S, &s_slot, [&](int64_t g) {
    const int32_t s = (int32_t)(g / nd);
    const int64_t h = g - (int64_t)s * nd;
    SlabSrc sr = src0;
    const int64_t nsrc = sr.bind(h, s);
    const int64_t c0 = (int64_t)s << ls;
    __syncthreads();
    auto fetch = [&](const Item& it, int64_t idx) { return (int32_t)(sr.col(it, idx) - c0); };
    auto apply = [&](int32_t c) {
      if ((uint32_t)c < cmax) atomicOr(&s_bm[c >> 5], 1u << (c & 31));
    };
    for_each_product<BS, kUnroll>(sr, nsrc, s_item, s_start, s_off, s_wave, fetch, apply);
    __syncthreads();
    int32_t* o2 = off2 + h * (T + 1);
    for (int tl = wave_id(); tl < G; tl += NW) {
      int32_t c = 0;
      for (int x = lane_id(); x < kTileWords; x += kWave) {
        const int wx = tl * kTileWords + x;
        c += __popc(s_bm[wx]);
        s_bm[wx] = 0u;
      }
      c = wave_sum(c);
      const int t = s * G + tl;
      if (lane_id() == 0 && t < T) o2[t] = c;
    }
  });
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

// ---- numeric ---------------------------------------------------------------------
// One numeric task per non-empty (dense row, slab), with everything the
// kernel needs up front (no dependent lookups before the sources).
struct SlabTask {
  int32_t h, s;   // position in the dense list, slab
  int64_t out;    // C position of the slab's first entry
  int64_t a0;     // first A entry of the row
  int32_t nsrc;   // A entries of the row
  int32_t m;      // C entries in the slab
};

// One thread per dense row; slab tasks go to per-slab buckets of nd slots
// (book[2*T + s] counts bucket s), entries are summed for the statistics.
template <int BS>
__global__ __launch_bounds__(BS) void k_slab_tasks(Bins bins, const DenseRow* dr, const int32_t* off2, int32_t T,
                                                   int32_t G, const int64_t* c_rowptr, SlabTask* tasks,
                                                   int32_t* book, int32_t* ctr) {
  __shared__ unsigned long long s_ent;
  if (threadIdx.x == 0) s_ent = 0ull;
  __syncthreads();
  const int64_t nd = dense_rows(bins);
  int32_t* cnt = book + 2 * T;
  unsigned long long ent = 0ull;
  for (int64_t h = (int64_t)blockIdx.x * BS + threadIdx.x; h < nd; h += (int64_t)gridDim.x * BS) {
    const DenseRow d = dr[h];
    const int32_t* o2 = off2 + h * (T + 1);
    const int64_t base = c_rowptr[d.i];
    int32_t s = 0;
    for (int32_t ta = 0; ta < T; ta += G, ++s) {
      const int32_t tb = ta + G < T ? ta + G : T;
      const int32_t lo = o2[ta], m = o2[tb] - lo;
      if (m <= 0) continue;
      tasks[(int64_t)s * nd + atomicAdd(&cnt[s], 1)] = SlabTask{(int32_t)h, s, base + lo, d.a0, d.nsrc, m};
      ent += (unsigned long long)m;
    }
  }
  ent = wave_sum(ent);
  if (lane_id() == 0 && ent) atomicAdd(&s_ent, ent);
  __syncthreads();
  if (threadIdx.x == 0 && s_ent) atomicAdd((unsigned long long*)(ctr + kCtrEntries) + kListSlab, s_ent);
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

// Entries of a task's LDS value array (32 KB of accumulators).
template <class Sr>
constexpr int slab_cap() {
  return 32768 / (int)sizeof(typename Sr::Acc);
}

constexpr int kBoffCache = 256;  // slab-bucket offsets kept in LDS

template <class Sr, class V, int BS, int CAP>
__global__ __launch_bounds__(BS) void k_num_slab(SlabB<V> b, const int32_t* a_col, const V* a_val,
                                                 const int32_t* off2, OutC C, const SlabTask* tasks,
                                                 const int32_t* boff, int32_t S, int32_t nd, int32_t* ctr,
                                                 int32_t* err) {
  constexpr int NW = BS / kWave;
  static_assert(NW * kWave <= kTileWords, "each wavefront owns a multiple of 64 words of a window");
  static_assert(CAP <= 65535, "ranks are 16-bit");
  using Acc = typename Sr::Acc;
  constexpr int64_t kBlock = (int64_t)kWave * kUnroll;
  __shared__ uint32_t s_bits[kSlabWordsMax];
  __shared__ uint16_t s_rank[kSlabWordsMax];
  __shared__ Acc s_val[CAP];
  __shared__ V s_a[BS];
  __shared__ int32_t s_k[BS], s_slen[BS], s_wo[BS];
  __shared__ int64_t s_sst[BS], s_off[BS], s_wave[NW];
  __shared__ int32_t s_wt[NW];
  __shared__ int32_t s_tc[kSlabTilesMax + 1];
  __shared__ int32_t s_boff[kBoffCache + 1];
  __shared__ int64_t s_slot;
  const int T = b.T, G = b.G;
  for (int x = threadIdx.x; x < kSlabWordsMax; x += BS) s_bits[x] = 0u;
  const bool bcache = S < kBoffCache;
  if (bcache)
    for (int x = threadIdx.x; x <= S; x += BS) s_boff[x] = boff[x];
  __syncthreads();
  const int wv = wave_id();
  for_each_queued(ctr, kListSlab, (int64_t)ctr[kListSlab], &s_slot, [&](int64_t g) {
    // task g: its slab bucket is the last s with boff[s] <= g
    int lo = 0, hi = S - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if ((bcache ? s_boff[mid] : boff[mid]) <= g) lo = mid;
      else hi = mid - 1;
    }
    const SlabTask tk = tasks[(int64_t)lo * nd + (g - (bcache ? s_boff[lo] : boff[lo]))];
    const int s = tk.s;
    const int ts0 = s * G, ts1 = ts0 + G < T ? ts0 + G : T;
    const bool split = tk.m > CAP;
    if (split && threadIdx.x <= ts1 - ts0) {
      const int32_t* o2 = off2 + (int64_t)tk.h * (T + 1);
      s_tc[threadIdx.x] = o2[ts0 + threadIdx.x] - o2[ts0];
    }
    auto load_src = [&](int64_t c0, int nc) {
      if (threadIdx.x < nc) {
        const int64_t e = tk.a0 + c0 + threadIdx.x;
        const int32_t k = a_col[e];
        s_k[threadIdx.x] = k;
        s_a[threadIdx.x] = a_val[e];
        const int64_t* pr = b.prow + (int64_t)s * b.nb + k;
        const int64_t st = pr[0];
        s_sst[threadIdx.x] = st;
        s_slen[threadIdx.x] = (int32_t)(pr[1] - st);
      }
    };
    const bool one = tk.nsrc <= BS;
    if (one) load_src(0, tk.nsrc);
    __syncthreads();
    int t0 = ts0;
    while (t0 < ts1) {
      int t1 = ts1;
      int32_t rel0 = 0, mw = tk.m;
      if (split) {
        t1 = t0 + 1;
        while (t1 < ts1 && s_tc[t1 + 1 - ts0] - s_tc[t0 - ts0] <= CAP) ++t1;
        rel0 = s_tc[t0 - ts0];
        mw = s_tc[t1 - ts0] - rel0;
      }
      if (mw > 0) {
        const int64_t cw0 = (int64_t)t0 << kTileLog;
        const int nwords = (t1 - t0) * kTileWords;
        const int wpw = nwords / NW;
        const uint32_t cmax = (uint32_t)nwords * 32u;
        // products of the window, source chunk by source chunk; pass 1 sets
        // the bitmap, pass 2 folds values whose rank lies in [r0, r0 + mc)
        auto gather = [&](bool vals, int32_t r0, int32_t mc) {
          for (int64_t c0 = 0; c0 < tk.nsrc; c0 += BS) {
            const int nc = (int)((tk.nsrc - c0) < BS ? (tk.nsrc - c0) : BS);
            if (!one) {
              __syncthreads();
              load_src(c0, nc);
              __syncthreads();
            }
            int64_t len = 0;
            int32_t wo = 0;
            if (threadIdx.x < nc) {
              if (!split) {
                len = s_slen[threadIdx.x];
              } else {
                const int32_t* r = b.rpt + ((int64_t)s * b.nb + s_k[threadIdx.x]) * (G + 1);
                wo = r[t0 - ts0];
                len = r[t1 - ts0] - wo;
              }
            }
            int64_t total;
            const int64_t off = block_excl_scan<NW, int64_t>(len, s_wave, &total);
            s_off[threadIdx.x] = off;
            s_wo[threadIdx.x] = wo;
            __syncthreads();
            for (int64_t qb = (int64_t)wv * kBlock; qb < total; qb += (int64_t)NW * kBlock) {
              const int64_t qe = (qb + kBlock - 1) < (total - 1) ? (qb + kBlock - 1) : (total - 1);
              int a = 0, bb = nc - 1;
              while (a < bb) {
                const int mid = (a + bb + 1) >> 1;
                if (s_off[mid] <= qb) a = mid;
                else bb = mid - 1;
              }
              int e = a, f = nc - 1;
              while (e < f) {
                const int mid = (e + f + 1) >> 1;
                if (s_off[mid] <= qe) e = mid;
                else f = mid - 1;
              }
              int32_t cc[kUnroll];
              Acc vv[kUnroll];
              int ow = a;
#pragma unroll
              for (int u = 0; u < kUnroll; ++u) {
                const int64_t q = qb + u * kWave + lane_id();
                cc[u] = -1;
                if (q < total) {
                  int h2 = e;
                  while (ow < h2) {
                    const int mid = (ow + h2 + 1) >> 1;
                    if (s_off[mid] <= q) ow = mid;
                    else h2 = mid - 1;
                  }
                  const int64_t idx = s_sst[ow] + s_wo[ow] + (q - s_off[ow]);
                  cc[u] = (int32_t)(b.pcol[idx] - cw0);
                  if (vals) vv[u] = Sr::mul(s_a[ow], b.pval[idx]);
                }
              }
#pragma unroll
              for (int u = 0; u < kUnroll; ++u) {
                const int32_t c = cc[u];
                if ((uint32_t)c >= cmax) continue;
                if (!vals) {
                  atomicOr(&s_bits[c >> 5], 1u << (c & 31));
                } else {
                  const int w = c >> 5;
                  const int32_t rr = (int32_t)s_rank[w] + __popc(s_bits[w] & ((1u << (c & 31)) - 1u)) - r0;
                  if ((uint32_t)rr < (uint32_t)mc) Sr::lds_acc(&s_val[rr], vv[u]);
                }
              }
            }
            __syncthreads();
          }
        };
        gather(false, 0, 0);
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
        __syncthreads();
        int32_t wbase = 0, tot = 0;
#pragma unroll
        for (int u = 0; u < NW; ++u) {
          const int32_t v = s_wt[u];
          wbase += u < wv ? v : 0;
          tot += v;
        }
        if (threadIdx.x == 0 && tot != mw) atomicOr(err, 1);
        if (wbase)
          for (int it = 0; it < wpw; it += kWave) {
            const int w = wv * wpw + it + lane_id();
            s_rank[w] = (uint16_t)(s_rank[w] + wbase);
          }
        for (int32_t r0 = 0; r0 < mw; r0 += CAP) {
          const int32_t mc = (mw - r0) < CAP ? (mw - r0) : CAP;
          const bool last = r0 + mc >= mw;
          for (int x = threadIdx.x; x < mc; x += BS) s_val[x] = Sr::ident();
          __syncthreads();
          gather(true, r0, mc);
          // column-ordered write-out of ranks [r0, r0 + mc)
          for (int it = 0; it < wpw; it += kWave) {
            const int w = wv * wpw + it + lane_id();
            uint32_t bits = s_bits[w];
            int32_t r = s_rank[w];
            if (r + __popc(bits) > r0 && r < r0 + mc) {
              while (bits) {
                const int bt = __ffs((int)bits) - 1;
                bits &= bits - 1u;
                const int32_t rr = r - r0;
                if ((uint32_t)rr < (uint32_t)mc) {
                  const int64_t pos = tk.out + rel0 + r;
                  C.col[pos] = (int32_t)(cw0 + w * 32 + bt);
                  ((V*)C.val)[pos] = Sr::out(s_val[rr]);
                }
                ++r;
              }
            }
            if (last) s_bits[w] = 0u;
          }
          __syncthreads();
        }
      }
      t0 = t1;
    }
  });
}

}  // namespace sg
