// Column-slab path for the dense rows of a single product C = A (x).(+) B.
//
// B's columns are cut into slabs of 2^ls columns (one to eight 16384-column
// tiles).  A partition of B keeps, for slab s and B row k, the entries of
// B_k inside the slab contiguous:  pcol/pval[prow[s*nb + k] .. prow[s*nb + k + 1]).
// A dense row's work is then one task per (row, slab); every task finds each
// source's segment with one read of prow, and the tasks run in slab-major
// order, so at any moment the whole chip gathers from one slab of B.
//
//   symbolic  per task an LDS bitmap of the slab (16 KB at 2^17 columns);
//             per-tile popcounts become the row's per-tile output counts
//   numeric   bitmap + rank accumulator: pass 1 sets the slab's bitmap, a
//             scan turns it into per-word ranks, pass 2 folds every product
//             into the compacted slot rank(column) of an LDS value array,
//             and the bitmap walk writes the slab's entries in column order
//             (no sort, no hash probing).  Slabs with more entries than the
//             value array holds go to the tile/range tasks instead.
#pragma once

#include "sg_kernels.hpp"

namespace sg {

constexpr int kSlabLogMin = kTileLog;  // a slab is 1..8 column tiles
constexpr int kSlabLogMax = 17;
constexpr int kSlabWordsMax = 1 << (kSlabLogMax - 5);

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

// Row i of A (x) B restricted to one slab: one source per stored A_ik, its
// segment = the slab part of B_k in the partition.
template <class V, bool kVals>
struct SlabSrc {
  const int64_t* a_rowptr;
  const int32_t* a_col;
  const V* a_val;
  const int64_t* prow;
  const int32_t* pcol;
  const V* pval;
  int64_t nb;
  int64_t a0;
  int64_t sb;

  struct Item {
    V a;
  };

  SG_DEV int64_t bind(int64_t i, int32_t s) {
    a0 = a_rowptr[i];
    sb = (int64_t)s * nb;
    return a_rowptr[i + 1] - a0;
  }
  SG_DEV void load(int64_t j, Item& it, int64_t& start, int64_t& len) const {
    const int64_t e = a0 + j;
    const int32_t k = a_col[e];
    if constexpr (kVals) it.a = a_val[e];
    const int64_t* r = prow + sb + k;
    start = r[0];
    len = r[1] - start;
  }
  SG_DEV int32_t col(const Item&, int64_t idx) const { return pcol[idx]; }
  template <class Sr>
  SG_DEV typename Sr::Acc value(const Item& it, int64_t idx) const {
    return Sr::mul(it.a, pval[idx]);
  }
};

// ---- symbolic --------------------------------------------------------------------
// Task g = (slab s, dense row h) with s = g / nd: per-tile popcounts of the
// slab's bitmap are written raw to off2[h*(Tmax+1) + t]; k_off2_finish turns
// them into per-row offsets.
template <class Src, int BS>
__global__ __launch_bounds__(BS) void k_sym_slab(Src src0, Bins bins, int32_t S, int32_t ls, int32_t T,
                                                 int32_t Tmax, int32_t* off2, int32_t* ctr) {
  constexpr int NW = BS / kWave;
  using Item = typename Src::Item;
  __shared__ uint32_t s_bm[kSlabWordsMax];
  __shared__ Item s_item[BS];
  __shared__ int64_t s_start[BS], s_off[BS], s_wave[NW];
  __shared__ int64_t s_slot;
  const int nwords = 1 << (ls - 5);
  const int G = 1 << (ls - kTileLog);
  for (int x = threadIdx.x; x < nwords; x += BS) s_bm[x] = 0u;
  const int32_t* L = bins.list + bins.start[kBinDense0];
  const int64_t nd = dense_rows(bins);
  const uint32_t cmax = (uint32_t)nwords * 32u;
  for_each_queued(ctr, kListSymSlab, nd * S, &s_slot, [&](int64_t g) {
    const int32_t s = (int32_t)(g / nd);
    const int64_t h = g - (int64_t)s * nd;
    const int64_t i = L[h];
    Src sr = src0;
    const int64_t nsrc = sr.bind(i, s);
    const int64_t c0 = (int64_t)s << ls;
    __syncthreads();
    auto fetch = [&](const Item& it, int64_t idx) { return (int32_t)(sr.col(it, idx) - c0); };
    auto apply = [&](int32_t c) {
      if ((uint32_t)c < cmax) atomicOr(&s_bm[c >> 5], 1u << (c & 31));
    };
    for_each_product<BS, kUnroll>(sr, nsrc, s_item, s_start, s_off, s_wave, fetch, apply);
    __syncthreads();
    int32_t* o2 = off2 + h * (Tmax + 1);
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
// entries T..Tmax = the row's count, which also goes to cnt_out.
template <int BS>
__global__ __launch_bounds__(BS) void k_off2_finish(Bins bins, int32_t* off2, int32_t T, int32_t Tmax,
                                                    int64_t* cnt_out) {
  const int32_t* L = bins.list + bins.start[kBinDense0];
  const int64_t nd = dense_rows(bins);
  const int64_t w0 = ((int64_t)blockIdx.x * BS + threadIdx.x) >> 6;
  const int64_t nw = ((int64_t)gridDim.x * BS) >> 6;
  for (int64_t h = w0; h < nd; h += nw) {
    int32_t* o2 = off2 + h * (Tmax + 1);
    int32_t run = 0;
    for (int t0 = 0; t0 < T; t0 += kWave) {
      const int t = t0 + lane_id();
      const int32_t v = t < T ? o2[t] : 0;
      const int32_t inc = wave_incl_scan(v);
      if (t < T) o2[t] = run + inc - v;
      run += shfl(inc, kWave - 1);
    }
    for (int t = T + lane_id(); t <= Tmax; t += kWave) o2[t] = run;
    if (lane_id() == 0) cnt_out[L[h]] = run;
  }
}

// ---- numeric ---------------------------------------------------------------------
// Entries of a slab task's LDS value array (32 KB of accumulators).
template <class Sr>
constexpr int slab_cap() {
  return 32768 / (int)sizeof(typename Sr::Acc);
}

template <class Sr, class Src, int BS, int CAP>
__global__ __launch_bounds__(BS) void k_num_slab(Src src0, Bins bins, OutC C, const int32_t* off2, int32_t Tmax,
                                                 int32_t ls, const Task* tasks, const int32_t* book_off,
                                                 int32_t* ctr, int32_t* err) {
  constexpr int NW = BS / kWave;
  static_assert(NW * kWave <= (1 << (kSlabLogMin - 5)), "each wavefront owns a multiple of 64 bitmap words");
  using Item = typename Src::Item;
  using Acc = typename Sr::Acc;
  using V = typename Sr::V;
  __shared__ uint2 s_w[kSlabWordsMax];  // .x occupancy bits, .y rank of the word's first entry
  __shared__ Acc s_val[CAP];
  __shared__ Item s_item[BS];
  __shared__ int64_t s_start[BS], s_off[BS], s_wave[NW];
  __shared__ int32_t s_wt[NW];
  __shared__ int64_t s_slot;
  const int nwords = 1 << (ls - 5);
  const int wpw = nwords / NW;  // words per wavefront (a multiple of 64 for ls >= 14)
  const int G = 1 << (ls - kTileLog);
  const uint32_t cmax = (uint32_t)nwords * 32u;
  for (int x = threadIdx.x; x < nwords; x += BS) s_w[x].x = 0u;
  const int32_t* L = bins.list + bins.start[kBinDense0];
  const int32_t nd = dense_rows(bins);
  const int wv = wave_id();
  for_each_queued(ctr, kListSlab, (int64_t)ctr[kListSlab], &s_slot, [&](int64_t g) {
    const Task tk = bucket_task(tasks, book_off, Tmax, nd, (int32_t)g);
    const int32_t* o2 = off2 + (int64_t)tk.h * (Tmax + 1);
    const int32_t lo = o2[tk.t0], hi = o2[tk.t1];
    const int32_t m = hi - lo;
    const int32_t mm = m < CAP ? m : CAP;
    const int64_t i = L[tk.h];
    const int64_t base = C.rowptr[i] + lo;
    const int32_t s = tk.t0 / G;
    const int64_t c0 = (int64_t)s << ls;
    Src sr = src0;
    const int64_t nsrc = sr.bind(i, s);
    __syncthreads();
    // pass 1: the slab's column set
    auto f1 = [&](const Item& it, int64_t idx) { return (int32_t)(sr.col(it, idx) - c0); };
    auto a1 = [&](int32_t c) {
      if ((uint32_t)c < cmax) atomicOr(&s_w[c >> 5].x, 1u << (c & 31));
    };
    for_each_product<BS, kUnroll>(sr, nsrc, s_item, s_start, s_off, s_wave, f1, a1);
    __syncthreads();
    // ranks: wavefront wv owns words [wv*wpw, (wv+1)*wpw), lanes consecutive
    int32_t run = 0;
    for (int it = 0; it < wpw; it += kWave) {
      const int w = wv * wpw + it + lane_id();
      const int32_t pc = __popc(s_w[w].x);
      const int32_t inc = wave_incl_scan(pc);
      s_w[w].y = (uint32_t)(run + inc - pc);
      run += shfl(inc, kWave - 1);
    }
    if (lane_id() == 0) s_wt[wv] = run;
    for (int x = threadIdx.x; x < mm; x += BS) s_val[x] = Sr::ident();
    __syncthreads();
    int32_t wbase = 0, tot = 0;
#pragma unroll
    for (int u = 0; u < NW; ++u) {
      const int32_t v = s_wt[u];
      wbase += u < wv ? v : 0;
      tot += v;
    }
    if (threadIdx.x == 0 && (tot != m || m > CAP)) atomicOr(err, 1);
    if (wbase)
      for (int it = 0; it < wpw; it += kWave) s_w[wv * wpw + it + lane_id()].y += (uint32_t)wbase;
    __syncthreads();
    // pass 2: fold every product into its compacted slot
    auto f2 = [&](const Item& it, int64_t idx) {
      return ColVal<Acc>{(int32_t)(sr.col(it, idx) - c0), sr.template value<Sr>(it, idx)};
    };
    auto a2 = [&](const ColVal<Acc>& p) {
      if ((uint32_t)p.c >= cmax) return;
      const uint2 w = s_w[p.c >> 5];
      const int32_t r = (int32_t)w.y + __popc(w.x & ((1u << (p.c & 31)) - 1u));
      if (r < mm) Sr::lds_acc(&s_val[r], p.v);
    };
    for_each_product<BS, kUnroll>(sr, nsrc, s_item, s_start, s_off, s_wave, f2, a2);
    __syncthreads();
    // column-ordered write-out; clears the bitmap for the next task
    for (int it = 0; it < wpw; it += kWave) {
      const int w = wv * wpw + it + lane_id();
      uint32_t bits = s_w[w].x;
      int32_t r = (int32_t)s_w[w].y;
      while (bits) {
        const int b = __ffs((int)bits) - 1;
        bits &= bits - 1u;
        if (r < mm) {
          C.col[base + r] = (int32_t)(c0 + w * 32 + b);
          ((V*)C.val)[base + r] = Sr::out(s_val[r]);
        }
        ++r;
      }
      s_w[w].x = 0u;
    }
  });
}

}  // namespace sg
