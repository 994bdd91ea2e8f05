// Structural kernels and their launchers: row analysis and binning, tile
// bounds, the symbolic pass (semiring independent), prefix sums, fills and
// input validation.
#include "sg_launch.hpp"

namespace sg {

namespace {
constexpr int kAnaBS = 256;

// Per-(bin, block) scatter offsets within each bin and the per-bin totals.
// The histogram is bin-major (hist[b*nblk + k]: rows of block k in bin b),
// so workgroup b scans one contiguous row of it.
constexpr int kBinScanBS = 1024, kBinScanPer = 4;
__global__ __launch_bounds__(kBinScanBS) void k_bin_offsets(const int32_t* hist, int32_t nblk, int32_t* blk_off,
                                                            int32_t* bin_count) {
  __shared__ int32_t s_wave[kBinScanBS / kWave];
  const int64_t row = (int64_t)blockIdx.x * nblk;
  int32_t carry = 0;
  for (int32_t k0 = 0; k0 < nblk; k0 += kBinScanBS * kBinScanPer) {
    const int32_t base = k0 + (int32_t)threadIdx.x * kBinScanPer;
    int32_t v[kBinScanPer];
    int32_t sum = 0;
#pragma unroll
    for (int q = 0; q < kBinScanPer; ++q) {
      v[q] = base + q < nblk ? hist[row + base + q] : 0;
      sum += v[q];
    }
    int32_t tot;
    int32_t run = carry + block_excl_scan<kBinScanBS / kWave, int32_t>(sum, s_wave, &tot);
#pragma unroll
    for (int q = 0; q < kBinScanPer; ++q) {
      if (base + q < nblk) blk_off[row + base + q] = run;
      run += v[q];
    }
    carry += tot;
  }
  if (threadIdx.x == 0) bin_count[blockIdx.x] = carry;
}

// Bin starts: one wavefront scans the kNB (= 64) bin totals.
__global__ __launch_bounds__(kWave) void k_bin_starts(const int32_t* bin_count, int32_t* bin_start) {
  static_assert(kNB == kWave, "one lane per bin");
  const int32_t v = bin_count[threadIdx.x];
  bin_start[threadIdx.x] = wave_incl_scan(v) - v;
}

void bin_offsets(const int32_t* hist, int64_t nblk, int32_t* blk_off, int32_t* bin_start, int32_t* bin_count,
                 hipStream_t st) {
  hipLaunchKernelGGL(k_bin_offsets, dim3(kNB), dim3(kBinScanBS), 0, st, hist, (int32_t)nblk, blk_off, bin_count);
  hipLaunchKernelGGL(k_bin_starts, dim3(1), dim3(kWave), 0, st, (const int32_t*)bin_count, bin_start);
}

// Per B row, rp2[k*(T+1) + t] = number of entries of row k with column below
// t*16384 (t = 0..T).  One wavefront per row, lanes over t, binary search.
__global__ __launch_bounds__(256) void k_tile_bounds(const int64_t* rowptr, const int32_t* col, int64_t nrows,
                                                     int32_t T, int32_t lg, int32_t* rp2) {
  const int64_t w0 = ((int64_t)blockIdx.x * 256 + threadIdx.x) >> 6;
  const int64_t nw = ((int64_t)gridDim.x * 256) >> 6;
  for (int64_t k = w0; k < nrows; k += nw) {
    const int64_t s = rowptr[k], e = rowptr[k + 1];
    int32_t* r = rp2 + k * (T + 1);
    for (int t = lane_id(); t <= T; t += kWave) {
      const int64_t pos = (t == 0) ? s : (t == T ? e : lower_bound_col(col, s, e, (int64_t)t << lg));
      r[t] = (int32_t)(pos - s);
    }
  }
}

// ---- prefix sums over int64 (in place, inclusive) -----------------------------------
__global__ __launch_bounds__(kScanBS) void k_scan_reduce(const int64_t* a, int64_t n, int64_t* partial) {
  __shared__ int64_t s_wave[kScanBS / kWave];
  const int64_t base = (int64_t)blockIdx.x * kScanChunk;
  int64_t sum = 0;
#pragma unroll
  for (int q = 0; q < kScanPer; ++q) {
    const int64_t x = base + (int64_t)q * kScanBS + threadIdx.x;
    if (x < n) sum += a[x];
  }
  const int64_t tot = block_sum<kScanBS / kWave, int64_t>(sum, s_wave);
  if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

// Exclusive scan of the block partials by one block.
__global__ __launch_bounds__(kScanBS) void k_scan_partials(int64_t* partial, int64_t nblk) {
  __shared__ int64_t s_wave[kScanBS / kWave];
  int64_t carry = 0;
  for (int64_t b0 = 0; b0 < nblk; b0 += kScanBS) {
    const int64_t x = b0 + threadIdx.x;
    const int64_t v = x < nblk ? partial[x] : 0;
    int64_t tot;
    const int64_t ex = block_excl_scan<kScanBS / kWave, int64_t>(v, s_wave, &tot);
    if (x < nblk) partial[x] = carry + ex;
    carry += tot;
  }
}

__global__ __launch_bounds__(kScanBS) void k_scan_apply(int64_t* a, int64_t n, const int64_t* partial) {
  __shared__ int64_t s_wave[kScanBS / kWave];
  const int64_t base = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * kScanPer;
  int64_t v[kScanPer];
  int64_t sum = 0;
#pragma unroll
  for (int q = 0; q < kScanPer; ++q) {
    const int64_t x = base + q;
    v[q] = x < n ? a[x] : 0;
    sum += v[q];
  }
  int64_t tot;
  int64_t run = partial[blockIdx.x] + block_excl_scan<kScanBS / kWave, int64_t>(sum, s_wave, &tot);
#pragma unroll
  for (int q = 0; q < kScanPer; ++q) {
    run += v[q];
    const int64_t x = base + q;
    if (x < n) a[x] = run;
  }
}


template <class Rows>
void analyze_rows(const Rows& rows, const RowSource& r, const Policy& pol, const int64_t* c_rowptr, int64_t* p,
                  int32_t* nt, uint8_t* bin, int32_t* hist, int32_t* blk_off, int32_t* bin_start, int32_t* bin_count,
                  int32_t* list, int64_t* cnt_out, hipStream_t st) {
  const int64_t nblk = analyze_blocks(r.nrows);
  hipLaunchKernelGGL((k_analyze<Rows, kAnaBS>), dim3(nblk), dim3(kAnaBS), 0, st, rows, r.nrows, pol, c_rowptr, p,
                     nt, bin, hist, cnt_out);
  bin_offsets(hist, nblk, blk_off, bin_start, bin_count, st);
  hipLaunchKernelGGL(k_bin_scatter<kAnaBS>, dim3(nblk), dim3(kAnaBS), 0, st, bin, r.nrows, blk_off, bin_start, list);
}

// Rows of a hash bin (up to 2^(LGS-1) products) whose B has at most 65536
// columns: a workgroup per row over an LDS bitmap of the columns (1024 words
// when B has at most 32768 columns, else 2048).  False: B is wider.
template <class Rows, int LGS>
bool sym_bitmap_rows(const Rows& rows, const BinPlan& plan, int bin, int64_t* cnt_out, int cus, hipStream_t st) {
  constexpr int kBS = 256, U = row_unroll(1 << (LGS - 1), kBS);
  const int64_t cols = (int64_t)rows.Tmax * kTile;
  const int n = plan.count[bin];
  if (cols <= (int64_t)32 * 1024) {
    auto kb = k_sym_bitmap_row<Rows, 1024, kBS, U>;
    static int occb = occupancy(kb, kBS);
    hipLaunchKernelGGL(kb, dim3(grid_for(n, 1, cus * occb * 4)), dim3(kBS), 0, st, rows, plan.bins, bin, cnt_out);
    return true;
  }
  if (cols <= (int64_t)32 * 2048) {
    auto kb = k_sym_bitmap_row<Rows, 2048, kBS, U>;
    static int occb = occupancy(kb, kBS);
    hipLaunchKernelGGL(kb, dim3(grid_for(n, 1, cus * occb * 4)), dim3(kBS), 0, st, rows, plan.bins, bin, cnt_out);
    return true;
  }
  return false;
}

template <class Rows, int LGS, int BS>
void sym_hash_one(const Rows& rows, const BinPlan& plan, int bin, int64_t* cnt_out, int cus, hipStream_t st,
                  bool merge) {
  const int n = plan.count[bin];
  if (n == 0) return;
  if (sym_bitmap_rows<Rows, LGS>(rows, plan, bin, cnt_out, cus, st)) return;
  if (merge) {
    // wider B: the rows' sorted segments merged in LDS, columns only
    auto km = k_sym_merge_row<Rows, 1 << (LGS - 1), 512>;
    static int occm = occupancy(km, 512);
    hipLaunchKernelGGL(km, dim3(grid_for(n, 1, cus * occm * 4)), dim3(512), 0, st, rows, plan.bins, bin, cnt_out);
    return;
  }
  auto k = k_sym_hash<Rows, LGS, BS>;
  static int occ = occupancy(k, BS);
  hipLaunchKernelGGL(k, dim3(grid_for(n, 1, cus * occ * 4)), dim3(BS), 0, st, rows, plan.bins, bin, cnt_out);
}

template <class Rows, int LGS>
void sym_hash_wave_one(const Rows& rows, const BinPlan& plan, int bin, int64_t* cnt_out, int cus, hipStream_t st) {
  const int n = plan.count[bin];
  if (n == 0) return;
  if constexpr (LGS >= 10) {
    if (sym_bitmap_rows<Rows, LGS>(rows, plan, bin, cnt_out, cus, st)) return;
  }
  constexpr int BS = 256;
  auto k = k_sym_hash_wave<Rows, LGS, BS>;
  static int occ = occupancy(k, BS);
  hipLaunchKernelGGL(k, dim3(grid_for(n, BS / kWave, cus * occ * 4)), dim3(BS), 0, st, rows, plan.bins, bin, cnt_out);
}

template <class Rows>
void sym_dense_rows(const Rows& rows, const BinPlan& plan, int64_t* cnt_out, int32_t* off2, int cus,
                    hipStream_t st) {
  const int nd = plan.ndense();
  if (nd == 0) return;
  if (rows.Tmax <= 2) {
    // narrow B: a bitmap of two or four tiles, 256-thread workgroups
    auto k = k_sym_dense<Rows, 2, 256>;
    static int occ = occupancy(k, 256);
    hipLaunchKernelGGL(k, dim3(grid_for(nd, 1, cus * occ * 2)), dim3(256), 0, st, rows, plan.bins, cnt_out, off2);
    return;
  }
  if (rows.Tmax <= 4) {
    auto k = k_sym_dense<Rows, 4, 256>;
    static int occ = occupancy(k, 256);
    hipLaunchKernelGGL(k, dim3(grid_for(nd, 1, cus * occ * 2)), dim3(256), 0, st, rows, plan.bins, cnt_out, off2);
    return;
  }
  // bitmaps of 16 or 32 tiles (32 or 64 KB) leave room for several
  // 512-thread workgroups per CU where the 64-tile one fits one
  if (rows.Tmax <= 16) {
    auto k = k_sym_dense<Rows, 16, 512>;
    static int occ = occupancy(k, 512);
    hipLaunchKernelGGL(k, dim3(grid_for(nd, 1, cus * occ * 2)), dim3(512), 0, st, rows, plan.bins, cnt_out, off2);
    return;
  }
  if (rows.Tmax <= 32) {
    auto k = k_sym_dense<Rows, 32, 512>;
    static int occ = occupancy(k, 512);
    hipLaunchKernelGGL(k, dim3(grid_for(nd, 1, cus * occ * 2)), dim3(512), 0, st, rows, plan.bins, cnt_out, off2);
    return;
  }
  constexpr int BS = sizeof(typename Rows::Src::Item) <= 8 ? 1024 : 512;
  auto k = k_sym_dense<Rows, kSymTiles, BS>;
  static int occ = occupancy(k, BS);
  hipLaunchKernelGGL(k, dim3(grid_for(nd, 1, cus * occ * 2)), dim3(BS), 0, st, rows, plan.bins, cnt_out, off2);
}

template <class Rows>
void symbolic_rows(const Rows& rows, const BinPlan& plan, int64_t* cnt_out, int32_t* off2, int cus,
                   const Marks& marks, hipStream_t st, bool dense, bool merge) {
  marks.mark(kPhSymSmall, 1);
  if (plan.count[kBinSmall]) {
    auto k = k_sym_small<Rows>;
    static int occ = occupancy(k, 256);
    hipLaunchKernelGGL(k, dim3(grid_for(plan.count[kBinSmall], 4, cus * occ * 4)), dim3(256), 0, st, rows,
                       plan.bins, kBinSmall, cnt_out);
  }
  marks.mark(kPhSymSmall, 0);
  marks.mark(kPhSymHash, 1);
  // hash bins hold tables of 2^8 .. 2^13 keys (symbolic tables start at 256);
  // rows of up to 1024 products take one wavefront each
  sym_hash_wave_one<Rows, 8>(rows, plan, kBinHash0 + 1, cnt_out, cus, st);
  sym_hash_wave_one<Rows, 9>(rows, plan, kBinHash0 + 2, cnt_out, cus, st);
  sym_hash_wave_one<Rows, 10>(rows, plan, kBinHash0 + 3, cnt_out, cus, st);
  sym_hash_wave_one<Rows, 11>(rows, plan, kBinHash0 + 4, cnt_out, cus, st);
  sym_hash_one<Rows, 12, 512>(rows, plan, kBinHash0 + 5, cnt_out, cus, st, merge);
  sym_hash_one<Rows, 13, 512>(rows, plan, kBinHash0 + 6, cnt_out, cus, st, merge);
  marks.mark(kPhSymHash, 0);
  if (!dense) return;
  marks.mark(kPhSymDense, 1);
  marks.mark(kPhSymDenseBitmap, 1);
  sym_dense_rows(rows, plan, cnt_out, off2, cus, st);
  marks.mark(kPhSymDenseBitmap, 0);
  marks.mark(kPhSymDense, 0);
}

// Dense rows of a single product over the column-slab partition.
void sym_slab(const RowSource& r, const BinPlan& plan, int64_t* cnt_out, int32_t* off2, int cus, const Marks& marks,
              hipStream_t st) {
  const int nd = plan.ndense();
  if (nd == 0) return;
  const int32_t G = 1 << (r.ls - kTileLog);
  const SlabB<uint8_t> b{r.prow, r.pbit, nullptr, r.rpt, r.b_nrows, G, r.T};
  hipLaunchKernelGGL(k_fill<int32_t>, dim3(grid_for(kCtrInts, 256, 64)), dim3(256), 0, st, r.qctr, (int64_t)kCtrInts,
                     (int32_t)0);
  constexpr int BS = 256;
  auto k = r.gather32 ? k_sym_slab<BS, true> : k_sym_slab<BS, false>;
  static int occ = occupancy(k_sym_slab<BS, true>, BS);
  const int grid = cus * occ > kQueues ? cus * occ : kQueues;
  marks.mark(kPhSymDenseBitmap, 1);
  hipLaunchKernelGGL(k, dim3(grid), dim3(BS), 0, st, b, r.drow, r.a_col, plan.bins, r.S, off2, r.spn, r.qctr);
  marks.mark(kPhSymDenseBitmap, 0);
  hipLaunchKernelGGL(k_off2_finish<256>, dim3(grid_for(nd, 4, cus * 16)), dim3(256), 0, st, plan.bins, r.drow, off2,
                     r.T, cnt_out);
}

bool use_slab(const RowSource& r) { return r.mode == kModeProduct && r.S > 0; }

__global__ __launch_bounds__(256) void k_validate(const int64_t* rowptr, const int32_t* col, int64_t nrows,
                                                  int64_t ncols, int64_t nnz, int32_t* flag) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < nrows; i += (int64_t)gridDim.x * 256) {
    const int64_t s = rowptr[i], e = rowptr[i + 1];
    bool bad = (i == 0 && s != 0) || e < s || (i == nrows - 1 && e != nnz) || s < 0 || e > nnz;
    if (!bad) {
      int64_t prev = -1;
      for (int64_t x = s; x < e; ++x) {
        const int64_t c = col[x];
        if (c <= prev || c >= ncols) {
          bad = true;
          break;
        }
        prev = c;
      }
    }
    if (bad) atomicOr(flag, 1);
  }
}
}  // namespace

int64_t analyze_blocks(int64_t nrows) { return (nrows + kAnaBS - 1) / kAnaBS; }

void launch_analyze(const RowSource& r, const Policy& pol, const int64_t* c_rowptr, int64_t* p, int32_t* nt,
                    uint8_t* bin, int32_t* hist, int32_t* blk_off, int32_t* bin_start, int32_t* bin_count,
                    int32_t* list, int64_t* cnt_out, hipStream_t st) {
  with_rows<uint8_t, false>(r, [&](const auto& rows) {
    analyze_rows(rows, r, pol, c_rowptr, p, nt, bin, hist, blk_off, bin_start, bin_count, list, cnt_out, st);
  });
}

void launch_rebin(const int64_t* p, const int32_t* nt, const int64_t* c_rowptr, int64_t nrows, const Policy& pol,
                  uint8_t* bin, int32_t* hist, int32_t* blk_off, int32_t* bin_start, int32_t* bin_count,
                  int32_t* list, hipStream_t st) {
  const int64_t nblk = analyze_blocks(nrows);
  hipLaunchKernelGGL(k_rebin<kAnaBS>, dim3(nblk), dim3(kAnaBS), 0, st, p, nt, c_rowptr, nrows, pol, bin, hist);
  bin_offsets(hist, nblk, blk_off, bin_start, bin_count, st);
  hipLaunchKernelGGL(k_bin_scatter<kAnaBS>, dim3(nblk), dim3(kAnaBS), 0, st, bin, nrows, blk_off,
                     (const int32_t*)bin_start, list);
}

void launch_tile_bounds(const int64_t* rowptr, const int32_t* col, int64_t nrows, int32_t T, int32_t* rp2, int cus,
                        hipStream_t st) {
  if (nrows == 0) return;
  hipLaunchKernelGGL(k_tile_bounds, dim3(grid_for(nrows, 4, cus * 16)), dim3(256), 0, st, rowptr, col, nrows, T,
                     (int32_t)kTileLog, rp2);
}

template <class V>
void slab_scatter(const int64_t* b_rowptr, const int32_t* b_col, const void* b_val, int64_t nb, int64_t nnz,
                  int32_t ls, int32_t S, const int32_t* bnd, const int64_t* prow, int32_t* pbit, void* pcv,
                  int32_t* perm, bool cols, bool vals, int32_t* err, int cus, hipStream_t st) {
  const dim3 g(grid_for(nb, 256, cus * 16)), b(256);
  const V* bv = (const V*)b_val;
  ColV<V>* cv = (ColV<V>*)pcv;
  if (cols && vals)
    hipLaunchKernelGGL((k_slab_scatter<V, true, true>), g, b, 0, st, b_rowptr, b_col, bv, nb, ls, S, bnd, prow, pbit,
                       cv, perm, err);
  else if (cols)
    hipLaunchKernelGGL((k_slab_scatter<V, true, false>), g, b, 0, st, b_rowptr, b_col, bv, nb, ls, S, bnd, prow,
                       pbit, cv, perm, err);
  else if (vals && perm)
    hipLaunchKernelGGL((k_slab_perm_cv<V>), dim3(grid_for(nnz, 256, cus * 16)), b, 0, st, b_col, bv,
                       (const int32_t*)perm, nnz, cv);
  else if (vals)
    hipLaunchKernelGGL((k_slab_scatter<V, false, true>), g, b, 0, st, b_rowptr, b_col, bv, nb, ls, S, bnd, prow,
                       pbit, cv, (int32_t*)nullptr, err);
}

void launch_slab_partition(const int64_t* b_rowptr, const int32_t* b_col, const void* b_val, int vbytes, int64_t nb,
                           int64_t nnz, int32_t ls, int32_t S, int32_t T, int32_t* bnd, int32_t* rpt, int64_t* prow,
                           int64_t* partial, int32_t* pbit, void* pval, int32_t* perm, bool cols, bool vals,
                           int32_t* err, int cus, hipStream_t st) {
  if (nb <= 0) return;
  if (cols) {
    // entries that contradict the bounds leave their slot unwritten; code 0
    // there keeps every bitmap code in range
    hipLaunchKernelGGL(k_fill<int32_t>, dim3(grid_for(nnz, 256, cus * 16)), dim3(256), 0, st, pbit, nnz, (int32_t)0);
    hipLaunchKernelGGL(k_slab_bounds<256>, dim3(grid_for(nb, 4, cus * 16)), dim3(256), 0, st, b_rowptr, b_col, nb, T,
                       (int32_t)(1 << (ls - kTileLog)), S, bnd, rpt);
    hipLaunchKernelGGL(k_slab_counts<256>, dim3(grid_for((int64_t)S * nb, 256, cus * 16)), dim3(256), 0, st,
                       (const int32_t*)bnd, nb, S, prow);
    launch_scan_inclusive(prow + 1, (int64_t)S * nb, partial, st);
  }
  switch (vbytes) {
    case 1:
      slab_scatter<uint8_t>(b_rowptr, b_col, b_val, nb, nnz, ls, S, bnd, prow, pbit, pval, perm, cols, vals, err, cus,
                            st);
      break;
    case 4:
      slab_scatter<uint32_t>(b_rowptr, b_col, b_val, nb, nnz, ls, S, bnd, prow, pbit, pval, perm, cols, vals, err,
                             cus, st);
      break;
    default:
      slab_scatter<uint64_t>(b_rowptr, b_col, b_val, nb, nnz, ls, S, bnd, prow, pbit, pval, perm, cols, vals, err,
                             cus, st);
      break;
  }
}

void launch_symbolic(const RowSource& r, const BinPlan& plan, int64_t* cnt_out, int32_t* off2, int cus,
                     const Marks& marks, hipStream_t st) {
  const bool slab = use_slab(r);
  with_rows<uint8_t, false>(r,
                            [&](const auto& rows) {
                              symbolic_rows(rows, plan, cnt_out, off2, cus, marks, st, !slab, r.merge_rows != 0);
                            });
  if (slab) {
    marks.mark(kPhSymDense, 1);
    sym_slab(r, plan, cnt_out, off2, cus, marks, st);
    marks.mark(kPhSymDense, 0);
  }
}

void launch_symbolic_dense(const RowSource& r, const BinPlan& plan, int64_t* cnt_out, int32_t* off2, int cus,
                           hipStream_t st) {
  if (use_slab(r)) {
    sym_slab(r, plan, cnt_out, off2, cus, Marks{}, st);
    return;
  }
  with_rows<uint8_t, false>(r, [&](const auto& rows) { sym_dense_rows(rows, plan, cnt_out, off2, cus, st); });
}

void launch_dense_rows(const BinPlan& plan, const int64_t* a_rowptr, DenseRow* dr, int cus, hipStream_t st) {
  const int nd = plan.ndense();
  if (nd == 0) return;
  hipLaunchKernelGGL(k_dense_rows<256>, dim3(grid_for(nd, 256, cus * 8)), dim3(256), 0, st, plan.bins, a_rowptr, dr);
}

int64_t scan_partials_len(int64_t n) { return (n + kScanChunk - 1) / kScanChunk + 1; }

void launch_scan_inclusive(int64_t* a, int64_t n, int64_t* partial, hipStream_t st) {
  if (n <= 0) return;
  const int64_t nblk = (n + kScanChunk - 1) / kScanChunk;
  hipLaunchKernelGGL(k_scan_reduce, dim3(nblk), dim3(kScanBS), 0, st, a, n, partial);
  hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(kScanBS), 0, st, partial, nblk);
  hipLaunchKernelGGL(k_scan_apply, dim3(nblk), dim3(kScanBS), 0, st, a, n, partial);
}

void launch_fill_i64(int64_t* p, int64_t n, int64_t v, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill<int64_t>, dim3(grid_for(n, 256, 4096)), dim3(256), 0, st, p, n, v);
}

void launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill<int32_t>, dim3(grid_for(n, 256, 4096)), dim3(256), 0, st, p, n, v);
}

void launch_validate(const int64_t* rowptr, const int32_t* col, int64_t nrows, int64_t ncols, int64_t nnz,
                     int32_t* flag, hipStream_t st) {
  if (nrows == 0) return;
  hipLaunchKernelGGL(k_validate, dim3(grid_for(nrows, 256, 4096)), dim3(256), 0, st, rowptr, col, nrows, ncols, nnz,
                     flag);
}

}  // namespace sg
