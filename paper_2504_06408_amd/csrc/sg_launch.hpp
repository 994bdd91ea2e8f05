// Host-side launch contexts and launcher templates.  The structural launchers
// (analysis, binning, tile bounds, symbolic, scans) live in k_struct.hip; one
// numeric launcher per semiring lives in num_<semiring>.hip.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "sg_kernels.hpp"
#include "sg_slab.hpp"

namespace sg {

enum RowMode { kModeProduct = 0, kModeMerge = 1, kModeBatchProducts = 2, kModeBatchMerges = 3 };

// Everything a symbolic or numeric launch needs to describe its rows.
struct RowSource {
  int mode;
  int merge_rows = 1;  // symbolic hash bins of 2^12 slots and up over wide B: the merge kernel
  // single product
  const int64_t* a_rowptr;
  const int32_t* a_col;
  const void* a_val;
  const int64_t* b_rowptr;
  const int32_t* b_col;
  const void* b_val;
  int64_t b_nrows;
  const int32_t* rp2;
  // single merge
  const PartDesc* parts;
  int32_t nparts;
  // batches
  const ProbDesc* probs;
  const GroupDesc* groups;
  const int64_t* rbase;
  const int32_t* coarse;  // owner of every 256th global row (see owner_of)
  int32_t ntable;
  // all
  int64_t nrows;  // (global) rows
  int64_t ncols;  // columns of C (single modes)
  int32_t T;      // column tiles (single modes) or the largest over the batch
  // column-slab partition of B (single product; S = 0: not used)
  const int64_t* prow;
  const int32_t* pbit;
  const void* pval;       // numeric partition: (column, value) pairs (ColV)
  const int32_t* rpt;     // tile offsets inside each slab segment
  const DenseRow* drow;   // per dense row: its A row
  uint4* spn;             // span counts of the dense rows' tiles (after off2 in its buffer)
  bool gather32;          // the symbolic slab pass may gather at 32-bit offsets
  int64_t b_nnz;          // entries of the partitioned B
  int32_t ls, S;
  int32_t* qctr;  // counter block (kCtrInts ints) of the slab symbolic pass
};

struct BinPlan {
  Bins bins;
  int32_t count[kNB];  // host copy (graph mode: a large placeholder per bin)
  int32_t start[kNB];
  bool graph = false;  // counts unknown on the host: launch every kernel
  int32_t ndense() const {
    int64_t s = 0;
    for (int b = kBinDense0; b < kNB; ++b) s += count[b];
    return s > INT32_MAX ? INT32_MAX : (int32_t)s;
  }
};

// Optional per-phase hook (records timing events); fn may be null.
struct Marks {
  void (*fn)(void* ctx, int phase, int begin) = nullptr;
  void* ctx = nullptr;
  void mark(int phase, int begin) const {
    if (fn) fn(ctx, phase, begin);
  }
};

// phase ids (mirror SG_PHASE_* of the public header)
enum { kPhSymAnalyze = 0, kPhSymBounds, kPhSymSmall, kPhSymHash, kPhSymDense, kPhSymScan, kPhNumAnalyze, kPhNumSmall,
       kPhNumHash, kPhNumDense, kPhSymDenseBitmap, kPhNumDenseSlab, kPhNumDenseTiles, kPhNumDenseRanges, kNPhases };

struct NumCtx {
  Marks marks;
  RowSource src;
  BinPlan plan;
  OutC C;
  const int32_t* off2;
  const uint4* spn;  // span counts of the slab path's tiles (after off2)
  int32_t* err;
  int32_t* task_ctr;  // counter block of kCtrInts ints (list totals, queue cursors)
  Task* tasks;        // tile, range and slab task lists of task_cap entries each
  int64_t task_cap;   // >= dense rows x tiles
  SlabTask* slab_tasks;  // slab path: dense rows x slabs tasks ...
  int32_t* slab_book;    // ... and their bucket bookkeeping (6*T + 3 ints)
  int32_t tile_min;
  int cus;
  int comp_dense;     // float sums: dense rows use compensated accumulation
  int32_t light_cap;  // slab path: most entries of a light task (0: the LDS capacity)
  int merge_rows;     // hash bins of 2^kMergeRowLgMin slots and up over wide B: merge kernel
};

// Bytes of the dense-row task buffer: three task lists of task_cap entries
// and the bucket bookkeeping (6*T + 3 ints) after them.
inline size_t task_buffer_bytes(int64_t task_cap, int32_t T) {
  return sizeof(Task) * 3 * (size_t)task_cap + sizeof(int32_t) * (6 * (size_t)T + 3);
}
inline int32_t* task_book(const NumCtx& c) { return (int32_t*)(c.tasks + 3 * c.task_cap); }

// Slab width 2^ls for a product with ncols columns: about an eighth of the
// columns, clamped to 1..8 column tiles.
inline int32_t slab_log(int64_t ncols) {
  int32_t ls = kSlabLogMin;
  while (ls < kSlabLogMax && ((int64_t)1 << ls) * 8 < ncols) ++ls;
  return ls;
}
// The same with a tuned width (0: the default above).
inline int32_t slab_log(int64_t ncols, int32_t tuned) {
  return tuned >= kSlabLogMin && tuned <= kSlabLogMax ? tuned : slab_log(ncols);
}
inline int32_t slab_count(int64_t ncols, int32_t ls) {
  return (int32_t)((ncols + ((int64_t)1 << ls) - 1) >> ls);
}

template <class V, bool kVals>
inline SpgemmSrc<V, kVals> make_spgemm_src(const RowSource& r) {
  SpgemmSrc<V, kVals> s{};
  s.a_rowptr = r.a_rowptr;
  s.a_col = r.a_col;
  s.a_val = (const V*)r.a_val;
  s.b_rowptr = r.b_rowptr;
  s.b_col = r.b_col;
  s.b_val = (const V*)r.b_val;
  s.rp2 = r.rp2;
  s.T = r.T;
  s.ncols = r.ncols;
  return s;
}

template <class V>
inline MergeSrc<V> make_merge_src(const RowSource& r) {
  MergeSrc<V> s{};
  s.parts = r.parts;
  s.nparts = r.nparts;
  s.T = r.T;
  s.ncols = r.ncols;
  return s;
}

// Calls f(rows) with the row set of r's mode; V is the value type the
// sources read (uint8_t and kVals = false for structure-only passes).
template <class V, bool kVals, class F>
inline void with_rows(const RowSource& r, F&& f) {
  switch (r.mode) {
    case kModeProduct: f(OneRows<SpgemmSrc<V, kVals>>{make_spgemm_src<V, kVals>(r), r.T}); break;
    case kModeMerge: f(OneRows<MergeSrc<V>>{make_merge_src<V>(r), r.T}); break;
    case kModeBatchProducts: f(TableRows<V, kVals>{r.probs, r.rbase, r.coarse, r.ntable, r.T}); break;
    case kModeBatchMerges: f(MergeTableRows<V>{r.groups, r.rbase, r.coarse, r.ntable, r.T}); break;
  }
}

template <class K>
inline int occupancy(K kernel, int bs) {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kernel, bs, 0) != hipSuccess || n < 1) n = 1;
  return n;
}

inline int grid_for(int64_t work, int per_block, int cap) {
  int64_t g = (work + per_block - 1) / per_block;
  if (g > cap) g = cap;
  return g < 1 ? 1 : (int)g;
}

// A numeric kernel to launch: a kernel compiled into the library (fn, its
// host stub) or a function of a module compiled at run time (mod), with the
// workgroups of its block size that fit one CU.
struct KRef {
  const void* fn = nullptr;
  hipFunction_t mod = nullptr;
  int occ = 1;
  bool ok() const { return fn != nullptr || mod != nullptr; }
};

inline KRef kref_static(const void* fn, int bs) {
  KRef k;
  k.fn = fn;
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, fn, bs, 0) == hipSuccess && n >= 1) k.occ = n;
  return k;
}

inline KRef kref_module(hipFunction_t f, int bs) {
  KRef k;
  k.mod = f;
  int n = 0;
  if (f && hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(&n, f, bs, 0) == hipSuccess && n >= 1) k.occ = n;
  return k;
}

// Launch k with kernel arguments args, which must have exactly the types of
// the kernel's parameters (they are passed by address).
template <class... A>
inline void klaunch(const KRef& k, dim3 grid, dim3 block, hipStream_t st, A... args) {
  void* p[] = {(void*)&args...};
  if (k.mod) (void)hipModuleLaunchKernel(k.mod, grid.x, grid.y, grid.z, block.x, block.y, block.z, 0, st, p, nullptr);
  else (void)hipLaunchKernel(k.fn, grid, block, p, 0, st);
}

// Dense rows: build the tile and range task lists from the per-tile counts,
// then run the two persistent task kernels.
constexpr int kRangeLg = 12;          // range tasks: hash table of 4096 slots
constexpr int kRangeCap = 2048;       // entries per range task
constexpr int kTileMinDefault = 2048; // entries that make a tile a dense-tile task (= kRangeCap)

// Block sizes of the numeric kernels (shared by the launchers and by the
// run-time compilation of semirings, which instantiates the same kernels).
// Hash bins: table of 2^(7+k) slots, k = 0..6; the largest table with 4-byte
// accumulators leaves LDS for 1024 threads.
constexpr int kHashBins = 7;
constexpr int hash_bs(int k, int acc_bytes) { return k < 4 ? 256 : (k < 6 ? 512 : (acc_bytes <= 4 ? 1024 : 512)); }
// Dense tiles: 8-byte accumulators need the whole LDS for one 16384-slot
// tile, so a 1024-thread workgroup (16 waves) when the per-source items are
// small.
constexpr int tiles_bs(int acc_bytes, int item_bytes) { return (acc_bytes >= 8 && item_bytes <= 8) ? 1024 : 512; }
constexpr int ranges_bs(int acc_bytes) { return acc_bytes >= 8 ? 256 : 512; }
constexpr int kSlabBS = 512;

// The library's own kernels (compiled in for the five semirings).
struct KLib {
  template <class Sr, class Rows>
  KRef small() const {
    static const KRef k = kref_static((const void*)k_num_small<Sr, Rows>, 256);
    return k;
  }
  template <class Sr, class Rows, int LGS, int BS>
  KRef hash() const {
    static const KRef k = kref_static((const void*)k_num_hash<Sr, Rows, LGS, BS>, BS);
    return k;
  }
  template <class Sr, int kCap, bool kNarrow>
  KRef slab() const {
    static const KRef k = kref_static((const void*)k_num_slab<Sr, typename Sr::V, kSlabBS, kCap, kNarrow>, kSlabBS);
    return k;
  }
  template <class Sr, bool kNarrow>
  KRef heavy() const {
    static const KRef k = kref_static((const void*)k_num_slab_heavy<Sr, typename Sr::V, kSlabBS, kNarrow>, kSlabBS);
    return k;
  }
  template <class Sr, class Rows, int BS>
  KRef tiles() const {
    static const KRef k = kref_static((const void*)k_num_tiles<Sr, Rows, BS>, BS);
    return k;
  }
  template <class Sr, class Rows, int LGS, int BS>
  KRef ranges() const {
    static const KRef k = kref_static((const void*)k_num_ranges<Sr, Rows, LGS, BS>, BS);
    return k;
  }
  template <class Sr, class Rows, int CAP, int BS>
  KRef merge_row() const {
    static const KRef k = kref_static((const void*)k_num_merge_row<Sr, Rows, CAP, BS>, BS);
    return k;
  }
  template <class Sr, class Rows, int WORDS, int CAP, int BS>
  KRef wave_bitmap() const {
    static const KRef k = kref_static((const void*)k_num_wave_bitmap<Sr, Rows, WORDS, CAP, BS>, BS);
    return k;
  }
  template <class Sr, class Rows, int WORDS, int CAP, int BS>
  KRef bitmap_row() const {
    static const KRef k = kref_static((const void*)k_num_bitmap_row<Sr, Rows, WORDS, CAP, BS>, BS);
    return k;
  }
  template <class Sr, class Rows, int WORDS, int CAP, int BS>
  KRef bitmap_dense() const {
    static const KRef k = kref_static((const void*)k_num_bitmap_dense<Sr, Rows, WORDS, CAP, BS>, BS);
    return k;
  }
  template <class Sr, class Rows, int WORDS, int CAP, int BS>
  KRef ranges_bitmap() const {
    static const KRef k = kref_static((const void*)k_num_ranges_bitmap<Sr, Rows, WORDS, CAP, BS>, BS);
    return k;
  }
  template <class Sr, class Rows, int WORDS, int CAP, int BS>
  KRef range_runs() const {
    static const KRef k = kref_static((const void*)k_num_range_runs<Sr, Rows, WORDS, CAP, BS>, BS);
    return k;
  }
};

// Hash rows whose columns all lie below 32 * kWaveWords (products whose B has
// at most four column tiles) need no hash table: a bitmap of the columns and
// per-word ranks place every entry.  Rows of up to 2^kWaveLgMax / 2 entries
// run one wavefront per row, larger ones one workgroup per row over a shared
// bitmap (the hash bins of 2^kRowBitmapLgMin slots and up).
constexpr int kWaveWords = 2048;
constexpr int kWaveWordsHalf = 1024;
constexpr int kWaveBS = 128;
constexpr int kWaveLgMax = 9;
constexpr int kRowBitmapBS = 256;
constexpr int kRowBitmapLgMin = 10;

// Hash rows over wider B of more than 2^(kMergeRowLgMin-2) products are
// merged from their sorted segments (k_num_merge_row): the (key, value)
// buffers take 2*CAP*(4+acc) bytes of LDS, so rows of 4096 products with
// 4-byte accumulators run two 512-thread workgroups per CU, and with 8-byte
// ones one of 1024 threads; rows of up to 256 products take one wavefront.
constexpr int kMergeRowLgMin = 8;
constexpr int merge_row_bs(int cap, int acc_bytes) {
  return cap <= 256 ? 64 : (cap <= 1024 ? 256 : (acc_bytes >= 8 && cap > 2048 ? 1024 : 512));
}

// Dense rows over narrow B: whole rows of up to dense_bitmap_cap entries in
// one 1024-thread workgroup per CU (bitmap, ranks, the accumulators with
// their 16-bit columns and the iterator's arrays fill the 160 KB of LDS).
constexpr int kDenseBitmapBS = 1024;
constexpr int kRangeBitmapBS = 256;
template <class Sr, class Rows, int WORDS>
constexpr int dense_bitmap_cap() {
  constexpr int fixed = WORDS * 6 + kDenseBitmapBS * ((int)sizeof(typename Rows::Src::Item) + 16) + 1024 +
                        (Rows::Src::kParts ? 16 * kLdsParts : 0);
  constexpr int cap = ((160 * 1024 - fixed) / ((int)sizeof(typename Sr::Acc) + 2)) & ~255;
  return cap < 65280 ? cap : 65280;  // ranks are 16-bit
}

// Bitmap words of the narrow-B kernels for a batch whose widest B has
// `cols` columns: 1024 (32768 columns) or 2048 (65536); 0: too wide.
inline int narrow_words(int64_t cols) {
  return cols <= (int64_t)32 * kWaveWordsHalf ? kWaveWordsHalf : (cols <= (int64_t)32 * kWaveWords ? kWaveWords : 0);
}

template <class Sr, class Rows, int LGS, int BS, class Kp>
inline void launch_num_hash_one(const Rows& rows, const NumCtx& c, int bin, hipStream_t st, const Kp& kp) {
  const int n = c.plan.count[bin];
  if (n == 0) return;
  const int words = narrow_words((int64_t)rows.Tmax * kTile);
  if constexpr (LGS >= kRowBitmapLgMin) {
    if (words) {
      constexpr int CAP = 1 << (LGS - 1);
      const KRef kb = words == kWaveWordsHalf ? kp.template bitmap_row<Sr, Rows, kWaveWordsHalf, CAP, kRowBitmapBS>()
                                              : kp.template bitmap_row<Sr, Rows, kWaveWords, CAP, kRowBitmapBS>();
      if (kb.ok()) {
        klaunch(kb, dim3(grid_for(n, 1, c.cus * kb.occ * 4)), dim3(kRowBitmapBS), st, rows, c.plan.bins, (int)bin,
                c.C, c.err);
        return;
      }
    }
  } else if constexpr (LGS <= kWaveLgMax) {
    if (words) {
      constexpr int CAP = 1 << (LGS - 1);
      const KRef kw = words == kWaveWordsHalf ? kp.template wave_bitmap<Sr, Rows, kWaveWordsHalf, CAP, kWaveBS>()
                                              : kp.template wave_bitmap<Sr, Rows, kWaveWords, CAP, kWaveBS>();
      if (kw.ok()) {
        klaunch(kw, dim3(grid_for(n, kWaveBS / kWave, c.cus * kw.occ * 4)), dim3(kWaveBS), st, rows, c.plan.bins,
                (int)bin, c.C, c.err);
        return;
      }
    }
  }
  if constexpr (LGS >= kMergeRowLgMin) {
    if (!words && c.merge_rows) {
      constexpr int CAP = 1 << (LGS - 1);
      constexpr int MBS = merge_row_bs(CAP, (int)sizeof(typename Sr::Acc));
      const KRef km = kp.template merge_row<Sr, Rows, CAP, MBS>();
      if (km.ok()) {
        klaunch(km, dim3(grid_for(n, 1, c.cus * km.occ * 4)), dim3(MBS), st, rows, c.plan.bins, (int)bin, c.C,
                c.err);
        return;
      }
    }
  }
  const KRef k = kp.template hash<Sr, Rows, LGS, BS>();
  klaunch(k, dim3(grid_for(n, 1, c.cus * k.occ * 4)), dim3(BS), st, rows, c.plan.bins, (int)bin, c.C, c.err);
}

template <class Sr, class Rows, class Kp>
inline void launch_num_hash_all(const Rows& rows, const NumCtx& c, int bin0, hipStream_t st, const Kp& kp) {
  constexpr int A = (int)sizeof(typename Sr::Acc);
  launch_num_hash_one<Sr, Rows, 7, hash_bs(0, A)>(rows, c, bin0 + 0, st, kp);
  launch_num_hash_one<Sr, Rows, 8, hash_bs(1, A)>(rows, c, bin0 + 1, st, kp);
  launch_num_hash_one<Sr, Rows, 9, hash_bs(2, A)>(rows, c, bin0 + 2, st, kp);
  launch_num_hash_one<Sr, Rows, 10, hash_bs(3, A)>(rows, c, bin0 + 3, st, kp);
  launch_num_hash_one<Sr, Rows, 11, hash_bs(4, A)>(rows, c, bin0 + 4, st, kp);
  launch_num_hash_one<Sr, Rows, 12, hash_bs(5, A)>(rows, c, bin0 + 5, st, kp);
  launch_num_hash_one<Sr, Rows, 13, hash_bs(6, A)>(rows, c, bin0 + 6, st, kp);
}

template <class Sr, class Rows, class Kp>
inline void launch_num_dense(const Rows& rows, const NumCtx& c, hipStream_t st, const Kp& kp) {
  if (c.plan.ndense() == 0) return;
  using V = typename Sr::V;
  constexpr bool kProduct = std::is_same_v<Rows, OneRows<SpgemmSrc<V, true>>>;
  const bool slab = kProduct && c.src.mode == kModeProduct && c.src.S > 0;
  const int32_t G = slab ? (1 << (c.src.ls - kTileLog)) : 0;
  constexpr int kSlabCap = slab_cap<Sr>();
  if constexpr (kProduct) {
    if (slab) {
      const int32_t cap = c.light_cap > 0 && c.light_cap < kSlabCap ? c.light_cap : kSlabCap;
      const int32_t T = c.src.T;
      const int32_t nd = c.plan.bins.nd_cap;  // bucket capacity (the count itself may only be on the device)
      int32_t* sbook = c.slab_book;
      SlabTask* light = c.slab_tasks;
      SlabTask* heavy = c.slab_tasks + (int64_t)nd * c.src.S;
      hipLaunchKernelGGL(k_fill<int32_t>, dim3(grid_for(kCtrInts, 256, 64)), dim3(256), 0, st, c.task_ctr,
                         (int64_t)kCtrInts, (int32_t)0);
      hipLaunchKernelGGL(k_fill<int32_t>, dim3(grid_for(3 * (int64_t)T, 256, 1024)), dim3(256), 0, st, sbook,
                         3 * (int64_t)T, (int32_t)0);
      hipLaunchKernelGGL(k_slab_tasks<256>, dim3(grid_for(nd, 256, c.cus * 8)), dim3(256), 0, st, c.plan.bins,
                         c.src.drow, c.off2, T, G, c.src.S, cap, (const int64_t*)c.C.rowptr, light,
                         heavy, sbook, c.task_ctr);
      hipLaunchKernelGGL(k_task_offsets<1024>, dim3(1), dim3(1024), 0, st, sbook, T, c.task_ctr);
      SlabB<V> b{c.src.prow, c.src.pbit, (const ColV<V>*)c.src.pval, c.src.rpt, c.src.b_nrows, G, T};
      // 32-bit gathers when the (column, value) partition spans less than 4 GiB
      const bool narrow = c.src.gather32 && c.src.b_nnz < ((int64_t)1 << 32) / (int64_t)sizeof(ColV<V>);
      {
        const KRef k = narrow ? kp.template slab<Sr, kSlabCap, true>() : kp.template slab<Sr, kSlabCap, false>();
        const int occ = kp.template slab<Sr, kSlabCap, true>().occ;
        const int grid = c.cus * occ > kQueues ? c.cus * occ : kQueues;
        c.marks.mark(kPhNumDenseSlab, 1);
        klaunch(k, dim3(grid), dim3(kSlabBS), st, b, (const int32_t*)c.src.a_col, (const V*)c.src.a_val, c.C,
                (const SlabTask*)light, (const int32_t*)book_off(sbook, T, kListSlab), (int32_t)nd, c.task_ctr,
                c.err);
        c.marks.mark(kPhNumDenseSlab, 0);
      }
      {
        const KRef k = narrow ? kp.template heavy<Sr, true>() : kp.template heavy<Sr, false>();
        const int occ = kp.template heavy<Sr, true>().occ;
        const int grid = c.cus * occ > kQueues ? c.cus * occ : kQueues;
        c.marks.mark(kPhNumDenseTiles, 1);
        klaunch(k, dim3(grid), dim3(kSlabBS), st, b, (const int32_t*)c.src.a_col, (const V*)c.src.a_val,
                (const int32_t*)c.off2, (const uint4*)c.spn, c.C, (const SlabTask*)heavy,
                (const int32_t*)book_off(sbook, T, kListTile), (int32_t)nd, c.task_ctr, c.err);
        c.marks.mark(kPhNumDenseTiles, 0);
      }
      return;
    }
  }
  int32_t* book = task_book(c);
  const int32_t Tmax = rows.Tmax;
  // over narrow B, whole rows of at most DCAP entries take the bitmap fold:
  // the task builder puts them on its slab list (one slab spanning the row)
  constexpr int DCAP = dense_bitmap_cap<Sr, Rows, kWaveWords>();
  constexpr int DCAPH = dense_bitmap_cap<Sr, Rows, kWaveWordsHalf>();
  KRef kb{};
  const int words = narrow_words((int64_t)Tmax * kTile);
  if (words == kWaveWordsHalf) kb = kp.template bitmap_dense<Sr, Rows, kWaveWordsHalf, DCAPH, kDenseBitmapBS>();
  else if (words == kWaveWords) kb = kp.template bitmap_dense<Sr, Rows, kWaveWords, DCAP, kDenseBitmapBS>();
  const bool bm = kb.ok();
  const int32_t dcap = words == kWaveWordsHalf ? DCAPH : DCAP;
  hipLaunchKernelGGL(k_fill<int32_t>, dim3(grid_for(kCtrInts, 256, 64)), dim3(256), 0, st, c.task_ctr,
                     (int64_t)kCtrInts, (int32_t)0);
  hipLaunchKernelGGL(k_fill<int32_t>, dim3(grid_for(3 * (int64_t)Tmax, 256, 1024)), dim3(256), 0, st, book,
                     3 * (int64_t)Tmax, (int32_t)0);
  // products: range tasks as runs over groups of kRunTiles tiles
  KRef krr{};
  if constexpr (!Rows::Src::kParts) krr = kp.template range_runs<Sr, Rows, kWaveWords, kRangeCap, kRangeBitmapBS>();
  const int32_t run_tiles = krr.ok() ? kRunTiles : 0;
  hipLaunchKernelGGL(k_dense_tasks<256>, dim3(grid_for(c.plan.ndense(), 256, c.cus * 8)), dim3(256), 0, st,
                     c.plan.bins, c.off2, Tmax, bm ? Tmax : 0, bm ? dcap : 0, c.tile_min, kRangeCap, run_tiles,
                     c.tasks, c.tasks + c.task_cap, c.tasks + 2 * c.task_cap, book, c.task_ctr);
  hipLaunchKernelGGL(k_task_offsets<1024>, dim3(1), dim3(1024), 0, st, book, Tmax, c.task_ctr);
  if (bm) {
    const int grid = c.cus * kb.occ > kQueues ? c.cus * kb.occ : kQueues;
    c.marks.mark(kPhNumDenseSlab, 1);
    klaunch(kb, dim3(grid), dim3(kDenseBitmapBS), st, rows, c.plan.bins, c.C, (const Task*)(c.tasks + 2 * c.task_cap),
            (const int32_t*)book, c.task_ctr, c.err);
    c.marks.mark(kPhNumDenseSlab, 0);
  }
  constexpr int BS = tiles_bs((int)sizeof(typename Sr::Acc), (int)sizeof(typename Rows::Src::Item));
  const KRef k = kp.template tiles<Sr, Rows, BS>();
  const int grid = c.cus * k.occ > kQueues ? c.cus * k.occ : kQueues;
  c.marks.mark(kPhNumDenseTiles, 1);
  klaunch(k, dim3(grid), dim3(BS), st, rows, c.plan.bins, c.C, (const int32_t*)c.off2, (const Task*)c.tasks,
          (const int32_t*)book, c.task_ctr, c.err);
  c.marks.mark(kPhNumDenseTiles, 0);
  // range tasks (at most kRangeSpanMax tiles): the bitmap fold, else (run-
  // time semirings) a hash table and a sort
  const KRef kr = kp.template ranges_bitmap<Sr, Rows, kWaveWords, kRangeCap, kRangeBitmapBS>();
  c.marks.mark(kPhNumDenseRanges, 1);
  if (run_tiles) {
    const int grid2 = c.cus * krr.occ > kQueues ? c.cus * krr.occ : kQueues;
    klaunch(krr, dim3(grid2), dim3(kRangeBitmapBS), st, rows, c.plan.bins, c.C, (const int32_t*)c.off2,
            (const Task*)(c.tasks + c.task_cap), (const int32_t*)book, c.task_ctr, c.tile_min, c.err);
  } else if (kr.ok()) {
    const int grid2 = c.cus * kr.occ > kQueues ? c.cus * kr.occ : kQueues;
    klaunch(kr, dim3(grid2), dim3(kRangeBitmapBS), st, rows, c.plan.bins, c.C, (const int32_t*)c.off2,
            (const Task*)(c.tasks + c.task_cap), (const int32_t*)book, c.task_ctr, c.err);
  } else {
    constexpr int RBS = ranges_bs((int)sizeof(typename Sr::Acc));
    const KRef k2 = kp.template ranges<Sr, Rows, kRangeLg, RBS>();
    const int grid2 = c.cus * k2.occ > kQueues ? c.cus * k2.occ : kQueues;
    klaunch(k2, dim3(grid2), dim3(RBS), st, rows, c.plan.bins, c.C, (const int32_t*)c.off2,
            (const Task*)(c.tasks + c.task_cap), (const int32_t*)book, c.task_ctr, c.err);
  }
  c.marks.mark(kPhNumDenseRanges, 0);
}

// Numeric pass for semiring Sr (SrC: its compensated variant, or Sr), with
// the kernels of provider kp.
template <class Sr, class SrC, class Rows, class Kp>
inline void launch_numeric_rows(const Rows& rows, const NumCtx& c, hipStream_t st, const Kp& kp) {
  c.marks.mark(kPhNumSmall, 1);
  if (c.plan.count[kBinSmall]) {
    const KRef k = kp.template small<Sr, Rows>();
    klaunch(k, dim3(grid_for(c.plan.count[kBinSmall], 4, c.cus * k.occ * 4)), dim3(256), st, rows, c.plan.bins,
            (int)kBinSmall, c.C, c.err);
  }
  c.marks.mark(kPhNumSmall, 0);
  c.marks.mark(kPhNumHash, 1);
  launch_num_hash_all<Sr, Rows>(rows, c, kBinHash0, st, kp);
  launch_num_hash_all<SrC, Rows>(rows, c, kBinHashC0, st, kp);
  c.marks.mark(kPhNumHash, 0);
  c.marks.mark(kPhNumDense, 1);
  if (c.comp_dense) launch_num_dense<SrC, Rows>(rows, c, st, kp);
  else launch_num_dense<Sr, Rows>(rows, c, st, kp);
  c.marks.mark(kPhNumDense, 0);
}

template <class Sr, class SrC, class Kp = KLib>
inline void launch_numeric(const NumCtx& c, hipStream_t st, const Kp& kp = Kp{}) {
  with_rows<typename Sr::V, true>(c.src, [&](const auto& rows) { launch_numeric_rows<Sr, SrC>(rows, c, st, kp); });
}

// ---- entry points implemented in the .hip translation units -------------------------

// k_struct.hip
void launch_analyze(const RowSource& r, const Policy& pol, const int64_t* c_rowptr, int64_t* p, int32_t* nt,
                    uint8_t* bin, int32_t* hist, int32_t* blk_off, int32_t* bin_start, int32_t* bin_count,
                    int32_t* list, int64_t* cnt_out, hipStream_t st);
// Numeric binning from the symbolic pass's per-row products p and terms nt.
void launch_rebin(const int64_t* p, const int32_t* nt, const int64_t* c_rowptr, int64_t nrows, const Policy& pol,
                  uint8_t* bin, int32_t* hist, int32_t* blk_off, int32_t* bin_start, int32_t* bin_count,
                  int32_t* list, hipStream_t st);
int64_t analyze_blocks(int64_t nrows);
void launch_tile_bounds(const int64_t* rowptr, const int32_t* col, int64_t nrows, int32_t T, int32_t* rp2, int cus,
                        hipStream_t st);
// Column-slab partition of B (slabs of 2^ls columns, S of them): with cols
// set, the bounds bnd (S+1 ints per B row), the tile offsets rpt, the
// segment starts prow (S*nb + 1), pbit and, when perm is given, each
// entry's destination; with vals set, pval (vbytes per entry), through perm
// when it is given and cols is not set.  partial: scan_partials_len(S*nb)
// int64 of scratch; err: flag set on entries that contradict the bounds
// (unsorted or out-of-range columns).
void launch_slab_partition(const int64_t* b_rowptr, const int32_t* b_col, const void* b_val, int vbytes, int64_t nb,
                           int64_t nnz, int32_t ls, int32_t S, int32_t T, int32_t* bnd, int32_t* rpt, int64_t* prow,
                           int64_t* partial, int32_t* pbit, void* pval, int32_t* perm, bool cols, bool vals,
                           int32_t* err, int cus, hipStream_t st);
// Per dense row of the plan: its A row (the slab path's row table).
void launch_dense_rows(const BinPlan& plan, const int64_t* a_rowptr, DenseRow* dr, int cus, hipStream_t st);
void launch_symbolic(const RowSource& r, const BinPlan& plan, int64_t* cnt_out, int32_t* off2, int cus,
                     const Marks& marks, hipStream_t st);
void launch_symbolic_dense(const RowSource& r, const BinPlan& plan, int64_t* cnt_out, int32_t* off2, int cus,
                           hipStream_t st);
int64_t scan_partials_len(int64_t n);
void launch_scan_inclusive(int64_t* a, int64_t n, int64_t* partial, hipStream_t st);
void launch_fill_i64(int64_t* p, int64_t n, int64_t v, hipStream_t st);
void launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t st);
void launch_validate(const int64_t* rowptr, const int32_t* col, int64_t nrows, int64_t ncols, int64_t nnz,
                     int32_t* flag, hipStream_t st);

// num_*.hip
void launch_numeric_i64(const NumCtx& c, hipStream_t st);
void launch_numeric_f32(const NumCtx& c, hipStream_t st);
void launch_numeric_f64(const NumCtx& c, hipStream_t st);
void launch_numeric_bool(const NumCtx& c, hipStream_t st);
void launch_numeric_minplus(const NumCtx& c, hipStream_t st);

}  // namespace sg
