// Host-side launch contexts and launcher templates.  The structural launchers
// (analysis, binning, tile bounds, symbolic, scans) live in k_struct.hip; one
// numeric launcher per semiring lives in num_<semiring>.hip.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sg_kernels.hpp"

namespace sg {

// Everything a symbolic or numeric launch needs to describe its rows.
struct RowSource {
  int merge;  // 0: product rows of A (x) B, 1: merge of parts
  // product
  const int64_t* a_rowptr;
  const int32_t* a_col;
  const void* a_val;
  const int64_t* b_rowptr;
  const int32_t* b_col;
  const void* b_val;
  int64_t b_nrows;
  const int32_t* rp2;
  // merge
  const PartDesc* parts;
  int32_t nparts;
  // both
  int64_t nrows;
  int64_t ncols;  // columns of C
  int32_t T;      // column tiles of C
};

struct BinPlan {
  Bins bins;
  int32_t count[kNB];  // host copy
  int32_t start[kNB];
  int32_t ndense() const {
    int32_t s = 0;
    for (int b = kBinDense0; b < kNB; ++b) s += count[b];
    return s;
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
       kPhNumHash, kPhNumDense, kNPhases };

struct NumCtx {
  Marks marks;
  RowSource src;
  BinPlan plan;
  OutC C;
  const int32_t* off2;
  int32_t* err;
  int32_t* task_ctr;
  int cus;
  int comp_dense;  // float sums: dense rows use compensated accumulation
};

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

template <class Sr, class Src, int LGS, int BS>
inline void launch_num_hash_one(const Src& s, const NumCtx& c, int bin, hipStream_t st) {
  const int n = c.plan.count[bin];
  if (n == 0) return;
  auto k = k_num_hash<Sr, Src, LGS, BS>;
  static int occ = occupancy(k, BS);
  hipLaunchKernelGGL(k, dim3(grid_for(n, 1, c.cus * occ * 4)), dim3(BS), 0, st, s, c.plan.bins, bin, c.C, c.err);
}

template <class Sr, class Src>
inline void launch_num_hash_all(const Src& s, const NumCtx& c, int bin0, hipStream_t st) {
  launch_num_hash_one<Sr, Src, 7, 256>(s, c, bin0 + 0, st);
  launch_num_hash_one<Sr, Src, 8, 256>(s, c, bin0 + 1, st);
  launch_num_hash_one<Sr, Src, 9, 256>(s, c, bin0 + 2, st);
  launch_num_hash_one<Sr, Src, 10, 256>(s, c, bin0 + 3, st);
  launch_num_hash_one<Sr, Src, 11, 512>(s, c, bin0 + 4, st);
  launch_num_hash_one<Sr, Src, 12, 512>(s, c, bin0 + 5, st);
  launch_num_hash_one<Sr, Src, 13, 512>(s, c, bin0 + 6, st);
}

template <class Sr, class Src>
inline void launch_num_dense(const Src& s, const NumCtx& c, hipStream_t st) {
  if (c.plan.ndense() == 0) return;
  // 8-byte accumulators need the whole LDS for one 16384-slot tile: use a
  // 1024-thread workgroup (16 waves) when the per-source items are small.
  constexpr int BS = (sizeof(typename Sr::Acc) >= 8 && sizeof(typename Src::Item) <= 8) ? 1024 : 512;
  auto k = k_num_dense<Sr, Src, BS>;
  static int occ = occupancy(k, BS);
  hipLaunchKernelGGL(k_fill<int32_t>, dim3(1), dim3(64), 0, st, c.task_ctr, (int64_t)1, (int32_t)0);
  hipLaunchKernelGGL(k, dim3(c.cus * occ), dim3(BS), 0, st, s, c.plan.bins, c.C, c.off2, c.task_ctr, c.err);
}

// Numeric pass for semiring Sr (SrC: its compensated variant, or Sr).
template <class Sr, class SrC, class Src>
inline void launch_numeric_src(const Src& s, const NumCtx& c, hipStream_t st) {
  c.marks.mark(kPhNumSmall, 1);
  if (c.plan.count[kBinSmall]) {
    auto k = k_num_small<Sr, Src>;
    static int occ = occupancy(k, 256);
    hipLaunchKernelGGL(k, dim3(grid_for(c.plan.count[kBinSmall], 4, c.cus * occ * 4)), dim3(256), 0, st, s,
                       c.plan.bins, kBinSmall, c.C, c.err);
  }
  c.marks.mark(kPhNumSmall, 0);
  c.marks.mark(kPhNumHash, 1);
  launch_num_hash_all<Sr, Src>(s, c, kBinHash0, st);
  launch_num_hash_all<SrC, Src>(s, c, kBinHashC0, st);
  c.marks.mark(kPhNumHash, 0);
  c.marks.mark(kPhNumDense, 1);
  if (c.comp_dense) launch_num_dense<SrC, Src>(s, c, st);
  else launch_num_dense<Sr, Src>(s, c, st);
  c.marks.mark(kPhNumDense, 0);
}

template <class Sr, class SrC>
inline void launch_numeric(const NumCtx& c, hipStream_t st) {
  using V = typename Sr::V;
  if (c.src.merge) launch_numeric_src<Sr, SrC>(make_merge_src<V>(c.src), c, st);
  else launch_numeric_src<Sr, SrC>(make_spgemm_src<V, true>(c.src), c, st);
}

// ---- entry points implemented in the .hip translation units -------------------------

// k_struct.hip
void launch_analyze(const RowSource& r, const Policy& pol, const int64_t* c_rowptr, int64_t* p, uint8_t* bin,
                    int32_t* hist, int32_t* blk_off, int32_t* bin_start, int32_t* bin_count, int32_t* list,
                    int64_t* cnt_out, hipStream_t st);
int64_t analyze_blocks(int64_t nrows);
void launch_tile_bounds(const int64_t* rowptr, const int32_t* col, int64_t nrows, int32_t T, int32_t* rp2, int cus,
                        hipStream_t st);
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
