// Batched persistent path (paper Section 2.1: the many stage-local block
// products of a 2D Sparse SUMMA and their merge, run here on one GPU).
//
// All products of a plan form one global row space: row r belongs to product
// q when rbase[q] <= r < rbase[q+1].  Every phase is one set of persistent
// kernels over the global bins of all products at once (TableRows), so a
// batch of many small or uneven products costs the same handful of launches
// as one product.  Merges form a second row space whose parts point straight
// at the products' outputs in the pool.  sg_batch_plan sizes everything with
// one eager pass (patterns are fixed after planning), then records the whole
// pipeline -- analysis, binning, tile bounds, symbolic, scan, pool guard,
// numeric, for products and then merges, and the per-result row pointers --
// into a hipGraph; sg_batch_execute only replays that graph.
#include <algorithm>
#include <cstring>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "sg_batch.hpp"
#include "sg_handle.hpp"

using namespace sg;

#define SG_HIP(h, call)                                        \
  do {                                                         \
    const sg_status _s = sg_check_hip((h), (call), #call);     \
    if (_s != SG_OK) return _s;                                \
  } while (0)

#define SG_TRY(expr)                \
  do {                              \
    const sg_status _s = (expr);    \
    if (_s != SG_OK) return _s;     \
  } while (0)

namespace {

struct Stage {
  RowSource src{};
  int64_t R = 0;
  int32_t nd = 0;
  int64_t nnz = 0;
  SgBuf work, off_buf, off2_buf, col_buf, val_buf, task_buf;
  // a single product recorded on the column-slab path: B's partition, its
  // scan scratch and B's descriptor
  bool slab = false;
  SlabBufs sb;
  SgBuf spart;
  sg_csr b{};
  // views into work
  int64_t* p = nullptr;
  int32_t* nt = nullptr;
  uint8_t* bin = nullptr;
  int32_t *hist = nullptr, *blk_off = nullptr, *bin_start = nullptr, *bin_count = nullptr, *list = nullptr;
  int64_t* partial = nullptr;
  int64_t* off = nullptr;

  sg_status alloc_work(sg_handle* h) {
    SgArena m;
    const int64_t nblk = analyze_blocks(R);
    m.take<int64_t>(R);
    m.take<uint8_t>(R);
    m.take<int32_t>(nblk * kNB);
    m.take<int32_t>(nblk * kNB);
    m.take<int32_t>(kNB);
    m.take<int32_t>(kNB);
    m.take<int32_t>(R);
    m.take<int32_t>(R);
    m.take<int64_t>(scan_partials_len(R));
    SG_HIP(h, work.ensure(m.off));
    SgArena a;
    a.base = (char*)work.p;
    p = a.take<int64_t>(R);
    bin = a.take<uint8_t>(R);
    hist = a.take<int32_t>(nblk * kNB);
    blk_off = a.take<int32_t>(nblk * kNB);
    bin_start = a.take<int32_t>(kNB);
    bin_count = a.take<int32_t>(kNB);
    list = a.take<int32_t>(R);
    nt = a.take<int32_t>(R);
    partial = a.take<int64_t>(scan_partials_len(R));
    SG_HIP(h, off_buf.ensure(sizeof(int64_t) * (size_t)(R + 1)));
    off = (int64_t*)off_buf.p;
    return SG_OK;
  }
  BinPlan graph_plan() const {
    BinPlan bp;
    bp.bins = Bins{list, bin_start, bin_count, nd};
    for (int b = 0; b < kNB; ++b) {
      bp.count[b] = 1 << 30;
      bp.start[b] = 0;
    }
    bp.graph = true;
    return bp;
  }
  void release() {
    work.release();
    off_buf.release();
    off2_buf.release();
    col_buf.release();
    val_buf.release();
    task_buf.release();
    sb.release();
    spart.release();
  }
  // dense-row task memory: the slab path's light and heavy lists, or the
  // tile and range lists
  size_t task_bytes() const {
    const int64_t n = nd > 0 ? nd : 1;
    if (slab) return 2 * sizeof(SlabTask) * (size_t)n * (size_t)src.S + sizeof(int32_t) * (6 * (size_t)src.T + 3);
    return task_buffer_bytes(n * src.T, src.T);
  }
};

}  // namespace

struct sg_plan {
  sg_handle* h = nullptr;
  sg_semiring sr{};
  int nprob = 0, ngroups = 0;
  std::vector<sg_csr> A, B;
  std::vector<int32_t> go;
  std::vector<int64_t> rbase_p, rbase_m;  // host copies
  SgBuf tables;                           // probs, groups, parts, rbase arrays, lbase arrays, local rowptrs, flag
  ProbDesc* d_probs = nullptr;
  GroupDesc* d_groups = nullptr;
  PartDesc* d_parts = nullptr;
  int64_t *d_rbase_p = nullptr, *d_rbase_m = nullptr, *d_lbase_p = nullptr, *d_lbase_m = nullptr;
  int32_t *d_coarse_p = nullptr, *d_coarse_m = nullptr;  // owners of every 256th row
  int64_t *d_lrow_p = nullptr, *d_lrow_m = nullptr;
  int64_t ltot_p = 0, ltot_m = 0;
  int32_t* d_flag = nullptr;  // [0] pool overflow, [1] consistency, [kCtrBase, ...) task counters
  std::vector<SgBuf> rp2;     // one per distinct B with more than one column tile
  std::vector<std::tuple<const int64_t*, const int32_t*, int64_t, int32_t, int32_t*>> bounds;  // B rows -> rp2
  Stage prod, merg;
  hipStream_t stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  bool ran = false;
};

namespace {

sg_status run_stage_eager(sg_plan* P, Stage& S, bool has_dense_inputs) {
  sg_handle* h = P->h;
  hipStream_t st = P->stream;
  // symbolic with host-known bin counts (this pass only sizes the plan)
  const Policy ps = make_policy(h, 0, nullptr);
  launch_analyze(S.src, ps, nullptr, S.p, S.nt, S.bin, S.hist, S.blk_off, S.bin_start, S.bin_count, S.list, S.off + 1, st);
  BinPlan bp;
  int32_t* hp = (int32_t*)h->h_pin;
  SG_HIP(h, hipMemcpyAsync(hp, S.bin_count, kNB * sizeof(int32_t), hipMemcpyDeviceToHost, st));
  SG_HIP(h, hipStreamSynchronize(st));
  std::memcpy(bp.count, hp, sizeof(bp.count));
  S.nd = bp.ndense();
  bp.bins = Bins{S.list, S.bin_start, S.bin_count, S.nd};
  if (S.slab && S.nd > 0) {
    // the slab path keeps span counts after the tile offsets
    SG_HIP(h, S.off2_buf.ensure(off2_span_bytes(S.nd, S.src.T)));
    S.src.spn = (uint4*)((char*)S.off2_buf.p + span_offset(S.nd, S.src.T));
    // structure once (patterns do not change after planning); values are
    // re-scattered by every replay
    SG_HIP(h, S.spart.ensure(sizeof(int64_t) * (slab_partials(h, S.src) + 1)));
    Scratch sc{h};
    SG_TRY(build_slabs(h, sc, S.sb, S.src, &S.b, P->sr.value_bytes, true, true, (int64_t*)S.spart.p, P->d_flag + 1,
                       P->d_flag + kCtrBase, st));
    SG_TRY(build_dense_rows(h, sc, S.sb, S.src, bp, st));
  } else {
    S.slab = false;
    S.src.S = 0;
    S.src.spn = nullptr;
    SG_HIP(h, S.off2_buf.ensure(sizeof(int32_t) * (size_t)(S.nd > 0 ? S.nd : 1) * (size_t)(S.src.T + 1)));
  }
  SG_HIP(h, S.task_buf.ensure(S.task_bytes()));
  if (S.nd > 0 && has_dense_inputs)
    for (auto& b : P->bounds)
      launch_tile_bounds(std::get<0>(b), std::get<1>(b), std::get<2>(b), std::get<3>(b), std::get<4>(b), h->cus, st);
  launch_symbolic(S.src, bp, S.off + 1, (int32_t*)S.off2_buf.p, h->cus, Marks{}, st);
  launch_fill_i64(S.off, 1, 0, st);
  launch_scan_inclusive(S.off + 1, S.R, S.partial, st);
  SG_HIP(h, hipGetLastError());
  SG_HIP(h, hipMemcpyAsync(h->h_pin, S.off + S.R, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  SG_HIP(h, hipStreamSynchronize(st));
  S.nnz = h->h_pin[0];
  return SG_OK;
}

sg_status alloc_pool(sg_plan* P, Stage& S) {
  const size_t vb = (size_t)P->sr.value_bytes;
  const size_t n = (size_t)(S.nnz > 0 ? S.nnz : 1);
  SG_HIP(P->h, S.col_buf.ensure(n * sizeof(int32_t), true));
  SG_HIP(P->h, S.val_buf.ensure(n * vb, true));
  return SG_OK;
}

int64_t pool_cap(const Stage& S, size_t vb) {
  const size_t c1 = S.col_buf.cap / sizeof(int32_t), c2 = S.val_buf.cap / vb;
  return (int64_t)(c1 < c2 ? c1 : c2);
}

// Queue one stage's full pipeline on the plan stream with device-side bin
// counts only (graph-capturable: no host reads, no memsets).
void record_stage(sg_plan* P, Stage& S, bool has_dense_inputs) {
  sg_handle* h = P->h;
  hipStream_t st = P->stream;
  const Policy ps = make_policy(h, 0, nullptr);
  const Policy pn = make_policy(h, 1, &P->sr, S.src.T);
  launch_analyze(S.src, ps, nullptr, S.p, S.nt, S.bin, S.hist, S.blk_off, S.bin_start, S.bin_count, S.list, S.off + 1, st);
  BinPlan bp = S.graph_plan();
  if (S.nd == 0) {
    for (int b = kBinDense0; b < kNB; ++b) bp.count[b] = 0;
  } else if (has_dense_inputs) {
    for (auto& b : P->bounds)
      launch_tile_bounds(std::get<0>(b), std::get<1>(b), std::get<2>(b), std::get<3>(b), std::get<4>(b), h->cus, st);
  }
  launch_symbolic(S.src, bp, S.off + 1, (int32_t*)S.off2_buf.p, h->cus, Marks{}, st);
  launch_fill_i64(S.off, 1, 0, st);
  launch_scan_inclusive(S.off + 1, S.R, S.partial, st);
  launch_rebin(S.p, S.nt, S.off, S.R, pn, S.bin, S.hist, S.blk_off, S.bin_start, S.bin_count, S.list, st);
  launch_pool_guard(S.off + S.R, pool_cap(S, (size_t)P->sr.value_bytes), S.bin_count, P->d_flag, st);
  Scratch sc{h};
  if (S.slab)  // the current values into the partition (buffers sized at plan time)
    (void)build_slabs(h, sc, S.sb, S.src, &S.b, P->sr.value_bytes, false, true, (int64_t*)S.spart.p, P->d_flag + 1,
                      P->d_flag + kCtrBase, st);
  NumCtx c{};
  c.src = S.src;
  c.plan = bp;
  c.C = OutC{S.off, (int32_t*)S.col_buf.p, S.val_buf.p};
  c.off2 = (const int32_t*)S.off2_buf.p;
  c.spn = S.src.spn;
  c.err = P->d_flag + 1;
  c.task_ctr = P->d_flag + kCtrBase;
  c.task_cap = (int64_t)(S.nd > 0 ? S.nd : 1) * S.src.T;
  c.tasks = (Task*)S.task_buf.p;
  if (S.slab) {
    const size_t tb = 2 * sizeof(SlabTask) * (size_t)S.nd * (size_t)S.src.S;
    c.slab_tasks = (SlabTask*)S.task_buf.p;
    c.slab_book = (int32_t*)((char*)S.task_buf.p + tb);
  }
  c.tile_min = h->tile_min;
  c.cus = h->cus;
  c.merge_rows = h->merge_rows;
  c.light_cap = light_cap_for(h, &P->sr);
  c.comp_dense = pn.comp_mode != kCompNone;
  switch (P->sr.id) {
    case SG_PLUS_TIMES_I64: launch_numeric_i64(c, st); break;
    case SG_PLUS_TIMES_F32: launch_numeric_f32(c, st); break;
    case SG_PLUS_TIMES_F64: launch_numeric_f64(c, st); break;
    case SG_OR_AND_BOOL: launch_numeric_bool(c, st); break;
    default: launch_numeric_minplus(c, st); break;
  }
}

void record_all(sg_plan* P) {
  hipStream_t st = P->stream;
  launch_fill_i32(P->d_flag, 8, 0, st);
  record_stage(P, P->prod, true);
  if (P->ngroups > 0) record_stage(P, P->merg, false);
  launch_local_rowptr(P->prod.off, P->d_rbase_p, P->d_lbase_p, P->nprob, P->ltot_p, P->d_lrow_p, P->h->cus, st);
  if (P->ngroups > 0)
    launch_local_rowptr(P->merg.off, P->d_rbase_m, P->d_lbase_m, P->ngroups, P->ltot_m, P->d_lrow_m, P->h->cus, st);
}

sg_status plan_build(sg_plan* P, size_t pool_bytes) {
  sg_handle* h = P->h;
  const int np = P->nprob, ng = P->ngroups;
  // ---- row spaces and tables (host) ----
  P->rbase_p.assign((size_t)np + 1, 0);
  int32_t Tmax_p = 1;
  for (int q = 0; q < np; ++q) {
    P->rbase_p[(size_t)q + 1] = P->rbase_p[(size_t)q] + P->A[(size_t)q].nrows;
    const int32_t T = tiles_of(P->B[(size_t)q].ncols);
    Tmax_p = T > Tmax_p ? T : Tmax_p;
  }
  P->rbase_m.assign((size_t)ng + 1, 0);
  int32_t Tmax_m = 1;
  for (int g = 0; g < ng; ++g) {
    const int q0 = P->go[(size_t)g];
    P->rbase_m[(size_t)g + 1] = P->rbase_m[(size_t)g] + P->A[(size_t)q0].nrows;
    const int32_t T = tiles_of(P->B[(size_t)q0].ncols);
    Tmax_m = T > Tmax_m ? T : Tmax_m;
  }
  const int64_t Rp = P->rbase_p[(size_t)np], Rm = P->rbase_m[(size_t)ng];
  if (Rp >= INT32_MAX || Rm >= INT32_MAX) return sg_fail(h, SG_ERR_OVERFLOW, "a batch holds 2^31 rows or more");
  P->ltot_p = Rp + np;
  P->ltot_m = Rm + ng;
  int nparts = 0;
  for (int g = 0; g < ng; ++g) nparts += P->go[(size_t)g + 1] - P->go[(size_t)g];

  // owner of every 256th row of each row space (and of its last row)
  auto coarse_of = [](const std::vector<int64_t>& rbase, int n, int64_t R) {
    std::vector<int32_t> c((size_t)(R > 0 ? ((R - 1) >> kOwnerShift) + 2 : 2), 0);
    for (size_t k = 0; k < c.size(); ++k) {
      int64_t r = (int64_t)k << kOwnerShift;
      r = r < R - 1 ? r : (R > 0 ? R - 1 : 0);
      c[k] = (int32_t)(std::upper_bound(rbase.begin(), rbase.begin() + n, r) - rbase.begin()) - 1;
      c[k] = c[k] < 0 ? 0 : c[k];
    }
    return c;
  };
  const std::vector<int32_t> coarse_p = coarse_of(P->rbase_p, np, Rp);
  const std::vector<int32_t> coarse_m = coarse_of(P->rbase_m, ng > 0 ? ng : 1, Rm);

  SgArena m;
  m.take<ProbDesc>((size_t)np);
  m.take<GroupDesc>((size_t)(ng > 0 ? ng : 1));
  m.take<PartDesc>((size_t)(nparts > 0 ? nparts : 1));
  m.take<int64_t>((size_t)np + 1);
  m.take<int64_t>((size_t)ng + 1);
  m.take<int64_t>((size_t)np + 1);
  m.take<int64_t>((size_t)ng + 1);
  m.take<int64_t>((size_t)P->ltot_p);
  m.take<int64_t>((size_t)(P->ltot_m > 0 ? P->ltot_m : 1));
  m.take<int32_t>(kFlagInts);
  m.take<int32_t>(coarse_p.size());
  m.take<int32_t>(coarse_m.size());
  SG_HIP(h, P->tables.ensure(m.off));
  SgArena a;
  a.base = (char*)P->tables.p;
  P->d_probs = a.take<ProbDesc>((size_t)np);
  P->d_groups = a.take<GroupDesc>((size_t)(ng > 0 ? ng : 1));
  P->d_parts = a.take<PartDesc>((size_t)(nparts > 0 ? nparts : 1));
  P->d_rbase_p = a.take<int64_t>((size_t)np + 1);
  P->d_rbase_m = a.take<int64_t>((size_t)ng + 1);
  P->d_lbase_p = a.take<int64_t>((size_t)np + 1);
  P->d_lbase_m = a.take<int64_t>((size_t)ng + 1);
  P->d_lrow_p = a.take<int64_t>((size_t)P->ltot_p);
  P->d_lrow_m = a.take<int64_t>((size_t)(P->ltot_m > 0 ? P->ltot_m : 1));
  P->d_flag = a.take<int32_t>(kFlagInts);
  P->d_coarse_p = a.take<int32_t>(coarse_p.size());
  P->d_coarse_m = a.take<int32_t>(coarse_m.size());

  // one product and no merges: recorded as a single product on the
  // column-slab path (no tile-bounds tables needed)
  const bool single = np == 1 && ng == 0 && h->slab;
  // distinct B operands that need column-tile bounds
  std::map<std::tuple<const int64_t*, const int32_t*, int64_t>, int32_t*> seen;
  std::vector<ProbDesc> probs((size_t)np);
  for (int q = 0; q < np; ++q) {
    const sg_csr& A = P->A[(size_t)q];
    const sg_csr& B = P->B[(size_t)q];
    ProbDesc d{};
    d.a_rowptr = A.rowptr;
    d.a_col = A.col;
    d.a_val = A.val;
    d.b_rowptr = B.rowptr;
    d.b_col = B.col;
    d.b_val = B.val;
    d.ncols = B.ncols;
    d.T = tiles_of(B.ncols);
    if (d.T > 1 && !single) {
      auto key = std::make_tuple((const int64_t*)B.rowptr, (const int32_t*)B.col, B.nrows);
      auto it = seen.find(key);
      if (it == seen.end()) {
        P->rp2.emplace_back();
        SG_HIP(h, P->rp2.back().ensure(sizeof(int32_t) * (size_t)B.nrows * (size_t)(d.T + 1)));
        int32_t* r2 = (int32_t*)P->rp2.back().p;
        it = seen.emplace(key, r2).first;
        P->bounds.emplace_back(B.rowptr, B.col, B.nrows, d.T, r2);
      }
      d.rp2 = it->second;
    }
    probs[(size_t)q] = d;
  }
  std::vector<int64_t> lb_p((size_t)np + 1, 0), lb_m((size_t)ng + 1, 0);
  for (int q = 0; q < np; ++q) lb_p[(size_t)q + 1] = lb_p[(size_t)q] + P->A[(size_t)q].nrows + 1;
  for (int g = 0; g < ng; ++g) lb_m[(size_t)g + 1] = lb_m[(size_t)g] + (P->rbase_m[(size_t)g + 1] - P->rbase_m[(size_t)g]) + 1;

  hipStream_t st = P->stream;
  SG_HIP(h, hipMemcpyAsync(P->d_probs, probs.data(), sizeof(ProbDesc) * (size_t)np, hipMemcpyHostToDevice, st));
  SG_HIP(h, hipMemcpyAsync(P->d_rbase_p, P->rbase_p.data(), sizeof(int64_t) * ((size_t)np + 1), hipMemcpyHostToDevice, st));
  SG_HIP(h, hipMemcpyAsync(P->d_rbase_m, P->rbase_m.data(), sizeof(int64_t) * ((size_t)ng + 1), hipMemcpyHostToDevice, st));
  SG_HIP(h, hipMemcpyAsync(P->d_coarse_p, coarse_p.data(), sizeof(int32_t) * coarse_p.size(), hipMemcpyHostToDevice, st));
  SG_HIP(h, hipMemcpyAsync(P->d_coarse_m, coarse_m.data(), sizeof(int32_t) * coarse_m.size(), hipMemcpyHostToDevice, st));
  SG_HIP(h, hipMemcpyAsync(P->d_lbase_p, lb_p.data(), sizeof(int64_t) * ((size_t)np + 1), hipMemcpyHostToDevice, st));
  SG_HIP(h, hipMemcpyAsync(P->d_lbase_m, lb_m.data(), sizeof(int64_t) * ((size_t)ng + 1), hipMemcpyHostToDevice, st));
  launch_fill_i32(P->d_flag, 8, 0, st);

  // ---- product stage: size it with an eager pass ----
  Stage& S = P->prod;
  if (single) {
    const sg_csr& A = P->A[0];
    const sg_csr& B = P->B[0];
    S.src.mode = kModeProduct;
    S.src.merge_rows = h->merge_rows;
    S.src.a_rowptr = A.rowptr;
    S.src.a_col = A.col;
    S.src.a_val = A.val;
    S.src.b_rowptr = B.rowptr;
    S.src.b_col = B.col;
    S.src.b_val = B.val;
    S.src.b_nrows = B.nrows;
    S.src.nrows = A.nrows;
    S.src.ncols = B.ncols;
    S.src.T = tiles_of(B.ncols);
    S.slab = true;
    S.b = B;
  } else {
    S.src.mode = kModeBatchProducts;
    S.src.merge_rows = h->merge_rows;
    S.src.probs = P->d_probs;
    S.src.rbase = P->d_rbase_p;
    S.src.coarse = P->d_coarse_p;
    S.src.ntable = np;
    S.src.nrows = Rp;
    S.src.T = Tmax_p;
  }
  S.R = Rp;
  SG_TRY(S.alloc_work(h));
  SG_TRY(run_stage_eager(P, S, true));
  const size_t vb = (size_t)P->sr.value_bytes;
  // ---- merge stage: its parts are the products' outputs ----
  Stage& M = P->merg;
  if (ng > 0) {
    SG_TRY(alloc_pool(P, S));
    // the merge symbolic reads the products' column ids: fill them now
    record_stage(P, S, true);
    std::vector<PartDesc> parts((size_t)(nparts > 0 ? nparts : 1));
    std::vector<GroupDesc> groups((size_t)ng);
    int k = 0;
    for (int g = 0; g < ng; ++g) {
      const int q0 = P->go[(size_t)g], q1 = P->go[(size_t)g + 1];
      groups[(size_t)g] = GroupDesc{P->d_parts + k, P->B[(size_t)q0].ncols, q1 - q0, tiles_of(P->B[(size_t)q0].ncols)};
      for (int q = q0; q < q1; ++q)
        parts[(size_t)k++] = PartDesc{S.off + P->rbase_p[(size_t)q], (const int32_t*)S.col_buf.p, S.val_buf.p, 0};
    }
    SG_HIP(h, hipMemcpyAsync(P->d_parts, parts.data(), sizeof(PartDesc) * parts.size(), hipMemcpyHostToDevice, st));
    SG_HIP(h, hipMemcpyAsync(P->d_groups, groups.data(), sizeof(GroupDesc) * (size_t)ng, hipMemcpyHostToDevice, st));
    M.src.mode = kModeBatchMerges;
    M.src.merge_rows = h->merge_rows;
    M.src.groups = P->d_groups;
    M.src.rbase = P->d_rbase_m;
    M.src.coarse = P->d_coarse_m;
    M.src.ntable = ng;
    M.src.nrows = Rm;
    M.src.T = Tmax_m;
    M.R = Rm;
    SG_TRY(M.alloc_work(h));
    SG_TRY(run_stage_eager(P, M, false));
  }
  const size_t need = (size_t)S.nnz * (4 + vb) + (ng > 0 ? (size_t)M.nnz * (4 + vb) : 0);
  if (pool_bytes > 0 && pool_bytes < need)
    return sg_fail(h, SG_ERR_NOMEM, "pool_bytes " + std::to_string(pool_bytes) + " < the " + std::to_string(need) +
                                        " bytes the batch's outputs need");
  SG_TRY(alloc_pool(P, S));
  if (ng > 0) SG_TRY(alloc_pool(P, M));
  SG_HIP(h, hipStreamSynchronize(st));

  // ---- record the graph ----
  SG_HIP(h, hipStreamBeginCapture(st, hipStreamCaptureModeRelaxed));
  record_all(P);
  hipGraph_t g = nullptr;
  const hipError_t ec = hipStreamEndCapture(st, &g);
  if (ec != hipSuccess) return sg_check_hip(h, ec, "hipStreamEndCapture");
  P->graph = g;
  SG_HIP(h, hipGraphInstantiate(&P->exec, g, nullptr, nullptr, 0));
  return SG_OK;
}

}  // namespace

extern "C" {

sg_status sg_batch_plan(sg_handle* h, const sg_semiring* sr, int nprob, const sg_csr* A, const sg_csr* B,
                        int ngroups, const int32_t* group_offsets, size_t pool_bytes, sg_plan** out) {
  if (!h || !out) return SG_ERR_INVALID;
  *out = nullptr;
  if (!sr) return sg_fail(h, SG_ERR_INVALID, "semiring descriptor is NULL");
  static const int bytes[6] = {0, 8, 4, 8, 1, 4};
  if (sr->id < 1 || sr->id > 5 || sr->value_bytes != bytes[sr->id] || sr->acc_flags > SG_ACC_PLAIN)
    return sg_fail(h, SG_ERR_SEMIRING, "bad semiring descriptor");
  if (nprob < 1 || !A || !B) return sg_fail(h, SG_ERR_INVALID, "a batch needs at least one product");
  if (ngroups < 0 || (ngroups > 0 && !group_offsets)) return sg_fail(h, SG_ERR_INVALID, "bad merge groups");
  for (int q = 0; q < nprob; ++q) {
    const sg_csr* M[2] = {&A[q], &B[q]};
    for (const sg_csr* X : M) {
      if (X->nrows < 0 || X->ncols < 0 || X->nnz < 0 || !X->rowptr || (X->nnz > 0 && (!X->col || !X->val)))
        return sg_fail(h, SG_ERR_INVALID, "product " + std::to_string(q) + ": bad operand descriptor");
      if (X->ncols > INT32_MAX || X->nrows > INT32_MAX)
        return sg_fail(h, SG_ERR_OVERFLOW, "product " + std::to_string(q) + ": operand too large");
    }
    if (A[q].ncols != B[q].nrows) return sg_fail(h, SG_ERR_SHAPE, "product " + std::to_string(q) + ": A.ncols != B.nrows");
  }
  if (ngroups > 0) {
    if (group_offsets[0] < 0) return sg_fail(h, SG_ERR_INVALID, "group offsets must start at 0 or above");
    for (int g = 0; g < ngroups; ++g) {
      const int q0 = group_offsets[g], q1 = group_offsets[g + 1];
      if (q1 <= q0 || q1 > nprob) return sg_fail(h, SG_ERR_INVALID, "group offsets must ascend within [0, nprob]");
      for (int q = q0; q < q1; ++q)
        if (A[q].nrows != A[q0].nrows || B[q].ncols != B[q0].ncols)
          return sg_fail(h, SG_ERR_SHAPE, "products merged in one group differ in shape");
    }
  }
  SG_HIP(h, hipSetDevice(h->device));
  sg_plan* P = new sg_plan;
  P->h = h;
  P->sr = *sr;
  P->nprob = nprob;
  P->ngroups = ngroups;
  P->A.assign(A, A + nprob);
  P->B.assign(B, B + nprob);
  if (ngroups > 0) P->go.assign(group_offsets, group_offsets + ngroups + 1);
  sg_status s = sg_check_hip(h, hipStreamCreateWithFlags(&P->stream, hipStreamNonBlocking), "hipStreamCreate");
  if (s == SG_OK) s = plan_build(P, pool_bytes);
  if (s != SG_OK) {
    sg_plan_destroy(P);
    return s;
  }
  *out = P;
  return SG_OK;
}

sg_status sg_batch_execute(sg_plan* P, void* stream) {
  if (!P || !P->exec) return SG_ERR_INVALID;
  sg_handle* h = P->h;
  SG_HIP(h, hipSetDevice(h->device));
  SG_HIP(h, hipGraphLaunch(P->exec, (hipStream_t)stream));
  P->ran = true;
  return SG_OK;
}

sg_status sg_batch_results(sg_plan* P, sg_csr* out_C) {
  if (!P || !out_C) return SG_ERR_INVALID;
  sg_handle* h = P->h;
  if (!P->ran) return sg_fail(h, SG_ERR_INVALID, "the plan has not been executed");
  SG_HIP(h, hipSetDevice(h->device));
  SG_HIP(h, hipDeviceSynchronize());
  int32_t flags[2] = {0, 0};
  SG_HIP(h, hipMemcpy(flags, P->d_flag, sizeof(flags), hipMemcpyDeviceToHost));
  if (flags[0]) return sg_fail(h, SG_ERR_NOMEM, "the batch's outputs overflowed the plan's pool (patterns changed?)");
  if (flags[1]) return sg_fail(h, SG_ERR_INVALID, "a numeric pass filled a different number of entries than counted");
  const size_t vb = (size_t)P->sr.value_bytes;
  auto fill = [&](Stage& S, const std::vector<int64_t>& rbase, int64_t* lrow, int nres, int first,
                  const std::vector<int64_t>& nrows_of, const std::vector<int64_t>& ncols_of) -> sg_status {
    std::vector<int64_t> off((size_t)S.R + 1);
    SG_HIP(h, hipMemcpy(off.data(), S.off, sizeof(int64_t) * off.size(), hipMemcpyDeviceToHost));
    int64_t lb = 0;
    for (int q = 0; q < nres; ++q) {
      const int64_t o0 = off[(size_t)rbase[(size_t)q]], o1 = off[(size_t)rbase[(size_t)q + 1]];
      sg_csr& C = out_C[first + q];
      C.nrows = nrows_of[(size_t)q];
      C.ncols = ncols_of[(size_t)q];
      C.nnz = o1 - o0;
      C.rowptr = lrow + lb;
      C.col = (int32_t*)S.col_buf.p + o0;
      C.val = (char*)S.val_buf.p + (size_t)o0 * vb;
      lb += C.nrows + 1;
    }
    return SG_OK;
  };
  std::vector<int64_t> nr((size_t)P->nprob), nc((size_t)P->nprob);
  for (int q = 0; q < P->nprob; ++q) {
    nr[(size_t)q] = P->A[(size_t)q].nrows;
    nc[(size_t)q] = P->B[(size_t)q].ncols;
  }
  SG_TRY(fill(P->prod, P->rbase_p, P->d_lrow_p, P->nprob, 0, nr, nc));
  if (P->ngroups > 0) {
    std::vector<int64_t> gr((size_t)P->ngroups), gc((size_t)P->ngroups);
    for (int g = 0; g < P->ngroups; ++g) {
      gr[(size_t)g] = P->A[(size_t)P->go[(size_t)g]].nrows;
      gc[(size_t)g] = P->B[(size_t)P->go[(size_t)g]].ncols;
    }
    SG_TRY(fill(P->merg, P->rbase_m, P->d_lrow_m, P->ngroups, P->nprob, gr, gc));
  }
  return SG_OK;
}

sg_status sg_plan_destroy(sg_plan* P) {
  if (!P) return SG_ERR_INVALID;
  (void)hipSetDevice(P->h->device);
  if (P->stream) (void)hipStreamSynchronize(P->stream);
  (void)hipDeviceSynchronize();
  if (P->exec) (void)hipGraphExecDestroy(P->exec);
  if (P->graph) (void)hipGraphDestroy(P->graph);
  if (P->stream) (void)hipStreamDestroy(P->stream);
  P->prod.release();
  P->merg.release();
  for (auto& b : P->rp2) b.release();
  P->tables.release();
  delete P;
  return SG_OK;
}

}  // extern "C"
