// C-ABI of the semiring sparse product and merge (declared in include/spgemm.h).
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "sg_handle.hpp"
#include "sg_user.hpp"

using namespace sg;

sg_status sg_fail(sg_handle* h, sg_status s, const std::string& msg) {
  if (h) h->err = msg;
  return s;
}

sg_status sg_check_hip(sg_handle* h, hipError_t e, const char* what) {
  if (e == hipSuccess) return SG_OK;
  if (e == hipErrorOutOfMemory) return sg_fail(h, SG_ERR_NOMEM, std::string(what) + ": out of device memory");
  return sg_fail(h, SG_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

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

// Scratch of sg_spgemm_numeric_noalloc: a fixed device array, one copy per
// GPU the library runs on, held until the process ends.  Host code never
// passes `scratch` itself to a kernel (on the host it only names the symbol):
// its device address is looked up once per device at handle creation and
// kept in g_scratch_ptr.
static __device__ __align__(256) unsigned char scratch[SG_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on `device` (the current device), looked up on
// the first call for that device.
hipError_t bind_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return hipSuccess;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  if (!ptr) return hipErrorInvalidSymbol;
  g_scratch_ptr[device] = ptr;
  return hipSuccess;
}

void* scratch_ptr(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return g_scratch_ptr[device];
}
}  // namespace

sg_status Scratch::take(SgBuf& b, size_t bytes) {
  if (!base) return sg_check_hip(h, b.ensure(bytes), "hipMalloc (scratch)");
  const size_t o = (off + 255) & ~(size_t)255;
  if (o > cap || bytes > cap - o)
    return sg_fail(h, SG_ERR_NOMEM, "the product needs more scratch than the fixed " + std::to_string(cap >> 20) +
                                        " MiB device array of the no-allocation entry point holds");
  b.p = base + o;
  b.cap = bytes;
  off = o + bytes;
  return SG_OK;
}

namespace sg {

int32_t tiles_of(int64_t ncols) {
  const int64_t t = (ncols + kTile - 1) / kTile;
  return t < 1 ? 1 : (int32_t)t;
}

Policy make_policy(const sg_handle* h, int numeric, const sg_semiring* sr, int32_t T) {
  Policy p{};
  // the library's semirings merge hash rows over B wider than the bitmap
  // kernels' 65,536 columns; such a row holds all its products in LDS, so its
  // bin is chosen by its products
  p.by_products = numeric && h->merge_rows && sr && sr->id >= 1 && sr->id <= 5 && T > 0 &&
                  narrow_words((int64_t)T * kTile) == 0;
  p.numeric = numeric;
  p.force = h->force;
  p.hash_max = h->hash_max;
  p.comp_mode = kCompNone;
  p.comp_min_terms = 64;
  p.comp_min_products = 0;
  if (sr && sr->id == SG_PLUS_TIMES_F32) {
    p.comp_mode = sr->acc_flags == SG_ACC_PLAIN ? kCompNone
                  : sr->acc_flags == SG_ACC_COMPENSATED ? kCompAll
                                                        : kCompRule;
    p.comp_min_terms = sr->comp_min_terms;
    p.comp_min_products = sr->comp_min_products;
  }
  return p;
}

static void handle_mark(void* ctx, int phase, int begin) {
  sg_handle* h = (sg_handle*)ctx;
  (void)hipEventRecord(h->ev[phase][begin ? 0 : 1], h->mark_stream);
  if (!begin) h->ev_rec[phase] = true;
}

Marks handle_marks(sg_handle* h, hipStream_t st) {
  Marks m;
  if (h->timing) {
    m.fn = handle_mark;
    m.ctx = h;
    h->mark_stream = st;
  }
  return m;
}

void clear_phases(sg_handle* h, int p0, int p1) {
  for (int p = p0; p < p1; ++p) h->ev_rec[p] = false;
}

size_t plan_rows_bytes(int64_t nrows) {
  SgArena a;
  const int64_t nblk = analyze_blocks(nrows);
  a.take<int64_t>(nrows);
  a.take<uint8_t>(nrows);
  a.take<int32_t>(nblk * kNB);
  a.take<int32_t>(nblk * kNB);
  a.take<int32_t>(kNB);
  a.take<int32_t>(kNB);
  a.take<int32_t>(nrows);
  a.take<int32_t>(nrows);
  return a.off;
}

sg_status plan_rows(sg_handle* h, const RowSource& r, const Policy& pol, const int64_t* c_rowptr, int64_t* cnt_out,
                    SgArena& ar, BinPlan& plan, hipStream_t st, int64_t* p_keep, int32_t* nt_keep, bool rebin) {
  const int64_t n = r.nrows;
  const int64_t nblk = analyze_blocks(n);
  int64_t* p = ar.take<int64_t>(n);
  uint8_t* bin = ar.take<uint8_t>(n);
  int32_t* hist = ar.take<int32_t>(nblk * kNB);
  int32_t* blk_off = ar.take<int32_t>(nblk * kNB);
  int32_t* bin_start = ar.take<int32_t>(kNB);
  int32_t* bin_count = ar.take<int32_t>(kNB);
  int32_t* list = ar.take<int32_t>(n);
  int32_t* nt = ar.take<int32_t>(n);
  if (p_keep) p = p_keep;
  if (nt_keep) nt = nt_keep;
  if (rebin) launch_rebin(p, nt, c_rowptr, n, pol, bin, hist, blk_off, bin_start, bin_count, list, st);
  else launch_analyze(r, pol, c_rowptr, p, nt, bin, hist, blk_off, bin_start, bin_count, list, cnt_out, st);
  int32_t* hp = (int32_t*)h->h_pin;
  SG_HIP(h, hipMemcpyAsync(hp, bin_count, kNB * sizeof(int32_t), hipMemcpyDeviceToHost, st));
  SG_HIP(h, hipMemcpyAsync(hp + kNB, bin_start, kNB * sizeof(int32_t), hipMemcpyDeviceToHost, st));
  SG_HIP(h, hipStreamSynchronize(st));
  std::memcpy(plan.count, hp, sizeof(plan.count));
  std::memcpy(plan.start, hp + kNB, sizeof(plan.start));
  plan.bins.list = list;
  plan.bins.start = bin_start;
  plan.bins.count = bin_count;
  plan.bins.nd_cap = plan.ndense();
  return SG_OK;
}

sg_status build_slabs(sg_handle* h, Scratch& sc, SlabBufs& sb, RowSource& r, const sg_csr* B, int vbytes, bool cols,
                      bool vals, int64_t* partial, int32_t* err, int32_t* qctr, hipStream_t st) {
  const int32_t ls = slab_log(r.ncols, h->slab_ls), S = slab_count(r.ncols, ls);
  const int64_t nb = B->nrows;
  const size_t ne = (size_t)(B->nnz > 0 ? B->nnz : 1);
  const int32_t G = 1 << (ls - kTileLog);
  if (cols) {
    SG_TRY(sc.take(sb.bnd, sizeof(int32_t) * (size_t)nb * (size_t)(S + 1)));
    SG_TRY(sc.take(sb.rpt, sizeof(int32_t) * (size_t)S * (size_t)nb * (size_t)(G + 1)));
    SG_TRY(sc.take(sb.prow, sizeof(int64_t) * ((size_t)S * (size_t)nb + 1)));
    SG_TRY(sc.take(sb.pbit, sizeof(int32_t) * ne));
  }
  // numeric partition entries: (column, value) pairs, 8 bytes (16 for 8-byte values)
  if (vals) SG_TRY(sc.take(sb.pcv, (size_t)(vbytes >= 8 ? 16 : 8) * ne));
  // destinations of B's entries (int32 positions) for the value scatters of
  // later numeric passes on the same structure
  const bool use_perm = B->nnz <= INT32_MAX;
  if (cols && use_perm) SG_TRY(sc.take(sb.perm, sizeof(int32_t) * ne));
  launch_slab_partition(B->rowptr, B->col, B->val, vbytes, nb, B->nnz, ls, S, r.T, (int32_t*)sb.bnd.p,
                        (int32_t*)sb.rpt.p, (int64_t*)sb.prow.p, partial, (int32_t*)sb.pbit.p,
                        vals ? sb.pcv.p : nullptr, use_perm ? (int32_t*)sb.perm.p : nullptr, cols, vals, err, h->cus,
                        st);
  r.rpt = (const int32_t*)sb.rpt.p;
  r.prow = (const int64_t*)sb.prow.p;
  r.pbit = (const int32_t*)sb.pbit.p;
  // 32-bit gathers need the bitmap-code array (4 bytes per entry) below 4 GiB
  r.gather32 = h->gather32 && B->nnz < ((int64_t)1 << 30);
  r.b_nnz = B->nnz;
  r.pval = vals ? sb.pcv.p : nullptr;
  r.ls = ls;
  r.S = S;
  r.qctr = qctr;
  return SG_OK;
}

sg_status build_dense_rows(sg_handle* h, Scratch& sc, SlabBufs& sb, RowSource& r, const BinPlan& plan,
                           hipStream_t st) {
  const int32_t nd = plan.bins.nd_cap;
  SG_TRY(sc.take(sb.dr, sizeof(DenseRow) * (size_t)(nd > 0 ? nd : 1)));
  launch_dense_rows(plan, r.a_rowptr, (DenseRow*)sb.dr.p, h->cus, st);
  r.drow = (const DenseRow*)sb.dr.p;
  return SG_OK;
}

int32_t light_cap_for(const sg_handle* h, const sg_semiring* sr) {
  // a tuned cap belongs to the semiring it was tuned on; a cap set as an
  // option (tuned_sr == 0) applies to every semiring
  if (h->light_cap <= 0) return 0;
  if (h->tuned_sr != 0 && (sr == nullptr || sr->id != h->tuned_sr || sr->value_bytes != h->tuned_vb)) return 0;
  return h->light_cap;
}

size_t slab_partials(const sg_handle* h, const RowSource& r) {
  if (r.mode != kModeProduct || !h->slab) return 0;
  const int32_t ls = slab_log(r.ncols, h->slab_ls);
  return (size_t)scan_partials_len((int64_t)slab_count(r.ncols, ls) * r.b_nrows);
}

}  // namespace sg

namespace {

const char* const kInconsistent =
    "inconsistent structure: a numeric pass filled a different number of entries than its symbolic pass, or B "
    "holds unsorted or out-of-range columns";

sg_status check_csr(sg_handle* h, const sg_csr* M, const char* name) {
  if (!M) return sg_fail(h, SG_ERR_INVALID, std::string(name) + " is NULL");
  if (M->nrows < 0 || M->ncols < 0 || M->nnz < 0) return sg_fail(h, SG_ERR_INVALID, std::string(name) + ": negative size");
  if (M->ncols > INT32_MAX || M->nrows > INT32_MAX)
    return sg_fail(h, SG_ERR_OVERFLOW, std::string(name) + ": more than 2^31-1 rows or columns");
  if (!M->rowptr) return sg_fail(h, SG_ERR_INVALID, std::string(name) + ".rowptr is NULL");
  if (M->nnz > 0 && !M->col) return sg_fail(h, SG_ERR_INVALID, std::string(name) + ".col is NULL");
  return SG_OK;
}

sg_status check_semiring(sg_handle* h, const sg_semiring* sr) {
  if (!sr) return sg_fail(h, SG_ERR_INVALID, "semiring descriptor is NULL");
  static const int bytes[6] = {0, 8, 4, 8, 1, 4};
  int vb = 0;
  if (sr->id >= kUserSemiringBase && user_semiring(sr->id, &vb, nullptr)) {
    if (sr->value_bytes != vb) return sg_fail(h, SG_ERR_SEMIRING, "value_bytes does not match the semiring");
    if (sr->acc_flags != SG_ACC_DEFAULT) return sg_fail(h, SG_ERR_SEMIRING, "run-time semirings take no accumulation flag");
    return SG_OK;
  }
  if (sr->id < 1 || sr->id > 5) return sg_fail(h, SG_ERR_SEMIRING, "unknown semiring id");
  if (sr->value_bytes != bytes[sr->id]) return sg_fail(h, SG_ERR_SEMIRING, "value_bytes does not match the semiring");
  if (sr->acc_flags > SG_ACC_PLAIN) return sg_fail(h, SG_ERR_SEMIRING, "unknown accumulation flag");
  return SG_OK;
}

sg_status validate_input(sg_handle* h, const sg_csr* M, const char* name, hipStream_t st) {
  if (!h->validate || M->nrows == 0) return SG_OK;
  int32_t* flag = h->d_flags + 2;
  launch_fill_i32(flag, 1, 0, st);
  launch_validate(M->rowptr, M->col, M->nrows, M->ncols, M->nnz, flag, st);
  int32_t v = 0;
  SG_HIP(h, hipMemcpyAsync(h->h_pin, flag, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  SG_HIP(h, hipStreamSynchronize(st));
  std::memcpy(&v, h->h_pin, sizeof(v));
  if (v) return sg_fail(h, SG_ERR_UNSORTED, std::string(name) + ": unsorted or duplicate column, or bad row offsets");
  return SG_OK;
}

SgCacheKey product_key(const sg_handle* h, const sg_csr* A, const sg_csr* B) {
  SgCacheKey k{};
  k.w[0] = 1;
  k.w[1] = (uint64_t)(uintptr_t)A->rowptr;
  k.w[2] = (uint64_t)(uintptr_t)A->col;
  k.w[3] = (uint64_t)A->nrows;
  k.w[4] = (uint64_t)A->ncols;
  k.w[5] = (uint64_t)A->nnz;
  k.w[6] = (uint64_t)(uintptr_t)B->rowptr;
  k.w[7] = (uint64_t)(uintptr_t)B->col;
  k.w[8] = (uint64_t)B->nrows;
  k.w[9] = (uint64_t)B->ncols;
  k.w[10] = (uint64_t)B->nnz;
  k.w[11] = (uint64_t)h->force;
  k.w[12] = (uint64_t)h->hash_max;
  k.w[13] = (uint64_t)h->slab;
  k.w[14] = (uint64_t)h->slab_ls;
  return k;
}

SgCacheKey merge_key(const sg_handle* h, int nparts, const sg_csr* parts) {
  SgCacheKey k{};
  k.w[0] = 2;
  uint64_t a = 1469598103934665603ull;
  for (int s = 0; s < nparts; ++s) {
    const uint64_t v[5] = {(uint64_t)(uintptr_t)parts[s].rowptr, (uint64_t)(uintptr_t)parts[s].col,
                           (uint64_t)parts[s].nrows, (uint64_t)parts[s].ncols, (uint64_t)parts[s].nnz};
    for (uint64_t x : v) a = (a ^ x) * 1099511628211ull;
  }
  k.w[1] = a;
  k.w[2] = (uint64_t)nparts;
  k.w[11] = (uint64_t)h->force;
  k.w[12] = (uint64_t)h->hash_max;
  return k;
}

sg_status upload_parts(sg_handle* h, int nparts, const sg_csr* parts, hipStream_t st) {
  h->parts_host.resize((size_t)nparts);
  for (int s = 0; s < nparts; ++s)
    h->parts_host[(size_t)s] = PartDesc{parts[s].rowptr, parts[s].col, parts[s].val, parts[s].nnz};
  SG_HIP(h, h->parts_buf.ensure(sizeof(PartDesc) * (size_t)nparts));
  SG_HIP(h, hipMemcpyAsync(h->parts_buf.p, h->parts_host.data(), sizeof(PartDesc) * (size_t)nparts,
                           hipMemcpyHostToDevice, st));
  return SG_OK;
}

// Shared body of the two symbolic entry points: counts into C_rowptr[1..n],
// dense-row tile offsets into the handle's cache, scan, readback of nnz.
sg_status run_symbolic(sg_handle* h, RowSource& r, const sg_csr* B, int64_t* C_rowptr, int64_t* nnzC,
                       const SgCacheKey& key, hipStream_t st) {
  const int64_t n = r.nrows;
  SgArena measure;
  measure.off = plan_rows_bytes(n);
  measure.take<int64_t>(scan_partials_len(n));
  measure.take<int64_t>(slab_partials(h, r));
  SG_HIP(h, h->ws.ensure(measure.off));
  SgArena ar;
  ar.base = (char*)h->ws.p;
  BinPlan plan;
  const Policy pol = make_policy(h, 0, nullptr);
  clear_phases(h, kPhSymAnalyze, kPhNumAnalyze);
  clear_phases(h, kPhSymDenseBitmap, kPhSymDenseBitmap + 1);
  const Marks mk = handle_marks(h, st);
  SG_HIP(h, h->p_buf.ensure(sizeof(int64_t) * (size_t)(n > 0 ? n : 1)));
  SG_HIP(h, h->nt_buf.ensure(sizeof(int32_t) * (size_t)(n > 0 ? n : 1)));
  mk.mark(kPhSymAnalyze, 1);
  SG_TRY(plan_rows(h, r, pol, nullptr, C_rowptr + 1, ar, plan, st, (int64_t*)h->p_buf.p, (int32_t*)h->nt_buf.p));
  mk.mark(kPhSymAnalyze, 0);
  const int32_t nd = plan.ndense();
  int32_t* off2 = nullptr;
  int64_t* partial = ar.take<int64_t>(scan_partials_len(n));
  int64_t* spartial = ar.take<int64_t>(slab_partials(h, r));
  if (nd > 0) {
    const bool slab = r.mode == kModeProduct && h->slab;
    const bool tiles = !slab && r.mode == kModeProduct && r.T > 1;
    if (tiles) SG_HIP(h, h->rp2_buf.ensure(sizeof(int32_t) * (size_t)B->nrows * (size_t)(r.T + 1)));
    // the slab path keeps span counts after the tile offsets
    SG_HIP(h, h->off2_buf.ensure(slab ? off2_span_bytes(nd, r.T) : sizeof(int32_t) * (size_t)nd * (size_t)(r.T + 1)));
    off2 = (int32_t*)h->off2_buf.p;
    if (slab) r.spn = (uint4*)((char*)h->off2_buf.p + span_offset(nd, r.T));
    mk.mark(kPhSymBounds, 1);
    if (tiles) {
      r.rp2 = (const int32_t*)h->rp2_buf.p;
      launch_tile_bounds(B->rowptr, B->col, B->nrows, r.T, (int32_t*)h->rp2_buf.p, h->cus, st);
    }
    if (slab) {
      Scratch sc{h};
      SG_TRY(build_slabs(h, sc, h->sb, r, B, 0, true, false, spartial, h->d_flags, h->d_flags + kCtrBase, st));
      SG_TRY(build_dense_rows(h, sc, h->sb, r, plan, st));
    }
    mk.mark(kPhSymBounds, 0);
  }
  r.merge_rows = h->merge_rows;
  launch_symbolic(r, plan, C_rowptr + 1, off2, h->cus, mk, st);
  mk.mark(kPhSymScan, 1);
  launch_fill_i64(C_rowptr, 1, 0, st);
  launch_scan_inclusive(C_rowptr + 1, n, partial, st);
  mk.mark(kPhSymScan, 0);
  SG_HIP(h, hipGetLastError());
  SG_HIP(h, hipMemcpyAsync(h->h_pin, C_rowptr + n, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  // the device-side consistency flag (set by an earlier numeric pass of this
  // handle, or by this pass's partition of B) comes back with nnz(C)
  SG_HIP(h, hipMemcpyAsync(h->h_pin + 1, h->d_flags, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  SG_HIP(h, hipStreamSynchronize(st));
  *nnzC = h->h_pin[0];
  int32_t flag = 0;
  std::memcpy(&flag, h->h_pin + 1, sizeof(flag));
  if (flag) {
    h->cache_valid = false;
    launch_fill_i32(h->d_flags, 1, 0, st);
    (void)hipStreamSynchronize(st);
    return sg_fail(h, SG_ERR_INVALID, kInconsistent);
  }
  h->cache_valid = true;
  h->cache_key = key;
  h->cache_T = r.T;
  h->cache_nd = nd;
  h->cache_n = n;
  return SG_OK;
}

// Buffers a numeric call draws its scratch from (the handle's own, or
// call-local views into the fixed array of the no-allocation entry point).
struct NumBufs {
  SgBuf& ws;
  SlabBufs& sb;
  SgBuf& off2;
  SgBuf& task;
  SgBuf& rp2;
};

// use_cache: the handle's saved structure of the last symbolic pass may be
// reused (per-row counts, B's partition, dense-row tile offsets).  Without it
// every structure-dependent table is rebuilt into `bufs`.
sg_status run_numeric(sg_handle* h, const sg_semiring* sr, RowSource& r, const sg_csr* B, sg_csr* C,
                      const SgCacheKey& key, hipStream_t st, Scratch& sc, const NumBufs& bufs, bool use_cache) {
  const int64_t n = r.nrows;
  SgArena measure;
  measure.off = plan_rows_bytes(n);
  measure.take<int64_t>(n);
  measure.take<int64_t>(slab_partials(h, r));
  SG_TRY(sc.take(bufs.ws, measure.off));
  SgArena ar;
  ar.base = (char*)bufs.ws.p;
  BinPlan plan;
  const Policy pol = make_policy(h, 1, sr, r.T);
  clear_phases(h, kPhNumAnalyze, kPhSymDenseBitmap);
  clear_phases(h, kPhNumDenseSlab, kNPhases);
  const Marks mk = handle_marks(h, st);
  // Same structure as the last symbolic call: its per-row counts give the bins
  // without touching A or B again.  Dense classification depends only on the
  // product count and the key's options, so the dense list is unchanged.
  const bool same =
      use_cache && h->cache_valid && h->cache_key == key && h->cache_T == r.T && h->cache_n == n;
  mk.mark(kPhNumAnalyze, 1);
  if (same)
    SG_TRY(plan_rows(h, r, pol, C->rowptr, nullptr, ar, plan, st, (int64_t*)h->p_buf.p, (int32_t*)h->nt_buf.p, true));
  else
    SG_TRY(plan_rows(h, r, pol, C->rowptr, nullptr, ar, plan, st));
  const int32_t nd = plan.ndense();
  const bool cached = same && h->cache_nd == nd;
  const bool slab = r.mode == kModeProduct && h->slab && nd > 0;
  if (nd > 0) {
    if (slab) {
      // structure from the last symbolic pass when cached; values every call
      int64_t* spartial = ar.take<int64_t>(slab_partials(h, r));
      SG_TRY(build_slabs(h, sc, bufs.sb, r, B, sr->value_bytes, !cached, true, spartial, h->d_flags,
                         h->d_flags + kCtrBase, st));
      SG_TRY(build_dense_rows(h, sc, bufs.sb, r, plan, st));
    } else if (r.mode == kModeProduct && r.T > 1) {
      if (!cached) {
        SG_TRY(sc.take(bufs.rp2, sizeof(int32_t) * (size_t)B->nrows * (size_t)(r.T + 1)));
        launch_tile_bounds(B->rowptr, B->col, B->nrows, r.T, (int32_t*)bufs.rp2.p, h->cus, st);
      }
      r.rp2 = (const int32_t*)bufs.rp2.p;
    }
    // the slab path keeps span counts after the tile offsets
    SG_TRY(sc.take(bufs.off2, slab ? off2_span_bytes(nd, r.T) : sizeof(int32_t) * (size_t)nd * (size_t)(r.T + 1)));
    if (slab) r.spn = (uint4*)((char*)bufs.off2.p + span_offset(nd, r.T));
    if (!cached) {
      int64_t* counts = ar.take<int64_t>(n);
      launch_symbolic_dense(r, plan, counts, (int32_t*)bufs.off2.p, h->cus, st);
      // off2 of the handle now belongs to this call's inputs only
      if (!sc.fixed()) h->cache_valid = false;
    }
  }
  mk.mark(kPhNumAnalyze, 0);
  NumCtx c{};
  c.marks = mk;
  c.src = r;
  c.plan = plan;
  c.C = OutC{C->rowptr, C->col, C->val};
  c.off2 = (const int32_t*)bufs.off2.p;
  c.spn = r.spn;
  c.err = h->d_flags;
  c.task_ctr = h->d_flags + kCtrBase;
  c.task_cap = (int64_t)(nd > 0 ? nd : 1) * r.T;
  if (slab) {
    const size_t tb = 2 * sizeof(SlabTask) * (size_t)nd * (size_t)r.S;  // light and heavy lists
    SG_TRY(sc.take(bufs.task, tb + sizeof(int32_t) * (6 * (size_t)r.T + 3)));
    c.slab_tasks = (SlabTask*)bufs.task.p;
    c.slab_book = (int32_t*)((char*)bufs.task.p + tb);
  } else if (nd > 0) {
    SG_TRY(sc.take(bufs.task, task_buffer_bytes(c.task_cap, r.T)));
    c.tasks = (Task*)bufs.task.p;
  }
  c.tile_min = h->tile_min;
  c.cus = h->cus;
  c.merge_rows = h->merge_rows;
  c.comp_dense = pol.comp_mode != kCompNone;
  c.light_cap = light_cap_for(h, sr);
  h->last_nd = nd;
  switch (sr->id) {
    case SG_PLUS_TIMES_I64: launch_numeric_i64(c, st); break;
    case SG_PLUS_TIMES_F32: launch_numeric_f32(c, st); break;
    case SG_PLUS_TIMES_F64: launch_numeric_f64(c, st); break;
    case SG_OR_AND_BOOL: launch_numeric_bool(c, st); break;
    case SG_MIN_PLUS_F32: launch_numeric_minplus(c, st); break;
    default: SG_TRY(launch_numeric_user(h, c, sr->id, st)); break;
  }
  SG_HIP(h, hipGetLastError());
  return SG_OK;
}

sg_status run_numeric(sg_handle* h, const sg_semiring* sr, RowSource& r, const sg_csr* B, sg_csr* C,
                      const SgCacheKey& key, hipStream_t st) {
  Scratch sc{h};
  const NumBufs bufs{h->ws, h->sb, h->off2_buf, h->task_buf, h->rp2_buf};
  return run_numeric(h, sr, r, B, C, key, st, sc, bufs, true);
}

const char* env(const char* name) {
  const char* v = std::getenv(name);
  return (v && *v) ? v : nullptr;
}

}  // namespace

extern "C" {

sg_status sg_semiring_make(sg_semiring_id id, uint32_t acc_flags, sg_semiring* out) {
  if (!out) return SG_ERR_INVALID;
  static const int bytes[6] = {0, 8, 4, 8, 1, 4};
  if ((int)id < 1 || (int)id > 5) return SG_ERR_SEMIRING;
  if (acc_flags > SG_ACC_PLAIN) return SG_ERR_SEMIRING;
  out->id = (int32_t)id;
  out->value_bytes = bytes[id];
  out->acc_flags = acc_flags;
  out->comp_min_terms = 64;
  out->comp_min_products = 0;
  return SG_OK;
}

sg_status sg_handle_set_option(sg_handle* h, const char* name, const char* value) {
  if (!h || !name || !value) return SG_ERR_INVALID;
  const std::string n(name), v(value);
  if (n == "hash_max_products") {
    char* end = nullptr;
    const long long x = std::strtoll(value, &end, 10);
    if (!end || *end || x < 0 || x > kHashCap) return sg_fail(h, SG_ERR_INVALID, "hash_max_products must be in [0, 4096]");
    h->hash_max = x;
  } else if (n == "dense_tile_min") {
    char* end = nullptr;
    const long long x = std::strtoll(value, &end, 10);
    if (!end || *end || x < 1 || x > kRangeCap)
      return sg_fail(h, SG_ERR_INVALID, "dense_tile_min must be in [1, 2048]");
    h->tile_min = (int32_t)x;
    return SG_OK;
  } else if (n == "slab_log") {
    char* end = nullptr;
    const long long x = std::strtoll(value, &end, 10);
    if (!end || *end || (x != 0 && (x < kSlabLogMin || x > kSlabLogMax)))
      return sg_fail(h, SG_ERR_INVALID, "slab_log must be 0 (automatic) or in [14, 17]");
    h->slab_ls = (int32_t)x;
  } else if (n == "light_cap") {
    char* end = nullptr;
    const long long x = std::strtoll(value, &end, 10);
    if (!end || *end || x < 0 || x > 32768)
      return sg_fail(h, SG_ERR_INVALID, "light_cap must be 0 (the LDS capacity) or in [1, 32768]");
    h->light_cap = (int32_t)x;
    h->tuned_sr = 0;  // set by hand: applies to every semiring
    h->tuned_vb = 0;
    return SG_OK;
  } else if (n == "dense_slab") {
    if (v != "0" && v != "1") return sg_fail(h, SG_ERR_INVALID, "dense_slab must be 0 or 1");
    h->slab = v == "1";
  } else if (n == "gather32") {
    if (v != "0" && v != "1") return sg_fail(h, SG_ERR_INVALID, "gather32 must be 0 or 1");
    h->gather32 = v == "1";
  } else if (n == "merge_rows") {
    if (v != "0" && v != "1") return sg_fail(h, SG_ERR_INVALID, "merge_rows must be 0 or 1");
    h->merge_rows = v == "1";
  } else if (n == "force_path") {
    if (v == "auto") h->force = kForceAuto;
    else if (v == "small") h->force = kForceSmall;
    else if (v == "hash") h->force = kForceHash;
    else if (v == "dense") h->force = kForceDense;
    else return sg_fail(h, SG_ERR_INVALID, "force_path must be auto, small, hash or dense");
  } else if (n == "validate") {
    if (v != "0" && v != "1") return sg_fail(h, SG_ERR_INVALID, "validate must be 0 or 1");
    h->validate = v == "1";
  } else if (n == "timing") {
    if (v != "0" && v != "1") return sg_fail(h, SG_ERR_INVALID, "timing must be 0 or 1");
    if (v == "1" && !h->ev[0][0]) {
      for (int p = 0; p < kNPhases; ++p)
        for (int b = 0; b < 2; ++b)
          if (hipEventCreate(&h->ev[p][b]) != hipSuccess) return sg_fail(h, SG_ERR_HIP, "hipEventCreate failed");
    }
    h->timing = v == "1";
    clear_phases(h, 0, kNPhases);
    return SG_OK;
  } else {
    return sg_fail(h, SG_ERR_INVALID, "unknown option " + n);
  }
  h->cache_valid = false;
  return SG_OK;
}


sg_status sg_handle_create(int device, const char* tuning_json, sg_handle** out) {
  if (!out) return SG_ERR_INVALID;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) return SG_ERR_HIP;
  if (device < 0 || device >= ndev) return SG_ERR_INVALID;
  if (hipSetDevice(device) != hipSuccess) return SG_ERR_HIP;
  sg_handle* h = new sg_handle;
  h->device = device;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) {
    delete h;
    return SG_ERR_HIP;
  }
  h->cus = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
  if (bind_scratch(device) != hipSuccess) {
    delete h;
    return SG_ERR_HIP;
  }
  if (hipMalloc(&h->d_flags, kFlagInts * sizeof(int32_t)) != hipSuccess) {
    delete h;
    return SG_ERR_NOMEM;
  }
  (void)hipMemset(h->d_flags, 0, kFlagInts * sizeof(int32_t));
  if (hipHostMalloc(&h->h_pin, 4096, hipHostMallocDefault) != hipSuccess) {
    (void)hipFree(h->d_flags);
    delete h;
    return SG_ERR_NOMEM;
  }
  if (const char* v = env("SG_VALIDATE")) h->validate = std::atoi(v) != 0;
  if (const char* v = env("SG_FORCE_PATH")) {
    if (sg_handle_set_option(h, "force_path", v) != SG_OK) {
      sg_handle_destroy(h);
      return SG_ERR_INVALID;
    }
  }
  if (const char* v = env("SG_HASH_MAX")) {
    if (sg_handle_set_option(h, "hash_max_products", v) != SG_OK) {
      sg_handle_destroy(h);
      return SG_ERR_INVALID;
    }
  }
  const char* tj = tuning_json ? tuning_json : env("SG_TUNING");
  if (tj) {
    const sg_status s = sg_tune_load(h, nullptr, tj);
    if (s != SG_OK) {
      sg_handle_destroy(h);
      return s;
    }
  }
  (void)hipDeviceSynchronize();
  *out = h;
  return SG_OK;
}

sg_status sg_handle_destroy(sg_handle* h) {
  if (!h) return SG_ERR_INVALID;
  (void)hipSetDevice(h->device);
  (void)hipDeviceSynchronize();
  h->ws.release();
  h->task_buf.release();
  h->p_buf.release();
  h->nt_buf.release();
  h->sb.release();
  h->rp2_buf.release();
  h->off2_buf.release();
  h->parts_buf.release();
  if (h->d_flags) (void)hipFree(h->d_flags);
  if (h->h_pin) (void)hipHostFree(h->h_pin);
  for (int p = 0; p < kNPhases; ++p)
    for (int b = 0; b < 2; ++b)
      if (h->ev[p][b]) (void)hipEventDestroy(h->ev[p][b]);
  delete h;
  return SG_OK;
}

sg_status sg_spgemm_symbolic(sg_handle* h, const sg_csr* A, const sg_csr* B, int64_t* C_rowptr, int64_t* nnzC,
                             void* stream) {
  if (!h) return SG_ERR_INVALID;
  SG_TRY(check_csr(h, A, "A"));
  SG_TRY(check_csr(h, B, "B"));
  if (!C_rowptr || !nnzC) return sg_fail(h, SG_ERR_INVALID, "C_rowptr or nnzC is NULL");
  if (A->ncols != B->nrows) return sg_fail(h, SG_ERR_SHAPE, "A.ncols != B.nrows");
  SG_HIP(h, hipSetDevice(h->device));
  hipStream_t st = (hipStream_t)stream;
  SG_TRY(validate_input(h, A, "A", st));
  SG_TRY(validate_input(h, B, "B", st));
  RowSource r{};
  r.a_rowptr = A->rowptr;
  r.a_col = A->col;
  r.b_rowptr = B->rowptr;
  r.b_col = B->col;
  r.b_nrows = B->nrows;
  r.nrows = A->nrows;
  r.ncols = B->ncols;
  r.T = tiles_of(B->ncols);
  if (A->nrows == 0 || A->nnz == 0 || B->nnz == 0) {
    // an empty operand: every row of C is empty (paper, Section 4.3 multiplies
    // only when both inputs hold a nonzero)
    launch_fill_i64(C_rowptr, A->nrows + 1, 0, st);
    SG_HIP(h, hipGetLastError());
    SG_HIP(h, hipStreamSynchronize(st));
    *nnzC = 0;
    h->cache_valid = false;
    return SG_OK;
  }
  return run_symbolic(h, r, B, C_rowptr, nnzC, product_key(h, A, B), st);
}

sg_status sg_spgemm_numeric(sg_handle* h, const sg_semiring* sr, const sg_csr* A, const sg_csr* B, sg_csr* C,
                            void* stream) {
  if (!h) return SG_ERR_INVALID;
  SG_TRY(check_semiring(h, sr));
  SG_TRY(check_csr(h, A, "A"));
  SG_TRY(check_csr(h, B, "B"));
  SG_TRY(check_csr(h, C, "C"));
  if (A->ncols != B->nrows || C->nrows != A->nrows || C->ncols != B->ncols)
    return sg_fail(h, SG_ERR_SHAPE, "shapes of A, B and C do not match");
  if ((A->nnz > 0 && !A->val) || (B->nnz > 0 && !B->val) || (C->nnz > 0 && !C->val))
    return sg_fail(h, SG_ERR_INVALID, "a value array is NULL");
  SG_HIP(h, hipSetDevice(h->device));
  hipStream_t st = (hipStream_t)stream;
  if (A->nrows == 0 || C->nnz == 0) return SG_OK;
  SG_TRY(validate_input(h, A, "A", st));
  SG_TRY(validate_input(h, B, "B", st));
  RowSource r{};
  r.a_rowptr = A->rowptr;
  r.a_col = A->col;
  r.a_val = A->val;
  r.b_rowptr = B->rowptr;
  r.b_col = B->col;
  r.b_val = B->val;
  r.b_nrows = B->nrows;
  r.nrows = A->nrows;
  r.ncols = B->ncols;
  r.T = tiles_of(B->ncols);
  return run_numeric(h, sr, r, B, C, product_key(h, A, B), st);
}

sg_status sg_spgemm_numeric_noalloc(sg_handle* h, const sg_semiring* sr, const sg_csr* A, const sg_csr* B,
                                    sg_csr* C, void* stream) {
  if (!h) return SG_ERR_INVALID;
  SG_TRY(check_semiring(h, sr));
  SG_TRY(check_csr(h, A, "A"));
  SG_TRY(check_csr(h, B, "B"));
  SG_TRY(check_csr(h, C, "C"));
  if (A->ncols != B->nrows || C->nrows != A->nrows || C->ncols != B->ncols)
    return sg_fail(h, SG_ERR_SHAPE, "shapes of A, B and C do not match");
  if ((A->nnz > 0 && !A->val) || (B->nnz > 0 && !B->val) || (C->nnz > 0 && !C->val))
    return sg_fail(h, SG_ERR_INVALID, "a value array is NULL");
  SG_HIP(h, hipSetDevice(h->device));
  char* base = (char*)scratch_ptr(h->device);
  if (!base) return sg_fail(h, SG_ERR_HIP, "the fixed scratch array is not bound on this device");
  hipStream_t st = (hipStream_t)stream;
  if (A->nrows == 0 || C->nnz == 0) return SG_OK;
  SG_TRY(validate_input(h, A, "A", st));
  SG_TRY(validate_input(h, B, "B", st));
  RowSource r{};
  r.a_rowptr = A->rowptr;
  r.a_col = A->col;
  r.a_val = A->val;
  r.b_rowptr = B->rowptr;
  r.b_col = B->col;
  r.b_val = B->val;
  r.b_nrows = B->nrows;
  r.nrows = A->nrows;
  r.ncols = B->ncols;
  r.T = tiles_of(B->ncols);
  Scratch sc{h, base, (size_t)SG_NOALLOC_SCRATCH_BYTES, 0};
  // call-local views into the fixed array; never released
  SgBuf ws, off2, task, rp2;
  SlabBufs sb;
  const NumBufs bufs{ws, sb, off2, task, rp2};
  return run_numeric(h, sr, r, B, C, product_key(h, A, B), st, sc, bufs, false);
}

static sg_status check_parts(sg_handle* h, int nparts, const sg_csr* parts) {
  if (nparts < 1 || nparts > 4096 || !parts) return sg_fail(h, SG_ERR_INVALID, "nparts must be in [1, 4096]");
  for (int s = 0; s < nparts; ++s) {
    SG_TRY(check_csr(h, &parts[s], "part"));
    if (parts[s].nrows != parts[0].nrows || parts[s].ncols != parts[0].ncols)
      return sg_fail(h, SG_ERR_SHAPE, "merge parts differ in shape");
  }
  return SG_OK;
}

sg_status sg_spgemm_merge_symbolic(sg_handle* h, int nparts, const sg_csr* parts, int64_t* C_rowptr, int64_t* nnzC,
                                   void* stream) {
  if (!h) return SG_ERR_INVALID;
  SG_TRY(check_parts(h, nparts, parts));
  if (!C_rowptr || !nnzC) return sg_fail(h, SG_ERR_INVALID, "C_rowptr or nnzC is NULL");
  SG_HIP(h, hipSetDevice(h->device));
  hipStream_t st = (hipStream_t)stream;
  for (int s = 0; s < nparts; ++s) SG_TRY(validate_input(h, &parts[s], "part", st));
  const int64_t n = parts[0].nrows;
  int64_t total = 0;
  for (int s = 0; s < nparts; ++s) total += parts[s].nnz;
  if (n == 0 || total == 0) {
    launch_fill_i64(C_rowptr, n + 1, 0, st);
    SG_HIP(h, hipGetLastError());
    SG_HIP(h, hipStreamSynchronize(st));
    *nnzC = 0;
    h->cache_valid = false;
    return SG_OK;
  }
  SG_TRY(upload_parts(h, nparts, parts, st));
  RowSource r{};
  r.mode = kModeMerge;
  r.parts = (const PartDesc*)h->parts_buf.p;
  r.nparts = nparts;
  r.nrows = n;
  r.ncols = parts[0].ncols;
  r.T = tiles_of(parts[0].ncols);
  return run_symbolic(h, r, nullptr, C_rowptr, nnzC, merge_key(h, nparts, parts), st);
}

sg_status sg_spgemm_merge_numeric(sg_handle* h, const sg_semiring* sr, int nparts, const sg_csr* parts, sg_csr* C,
                                  void* stream) {
  if (!h) return SG_ERR_INVALID;
  SG_TRY(check_semiring(h, sr));
  SG_TRY(check_parts(h, nparts, parts));
  SG_TRY(check_csr(h, C, "C"));
  if (C->nrows != parts[0].nrows || C->ncols != parts[0].ncols)
    return sg_fail(h, SG_ERR_SHAPE, "C does not have the parts' shape");
  for (int s = 0; s < nparts; ++s)
    if (parts[s].nnz > 0 && !parts[s].val) return sg_fail(h, SG_ERR_INVALID, "a part's value array is NULL");
  if (C->nnz > 0 && !C->val) return sg_fail(h, SG_ERR_INVALID, "C.val is NULL");
  SG_HIP(h, hipSetDevice(h->device));
  hipStream_t st = (hipStream_t)stream;
  if (C->nrows == 0 || C->nnz == 0) return SG_OK;
  for (int s = 0; s < nparts; ++s) SG_TRY(validate_input(h, &parts[s], "part", st));
  SG_TRY(upload_parts(h, nparts, parts, st));
  RowSource r{};
  r.mode = kModeMerge;
  r.parts = (const PartDesc*)h->parts_buf.p;
  r.nparts = nparts;
  r.nrows = C->nrows;
  r.ncols = C->ncols;
  r.T = tiles_of(C->ncols);
  return run_numeric(h, sr, r, nullptr, C, merge_key(h, nparts, parts), st);
}

sg_status sg_handle_check(sg_handle* h) {
  if (!h) return SG_ERR_INVALID;
  SG_HIP(h, hipSetDevice(h->device));
  SG_HIP(h, hipDeviceSynchronize());
  int32_t v = 0;
  SG_HIP(h, hipMemcpy(&v, h->d_flags, sizeof(int32_t), hipMemcpyDeviceToHost));
  if (v) {
    SG_HIP(h, hipMemset(h->d_flags, 0, sizeof(int32_t)));
    return sg_fail(h, SG_ERR_INVALID, kInconsistent);
  }
  return SG_OK;
}

sg_status sg_handle_timings(sg_handle* h, double* ms, int n) {
  if (!h || !ms || n < 0) return SG_ERR_INVALID;
  if (!h->timing) return sg_fail(h, SG_ERR_INVALID, "the timing option is off");
  SG_HIP(h, hipSetDevice(h->device));
  for (int p = 0; p < n && p < kNPhases; ++p) {
    ms[p] = 0.0;
    if (!h->ev_rec[p]) continue;
    SG_HIP(h, hipEventSynchronize(h->ev[p][1]));
    float t = 0.f;
    SG_HIP(h, hipEventElapsedTime(&t, h->ev[p][0], h->ev[p][1]));
    ms[p] = t;
  }
  return SG_OK;
}

sg_status sg_handle_stats(sg_handle* h, int64_t* out, int n) {
  if (!h || !out || n < 0) return SG_ERR_INVALID;
  SG_HIP(h, hipSetDevice(h->device));
  SG_HIP(h, hipDeviceSynchronize());
  int32_t blk[kCtrEntries + 6] = {};
  SG_HIP(h, hipMemcpy(blk, h->d_flags + kCtrBase, sizeof(blk), hipMemcpyDeviceToHost));
  uint64_t ent[3];
  std::memcpy(ent, blk + kCtrEntries, sizeof(ent));
  const int64_t v[SG_NSTATS] = {h->last_nd, blk[kListSlab], blk[kListTile], blk[kListRange],
                                (int64_t)ent[kListSlab], (int64_t)ent[kListTile], (int64_t)ent[kListRange]};
  for (int i = 0; i < n && i < SG_NSTATS; ++i) out[i] = v[i];
  return SG_OK;
}

const char* sg_status_string(sg_status s) {
  switch (s) {
    case SG_OK: return "SG_OK";
    case SG_ERR_INVALID: return "SG_ERR_INVALID";
    case SG_ERR_SHAPE: return "SG_ERR_SHAPE";
    case SG_ERR_SEMIRING: return "SG_ERR_SEMIRING";
    case SG_ERR_NOMEM: return "SG_ERR_NOMEM";
    case SG_ERR_OVERFLOW: return "SG_ERR_OVERFLOW";
    case SG_ERR_UNSORTED: return "SG_ERR_UNSORTED";
    case SG_ERR_HIP: return "SG_ERR_HIP";
  }
  return "unknown status";
}

const char* sg_last_error(const sg_handle* h) { return h ? h->err.c_str() : "no handle"; }

}  // extern "C"
