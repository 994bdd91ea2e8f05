// Handle, scratch memory and shared host-side helpers of the C-ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/spgemm.h"
#include "sg_launch.hpp"

// Device flag block of a handle or plan: error flags in the first ints, the
// task-queue counter block (sg::kCtrInts ints) from kCtrBase.
constexpr int kCtrBase = 256;
constexpr int kFlagInts = kCtrBase + sg::kCtrInts;

// Grow-only device buffer.
struct SgBuf {
  void* p = nullptr;
  size_t cap = 0;
  // exact: allocate bytes only, with no headroom for later growth (pools
  // sized once, where a quarter more can be tens of GB)
  hipError_t ensure(size_t bytes, bool exact = false) {
    if (bytes <= cap && p) return hipSuccess;
    release();
    const size_t nb = exact ? (bytes > 0 ? bytes : 1) : bytes + bytes / 4 + 4096;
    hipError_t e = hipMalloc(&p, nb);
    if (e != hipSuccess) {
      p = nullptr;
      return e;
    }
    cap = nb;
    return hipSuccess;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    cap = 0;
  }
};

// Where a call's device scratch comes from: the grow-only buffers (grown
// with hipMalloc when too small), or consecutive pieces of one fixed device
// array that is never grown or freed (base != nullptr).  In the fixed mode
// the SgBuf handed to take() becomes a view into the array; such views are
// call-local and must never be released.
struct Scratch {
  struct sg_handle* h = nullptr;
  char* base = nullptr;
  size_t cap = 0, off = 0;
  bool fixed() const { return base != nullptr; }
  sg_status take(SgBuf& b, size_t bytes);
};

// Column-slab partition of one B (per-row slab bounds, tile offsets inside
// the segments, segment starts, column ids, (column, value) pairs, each B
// entry's position) and the dense-row table of the product using it.
struct SlabBufs {
  SgBuf bnd, rpt, prow, pbit, pcv, perm, dr;
  void release() {
    bnd.release();
    rpt.release();
    prow.release();
    pbit.release();
    pcv.release();
    perm.release();
    dr.release();
  }
};

// Bump allocator over a buffer; with base == nullptr it only measures.
struct SgArena {
  char* base = nullptr;
  size_t off = 0;
  template <class T>
  T* take(size_t n) {
    off = (off + 255) & ~(size_t)255;
    T* r = base ? (T*)(base + off) : nullptr;
    off += n * sizeof(T) + 1;
    return r;
  }
};

struct SgCacheKey {
  uint64_t w[16];
  bool operator==(const SgCacheKey& o) const {
    for (int i = 0; i < 16; ++i)
      if (w[i] != o.w[i]) return false;
    return true;
  }
};

struct sg_handle {
  int device = 0;
  int cus = 256;
  std::string err;
  // options
  int force = sg::kForceAuto;
  int64_t hash_max = sg::kHashCap;
  int validate = 0;
  int timing = 0;
  hipEvent_t ev[sg::kNPhases][2] = {};
  bool ev_rec[sg::kNPhases] = {};
  hipStream_t mark_stream = nullptr;
  // scratch
  SgBuf ws;                  // per call
  SgBuf rp2_buf, off2_buf;   // dense-path data kept from symbolic for numeric
  SgBuf parts_buf;           // device table of merge parts
  SgBuf task_buf;            // dense-row task lists of the numeric pass
  SgBuf p_buf, nt_buf;       // per-row products and terms from symbolic, reused to re-bin numeric
  SlabBufs sb;               // column-slab partition of B and the dense-row table
  int slab = 1;              // dense rows of single products use the column-slab path
  int gather32 = 1;          // slab symbolic gathers at 32-bit offsets where B allows
  int merge_rows = 1;        // hash rows of 512+ products over wide B merged from their sorted segments
  int32_t tile_min = sg::kTileMinDefault;
  int32_t slab_ls = 0;     // slab width 2^slab_ls of the column-slab path (0: chosen from ncols)
  int32_t light_cap = 0;   // most entries of a light slab task (0: the LDS capacity)
  int32_t tuned_sr = 0;    // semiring (id, value bytes) a loaded tuning table was made for
  int32_t tuned_vb = 0;
  std::vector<sg::PartDesc> parts_host;
  bool cache_valid = false;
  SgCacheKey cache_key{};
  int32_t cache_T = 0, cache_nd = 0;
  int64_t cache_n = -1;
  int64_t last_nd = 0;  // dense rows of the last numeric call
  int32_t* d_flags = nullptr;  // kFlagInts: [0] consistency error, [2] validation, task counters from kCtrBase
  int64_t* h_pin = nullptr;    // pinned readback area (>= 256 int64)
};

// Status with message.
sg_status sg_fail(sg_handle* h, sg_status s, const std::string& msg);
sg_status sg_check_hip(sg_handle* h, hipError_t e, const char* what);

namespace sg {
int32_t tiles_of(int64_t ncols);
Policy make_policy(const sg_handle* h, int numeric, const sg_semiring* sr, int32_t T = 0);
// Analysis + binning of the rows of r; waits for the stream to read the bin
// counts.  Scratch comes from `ar`.  p_keep / nt_keep (optional) receive the
// per-row product and term counts; with rebin set they are read instead and
// no gathers are made.
sg_status plan_rows(sg_handle* h, const RowSource& r, const Policy& pol, const int64_t* c_rowptr, int64_t* cnt_out,
                    SgArena& ar, BinPlan& plan, hipStream_t st, int64_t* p_keep = nullptr,
                    int32_t* nt_keep = nullptr, bool rebin = false);
size_t plan_rows_bytes(int64_t nrows);
// Column-slab partition of B for the dense rows of single product r: with
// cols, the structure (bounds, tile offsets, segment starts, column ids and
// each entry's position); with vals, the (column, value) pairs.  partial:
// slab_partials() int64 of scratch.  Fills r's slab fields.
sg_status build_slabs(sg_handle* h, Scratch& sc, SlabBufs& sb, RowSource& r, const sg_csr* B, int vbytes, bool cols, bool vals,
                      int64_t* partial, int32_t* err, int32_t* qctr, hipStream_t st);
// Per dense row of the plan: its A row (first entry, length, row id).
sg_status build_dense_rows(sg_handle* h, Scratch& sc, SlabBufs& sb, RowSource& r, const BinPlan& plan, hipStream_t st);
// Light-task cap of a numeric call with semiring sr (0: the kernel's LDS
// capacity); a tuned cap applies only to the semiring it was tuned on.
int32_t light_cap_for(const sg_handle* h, const sg_semiring* sr);
// int64 scratch the partition's scan needs (0 when r does not use slabs).
size_t slab_partials(const sg_handle* h, const RowSource& r);
// Timing hooks of the handle for a call on stream st (inactive unless the
// "timing" option is on); clear_phases forgets phases [p0, p1).
Marks handle_marks(sg_handle* h, hipStream_t st);
void clear_phases(sg_handle* h, int p0, int p1);
}  // namespace sg
