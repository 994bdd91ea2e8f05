// Column-major operands and powers of a matrix, built on the product entry
// points.
//
// Column-major operands (paper, Section 4.1 and Algorithm 1): the arrays of a
// matrix in CSC are the CSR arrays of its transpose, and C = A B equals
// (B^T A^T)^T, so a product of CSC operands is the CSR product of the
// swapped operands, whose CSR result is C in CSC; no array is copied or
// transposed.  DCSC, which lists only the non-empty columns, is decompressed
// to CSC column pointers first, and a result can be compressed back.
//
// Powers (paper, Section 2.2): over (min,+) the powers of W' = I (+) W hold
// the shortest paths of at most k edges and stop changing at the distance
// matrix; over (or,and) they give reachability.  The driver runs linear
// steps D W' or squarings D D through sg_spgemm_symbolic/numeric and, when
// asked, stops at the first product that equals its left operand.
#include <cstring>
#include <string>

#include "sg_adapt.hpp"
#include "sg_handle.hpp"
#include "sg_user.hpp"

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

struct sg_power {
  sg_handle* h = nullptr;
  int64_t n = 0;
  SgBuf rp[3], col[3], val[3];  // slots 0 and 1: successive powers; slot 2: I (+) W
  SgBuf id_rp, id_col, id_val;  // the identity
  SgBuf flag;                   // device int of the equality test
  sg_csr D{};
  int32_t hops = 0, products = 0, converged = 0;
  void release() {
    for (int s = 0; s < 3; ++s) {
      rp[s].release();
      col[s].release();
      val[s].release();
    }
    id_rp.release();
    id_col.release();
    id_val.release();
    flag.release();
  }
};

namespace {

// The semiring's multiplicative identity as value bits.
uint64_t one_bits(int32_t id) {
  switch (id) {
    case SG_PLUS_TIMES_I64: return 1ull;
    case SG_PLUS_TIMES_F32: return 0x3F800000ull;          // 1.0f
    case SG_PLUS_TIMES_F64: return 0x3FF0000000000000ull;  // 1.0
    case SG_OR_AND_BOOL: return 1ull;
    default: return 0ull;  // (min,+): +0.0f
  }
}

// Grow slot s of P to a matrix of n rows and nnz entries of vb bytes.
sg_status slot_reserve(sg_power* P, int s, int64_t nnz, int vb) {
  sg_handle* h = P->h;
  SG_HIP(h, P->rp[s].ensure(sizeof(int64_t) * (size_t)(P->n + 1)));
  SG_HIP(h, P->col[s].ensure(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1)));
  SG_HIP(h, P->val[s].ensure((size_t)vb * (size_t)(nnz > 0 ? nnz : 1)));
  return SG_OK;
}

sg_csr slot_view(sg_power* P, int s, int64_t nnz) {
  return sg_csr{P->n, P->n, nnz, (int64_t*)P->rp[s].p, (int32_t*)P->col[s].p, P->val[s].p};
}

// X = L (x).(+) R into slot s.
sg_status product_into(sg_power* P, const sg_semiring* sr, const sg_csr& L, const sg_csr& R, int s, sg_csr* X,
                       hipStream_t st) {
  sg_handle* h = P->h;
  // slot s may still be read by the previous product's kernels: let them
  // finish before its buffers are regrown
  SG_HIP(h, hipStreamSynchronize(st));
  SG_HIP(h, P->rp[s].ensure(sizeof(int64_t) * (size_t)(P->n + 1)));
  int64_t nnz = 0;
  SG_TRY(sg_spgemm_symbolic(h, &L, &R, (int64_t*)P->rp[s].p, &nnz, st));
  SG_TRY(slot_reserve(P, s, nnz, sr->value_bytes));
  *X = slot_view(P, s, nnz);
  return sg_spgemm_numeric(h, sr, &L, &R, X, st);
}

sg_status power_run(sg_power* P, const sg_semiring* sr, const sg_csr* W, int32_t max_hops, uint32_t flags,
                    hipStream_t st) {
  sg_handle* h = P->h;
  const int64_t n = P->n;
  const int vb = sr->value_bytes;
  const bool squaring = flags & SG_POWER_SQUARING, fixpoint = flags & SG_POWER_FIXPOINT;
  sg_csr Wp = *W;
  int cur = -1;  // slot holding D (-1: the caller's W)
  if (flags & SG_POWER_SELF_LOOPS) {
    SG_HIP(h, P->id_rp.ensure(sizeof(int64_t) * (size_t)(n + 1)));
    SG_HIP(h, P->id_col.ensure(sizeof(int32_t) * (size_t)(n > 0 ? n : 1)));
    SG_HIP(h, P->id_val.ensure((size_t)vb * (size_t)(n > 0 ? n : 1)));
    uint64_t one = one_bits(sr->id);
    if (sr->id >= kUserSemiringBase) SG_TRY(user_semiring_identities(h, sr->id, nullptr, &one));
    launch_identity(n, one, vb, (int64_t*)P->id_rp.p, (int32_t*)P->id_col.p, P->id_val.p, h->cus, st);
    const sg_csr parts[2] = {sg_csr{n, n, n, (int64_t*)P->id_rp.p, (int32_t*)P->id_col.p, P->id_val.p}, *W};
    SG_HIP(h, P->rp[2].ensure(sizeof(int64_t) * (size_t)(n + 1)));
    int64_t nnz = 0;
    SG_TRY(sg_spgemm_merge_symbolic(h, 2, parts, (int64_t*)P->rp[2].p, &nnz, st));
    SG_TRY(slot_reserve(P, 2, nnz, vb));
    Wp = slot_view(P, 2, nnz);
    SG_TRY(sg_spgemm_merge_numeric(h, sr, 2, parts, &Wp, st));
    cur = 2;
  }
  sg_csr D = Wp;
  int32_t hops = 1;
  const int64_t limit = max_hops > 0 ? (int64_t)max_hops : 2 * (n > 0 ? n : 1);
  SG_HIP(h, P->flag.ensure(sizeof(int32_t)));
  while (hops < limit) {
    const int nx = cur == 0 ? 1 : 0;
    sg_csr X{};
    SG_TRY(product_into(P, sr, D, squaring ? D : Wp, nx, &X, st));
    ++P->products;
    hops = squaring ? 2 * hops : hops + 1;
    bool same = false;
    if (fixpoint && X.nnz == D.nnz) {
      int32_t* f = (int32_t*)P->flag.p;
      launch_fill_i32(f, 1, 0, st);
      launch_csr_equal(D.rowptr, D.col, D.val, X.rowptr, X.col, X.val, n, X.nnz, vb, f, h->cus, st);
      SG_HIP(h, hipMemcpyAsync(h->h_pin, f, sizeof(int32_t), hipMemcpyDeviceToHost, st));
      SG_HIP(h, hipStreamSynchronize(st));
      int32_t v = 1;
      std::memcpy(&v, h->h_pin, sizeof(v));
      same = v == 0;
    }
    D = X;
    cur = nx;
    if (same) {
      P->converged = 1;
      break;
    }
  }
  if (cur < 0) {  // no product ran: the result is a copy of W
    SG_TRY(slot_reserve(P, 0, W->nnz, vb));
    SG_HIP(h, hipMemcpyAsync(P->rp[0].p, W->rowptr, sizeof(int64_t) * (size_t)(n + 1), hipMemcpyDeviceToDevice, st));
    if (W->nnz > 0) {
      SG_HIP(h, hipMemcpyAsync(P->col[0].p, W->col, sizeof(int32_t) * (size_t)W->nnz, hipMemcpyDeviceToDevice, st));
      SG_HIP(h, hipMemcpyAsync(P->val[0].p, W->val, (size_t)vb * (size_t)W->nnz, hipMemcpyDeviceToDevice, st));
    }
    D = slot_view(P, 0, W->nnz);
  }
  SG_HIP(h, hipStreamSynchronize(st));
  P->D = D;
  P->hops = hops;
  return SG_OK;
}

sg_csr csc_as_transpose(const sg_csc* M) {
  return sg_csr{M->ncols, M->nrows, M->nnz, M->colptr, M->row, M->val};
}

sg_status check_csc(sg_handle* h, const sg_csc* M, const char* name) {
  if (!M) return sg_fail(h, SG_ERR_INVALID, std::string(name) + " is NULL");
  if (M->nrows < 0 || M->ncols < 0 || M->nnz < 0) return sg_fail(h, SG_ERR_INVALID, std::string(name) + ": negative size");
  if (!M->colptr) return sg_fail(h, SG_ERR_INVALID, std::string(name) + ".colptr is NULL");
  return SG_OK;
}

}  // namespace

extern "C" {

sg_status sg_power_run(sg_handle* h, const sg_semiring* sr, const sg_csr* W, int32_t max_hops, uint32_t flags,
                       void* stream, sg_power** out) {
  if (!h || !out) return SG_ERR_INVALID;
  *out = nullptr;
  if (!sr || !W) return sg_fail(h, SG_ERR_INVALID, "semiring or W is NULL");
  bool idem = sr->id == SG_OR_AND_BOOL || sr->id == SG_MIN_PLUS_F32;
  const bool user = sr->id >= kUserSemiringBase && user_semiring(sr->id, nullptr, &idem);
  if (!user && (sr->id < 1 || sr->id > 5)) return sg_fail(h, SG_ERR_SEMIRING, "unknown semiring id");
  if (W->nrows != W->ncols) return sg_fail(h, SG_ERR_SHAPE, "W must be square");
  if (W->nrows < 0 || W->nnz < 0 || !W->rowptr || (W->nnz > 0 && (!W->col || !W->val)))
    return sg_fail(h, SG_ERR_INVALID, "bad W descriptor");
  if (flags & ~(uint32_t)(SG_POWER_SELF_LOOPS | SG_POWER_SQUARING | SG_POWER_FIXPOINT))
    return sg_fail(h, SG_ERR_INVALID, "unknown power flag");
  if ((flags & SG_POWER_FIXPOINT) && (!(flags & SG_POWER_SELF_LOOPS) || !idem))
    return sg_fail(h, SG_ERR_INVALID,
                   "a fixed point needs self loops and an idempotent (+): (or,and), (min,+) or a run-time "
                   "semiring defined with SG_SR_IDEMPOTENT");
  SG_HIP(h, hipSetDevice(h->device));
  sg_power* P = new sg_power;
  P->h = h;
  P->n = W->nrows;
  const sg_status s = power_run(P, sr, W, max_hops, flags, (hipStream_t)stream);
  if (s != SG_OK) {
    (void)hipStreamSynchronize((hipStream_t)stream);
    P->release();
    delete P;
    return s;
  }
  *out = P;
  return SG_OK;
}

sg_status sg_power_result(const sg_power* P, sg_csr* D, int32_t* hops, int32_t* products, int32_t* converged) {
  if (!P || !D) return SG_ERR_INVALID;
  *D = P->D;
  if (hops) *hops = P->hops;
  if (products) *products = P->products;
  if (converged) *converged = P->converged;
  return SG_OK;
}

sg_status sg_power_destroy(sg_power* P) {
  if (!P) return SG_ERR_INVALID;
  (void)hipSetDevice(P->h->device);
  (void)hipDeviceSynchronize();
  P->release();
  delete P;
  return SG_OK;
}

sg_status sg_dcsc_decompress(sg_handle* h, const sg_dcsc* A, int64_t* colptr, void* stream) {
  if (!h) return SG_ERR_INVALID;
  if (!A || !colptr) return sg_fail(h, SG_ERR_INVALID, "A or colptr is NULL");
  if (A->ncols < 0 || A->nzc < 0 || A->nzc > A->ncols || A->nnz < 0)
    return sg_fail(h, SG_ERR_INVALID, "bad DCSC sizes (0 <= nzc <= ncols)");
  if (A->ncols > INT32_MAX) return sg_fail(h, SG_ERR_OVERFLOW, "more than 2^31-1 columns");
  if (!A->cp || (A->nzc > 0 && !A->jc)) return sg_fail(h, SG_ERR_INVALID, "A.jc or A.cp is NULL");
  SG_HIP(h, hipSetDevice(h->device));
  hipStream_t st = (hipStream_t)stream;
  launch_dcsc_decompress(A->jc, A->cp, A->nzc, A->ncols, colptr, h->cus, st);
  SG_HIP(h, hipGetLastError());
  return SG_OK;
}

sg_status sg_dcsc_compress(sg_handle* h, int64_t ncols, const int64_t* colptr, int32_t* jc, int64_t* cp, int64_t* nzc,
                           void* stream) {
  if (!h) return SG_ERR_INVALID;
  if (!colptr || !cp || !nzc || (ncols > 0 && !jc)) return sg_fail(h, SG_ERR_INVALID, "a pointer argument is NULL");
  if (ncols < 0) return sg_fail(h, SG_ERR_INVALID, "negative column count");
  if (ncols > INT32_MAX) return sg_fail(h, SG_ERR_OVERFLOW, "more than 2^31-1 columns");
  SG_HIP(h, hipSetDevice(h->device));
  hipStream_t st = (hipStream_t)stream;
  SgArena m;
  m.take<int64_t>((size_t)(ncols > 0 ? ncols : 1));
  m.take<int64_t>((size_t)scan_partials_len(ncols));
  SG_HIP(h, h->ws.ensure(m.off));
  SgArena a;
  a.base = (char*)h->ws.p;
  int64_t* incl = a.take<int64_t>((size_t)(ncols > 0 ? ncols : 1));
  int64_t* partial = a.take<int64_t>((size_t)scan_partials_len(ncols));
  launch_dcsc_compress(colptr, ncols, incl, partial, jc, cp, h->cus, st);
  SG_HIP(h, hipGetLastError());
  if (ncols > 0) SG_HIP(h, hipMemcpyAsync(h->h_pin, incl + ncols - 1, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  SG_HIP(h, hipStreamSynchronize(st));
  *nzc = ncols > 0 ? h->h_pin[0] : 0;
  return SG_OK;
}

sg_status sg_spgemm_csc_symbolic(sg_handle* h, const sg_csc* A, const sg_csc* B, int64_t* C_colptr, int64_t* nnzC,
                                 void* stream) {
  if (!h) return SG_ERR_INVALID;
  SG_TRY(check_csc(h, A, "A"));
  SG_TRY(check_csc(h, B, "B"));
  if (A->ncols != B->nrows) return sg_fail(h, SG_ERR_SHAPE, "A.ncols != B.nrows");
  const sg_csr At = csc_as_transpose(A), Bt = csc_as_transpose(B);
  return sg_spgemm_symbolic(h, &Bt, &At, C_colptr, nnzC, stream);
}

sg_status sg_spgemm_csc_numeric(sg_handle* h, const sg_semiring* sr, const sg_csc* A, const sg_csc* B, sg_csc* C,
                                void* stream) {
  if (!h) return SG_ERR_INVALID;
  SG_TRY(check_csc(h, A, "A"));
  SG_TRY(check_csc(h, B, "B"));
  SG_TRY(check_csc(h, C, "C"));
  if (A->ncols != B->nrows || C->nrows != A->nrows || C->ncols != B->ncols)
    return sg_fail(h, SG_ERR_SHAPE, "shapes of A, B and C do not match");
  const sg_csr At = csc_as_transpose(A), Bt = csc_as_transpose(B);
  sg_csr Ct = csc_as_transpose(C);
  return sg_spgemm_numeric(h, sr, &Bt, &At, &Ct, stream);
}

}  // extern "C"
