// CPU oracle for the semiring sparse product and the merge of partial
// products.  TEST INFRASTRUCTURE ONLY: nothing in the library's product path
// may link, load or call this file; only the test suite, the smoke check and
// the benchmark's CPU-baseline leg use it.
//
// What it computes (paper, Section 2.2 "Semiring Abstraction"): the product
// C = A (x).(+) B over a semiring (S, (+), (x), 0, 1), i.e.
//     C_ij = (+)_{k : A_ik and B_kj stored} A_ik (x) B_kj,
// with the pattern of C being every (i, j) reached by at least one product
// (structural: an entry whose value equals the semiring zero is kept).
// The merge (Section 4.4 "Merging Operation"; Section 2.1 on combining the
// stage results) is C = P_0 (+) P_1 (+) ... (+) P_{S-1} entry by entry, with
// the union of the parts' patterns.
//
// How: row by row Gustavson.  For row i an empty std::map from column to
// accumulator is filled by walking A's row i in ascending k and, for each k,
// B's row k in ascending j; the first product for a column initialises its
// slot and later ones are folded in with (+).  The map is then emitted in key
// order.  Rows are independent, so rows run in parallel (OpenMP) without
// changing any result.  Built with -O2 -ffp-contract=off so that (x) and (+)
// are never fused.
//
// Semirings (ids 1..5):
//   1  (+, x) int64   : wrapping arithmetic modulo 2^64
//   2  (+, x) float32 : inputs upcast to float64; each product is then exact
//                       and the sum is taken in float64 (reference precision)
//   3  (+, x) float64 : IEEE float64, round to nearest even
//   4  (or, and) bool : uint8, nonzero means true; result 0/1
//   5  (min, +) f32   : (x) is float32 addition (rounded), (+) is the minimum
//                       under IEEE '<'; 0 = +inf, 1 = +0.0
//   6  (max, +) f32   : (x) is float32 addition (rounded), (+) the maximum
//   7  (max, x) f64   : (x) is float64 multiplication (rounded), (+) the
//                       maximum
//   8  (min, max) i64 : (x) is the maximum, (+) the minimum (bottleneck
//                       paths)
// Ids 6..8 are semirings the paper's abstraction lets a user define (the
// entry type, (+) and (x) redefined); the library builds such semirings at
// run time, and these are the oracle's own definitions of three of them.
// For the float sums it also returns, per entry, sum_k |A_ik * B_kj| in
// float64 (the scale a rounding-error bound is relative to).
//
// Compile-time switch ORACLE_MUTANT plants one of several deliberate mistakes;
// the test suite builds those variants to show that its pins catch them.

#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>
#include <type_traits>
#include <vector>
#include <omp.h>

#ifndef ORACLE_MUTANT
#define ORACLE_MUTANT 0
#endif

namespace {

struct Csr {
  int64_t nrows, ncols;
  const int64_t* rowptr;
  const int32_t* col;
  const void* val;
};

// ---- semiring definitions -------------------------------------------------

struct PlusTimesI64 {
  using in_t = int64_t;
  using acc_t = uint64_t;
  using out_t = int64_t;
  static constexpr bool has_abs = false;
  static acc_t mul(in_t a, in_t b) {
#if ORACLE_MUTANT == 8
    return (uint64_t)(uint32_t)((uint64_t)a * (uint64_t)b);  // truncated product
#else
    return (uint64_t)a * (uint64_t)b;
#endif
  }
  static acc_t add(acc_t x, acc_t y) { return x + y; }
  static out_t out(acc_t x) { return (int64_t)x; }
  static double mag(acc_t) { return 0.0; }
};

struct PlusTimesF32 {
  using in_t = float;
  using acc_t = double;
  using out_t = double;
  static constexpr bool has_abs = true;
  static acc_t mul(in_t a, in_t b) { return (double)a * (double)b; }
  static acc_t add(acc_t x, acc_t y) { return x + y; }
  static out_t out(acc_t x) { return x; }
  static double mag(acc_t v) { return std::fabs(v); }
};

struct PlusTimesF64 {
  using in_t = double;
  using acc_t = double;
  using out_t = double;
  static constexpr bool has_abs = true;
  static acc_t mul(in_t a, in_t b) { return a * b; }
  static acc_t add(acc_t x, acc_t y) {
#if ORACLE_MUTANT == 4
    (void)x;
    return y;  // overwrite instead of accumulate
#else
    return x + y;
#endif
  }
  static out_t out(acc_t x) { return x; }
  static double mag(acc_t v) {
#if ORACLE_MUTANT == 6
    return v;  // signed instead of absolute
#else
    return std::fabs(v);
#endif
  }
};

struct OrAnd {
  using in_t = uint8_t;
  using acc_t = uint8_t;
  using out_t = uint8_t;
  static constexpr bool has_abs = false;
  static acc_t mul(in_t a, in_t b) { return (a != 0 && b != 0) ? 1 : 0; }
  static acc_t add(acc_t x, acc_t y) { return (x != 0 || y != 0) ? 1 : 0; }
  static out_t out(acc_t x) { return x; }
  static double mag(acc_t) { return 0.0; }
};

struct MinPlusF32 {
  using in_t = float;
  using acc_t = float;
  using out_t = float;
  static constexpr bool has_abs = false;
  static acc_t mul(in_t a, in_t b) {
    volatile float s = a + b;  // float32 addition, rounded to nearest
    return s;
  }
  static acc_t add(acc_t x, acc_t y) {
#if ORACLE_MUTANT == 3
    return (y > x) ? y : x;  // max instead of min
#else
    return (y < x) ? y : x;
#endif
  }
  static out_t out(acc_t x) { return x; }
  static double mag(acc_t) { return 0.0; }
};

struct MaxPlusF32 {
  using in_t = float;
  using acc_t = float;
  using out_t = float;
  static constexpr bool has_abs = false;
  static acc_t mul(in_t a, in_t b) {
    volatile float s = a + b;  // float32 addition, rounded to nearest
    return s;
  }
  static acc_t add(acc_t x, acc_t y) { return (y > x) ? y : x; }
  static out_t out(acc_t x) { return x; }
  static double mag(acc_t) { return 0.0; }
};

struct MaxTimesF64 {
  using in_t = double;
  using acc_t = double;
  using out_t = double;
  static constexpr bool has_abs = false;
  static acc_t mul(in_t a, in_t b) { return a * b; }
  static acc_t add(acc_t x, acc_t y) {
#if ORACLE_MUTANT == 9
    return (y < x) ? y : x;  // min instead of max
#else
    return (y > x) ? y : x;
#endif
  }
  static out_t out(acc_t x) { return x; }
  static double mag(acc_t) { return 0.0; }
};

struct MinMaxI64 {
  using in_t = int64_t;
  using acc_t = int64_t;
  using out_t = int64_t;
  static constexpr bool has_abs = false;
  static acc_t mul(in_t a, in_t b) {
#if ORACLE_MUTANT == 10
    return (b < a) ? b : a;  // min instead of max
#else
    return (b > a) ? b : a;
#endif
  }
  static acc_t add(acc_t x, acc_t y) { return (y < x) ? y : x; }
  static out_t out(acc_t x) { return x; }
  static double mag(acc_t) { return 0.0; }
};

// ---- result container -------------------------------------------------------

struct Result {
  int sr = 0;
  int64_t nrows = 0;
  std::vector<int64_t> rowptr;
  std::vector<int32_t> col;
  std::vector<uint8_t> val;  // raw bytes, out_t each
  std::vector<double> mag;   // float sums only
  int out_bytes = 0;
};

template <class Sr>
struct RowOut {
  std::vector<int32_t> col;
  std::vector<typename Sr::out_t> val;
  std::vector<double> mag;
};

template <class Sr>
void product_row(const Csr& A, const Csr& B, int64_t i, RowOut<Sr>& o) {
  using in_t = typename Sr::in_t;
  using acc_t = typename Sr::acc_t;
  const in_t* av = (const in_t*)A.val;
  const in_t* bv = (const in_t*)B.val;
  std::map<int32_t, acc_t> m;
  std::map<int32_t, double> mag;
  int64_t a_begin = A.rowptr[i];
#if ORACLE_MUTANT == 5
  a_begin += 1;  // skip the first stored entry of the row
#endif
  for (int64_t e = a_begin; e < A.rowptr[i + 1]; ++e) {
#if ORACLE_MUTANT == 2
    const int64_t k = i % B.nrows;  // walks B's row i instead of row k
#else
    const int64_t k = A.col[e];
#endif
    const in_t a = av[e];
    int64_t b_end = B.rowptr[k + 1];
#if ORACLE_MUTANT == 1
    if (b_end > B.rowptr[k]) b_end -= 1;  // drop the last product of each B row
#endif
    for (int64_t f = B.rowptr[k]; f < b_end; ++f) {
      const int32_t j = B.col[f];
      const acc_t v = Sr::mul(a, bv[f]);
      auto it = m.find(j);
      if (it == m.end()) m.emplace(j, v);
      else it->second = Sr::add(it->second, v);
      if (Sr::has_abs) mag[j] += Sr::mag(v);
    }
  }
  o.col.reserve(m.size());
  o.val.reserve(m.size());
  for (const auto& kv : m) {
    o.col.push_back(kv.first);
    o.val.push_back(Sr::out(kv.second));
  }
  if (Sr::has_abs)
    for (const auto& kv : mag) o.mag.push_back(kv.second);
}

template <class Sr>
void merge_row(int nparts, const Csr* parts, int64_t i, RowOut<Sr>& o) {
  using in_t = typename Sr::in_t;
  using acc_t = typename Sr::acc_t;
  std::map<int32_t, acc_t> m;
  std::map<int32_t, double> mag;
  int np = nparts;
#if ORACLE_MUTANT == 7
  if (np > 1) np -= 1;  // forget the last part
#endif
  for (int s = 0; s < np; ++s) {
    const Csr& P = parts[s];
    const in_t* pv = (const in_t*)P.val;
    for (int64_t e = P.rowptr[i]; e < P.rowptr[i + 1]; ++e) {
      const int32_t j = P.col[e];
      acc_t v;
      if constexpr (std::is_same<Sr, PlusTimesF32>::value) v = (double)pv[e];
      else if constexpr (std::is_same<Sr, PlusTimesI64>::value) v = (uint64_t)pv[e];
      else if constexpr (std::is_same<Sr, OrAnd>::value) v = pv[e] != 0 ? 1 : 0;
      else v = (acc_t)pv[e];
      auto it = m.find(j);
      if (it == m.end()) m.emplace(j, v);
      else it->second = Sr::add(it->second, v);
      if (Sr::has_abs) mag[j] += Sr::mag(v);
    }
  }
  for (const auto& kv : m) {
    o.col.push_back(kv.first);
    o.val.push_back(Sr::out(kv.second));
  }
  if (Sr::has_abs)
    for (const auto& kv : mag) o.mag.push_back(kv.second);
}

template <class Sr, class RowFn>
Result* run_rows(int sr, int64_t nsel, const int64_t* rows, int nthreads, RowFn fn) {
  std::vector<RowOut<Sr>> outs((size_t)nsel);
  if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
  for (int64_t r = 0; r < nsel; ++r) fn(rows ? rows[r] : r, outs[(size_t)r]);
  Result* res = new Result;
  res->sr = sr;
  res->nrows = nsel;
  res->out_bytes = (int)sizeof(typename Sr::out_t);
  res->rowptr.assign((size_t)nsel + 1, 0);
  for (int64_t r = 0; r < nsel; ++r) res->rowptr[(size_t)r + 1] = res->rowptr[(size_t)r] + (int64_t)outs[(size_t)r].col.size();
  const int64_t nnz = res->rowptr[(size_t)nsel];
  res->col.resize((size_t)nnz);
  res->val.resize((size_t)nnz * sizeof(typename Sr::out_t));
  if (Sr::has_abs) res->mag.resize((size_t)nnz);
  for (int64_t r = 0; r < nsel; ++r) {
    const auto& o = outs[(size_t)r];
    const int64_t b = res->rowptr[(size_t)r];
    if (!o.col.empty()) {
      std::memcpy(res->col.data() + b, o.col.data(), o.col.size() * sizeof(int32_t));
      std::memcpy(res->val.data() + b * sizeof(typename Sr::out_t), o.val.data(),
                  o.val.size() * sizeof(typename Sr::out_t));
      if (Sr::has_abs) std::memcpy(res->mag.data() + b, o.mag.data(), o.mag.size() * sizeof(double));
    }
  }
  return res;
}

template <class Sr>
Result* spgemm_t(int sr, const Csr& A, const Csr& B, const int64_t* rows, int64_t nsel, int nthreads) {
  return run_rows<Sr>(sr, nsel, rows, nthreads, [&](int64_t i, RowOut<Sr>& o) { product_row<Sr>(A, B, i, o); });
}

template <class Sr>
Result* merge_t(int sr, int nparts, const Csr* parts, const int64_t* rows, int64_t nsel, int nthreads) {
  return run_rows<Sr>(sr, nsel, rows, nthreads, [&](int64_t i, RowOut<Sr>& o) { merge_row<Sr>(nparts, parts, i, o); });
}

}  // namespace

extern "C" {

// Rows `rows[0..nsel)` of A (x).(+) B (all rows in order when rows is NULL,
// then nsel must equal A's row count).  Returns NULL on a bad semiring id or
// a shape mismatch.  Free with oracle_result_free.
void* oracle_spgemm(int sr, int64_t a_nrows, int64_t a_ncols, const int64_t* a_rowptr, const int32_t* a_col,
                    const void* a_val, int64_t b_nrows, int64_t b_ncols, const int64_t* b_rowptr,
                    const int32_t* b_col, const void* b_val, const int64_t* rows, int64_t nsel, int nthreads) {
  if (a_ncols != b_nrows) return nullptr;
  Csr A{a_nrows, a_ncols, a_rowptr, a_col, a_val};
  Csr B{b_nrows, b_ncols, b_rowptr, b_col, b_val};
  switch (sr) {
    case 1: return spgemm_t<PlusTimesI64>(sr, A, B, rows, nsel, nthreads);
    case 2: return spgemm_t<PlusTimesF32>(sr, A, B, rows, nsel, nthreads);
    case 3: return spgemm_t<PlusTimesF64>(sr, A, B, rows, nsel, nthreads);
    case 4: return spgemm_t<OrAnd>(sr, A, B, rows, nsel, nthreads);
    case 5: return spgemm_t<MinPlusF32>(sr, A, B, rows, nsel, nthreads);
    case 6: return spgemm_t<MaxPlusF32>(sr, A, B, rows, nsel, nthreads);
    case 7: return spgemm_t<MaxTimesF64>(sr, A, B, rows, nsel, nthreads);
    case 8: return spgemm_t<MinMaxI64>(sr, A, B, rows, nsel, nthreads);
    default: return nullptr;
  }
}

// Rows of P_0 (+) ... (+) P_{nparts-1}; parts share one shape (nrows x ncols).
void* oracle_merge(int sr, int nparts, int64_t nrows, int64_t ncols, const int64_t* const* rowptrs,
                   const int32_t* const* cols, const void* const* vals, const int64_t* rows, int64_t nsel,
                   int nthreads) {
  std::vector<Csr> parts((size_t)nparts);
  for (int s = 0; s < nparts; ++s) parts[(size_t)s] = Csr{nrows, ncols, rowptrs[s], cols[s], vals[s]};
  switch (sr) {
    case 1: return merge_t<PlusTimesI64>(sr, nparts, parts.data(), rows, nsel, nthreads);
    case 2: return merge_t<PlusTimesF32>(sr, nparts, parts.data(), rows, nsel, nthreads);
    case 3: return merge_t<PlusTimesF64>(sr, nparts, parts.data(), rows, nsel, nthreads);
    case 4: return merge_t<OrAnd>(sr, nparts, parts.data(), rows, nsel, nthreads);
    case 5: return merge_t<MinPlusF32>(sr, nparts, parts.data(), rows, nsel, nthreads);
    case 6: return merge_t<MaxPlusF32>(sr, nparts, parts.data(), rows, nsel, nthreads);
    case 7: return merge_t<MaxTimesF64>(sr, nparts, parts.data(), rows, nsel, nthreads);
    case 8: return merge_t<MinMaxI64>(sr, nparts, parts.data(), rows, nsel, nthreads);
    default: return nullptr;
  }
}

int64_t oracle_result_nnz(const void* r) { return ((const Result*)r)->rowptr.back(); }
int oracle_result_val_bytes(const void* r) { return ((const Result*)r)->out_bytes; }
int oracle_result_has_mag(const void* r) { return ((const Result*)r)->mag.empty() ? 0 : 1; }

void oracle_result_copy(const void* rp, int64_t* rowptr, int32_t* col, void* val, double* mag) {
  const Result* r = (const Result*)rp;
  std::memcpy(rowptr, r->rowptr.data(), r->rowptr.size() * sizeof(int64_t));
  if (!r->col.empty()) {
    std::memcpy(col, r->col.data(), r->col.size() * sizeof(int32_t));
    std::memcpy(val, r->val.data(), r->val.size());
    if (mag && !r->mag.empty()) std::memcpy(mag, r->mag.data(), r->mag.size() * sizeof(double));
  }
}

void oracle_result_free(void* r) { delete (Result*)r; }

int oracle_num_threads(void) { return omp_get_max_threads(); }

}  // extern "C"
