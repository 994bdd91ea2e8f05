// Memory-budgeted waves of a batch (paper, Section 2.1: the stage products
// of a 2D Sparse SUMMA and their merge, at a scale whose stage outputs do not
// fit one GPU at once).
//
// sg_waves_plan sizes every product of the batch with one symbolic pass (its
// nnz), then cuts the merge groups, in order, into waves whose outputs -- the
// group's stage products plus its merged result, which holds at most as many
// entries as they do together -- stay under a byte budget.  sg_waves_run
// builds the batched plan of one wave (sg_batch_plan: one graph of persistent
// kernels over all of the wave's products and merges), replays it, and frees
// the previous wave's plan first, so only one wave's pool is alive at a time.
#include <string>
#include <vector>

#include "sg_handle.hpp"

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

struct sg_waves {
  sg_handle* h = nullptr;
  sg_semiring sr{};
  std::vector<sg_csr> A, B;
  std::vector<int32_t> go;     // group offsets over the products
  std::vector<int64_t> nnz;    // per product: entries of its output
  std::vector<int32_t> wg;     // wave offsets over the groups
  std::vector<size_t> wbytes;  // per wave: output bytes of its products and merges (upper bound)
  int cur = -1;                // wave whose plan is alive
  sg_plan* plan = nullptr;
};

namespace {

size_t group_bytes(const sg_waves* W, int g) {
  const size_t eb = 4 + (size_t)W->sr.value_bytes;
  size_t e = 0;
  for (int q = W->go[(size_t)g]; q < W->go[(size_t)g + 1]; ++q) e += (size_t)W->nnz[(size_t)q];
  return 2 * e * eb;  // stage outputs, and their merge (at most as many entries)
}

sg_status size_products(sg_waves* W, hipStream_t st) {
  sg_handle* h = W->h;
  int64_t rows = 1;
  for (const sg_csr& a : W->A) rows = a.nrows + 1 > rows ? a.nrows + 1 : rows;
  int64_t* rp = nullptr;
  SG_HIP(h, hipMalloc(&rp, sizeof(int64_t) * (size_t)rows));
  sg_status s = SG_OK;
  W->nnz.assign(W->A.size(), 0);
  for (size_t q = 0; q < W->A.size() && s == SG_OK; ++q) s = sg_spgemm_symbolic(h, &W->A[q], &W->B[q], rp, &W->nnz[q], st);
  (void)hipFree(rp);
  return s;
}

}  // namespace

extern "C" {

sg_status sg_waves_plan(sg_handle* h, const sg_semiring* sr, int nprob, const sg_csr* A, const sg_csr* B,
                        int ngroups, const int32_t* group_offsets, size_t budget_bytes, sg_waves** out) {
  if (!h || !out) return SG_ERR_INVALID;
  *out = nullptr;
  if (!sr || !A || !B || nprob < 1) return sg_fail(h, SG_ERR_INVALID, "a wave plan needs products");
  if (ngroups < 1 || !group_offsets || group_offsets[0] != 0 || group_offsets[ngroups] != nprob)
    return sg_fail(h, SG_ERR_INVALID, "merge groups must cover the products 0..nprob-1 in order");
  for (int g = 0; g < ngroups; ++g)
    if (group_offsets[g + 1] <= group_offsets[g]) return sg_fail(h, SG_ERR_INVALID, "group offsets must ascend");
  if (budget_bytes == 0) return sg_fail(h, SG_ERR_INVALID, "budget_bytes must be positive");
  SG_HIP(h, hipSetDevice(h->device));
  sg_waves* W = new sg_waves;
  W->h = h;
  W->sr = *sr;
  W->A.assign(A, A + nprob);
  W->B.assign(B, B + nprob);
  W->go.assign(group_offsets, group_offsets + ngroups + 1);
  sg_status s = size_products(W, nullptr);
  if (s == SG_OK) {
    W->wg.push_back(0);
    size_t acc = 0;
    for (int g = 0; g < ngroups; ++g) {
      const size_t b = group_bytes(W, g);
      if (b > budget_bytes) {
        s = sg_fail(h, SG_ERR_NOMEM, "merge group " + std::to_string(g) + " needs " + std::to_string(b) +
                                         " output bytes, more than the wave budget of " +
                                         std::to_string(budget_bytes));
        break;
      }
      if (acc + b > budget_bytes) {
        W->wg.push_back(g);
        W->wbytes.push_back(acc);
        acc = 0;
      }
      acc += b;
    }
    W->wg.push_back(ngroups);
    W->wbytes.push_back(acc);
  }
  if (s != SG_OK) {
    delete W;
    return s;
  }
  *out = W;
  return SG_OK;
}

sg_status sg_waves_info(const sg_waves* W, int* nwaves, int64_t* product_nnz, int32_t* wave_groups,
                        size_t* wave_bytes) {
  if (!W || !nwaves) return SG_ERR_INVALID;
  const int nw = (int)W->wbytes.size();
  *nwaves = nw;
  if (product_nnz)
    for (size_t q = 0; q < W->nnz.size(); ++q) product_nnz[q] = W->nnz[q];
  if (wave_groups)
    for (int w = 0; w <= nw; ++w) wave_groups[w] = W->wg[(size_t)w];
  if (wave_bytes)
    for (int w = 0; w < nw; ++w) wave_bytes[w] = W->wbytes[(size_t)w];
  return SG_OK;
}

sg_status sg_waves_run(sg_waves* W, int wave, void* stream) {
  if (!W) return SG_ERR_INVALID;
  sg_handle* h = W->h;
  if (wave < 0 || wave >= (int)W->wbytes.size()) return sg_fail(h, SG_ERR_INVALID, "no such wave");
  SG_HIP(h, hipSetDevice(h->device));
  if (W->cur != wave) {
    if (W->plan) {
      SG_TRY(sg_plan_destroy(W->plan));
      W->plan = nullptr;
      W->cur = -1;
    }
    const int g0 = W->wg[(size_t)wave], g1 = W->wg[(size_t)wave + 1];
    const int q0 = W->go[(size_t)g0], q1 = W->go[(size_t)g1];
    std::vector<int32_t> go((size_t)(g1 - g0) + 1);
    for (int g = g0; g <= g1; ++g) go[(size_t)(g - g0)] = W->go[(size_t)g] - q0;
    SG_TRY(sg_batch_plan(h, &W->sr, q1 - q0, W->A.data() + q0, W->B.data() + q0, g1 - g0, go.data(), 0, &W->plan));
    W->cur = wave;
  }
  return sg_batch_execute(W->plan, stream);
}

sg_status sg_waves_results(sg_waves* W, sg_csr* out_C) {
  if (!W || !out_C) return SG_ERR_INVALID;
  if (!W->plan) return sg_fail(W->h, SG_ERR_INVALID, "no wave has run");
  return sg_batch_results(W->plan, out_C);
}

sg_status sg_waves_destroy(sg_waves* W) {
  if (!W) return SG_ERR_INVALID;
  if (W->plan) (void)sg_plan_destroy(W->plan);
  delete W;
  return SG_OK;
}

}  // extern "C"
