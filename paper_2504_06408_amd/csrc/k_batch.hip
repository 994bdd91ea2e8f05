// Kernels used only by the batched path: the pool guard that disables the
// numeric pass when the outputs would not fit the plan's pool, and the
// extraction of per-result (0-based) row pointers from the global offsets.
#include "sg_batch.hpp"

namespace sg {

namespace {

// If the scanned global offsets ask for more entries than the pool holds,
// zero every bin count (so the numeric kernels that follow find no rows)
// and raise the overflow flag.
__global__ void k_pool_guard(const int64_t* off_end, int64_t cap_entries, int32_t* bin_count, int32_t* flag) {
  const bool over = *off_end > cap_entries;
  if (over) {
    for (int b = threadIdx.x; b < kNB; b += blockDim.x) bin_count[b] = 0;
    if (threadIdx.x == 0) atomicOr(flag, 1);
  }
}

// out[x] for x over the concatenated (n_q + 1)-entry row pointers of all
// results: out[lbase[q] + i] = off[rbase[q] + i] - off[rbase[q]].
__global__ __launch_bounds__(256) void k_local_rowptr(const int64_t* off, const int64_t* rbase, const int64_t* lbase,
                                                      int32_t nres, int64_t total, int64_t* out) {
  for (int64_t x = (int64_t)blockIdx.x * 256 + threadIdx.x; x < total; x += (int64_t)gridDim.x * 256) {
    const int q = owner_search(lbase, nres, x);
    const int64_t i = x - lbase[q];
    out[x] = off[rbase[q] + i] - off[rbase[q]];
  }
}

}  // namespace

void launch_pool_guard(const int64_t* off_end, int64_t cap_entries, int32_t* bin_count, int32_t* flag,
                       hipStream_t st) {
  hipLaunchKernelGGL(k_pool_guard, dim3(1), dim3(64), 0, st, off_end, cap_entries, bin_count, flag);
}

void launch_local_rowptr(const int64_t* off, const int64_t* rbase, const int64_t* lbase, int32_t nres, int64_t total,
                         int64_t* out, int cus, hipStream_t st) {
  if (total <= 0) return;
  hipLaunchKernelGGL(k_local_rowptr, dim3(grid_for(total, 256, cus * 8)), dim3(256), 0, st, off, rbase, lbase, nres,
                     total, out);
}

}  // namespace sg
