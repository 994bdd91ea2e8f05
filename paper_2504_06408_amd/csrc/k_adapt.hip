// Kernels of the column-major adapter (paper, Section 4.1, Algorithm 1) and
// of the power driver (Section 2.2): DCSC column-pointer decompression and
// compression, the identity matrix of a semiring, and an exact comparison of
// two CSR matrices.
#include "sg_adapt.hpp"

namespace sg {

namespace {

// colptr[j] = cp[#{i : jc[i] < j}] for j = 0..ncols: every column id that
// the compressed list skips gets an empty segment at the running offset.
__global__ __launch_bounds__(256) void k_dcsc_decompress(const int32_t* jc, const int64_t* cp, int64_t nzc,
                                                         int64_t ncols, int64_t* colptr) {
  for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j <= ncols; j += (int64_t)gridDim.x * 256) {
    int64_t lo = 0, hi = nzc;  // first i with jc[i] >= j
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if ((int64_t)jc[mid] < j) lo = mid + 1;
      else hi = mid;
    }
    colptr[j] = cp[lo];
  }
}

// flag[j] = 1 when column j holds an entry.
__global__ __launch_bounds__(256) void k_nonempty(const int64_t* colptr, int64_t ncols, int64_t* flag) {
  for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < ncols; j += (int64_t)gridDim.x * 256)
    flag[j] = colptr[j + 1] > colptr[j] ? 1 : 0;
}

// With incl[j] the inclusive count of non-empty columns up to j: the i-th
// non-empty column j goes to jc[i], its first entry to cp[i]; cp[nzc] = nnz.
__global__ __launch_bounds__(256) void k_dcsc_compress(const int64_t* colptr, const int64_t* incl, int64_t ncols,
                                                       int32_t* jc, int64_t* cp) {
  for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < ncols; j += (int64_t)gridDim.x * 256) {
    const int64_t c0 = colptr[j];
    if (colptr[j + 1] > c0) {
      const int64_t i = incl[j] - 1;
      jc[i] = (int32_t)j;
      cp[i] = c0;
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) cp[ncols > 0 ? incl[ncols - 1] : 0] = colptr[ncols];
}

// The n x n identity of a semiring: row i holds (i, one).
__global__ __launch_bounds__(256) void k_identity(int64_t n, uint64_t one, int vbytes, int64_t* rowptr, int32_t* col,
                                                  void* val) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i <= n; i += (int64_t)gridDim.x * 256) {
    rowptr[i] = i;
    if (i == n) break;
    col[i] = (int32_t)i;
    switch (vbytes) {
      case 8: ((uint64_t*)val)[i] = one; break;
      case 4: ((uint32_t*)val)[i] = (uint32_t)one; break;
      default: ((uint8_t*)val)[i] = (uint8_t)one; break;
    }
  }
}

// flag |= 1 when the row offsets, column ids or value bits of X and Y
// differ (both hold nnz entries).
__global__ __launch_bounds__(256) void k_csr_equal(const int64_t* xr, const int32_t* xc, const void* xv,
                                                   const int64_t* yr, const int32_t* yc, const void* yv, int64_t n,
                                                   int64_t nnz, int vbytes, int32_t* flag) {
  bool diff = false;
  const int64_t stride = (int64_t)gridDim.x * 256;
  const int64_t t0 = (int64_t)blockIdx.x * 256 + threadIdx.x;
  for (int64_t i = t0; i <= n; i += stride) diff |= xr[i] != yr[i];
  for (int64_t e = t0; e < nnz; e += stride) {
    diff |= xc[e] != yc[e];
    switch (vbytes) {
      case 8: diff |= ((const uint64_t*)xv)[e] != ((const uint64_t*)yv)[e]; break;
      case 4: diff |= ((const uint32_t*)xv)[e] != ((const uint32_t*)yv)[e]; break;
      default: diff |= ((const uint8_t*)xv)[e] != ((const uint8_t*)yv)[e]; break;
    }
  }
  if (__ballot(diff) != 0ull && lane_id() == 0) atomicOr(flag, 1);
}

}  // namespace

void launch_dcsc_decompress(const int32_t* jc, const int64_t* cp, int64_t nzc, int64_t ncols, int64_t* colptr,
                            int cus, hipStream_t st) {
  hipLaunchKernelGGL(k_dcsc_decompress, dim3(grid_for(ncols + 1, 256, cus * 16)), dim3(256), 0, st, jc, cp, nzc,
                     ncols, colptr);
}

void launch_dcsc_compress(const int64_t* colptr, int64_t ncols, int64_t* incl, int64_t* partial, int32_t* jc,
                          int64_t* cp, int cus, hipStream_t st) {
  if (ncols > 0) {
    hipLaunchKernelGGL(k_nonempty, dim3(grid_for(ncols, 256, cus * 16)), dim3(256), 0, st, colptr, ncols, incl);
    launch_scan_inclusive(incl, ncols, partial, st);
  }
  hipLaunchKernelGGL(k_dcsc_compress, dim3(grid_for(ncols, 256, cus * 16)), dim3(256), 0, st, colptr, incl, ncols,
                     jc, cp);
}

void launch_identity(int64_t n, uint64_t one, int vbytes, int64_t* rowptr, int32_t* col, void* val, int cus,
                     hipStream_t st) {
  hipLaunchKernelGGL(k_identity, dim3(grid_for(n + 1, 256, cus * 16)), dim3(256), 0, st, n, one, vbytes, rowptr, col,
                     val);
}

void launch_csr_equal(const int64_t* xr, const int32_t* xc, const void* xv, const int64_t* yr, const int32_t* yc,
                      const void* yv, int64_t n, int64_t nnz, int vbytes, int32_t* flag, int cus, hipStream_t st) {
  const int64_t work = nnz > n + 1 ? nnz : n + 1;
  hipLaunchKernelGGL(k_csr_equal, dim3(grid_for(work, 256, cus * 16)), dim3(256), 0, st, xr, xc, xv, yr, yc, yv, n,
                     nnz, vbytes, flag);
}

}  // namespace sg
