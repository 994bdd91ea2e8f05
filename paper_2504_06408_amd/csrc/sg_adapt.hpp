// Launchers of the column-major adapter and power-driver kernels (k_adapt.hip).
#pragma once

#include "sg_launch.hpp"

namespace sg {

// colptr[0..ncols] of a DCSC matrix from its non-empty column ids jc and
// their offsets cp (nzc + 1 entries).
void launch_dcsc_decompress(const int32_t* jc, const int64_t* cp, int64_t nzc, int64_t ncols, int64_t* colptr,
                            int cus, hipStream_t st);
// jc, cp of the non-empty columns of colptr; incl: ncols int64 of scratch
// (ends as the inclusive count of non-empty columns), partial: scan scratch.
void launch_dcsc_compress(const int64_t* colptr, int64_t ncols, int64_t* incl, int64_t* partial, int32_t* jc,
                          int64_t* cp, int cus, hipStream_t st);
// The n x n identity with value bits `one` (vbytes 8, 4 or 1).
void launch_identity(int64_t n, uint64_t one, int vbytes, int64_t* rowptr, int32_t* col, void* val, int cus,
                     hipStream_t st);
// *flag |= 1 unless X and Y (n rows, nnz entries each) agree in row offsets,
// column ids and value bits.
void launch_csr_equal(const int64_t* xr, const int32_t* xc, const void* xv, const int64_t* yr, const int32_t* yc,
                      const void* yv, int64_t n, int64_t nnz, int vbytes, int32_t* flag, int cus, hipStream_t st);

}  // namespace sg
