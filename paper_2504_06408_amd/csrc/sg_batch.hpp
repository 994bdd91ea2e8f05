// Batched-path helpers shared by batch.cpp and k_batch.hip.
#pragma once

#include "sg_launch.hpp"

namespace sg {

void launch_pool_guard(const int64_t* off_end, int64_t cap_entries, int32_t* bin_count, int32_t* flag,
                       hipStream_t st);
void launch_local_rowptr(const int64_t* off, const int64_t* rbase, const int64_t* lbase, int32_t nres, int64_t total,
                         int64_t* out, int cus, hipStream_t st);

}  // namespace sg
