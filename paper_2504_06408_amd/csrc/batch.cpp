// Batched persistent path (placeholder until the persistent kernels land).
#include "sg_handle.hpp"

struct sg_plan {
  sg_handle* h;
};

extern "C" {
sg_status sg_batch_plan(sg_handle* h, const sg_semiring*, int, const sg_csr*, const sg_csr*, int, const int32_t*,
                        size_t, sg_plan** out) {
  if (out) *out = nullptr;
  return sg_fail(h, SG_ERR_INVALID, "batched path not available in this build");
}
sg_status sg_batch_execute(sg_plan*, void*) { return SG_ERR_INVALID; }
sg_status sg_batch_results(sg_plan*, sg_csr*) { return SG_ERR_INVALID; }
sg_status sg_plan_destroy(sg_plan*) { return SG_ERR_INVALID; }
}
