// Numeric pass (product and merge) for the I64 semiring.
#include "sg_launch.hpp"

namespace sg {
void launch_numeric_i64(const NumCtx& c, hipStream_t st) { launch_numeric<SrI64, SrI64>(c, st); }
}  // namespace sg
