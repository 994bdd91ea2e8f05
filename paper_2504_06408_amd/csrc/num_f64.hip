// Numeric pass (product and merge) for the F64 semiring.
#include "sg_launch.hpp"

namespace sg {
void launch_numeric_f64(const NumCtx& c, hipStream_t st) { launch_numeric<SrF64, SrF64>(c, st); }
}  // namespace sg
