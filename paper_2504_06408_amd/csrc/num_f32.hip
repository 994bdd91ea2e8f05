// Numeric pass (product and merge) for the F32 semiring.
#include "sg_launch.hpp"

namespace sg {
void launch_numeric_f32(const NumCtx& c, hipStream_t st) { launch_numeric<SrF32, SrF32Comp>(c, st); }
}  // namespace sg
