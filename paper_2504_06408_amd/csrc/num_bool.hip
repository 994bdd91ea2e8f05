// Numeric pass (product and merge) for the Bool semiring.
#include "sg_launch.hpp"

namespace sg {
void launch_numeric_bool(const NumCtx& c, hipStream_t st) { launch_numeric<SrBool, SrBool>(c, st); }
}  // namespace sg
