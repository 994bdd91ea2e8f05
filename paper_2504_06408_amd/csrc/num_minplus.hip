// Numeric pass (product and merge) for the MinPlus semiring.
#include "sg_launch.hpp"

namespace sg {
void launch_numeric_minplus(const NumCtx& c, hipStream_t st) { launch_numeric<SrMinPlus, SrMinPlus>(c, st); }
}  // namespace sg
