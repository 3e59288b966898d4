// Kernel instantiations: direction passes with learned weights (float
// compute type, two fluids).
#include "launch_impl.h"

namespace mfx {
template void launch_dispatch<float, true, SCHEME_WENO5, Fl2>(int, bool, int, const LaunchArgs&);
}  // namespace mfx
