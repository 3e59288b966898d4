// Kernel instantiations: the fused x-y pass, double compute type.
#include "launch_impl.h"

namespace mfx {
template void launch_xy<double, SCHEME_WENO5>(int, const XYArgs&);
template void launch_xy<double, SCHEME_WENO3>(int, const XYArgs&);
template void launch_xy<double, SCHEME_WENO5Z>(int, const XYArgs&);
}  // namespace mfx
