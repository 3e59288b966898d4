// Kernel instantiations: the fused x-y pass, double compute type.
#include "launch_impl.h"

namespace mfx {
template void launch_xy<double, SCHEME_WENO5, Fl2>(int, const XYArgs&);
template void launch_xy<double, SCHEME_WENO3, Fl2>(int, const XYArgs&);
template void launch_xy<double, SCHEME_WENO5Z, Fl2>(int, const XYArgs&);
}  // namespace mfx
