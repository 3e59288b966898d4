// Kernel instantiations: the fused x-y pass, fluid model Fl<3>, float compute type.
#include "launch_impl.h"

namespace mfx {
template void launch_xy<float, SCHEME_WENO5, Fl<3>>(int, const XYArgs&);
template void launch_xy<float, SCHEME_WENO3, Fl<3>>(int, const XYArgs&);
template void launch_xy<float, SCHEME_WENO5Z, Fl<3>>(int, const XYArgs&);
}  // namespace mfx
