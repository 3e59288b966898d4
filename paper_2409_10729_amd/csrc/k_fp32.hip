// Kernel instantiations: direction passes, float compute type, fluid model Fl2,
// every Jiang-Shu-family scheme.
#include "launch_impl.h"

namespace mfx {
template void launch_dispatch<float, false, SCHEME_WENO5, Fl2>(int, bool, int, const LaunchArgs&);
template void launch_dispatch<float, false, SCHEME_WENO3, Fl2>(int, bool, int, const LaunchArgs&);
template void launch_dispatch<float, false, SCHEME_WENO5Z, Fl2>(int, bool, int, const LaunchArgs&);
template void launch_dispatch<float, false, SCHEME_WENO5NU, Fl2>(int, bool, int, const LaunchArgs&);
}  // namespace mfx
