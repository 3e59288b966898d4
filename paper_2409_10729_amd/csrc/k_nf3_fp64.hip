// Kernel instantiations: direction passes, double compute type, fluid model Fl<3>,
// every Jiang-Shu-family scheme.
#include "launch_impl.h"

namespace mfx {
template void launch_dispatch<double, false, SCHEME_WENO5, Fl<3>>(int, bool, int, const LaunchArgs&);
template void launch_dispatch<double, false, SCHEME_WENO3, Fl<3>>(int, bool, int, const LaunchArgs&);
template void launch_dispatch<double, false, SCHEME_WENO5Z, Fl<3>>(int, bool, int, const LaunchArgs&);
template void launch_dispatch<double, false, SCHEME_WENO5NU, Fl<3>>(int, bool, int, const LaunchArgs&);
}  // namespace mfx
