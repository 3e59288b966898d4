// Launch of the sweep kernels of one direction pass and of the fused x-y
// pass.  The host code (mfx.hip) calls launch_dispatch and launch_xy; their
// definitions (launch_impl.h) are instantiated in the k_*.hip translation
// units, one per family of kernels, so the library compiles in parallel.
#pragma once

#include <hip/hip_runtime.h>

#include "sweep.h"

namespace mfx {

// Geometry of one sweep launch for direction d.
struct SweepGeom {
    dim3 grid;
    int block;
    int seg;     // segment length (marching sweeps) or rows per block (x row sweep)
    size_t lds;  // dynamic LDS bytes
    bool xrows;  // x sweep by whole rows
};

// Pointers and scalars of one sweep launch.
struct LaunchArgs {
    const SweepGeom* sg;
    hipStream_t st;
    const Grid* g;
    const double* qs;
    const double* qn;
    void* r;  // partial RHS buffer (compute type)
    double* out;
    const double* dt_dev;
    double dt_arg;
    void* bface;             // boundary faces of the x row sweep (compute type)
    const MlpNet* mlp;      // packed network (learned weights only)
    unsigned long long* fb;  // fallback counter (learned weights only)
    double* partial;         // CFL block maxima (stage-3 y/z sweep with cfl)
    unsigned* status;
    bool cfl;  // this stage-3 sweep also reduces the CFL speed of its output
};

// Pointers and scalars of one fused x-y pass.
struct XYArgs {
    const Grid* g;
    hipStream_t st;
    const double* qs;
    const double* qn;
    void* r;  // partial RHS buffer (compute type)
    double* out;
    const double* dt_dev;
    double dt_arg;
    void* bface;  // boundary faces of the x rows (compute type)
    const MlpNet* mlp;
    unsigned long long* fb;
    int seg_override;  // segment length along y (0: automatic)
};

// One direction pass: direction d (0, 1, 2), whether it is the pass's first
// direction, output mode (OUT_*).  T: compute type; L: learned weights;
// SCHEME: reconstruction (SCHEME_*); F: fluid model.
template <typename T, bool L, int SCHEME, class F>
void launch_dispatch(int d, bool first, int mode, const LaunchArgs& a);

// The fused x-y pass (equal cells, Jiang-Shu-family weights); F: fluid model.
template <typename T, int SCHEME, class F>
void launch_xy(int mode, const XYArgs& a);

}  // namespace mfx
