// Definitions of the launch functions declared in launch.h, included only by
// the k_*.hip translation units that instantiate them.
#pragma once

#include "launch.h"
#include "sweep.h"
#include "xrow.h"

namespace mfx {

// The x row sweep reads the boundary faces that boundary_faces_x leaves in
// `bface` (launched just before it on the same stream).
// F: the fluid model (Fl2 or Fl<3>).
template <int DIR, typename T, bool FIRST, int MODE, bool L, int SCHEME, class F>
void launch_one(const LaunchArgs& a)
{
    const SweepGeom& sg = *a.sg;
    T* r = static_cast<T*>(a.r);
    if constexpr (DIR == 0) {
        if (sg.xrows) {
            T* bf = static_cast<T*>(a.bface);
            const long long rows = (long long)a.g->n[1] * a.g->n[2];
            boundary_faces_x<T, L, SCHEME, F><<<(unsigned)((rows + 255) / 256), 256, 0, a.st>>>(*a.g, a.qs, bf,
                                                                                                a.mlp, a.fb);
            sweep_x_rows<T, FIRST, MODE, L, SCHEME, F><<<sg.grid, sg.block, sg.lds, a.st>>>(
                *a.g, a.qs, a.qn, r, a.out, sg.seg, bf, a.dt_dev, a.dt_arg, a.mlp, a.fb);
            return;
        }
        sweep_x_march<T, FIRST, MODE, L, SCHEME, F><<<sg.grid, XROWS, 0, a.st>>>(
            *a.g, a.qs, a.qn, r, a.out, sg.seg, a.dt_dev, a.dt_arg, a.mlp, a.fb);
    } else {
        if constexpr (MODE == OUT_STAGE3 && !L) {
            if (a.cfl) {
                sweep_yz<DIR, T, FIRST, MODE, L, true, SCHEME, F><<<sg.grid, sg.block, 0, a.st>>>(
                    *a.g, a.qs, a.qn, r, a.out, sg.seg, a.dt_dev, a.dt_arg, a.mlp, a.fb, a.partial, a.status);
                return;
            }
        }
        sweep_yz<DIR, T, FIRST, MODE, L, false, SCHEME, F><<<sg.grid, sg.block, 0, a.st>>>(
            *a.g, a.qs, a.qn, r, a.out, sg.seg, a.dt_dev, a.dt_arg, a.mlp, a.fb, nullptr, a.status);
    }
}

template <int DIR, typename T, bool FIRST, bool L, int SCHEME, class F>
void launch_mode(int mode, const LaunchArgs& a)
{
    switch (mode) {
    case OUT_ACCUM: launch_one<DIR, T, FIRST, OUT_ACCUM, L, SCHEME, F>(a); break;
    case OUT_RHS: launch_one<DIR, T, FIRST, OUT_RHS, L, SCHEME, F>(a); break;
    case OUT_STAGE1: launch_one<DIR, T, FIRST, OUT_STAGE1, L, SCHEME, F>(a); break;
    case OUT_STAGE2: launch_one<DIR, T, FIRST, OUT_STAGE2, L, SCHEME, F>(a); break;
    default: launch_one<DIR, T, FIRST, OUT_STAGE3, L, SCHEME, F>(a); break;
    }
}

// The x sweep, when active, is always the first direction of a pass.
template <typename T, bool L, int SCHEME, class F>
void launch_dispatch(int d, bool first, int mode, const LaunchArgs& a)
{
    if (d == 0)
        launch_mode<0, T, true, L, SCHEME, F>(mode, a);
    else if (d == 1)
        first ? launch_mode<1, T, true, L, SCHEME, F>(mode, a) : launch_mode<1, T, false, L, SCHEME, F>(mode, a);
    else
        first ? launch_mode<2, T, true, L, SCHEME, F>(mode, a) : launch_mode<2, T, false, L, SCHEME, F>(mode, a);
}

template <typename T, int MODE, int SCHEME, class F>
void launch_xy_mode(const XYArgs& a)
{
    const Grid& g = *a.g;
    const long long rows = (long long)g.n[1] * g.n[2];
    // segments along y as for the y sweep (lanes = x, blocks over z and segments)
    int seg = a.seg_override > 0 ? a.seg_override : 64;
    const long long pencils = (long long)g.n[0] * g.n[2];
    while (seg > 16 && pencils * ((g.n[1] + seg - 1) / seg) < 256LL * 64 * 16) seg /= 2;
    seg = std::min(seg, g.n[1]);
    const dim3 grid(1, (unsigned)g.n[2], (unsigned)((g.n[1] + seg - 1) / seg));
    const int block = 64 * ((g.n[0] + 63) / 64);
    T* bf = static_cast<T*>(a.bface);
    boundary_faces_x<T, false, SCHEME, F><<<(unsigned)((rows + 255) / 256), 256, 0, a.st>>>(g, a.qs, bf, a.mlp, a.fb);
    const size_t lds = xrow_lds_bytes(g.n[0], sizeof(T), F::NV);
    sweep_xy<T, MODE, SCHEME, F><<<grid, block, lds, a.st>>>(g, a.qs, a.qn, static_cast<T*>(a.r), a.out, seg, bf,
                                                          a.dt_dev, a.dt_arg);
}

template <typename T, int SCHEME, class F>
void launch_xy(int mode, const XYArgs& a)
{
    switch (mode) {
    case OUT_ACCUM: launch_xy_mode<T, OUT_ACCUM, SCHEME, F>(a); break;
    case OUT_RHS: launch_xy_mode<T, OUT_RHS, SCHEME, F>(a); break;
    case OUT_STAGE1: launch_xy_mode<T, OUT_STAGE1, SCHEME, F>(a); break;
    case OUT_STAGE2: launch_xy_mode<T, OUT_STAGE2, SCHEME, F>(a); break;
    default: launch_xy_mode<T, OUT_STAGE3, SCHEME, F>(a); break;
    }
}

}  // namespace mfx
