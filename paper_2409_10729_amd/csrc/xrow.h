// x sweep by whole rows: one lane per cell, rows of up to XROW_MAX cells.
//
// A block of ceil(nx/64) waves owns a run of rows (row = k*ny + j, contiguous
// in memory) and walks them in order.  For each row every lane loads and
// converts its own cell (coalesced 512-byte segments), the x stencil is read
// from an LDS copy of the row's primitives, and each face is solved once by
// the lane on its left.  Ghost primitives are plain LDS copies of the cells
// the boundary map points at, so no cell is loaded or converted twice.  The
// two boundary faces of every row (x = -1/2 and nx - 1/2), whose stencils
// reach ghost cells on both sides, are solved beforehand by
// boundary_faces_x for all rows at once, which keeps every lane of the row
// kernel on the same path.
#pragma once

#include "sweep.h"

namespace mfx {

constexpr int XROW_MAX = 512;       // longest row the row kernel takes
constexpr int XROW_THREADS = 512;   // launch bound (blockDim = 64 * ceil(nx / 64))
// Values per boundary face: the flux components and the face velocity.
template <class F>
constexpr int bface_of() { return F::NV + 1; }

// Boundary faces of every row, one lane per row: face 0 lies between ghost
// cell -1 and cell 0, face 1 between cell nx-1 and ghost cell nx; output
// bface[(row*2 + side) * (F::NV + 1) + k].  For nx >= 6 every stencil position
// either face reaches maps onto one of six anchor cells (0, 1, 2, nx-3,
// nx-2, nx-1) at both periodic and transmissive ends, so each lane loads
// and converts those six cells once and assembles both 6-cell stencils from
// them; with periodic ends the two faces are one face, solved once.
// Shorter rows map every position through the boundary rule.
template <typename T, bool LEARNED, int SCHEME = 5, class F = Fl2>
__global__ void __launch_bounds__(256) boundary_faces_x(Grid g, const double* __restrict__ qs, T* __restrict__ bface,
                                                        const MlpNet* __restrict__ mlp, unsigned long long* fb)
{
    const long long nrows = (long long)g.n[1] * g.n[2];
    const long long r_raw = (long long)blockIdx.x * 256 + threadIdx.x;
    const bool valid = r_raw < nrows;  // every lane computes (the learned weights need whole waves)
    const long long row = valid ? r_raw : nrows - 1;
    const int nx = g.n[0];
    const int blo = g.bc[0][0], bhi = g.bc[0][1];
    const bool anchored = nx >= 6;
    constexpr int V = F::NV, BF = bface_of<F>();
    const MixOf<F> mixd = make_mix<double, F>(g);
    const auto mix = make_mix<T, F>(g);
    const T eps = (T)g.eps;
    T a[6][V];
    if (anchored) {
#pragma unroll
        for (int j = 0; j < 6; ++j) {
            const int cell = j < 3 ? j : nx - 6 + j;
            double q[V];
#pragma unroll
            for (int v = 0; v < V; ++v) q[v] = qs[v * g.N + row * nx + cell];
            prim_of<T, F>(mixd, q, a[j]);
        }
    }
    auto recon = make_recon<T, LEARNED, SCHEME>(g, mlp, valid);
    recon.template bind<0>(g);  // (unequal cells: coefficients per face position)
    const int sides = blo == BC_PERIODIC ? 1 : 2;  // periodic ends pair up
#pragma unroll 1
    for (int side = 0; side < sides; ++side) {
        // stencil positions -3..2 (face 0) or nx-3..nx+2 (face 1)
        T w[6][V];
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const int pos = side == 0 ? k - 3 : nx - 3 + k;
            const int cell = map_cell(pos, nx, blo, bhi);
            if (anchored) {
                const int j = cell < 3 ? cell : cell - nx + 6;
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    T x = a[0][v];
#pragma unroll
                    for (int m = 1; m < 6; ++m) x = j == m ? a[m][v] : x;
                    w[k][v] = x;
                }
            } else {
                double q[V];
#pragma unroll
                for (int v = 0; v < V; ++v) q[v] = qs[v * g.N + row * nx + cell];
                prim_of<T, F>(mixd, q, w[k]);
            }
            if (special_ghost(pos, nx, blo, bhi)) ghost_fix<0, T, F>(g, mixd, pos, blo, bhi, w[k]);
        }
        // right edge of the cell before the face (window w[0..4]) and left
        // edge of the cell after it (window w[1..5])
        T wl[V], wr[V], dummy[V];
        recon.count_edges(true, false);  // the face uses this cell's right edge
        recon.at(side == 0 ? -1 : nx - 1);
        recon.cell_win(ArrayWindow<T, V>{w}, eps, dummy, wl);
        recon.count_edges(false, true);  // and the next cell's left edge
        recon.at(side == 0 ? 0 : nx);
        recon.cell_win(ArrayWindow<T, V>{w + 1}, eps, wr, dummy);
        T Fx[V], uf;
        hllc_f<0, T, F>(mix, wl, wr, Fx, uf);
        if (valid) {
            for (int out = side; out < 2; out += sides) {
                T* o = bface + (row * 2 + out) * BF;
#pragma unroll
                for (int v = 0; v < V; ++v) o[v] = Fx[v];
                o[V] = uf;
            }
        }
    }
    recon.flush(fb);
}

// LDS layout of the row kernel for nv variables (offsets in elements of
// T): primitives P[nv][nx+4] (two ghost slots on each side), face fluxes
// Fs[nv+1][nx] and left-edge states L[nv][nx].  P and Fs get storage of their own when all
// three fit in 64 KB; then a row can start overwriting P without waiting for
// the previous row's flux reads (the barriers inside the row order every
// other reuse).  Longer rows let Fs share P's storage (P is dead once every
// lane has reconstructed) and start each row with a barrier.
struct XrowLayout {
    size_t p, fs, l, elems;
    bool alias;
};

__host__ __device__ inline XrowLayout xrow_layout(int nx, size_t elem, int nv)
{
    const size_t np = (size_t)nx + 4;
    const size_t pe = (size_t)nv * np, fe = (size_t)(nv + 1) * nx, le = (size_t)nv * nx;
    XrowLayout L{};
    if (elem * (pe + fe + le) <= 64 * 1024) {
        L.p = 0;
        L.fs = pe;
        L.l = pe + fe;
        L.elems = pe + fe + le;
        L.alias = false;
    } else {
        const size_t pf = pe > fe ? pe : fe;
        L.p = 0;
        L.fs = 0;
        L.l = pf;
        L.elems = pf + le;
        L.alias = true;
    }
    return L;
}

inline size_t xrow_lds_bytes(int nx, size_t elem, int nv) { return elem * xrow_layout(nx, elem, nv).elems; }

// Ghost slot of the row buffer (p = P + slot, stride np between variables)
// filled, row by row, by the lane whose cell the index map names: a copy of
// its primitives w, with the normal velocity negated on a reflective side.
template <typename T, class F>
__device__ __forceinline__ void put_ghost_slot(T* p, int np, const T* w, unsigned refl)
{
#pragma unroll
    for (int v = 0; v < F::NV; ++v) p[v * np] = v == F::IM && refl ? -w[v] : w[v];
}

// Ghost slots of an inflow side hold the primitives of the side's state for
// every row: written once per block (mask: the inflow slots this lane
// owns).  Only the unaliased row buffer keeps them between rows; the host
// sends rows that need the aliased layout and have an inflow x side to the
// marching x sweep.
template <typename T, class F>
__device__ __forceinline__ void inflow_slots_init(const Grid& g, const MixOf<F>& mixd, unsigned mask, T* P, int np,
                                                  int nx)
{
    if (!mask) return;
#pragma unroll 1
    for (int s = 0; s < 2; ++s) {
        if ((mask >> (2 * s)) & 3u) {
            double qi[F::NV];
#pragma unroll
            for (int v = 0; v < F::NV; ++v) qi[v] = g.inflow[0][s][v];
            T wi[F::NV];
            prim_of<T, F>(mixd, qi, wi);
            const int slot0 = s == 0 ? 0 : nx + 2;
#pragma unroll
            for (int v = 0; v < F::NV; ++v) P[v * np + slot0] = P[v * np + slot0 + 1] = wi[v];
        }
    }
}

// Window of cell x inside the row's primitives in LDS: w(k, v) = P[v][x + k]
// (cell x-2+k; ghost slots included).
template <typename T, int NVV = NV>
struct RowWindow {
    static constexpr int nv = NVV;
    const T* p;  // P + x
    int np;
    __device__ __forceinline__ T operator()(int k, int v) const { return p[v * np + k]; }
};

// Row kernel.
template <typename T, bool FIRST, int MODE, bool LEARNED, int SCHEME = 5, class F = Fl2>
__global__ void __launch_bounds__(XROW_THREADS) __attribute__((amdgpu_waves_per_eu(LEARNED ? 3 : 1))) sweep_x_rows(Grid g, const double* __restrict__ qs, const double* qn,
                                                             T* __restrict__ racc, double* out, int rows_per_block,
                                                             const T* __restrict__ bface,
                                                             const double* __restrict__ dt_dev, double dt_arg,
                                                             const MlpNet* __restrict__ mlp, unsigned long long* fb)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    T* lds = reinterpret_cast<T*>(lds_raw);
    const int nx = g.n[0];
    const int np = nx + 4;
    constexpr int V = F::NV, BF = bface_of<F>();
    const XrowLayout lay = xrow_layout(nx, sizeof(T), V);
    T* P = lds + lay.p;    // [V][np], cell x at index x + 2
    T* Fs = lds + lay.fs;  // [V + 1][nx]
    T* L = lds + lay.l;    // [V][nx]
    const long long nrows = (long long)g.n[1] * g.n[2];
    const long long r0 = (long long)blockIdx.x * rows_per_block;
    const long long r1 = min(r0 + rows_per_block, nrows);
    const int x = threadIdx.x;
    const bool has = x < nx;
    const int xc = has ? x : nx - 1;
    const T idx = (T)g.inv_dx[0];
    const T eps = (T)g.eps;
    const MixOf<F> mixd = make_mix<double, F>(g);
    const auto mix = make_mix<T, F>(g);
    const OutArgs<T> o{qs, qn, racc, out, dt_dev ? *dt_dev : dt_arg};
    // ghost slots (positions -2, -1, nx, nx+1) this lane's cell fills, which
    // of them are reflective ghosts, and the inflow slots (written once)
    const unsigned gref = ghost_reflect(g.bc[0][0], g.bc[0][1]);
    const unsigned ginf = ghost_inflow(g.bc[0][0], g.bc[0][1]);
    const unsigned gall = has ? ghost_slots_of(x, nx, g.bc[0][0], g.bc[0][1]) : 0u;
    inflow_slots_init<T, F>(g, mixd, gall & ginf, P, np, nx);
    const unsigned gmine = gall & ~ginf;  // slots this lane refills every row

    auto recon = make_recon<T, LEARNED, SCHEME, true, false>(g, mlp, has);  // (tiles in turn: registers)
    // unequal cells: each lane keeps the coefficients and the reciprocal
    // width of its own position for every row of the block
    recon.template bind<0>(g);
    recon.at(xc);
    const T ih = recon.inv_width(xc, idx);
    double qc[V];
    if (r0 < r1) {
#pragma unroll
        for (int v = 0; v < V; ++v) qc[v] = qs[v * g.N + r0 * nx + xc];
    }
    for (long long row = r0; row < r1; ++row) {
        if (lay.alias) __syncthreads();  // the previous row's fluxes (P's storage) are consumed
        // 1. own cell -> primitives in LDS (and the ghost slots that copy it)
        T w[V];
        prim_of<T, F>(mixd, qc, w);
        if (has) {
#pragma unroll
            for (int v = 0; v < V; ++v) P[v * np + x + 2] = w[v];
            // ghost slots: at most four lanes take them, one test per lane
            const int gslot[4] = {0, 1, nx + 2, nx + 3};
            if (gmine) {
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    if (gmine >> k & 1u) put_ghost_slot<T, F>(P + gslot[k], np, w, gref >> k & 1u);
                }
            }
        }
        __syncthreads();
        // prefetch the next row (with learned weights after the
        // reconstruction: the loads would hold 14 registers across the
        // network evaluations)
        auto prefetch = [&]() {
            if (row + 1 < r1) {
#pragma unroll
                for (int v = 0; v < V; ++v) qc[v] = qs[v * g.N + (row + 1) * nx + xc];
            }
        };
        if constexpr (!LEARNED) prefetch();
        // 2. reconstruct own cell (window read from the LDS row as it goes):
        // left edge to LDS, right edge kept
        T rgt[V], lft[V];
        // interior faces only: the row's end faces come from boundary_faces_x
        recon.count_edges(xc < nx - 1, xc > 0);
        recon.cell_win(RowWindow<T, V>{P + xc, np}, eps, lft, rgt);
        if constexpr (LEARNED) prefetch();
        if (has) {
#pragma unroll
            for (int v = 0; v < V; ++v) L[v * nx + x] = lft[v];
        }
        __syncthreads();
        // 3. face x+1/2 (the row's last face comes from boundary_faces_x)
        T Fx[BF];
        {
            T wr[V];
            const int xr = min(xc + 1, nx - 1);
#pragma unroll
            for (int v = 0; v < V; ++v) wr[v] = L[v * nx + xr];
            T Fh[V], ufh;
            hllc_f<0, T, F>(mix, rgt, wr, Fh, ufh);
            const T* b = bface + (row * 2 + 1) * BF;
            const bool last = xc == nx - 1;
#pragma unroll
            for (int v = 0; v < V; ++v) Fx[v] = last ? b[v] : Fh[v];
            Fx[V] = last ? b[V] : ufh;
        }
        if (has) {
#pragma unroll
            for (int k = 0; k < BF; ++k) Fs[k * nx + x] = Fx[k];
        }
        __syncthreads();
        // 4. cell x: faces x-1/2 (left neighbour, or the row's first face) and x+1/2
        if (has) {
            T Fm[BF];
            if (x == 0) {
                const T* b = bface + (row * 2 + 0) * BF;
#pragma unroll
                for (int k = 0; k < BF; ++k) Fm[k] = b[k];
            } else {
#pragma unroll
                for (int k = 0; k < BF; ++k) Fm[k] = Fs[k * nx + x - 1];
            }
            T fd[V];
#pragma unroll
            for (int v = 0; v < V; ++v) fd[v] = (Fm[v] - Fx[v]) * ih;
            // every volume fraction's source alpha_a div(u)
            T src[F::NA];
#pragma unroll
            for (int a = 0; a < F::NA; ++a) src[a] = w[F::IA + a] * ((Fx[V] - Fm[V]) * ih);
            emit_cell<T, FIRST, MODE, F>(g, o, row * nx + x, fd, src);
        }
    }
    recon.flush(fb);
}

// Fused x and y passes: a block of 64 * ceil(nx / 64) lanes owns whole x
// rows of one z plane and marches along y over a segment (lane = x, as in
// the y sweep).  When the march puts cell row j (window slot W(1)), the
// block also computes that row's x contribution from the row's primitives,
// which every lane already holds: the same three-barrier row procedure as
// sweep_x_rows, with the row's end faces from boundary_faces_x.  Each cell
// then stores the sum (x part, then y part: the same additions in the same
// order as the x pass followed by the y pass) once, so the state is read
// once and the running sum never goes through memory.  The window lives in
// registers; LDS holds the row buffers of the x part (xrow_layout).
template <typename T, int MODE, int SCHEME = 5, class F = Fl2>
struct XYSink {
    static constexpr bool keeps_q = false;
    static constexpr int enter_at = ENTER_AFTER;  // see march
    static constexpr int V = F::NV, BF = bface_of<F>();
    using MixT = decltype(make_mix<T, F>(std::declval<const Grid&>()));
    __device__ __forceinline__ void prefetch(const Grid&, int) {}
    OutArgs<T> o;
    T* P;   // [V][nx+4]
    T* L;   // [V][nx]
    T* Fs;  // [V + 1][nx]
    const T* bface;
    long long base_z;  // first cell of the z plane
    long long row_z;   // first row (k * ny) of the z plane
    int nx, np, x, xc;
    bool has, alias;
    unsigned gmine;  // bit k: this lane's cell fills ghost slot k (positions -2, -1, nx, nx+1)
    unsigned gref;   // bit k: ghost slot k is on a reflective side (normal velocity negated)
    T idx, eps;
    MixT mix;

    template <class Win>
    __device__ __forceinline__ void put(const Grid& g, int c, const T* fdy, const T* srcy, const Win& W, const double*)
    {
        const long long row = row_z + c;
        T w[V];
#pragma unroll
        for (int v = 0; v < V; ++v) w[v] = W(1, v);
        if (alias) __syncthreads();  // the previous row's fluxes (P's storage) are consumed
        if (has) {
#pragma unroll
            for (int v = 0; v < V; ++v) P[v * np + x + 2] = w[v];
            const int gslot[4] = {0, 1, nx + 2, nx + 3};
            if (gmine) {  // at most four lanes
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    if (gmine >> k & 1u) put_ghost_slot<T, F>(P + gslot[k], np, w, gref >> k & 1u);
                }
            }
        }
        __syncthreads();
        T rgt[V], lft[V];
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const T* pv = P + v * np + xc;
            recon_scheme<T, SCHEME>(pv[0], pv[1], pv[2], pv[3], pv[4], eps, lft[v], rgt[v]);
            settle(lft[v], rgt[v]);
        }
        if (has) {
#pragma unroll
            for (int v = 0; v < V; ++v) L[v * nx + x] = lft[v];
        }
        __syncthreads();
        T Fx[BF];
        {
            T wr[V];
            const int xr = min(xc + 1, nx - 1);
#pragma unroll
            for (int v = 0; v < V; ++v) wr[v] = L[v * nx + xr];
            T Fh[V], ufh;
            hllc_f<0, T, F>(mix, rgt, wr, Fh, ufh);
            const T* b = bface + (row * 2 + 1) * BF;
            const bool last = xc == nx - 1;
#pragma unroll
            for (int v = 0; v < V; ++v) Fx[v] = last ? b[v] : Fh[v];
            Fx[V] = last ? b[V] : ufh;
        }
        if (has) {
#pragma unroll
            for (int k = 0; k < BF; ++k) Fs[k * nx + x] = Fx[k];
        }
        __syncthreads();
        if (has) {
            T Fm[BF];
            if (x == 0) {
                const T* b = bface + (row * 2 + 0) * BF;
#pragma unroll
                for (int k = 0; k < BF; ++k) Fm[k] = b[k];
            } else {
#pragma unroll
                for (int k = 0; k < BF; ++k) Fm[k] = Fs[k * nx + x - 1];
            }
            // x part, rounded as the x pass stores it
            T r[V];
#pragma unroll
            for (int v = 0; v < V; ++v) r[v] = (Fm[v] - Fx[v]) * idx;
#pragma unroll
            for (int a = 0; a < F::NA; ++a) r[F::IA + a] += w[F::IA + a] * ((Fx[V] - Fm[V]) * idx);
#pragma unroll
            for (int v = 0; v < V; ++v) asm volatile("" : "+v"(r[v]));
            // plus the y part
#pragma unroll
            for (int v = 0; v < V; ++v) r[v] = r[v] + fdy[v];
#pragma unroll
            for (int a = 0; a < F::NA; ++a) r[F::IA + a] += srcy[a];
            store_cell<T, MODE, F>(g, o, base_z + (long long)c * nx + x, r);
        }
    }
};

template <typename T, int MODE, int SCHEME = 5, class F = Fl2>
__global__ void __launch_bounds__(XROW_THREADS) sweep_xy(Grid g, const double* __restrict__ qs, const double* qn,
                                                         T* __restrict__ racc, double* out, int seg,
                                                         const T* __restrict__ bface,
                                                         const double* __restrict__ dt_dev, double dt_arg)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    T* lds = reinterpret_cast<T*>(lds_raw);
    const int nx = g.n[0], ny = g.n[1];
    const XrowLayout lay = xrow_layout(nx, sizeof(T), F::NV);
    const int x = threadIdx.x;
    const bool has = x < nx;
    const int xc = has ? x : nx - 1;
    const int z = blockIdx.y;
    const int c0 = blockIdx.z * seg;
    const int c1 = min(c0 + seg, ny);
    const long long base_z = (long long)z * g.stride[2];

    GlobalSrc<1, F> src{qs, g.inflow_dev + 1 * 2 * NVMAX, base_z + xc, g.stride[1], g.N, ny, g.bc[1][0], g.bc[1][1]};
    XYSink<T, MODE, SCHEME, F> sink{OutArgs<T>{qs, qn, racc, out, dt_dev ? *dt_dev : dt_arg},
                         lds + lay.p,
                         lds + lay.l,
                         lds + lay.fs,
                         bface,
                         base_z,
                         (long long)z * ny,
                         nx,
                         nx + 4,
                         x,
                         xc,
                         has,
                         lay.alias,
                         (has ? ghost_slots_of(x, nx, g.bc[0][0], g.bc[0][1]) : 0u) & ~ghost_inflow(g.bc[0][0], g.bc[0][1]),
                         ghost_reflect(g.bc[0][0], g.bc[0][1]),
                         (T)g.inv_dx[0],
                         (T)g.eps,
                         make_mix<T, F>(g)};
    inflow_slots_init<T, F>(g, make_mix<double, F>(g),
                         (has ? ghost_slots_of(x, nx, g.bc[0][0], g.bc[0][1]) : 0u) & ghost_inflow(g.bc[0][0], g.bc[0][1]),
                         lds + lay.p, nx + 4, nx);
    ReconJS<T, SCHEME> recon{};
    RegWindow<T, F::NV> W;
    march<1, T, F>(g, src, sink, recon, c0, c1, W);
}

}  // namespace mfx
