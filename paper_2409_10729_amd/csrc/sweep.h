// One fused pass per direction of the finite-volume right-hand side
// (arXiv 2409.10729, Sec. II-B, eq. rhs): ghost-cell index map, conserved ->
// primitive, WENO5 face states, HLLC flux + face velocity, flux difference
// and alpha1 div(u) source, and -- in the last active direction of a stage --
// the SSP-RK3 combine and the CFL wave-speed maximum.
//
// Work decomposition: one thread marches along the sweep direction over a
// segment of `seg` cells of one pencil, keeping a 5-cell window of
// primitives in registers; each cell is reconstructed once (both edges from
// one set of smoothness indicators), each face solved once, each output
// written once.  Lanes of a wave are consecutive pencils: consecutive x for
// the y and z sweeps (coalesced 512-byte rows), consecutive y for the x sweep.
// Every lane of a wave sits at the same position along the sweep, so the
// boundary branches are wave-uniform.
#pragma once

#include "physics.h"

namespace mfx {

enum : int { BC_PERIODIC = 0, BC_TRANSMISSIVE = 1 };

// What the pass does with the accumulated right-hand side of a cell.
enum : int {
    OUT_ACCUM = 0,   // write the partial sum to the RHS buffer (not the last direction)
    OUT_RHS = 1,     // write the total to the caller's RHS array
    OUT_STAGE1 = 2,  // q1 = q + dt L
    OUT_STAGE2 = 3,  // q2 = 3/4 q + 1/4 (q1 + dt L)
    OUT_STAGE3 = 4,  // q  = 1/3 q + 2/3 (q2 + dt L), plus CFL partial maxima
};

struct Grid {
    int n[3];
    long long stride[3];  // 1, nx, nx*ny
    long long N;          // cells
    double dx[3];
    double inv_dx[3];
    int bc[3][2];
    int active[3];
    double G1, G2, P1, P2;  // per-fluid 1/(gamma-1) and gamma pi/(gamma-1)
    double eps;
    double cfl;
};

__device__ __forceinline__ int map_cell(int c, int n, int bclo, int bchi)
{
    if (c < 0) return bclo == BC_PERIODIC ? ((c % n) + n) % n : 0;
    if (c >= n) return bchi == BC_PERIODIC ? c % n : n - 1;
    return c;
}

// CFL wave speed sum_d (|u_d| + c) / dx_d of one cell, written in the same
// operation order as the plain definition and without contraction, so the
// reduced time step is reproducible across implementations.
__device__ __forceinline__ double cfl_speed(const Grid& g, const double q[NV], unsigned& bad)
{
#pragma clang fp contract(off)
    const double rho = q[0] + q[1];
    const double u = q[2] / rho, v = q[3] / rho, w = q[4] / rho;
    const double ke = 0.5 * rho * (u * u + v * v + w * w);
    const double a1 = q[6];
    const double G = a1 * g.G1 + (1.0 - a1) * g.G2;
    const double P = a1 * g.P1 + (1.0 - a1) * g.P2;
    const double p = (q[5] - ke - P) / G;
    const double c2 = ((G + 1.0) * p + P) / (G * rho);
    const double c = sqrt(c2);
    double s = 0.0;
    const double vel[3] = {u, v, w};
#pragma unroll
    for (int d = 0; d < 3; ++d)
        if (g.active[d]) s = s + (fabs(vel[d]) + c) / g.dx[d];
    if (!(rho > 0.0)) bad |= 1u;
    if (!(c2 > 0.0)) bad |= 2u;
    if (!isfinite(s)) bad |= 4u;
    return s;
}

template <int BLOCK>
__device__ __forceinline__ void block_max_to(double v, double* slot)
{
    __shared__ double red[BLOCK / 64];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) red[wid] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = red[0];
#pragma unroll
        for (int i = 1; i < BLOCK / 64; ++i) m = fmax(m, red[i]);
        *slot = m;
    }
}

// SSP-RK3 stage combination of one cell, in the operation order of the
// plain definition and without contraction: rho E feeds the pressure
// inversion, which turns one unit in the last place of rho E into ~1e-7 Pa
// in water at 1e5 Pa, so the stage update is kept reproducible.
__device__ __forceinline__ double rk3_combine(int mode, double qn, double qs, double dt, double r)
{
#pragma clang fp contract(off)
    const double a = qs + dt * r;
    if (mode == OUT_STAGE1) return a;
    if (mode == OUT_STAGE2) return 0.75 * qn + 0.25 * a;
    return (1.0 / 3.0) * qn + (2.0 / 3.0) * a;
}

// Everything a marching thread needs besides its cell source.
struct MarchArgs {
    const double* qs;  // stage state (for the stage update)
    const double* qn;  // step's initial state (aliases out in stage 3)
    double* racc;      // partial RHS buffer
    double* out;       // caller RHS or new state
    long long base;    // offset of the pencil's cell 0
    long long sd;      // stride along the sweep
    int c0, c1;        // segment [c0, c1)
    int first, mode;
    bool valid;        // this lane owns a real pencil (else compute, never store)
    double dt;
};

// The marching loop.  Src::load(pos, q) returns the conserved state of cell
// `pos` along the sweep (boundary map applied); it is called for positions
// c0-3, c0-2, ..., c1+2 in that order, the same sequence on every lane.
template <int DIR, class Src>
__device__ __forceinline__ double march(const Grid& g, Src& src, const MarchArgs& a, unsigned& bad)
{
    const long long N = g.N;
    const double idx = g.inv_dx[DIR];
    const double eps = g.eps;
    const Mix<double> mix{g.G1, g.G2, g.P1, g.P2};

    // window: W[k] = primitives of cell c-2+k while reconstructing cell c
    double W[5][NV];
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        double qc[NV];
        src.load(a.c0 - 3 + k, qc);
        cons_to_prim(mix, qc, W[k]);
    }

    double rprev[NV], Fprev[NV], ufprev = 0.0;
#pragma unroll
    for (int v = 0; v < NV; ++v) rprev[v] = Fprev[v] = 0.0;
    double smax = 0.0;

    for (int c = a.c0 - 1; c <= a.c1; ++c) {
        // next cell entering the window (c+3), fetched early
        double qnext[NV];
        if (c < a.c1) src.load(c + 3, qnext);

        double lft[NV], rgt[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) weno5_js<double>(W[0][v], W[1][v], W[2][v], W[3][v], W[4][v], eps, lft[v], rgt[v]);

        if (c >= a.c0) {
            double F[NV], uf;
            hllc<DIR, double>(mix, rprev, lft, F, uf);
            if (c > a.c0) {
                // cell c-1: faces c-3/2 (Fprev) and c-1/2 (F)
                const long long cell = a.base + (long long)(c - 1) * a.sd;
                double r[NV];
                if (a.first) {
#pragma unroll
                    for (int v = 0; v < NV; ++v) r[v] = (Fprev[v] - F[v]) * idx;
                } else {
#pragma unroll
                    for (int v = 0; v < NV; ++v) r[v] = a.racc[v * N + cell] + (Fprev[v] - F[v]) * idx;
                }
                r[6] += W[1][6] * ((uf - ufprev) * idx);
                if (a.valid) {
                    if (a.mode == OUT_ACCUM) {
#pragma unroll
                        for (int v = 0; v < NV; ++v) a.racc[v * N + cell] = r[v];
                    } else if (a.mode == OUT_RHS) {
#pragma unroll
                        for (int v = 0; v < NV; ++v) a.out[v * N + cell] = r[v];
                    } else {
                        double qo[NV];
#pragma unroll
                        for (int v = 0; v < NV; ++v) {
                            const double qnv = a.mode == OUT_STAGE1 ? 0.0 : a.qn[v * N + cell];
                            qo[v] = rk3_combine(a.mode, qnv, a.qs[v * N + cell], a.dt, r[v]);
                        }
#pragma unroll
                        for (int v = 0; v < NV; ++v) a.out[v * N + cell] = qo[v];
                        if (a.mode == OUT_STAGE3) smax = fmax(smax, cfl_speed(g, qo, bad));
                    }
                }
            }
#pragma unroll
            for (int v = 0; v < NV; ++v) Fprev[v] = F[v];
            ufprev = uf;
        }
#pragma unroll
        for (int v = 0; v < NV; ++v) rprev[v] = rgt[v];

        if (c < a.c1) {
#pragma unroll
            for (int k = 0; k < 4; ++k)
#pragma unroll
                for (int v = 0; v < NV; ++v) W[k][v] = W[k + 1][v];
            cons_to_prim(mix, qnext, W[4]);
        }
    }
    return smax;
}

// Cell source for the y and z sweeps: straight from global memory; the
// lanes of a wave are consecutive x, so each load is a contiguous row.
struct GlobalSrc {
    const double* __restrict__ qs;
    long long base, sd, N;
    int n, bclo, bchi;
    __device__ __forceinline__ void load(int pos, double q[NV]) const
    {
        const long long off = base + (long long)map_cell(pos, n, bclo, bchi) * sd;
#pragma unroll
        for (int v = 0; v < NV; ++v) q[v] = qs[v * N + off];
    }
};

// Launch geometry of the y and z sweeps: blockIdx.x * BLOCK + threadIdx.x =
// x index, blockIdx.y = the other transverse index (z for the y sweep, y for
// the z sweep), blockIdx.z = segment along the sweep.
// qn and out alias in the third stage (the new state overwrites q in place;
// each cell's q is read only by the thread that then writes it), so neither
// is declared __restrict__.
template <int DIR, int BLOCK, int MINW>
__global__ void __launch_bounds__(BLOCK, MINW) sweep_yz_fp64(Grid g, const double* __restrict__ qs,
                                                             const double* qn, double* __restrict__ racc,
                                                             double* out, int first, int mode, int seg,
                                                             const double* __restrict__ dt_dev, double dt_arg,
                                                             double* __restrict__ partial,
                                                             unsigned* __restrict__ status)
{
    static_assert(DIR == 1 || DIR == 2, "y or z sweep");
    constexpr int SA = (DIR == 2) ? 1 : 2;  // slow transverse axis
    const int n = g.n[DIR];
    const int nx = g.n[0];
    const int i_raw = blockIdx.x * BLOCK + threadIdx.x;
    const bool valid = i_raw < nx;
    const int i = valid ? i_raw : nx - 1;

    MarchArgs a;
    a.qs = qs;
    a.qn = qn;
    a.racc = racc;
    a.out = out;
    a.base = (long long)i + (long long)blockIdx.y * g.stride[SA];
    a.sd = g.stride[DIR];
    a.c0 = blockIdx.z * seg;
    a.c1 = min(a.c0 + seg, n);
    a.first = first;
    a.mode = mode;
    a.valid = valid;
    a.dt = dt_dev ? *dt_dev : dt_arg;

    GlobalSrc src{qs, a.base, a.sd, g.N, n, g.bc[DIR][0], g.bc[DIR][1]};
    unsigned bad = 0;
    const double smax = march<DIR>(g, src, a, bad);

    if (mode == OUT_STAGE3) {
        if (bad) atomicOr(status, bad);
        const long long bid = ((long long)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
        block_max_to<BLOCK>(smax, partial + bid);
    }
}

// Cell source for the x sweep.  The 64 lanes of the (one-wave) block own 64
// consecutive rows and march along x together; every XCHUNK positions the
// block stages the next XCHUNK cells of all 64 rows through LDS with
// row-contiguous reads (XCHUNK consecutive doubles per row and variable),
// then each lane reads its own row from LDS.
constexpr int XROWS = 64;
constexpr int XCHUNK = 4;

struct LdsSrc {
    double (*buf)[NV][XROWS];  // [XCHUNK][NV][XROWS]
    const double* __restrict__ qs;
    long long N;
    long long row0;  // first row of the block
    long long nrows;
    int nx, bclo, bchi;
    int pstart;  // first position fetched (c0 - 3)

    __device__ __forceinline__ void load(int pos, double q[NV]) const
    {
        const int slot = (pos - pstart) % XCHUNK;
        if (slot == 0) {
            __syncthreads();  // every lane has consumed the previous chunk
            const int lane = threadIdx.x;
#pragma unroll
            for (int it = 0; it < XCHUNK; ++it) {
                const int item = lane + it * XROWS;
                const int r = item / XCHUNK, cx = item % XCHUNK;
                const long long row = min(row0 + r, nrows - 1);
                const long long off = row * nx + map_cell(pos + cx, nx, bclo, bchi);
#pragma unroll
                for (int v = 0; v < NV; ++v) buf[cx][v][r] = qs[v * N + off];
            }
            __syncthreads();
        }
#pragma unroll
        for (int v = 0; v < NV; ++v) q[v] = buf[slot][v][threadIdx.x];
    }
};

// Launch geometry of the x sweep: blockIdx.x = group of 64 rows (row =
// k * ny + j, x-contiguous in memory), blockIdx.z = segment along x.
template <int MINW>
__global__ void __launch_bounds__(XROWS, MINW) sweep_x_fp64(Grid g, const double* __restrict__ qs,
                                                            const double* qn, double* __restrict__ racc,
                                                            double* out, int first, int mode, int seg,
                                                            const double* __restrict__ dt_dev, double dt_arg,
                                                            double* __restrict__ partial,
                                                            unsigned* __restrict__ status)
{
    __shared__ double buf[XCHUNK][NV][XROWS];
    const int nx = g.n[0];
    const long long nrows = (long long)g.n[1] * g.n[2];
    const long long row0 = (long long)blockIdx.x * XROWS;
    const long long row_raw = row0 + threadIdx.x;
    const bool valid = row_raw < nrows;
    const long long row = valid ? row_raw : nrows - 1;

    MarchArgs a;
    a.qs = qs;
    a.qn = qn;
    a.racc = racc;
    a.out = out;
    a.base = row * nx;
    a.sd = 1;
    a.c0 = blockIdx.z * seg;
    a.c1 = min(a.c0 + seg, nx);
    a.first = first;
    a.mode = mode;
    a.valid = valid;
    a.dt = dt_dev ? *dt_dev : dt_arg;

    LdsSrc src{buf, qs, g.N, row0, nrows, nx, g.bc[0][0], g.bc[0][1], a.c0 - 3};
    unsigned bad = 0;
    const double smax = march<0>(g, src, a, bad);

    if (mode == OUT_STAGE3) {
        if (bad) atomicOr(status, bad);
        const long long bid = (long long)blockIdx.z * gridDim.x + blockIdx.x;
        block_max_to<XROWS>(smax, partial + bid);
    }
}

}  // namespace mfx
