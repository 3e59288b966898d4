// Fused passes of the finite-volume right-hand side (arXiv 2409.10729,
// Sec. II-B, eq. rhs): ghost-cell index map, conserved -> primitive, WENO
// face states (fifth order, or third), HLLC flux + face velocity, flux
// difference and alpha1 div(u) source, and -- in the last active direction
// of a stage -- the SSP-RK3 combine; the stage-3 pass also reduces the CFL
// wave speed of the new state.
//
// T is the arithmetic of reconstruction, Riemann solve and flux difference
// (double, or float for the mixed-precision form).  The conserved ->
// primitive conversion, the stage update and the CFL reduction are always
// float64; the partial RHS buffer holds T.
//
// Work decomposition of a marching pass: one thread marches along the sweep
// direction over a segment of `seg` cells of one pencil, keeping a 5-cell
// window of primitives (a ring in the lane's own LDS column, or in
// registers); each cell is reconstructed once (both edges from one set of
// smoothness indicators), each face solved once, each output written once.
// Lanes of a wave are consecutive pencils: consecutive x for the y and z
// sweeps (coalesced 512-byte rows), consecutive y for the marching x sweep.
// Every lane of a wave sits at the same position along the sweep, so the
// boundary branches are wave-uniform.  The x direction normally goes
// through whole rows in LDS (xrow.h), inside the y march where both are
// active.
#pragma once

#include <climits>

#include "learned.h"
#include "physics.h"

namespace mfx {

enum : int { BC_PERIODIC = 0, BC_TRANSMISSIVE = 1, BC_REFLECTIVE = 2, BC_INFLOW = 3 };

// What the pass does with the accumulated right-hand side of a cell.
enum : int {
    OUT_ACCUM = 0,   // write the partial sum to the RHS buffer (not the last direction)
    OUT_RHS = 1,     // write the total to the caller's RHS array
    OUT_STAGE1 = 2,  // q1 = q + dt L
    OUT_STAGE2 = 3,  // q2 = 3/4 q + 1/4 (q1 + dt L)
    OUT_STAGE3 = 4,  // q  = 1/3 q + 2/3 (q2 + dt L)
};

struct Grid {
    int n[3];
    long long stride[3];  // 1, nx, nx*ny
    long long N;          // cells
    double dx[3];
    double inv_dx[3];
    int bc[3][2];
    int active[3];
    double G1, G2, P1, P2;  // per-fluid 1/(gamma-1) and gamma pi/(gamma-1) (two fluids)
    int nf;                 // fluids
    double Gn[MAXF], Pn[MAXF];  // the same for every fluid
    double eps;
    double cfl;
    int edge_weights;  // learned weights: one network evaluation per edge for all variables
    double inflow[3][2][NVMAX];  // conserved state of the ghost cells of an inflow side
    const double* inflow_dev;    // the same states in device memory, [3][2][NVMAX]
    const double* nu[3];         // per-position tables of a non-uniform direction (NU_* below), else null
    int nonuniform;              // some direction has unequal cell widths
};

// Table of a direction with unequal cell widths (filled on the host from the
// face coordinates): the NU_K values of stencil position c (c = -1 .. n:
// every cell whose edges a face of the direction uses, ghosts included) at
// nu[(c + 1) * NU_K + k].  One position's values are contiguous, and every
// lane of a marching sweep reads the same position.
enum : int {
    NU_A = 0,    // NuCoef::a[3][3]
    NU_B = 9,    // NuCoef::b[3][3]
    NU_C = 18,   // NuCoef::c[3][3]
    NU_DR = 27,  // ideal weights of the right edge
    NU_DL = 30,  // ideal weights of the left edge
    NU_H = 33,   // the cell's width (CFL reduction)
    NU_IH = 34,  // its reciprocal (flux difference)
    NU_K = 36,   // values per position (padded to 32-byte rows)
};

// Mixture constants of the model F from the grid, in the type T.
template <typename T, class F>
__device__ __forceinline__ auto make_mix(const Grid& g)
{
    if constexpr (F::NF == 2) {
        return Mix<T>{(T)g.G1, (T)g.G2, (T)g.P1, (T)g.P2};
    } else {
        MixN<T, F::NF> m;
#pragma unroll
        for (int i = 0; i < F::NF; ++i) {
            m.G[i] = (T)g.Gn[i];
            m.P[i] = (T)g.Pn[i];
        }
        return m;
    }
}

// Cell whose state stencil position c takes.  Ghost positions (outside
// 0..n-1): periodic wraps around, transmissive repeats the edge cell,
// reflective mirrors about the wall face (-1-k <- k, n+k <- n-1-k; the three
// ghosts a stencil reaches need n >= 3) and the ghost carries the mirrored
// cell with its momentum normal to the wall negated (the loaders' finish(),
// the x-row ghost slots, ghost_fix()), a stationary slip wall.  An inflow
// ghost holds the side's fixed state: the loaders read it from the device
// copy instead, and the map's edge cell is only a placeholder.
// Positions further out (the marching x sweep stages whole chunks, up to
// n+5) are clamped into the row; no stencil uses them.
__host__ __device__ __forceinline__ int map_cell(int c, int n, int bclo, int bchi)
{
    if (c < 0) return bclo == BC_PERIODIC ? ((c % n) + n) % n : (bclo == BC_REFLECTIVE ? min(-1 - c, n - 1) : 0);
    if (c >= n) return bchi == BC_PERIODIC ? c % n : (bchi == BC_REFLECTIVE ? max(2 * n - 1 - c, 0) : n - 1);
    return c;
}

// Sides whose ghosts are not a plain copy of a cell: reflective and inflow.
__device__ __forceinline__ bool special_side(int bc) { return bc == BC_REFLECTIVE || bc == BC_INFLOW; }

// Ghost slots of the x-row kernels taking the inflow state: bit k set when
// slot k (positions -2, -1, n, n+1) lies on an inflow side.
__device__ __forceinline__ unsigned ghost_inflow(int bclo, int bchi)
{
    return (bclo == BC_INFLOW ? 3u : 0u) | (bchi == BC_INFLOW ? 12u : 0u);
}

// Ghost slots of the x-row kernels on a reflective side.
__device__ __forceinline__ unsigned ghost_reflect(int bclo, int bchi)
{
    return (bclo == BC_REFLECTIVE ? 3u : 0u) | (bchi == BC_REFLECTIVE ? 12u : 0u);
}

// True when stencil position c is a ghost of a reflective or inflow side.
__device__ __forceinline__ bool special_ghost(int c, int n, int bclo, int bchi)
{
    return (c < 0 && special_side(bclo)) || (c >= n && special_side(bchi));
}


// Ghost slots of the x-row kernels that cell x fills: bit k set when slot k
// (positions -2, -1, n, n+1) takes cell x's state.
__device__ __forceinline__ unsigned ghost_slots_of(int x, int n, int bclo, int bchi)
{
    return (map_cell(-2, n, bclo, bchi) == x ? 1u : 0u) | (map_cell(-1, n, bclo, bchi) == x ? 2u : 0u) |
           (map_cell(n, n, bclo, bchi) == x ? 4u : 0u) | (map_cell(n + 1, n, bclo, bchi) == x ? 8u : 0u);
}


// CFL wave speed sum_d (|u_d| + c) / dx_d of one cell, written in the same
// operation order as the plain definition and without contraction, so the
// reduced time step is reproducible across implementations.
// Volume fractions outside [0, 1]: alpha_1 .. alpha_{NF-1} and the last
// fluid's 1 - sum.
template <class F>
__device__ __forceinline__ bool alpha_out(const double* q)
{
    if constexpr (F::NF == 2) {
        return !(q[6] >= 0.0 && q[6] <= 1.0);
    } else {
        bool out = false;
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < F::NA; ++i) {
            out = out || !(q[F::IA + i] >= 0.0 && q[F::IA + i] <= 1.0);
            s += q[F::IA + i];
        }
        return out || !(s <= 1.0);
    }
}

// hw: the cell's widths per direction where they differ from g.dx (unequal
// cells), else null.
template <class F = Fl2>
__device__ __forceinline__ double cfl_speed(const Grid& g, const double* q, unsigned& bad, const double* hw = nullptr)
{
#pragma clang fp contract(off)
    double c2, u, v, w, rho;
    if constexpr (F::NF == 2) {
        rho = q[0] + q[1];
        const double ir = 1.0 / rho;
        u = q[2] * ir, v = q[3] * ir, w = q[4] * ir;
        const double ke = 0.5 * rho * (u * u + v * v + w * w);
        const double a1 = q[6];
        const double G = a1 * g.G1 + (1.0 - a1) * g.G2;
        const double P = a1 * g.P1 + (1.0 - a1) * g.P2;
        const double p = (q[5] - ke - P) / G;
        c2 = ((G + 1.0) * p + P) / (G * rho);
    } else {
        const MixN<double, F::NF> mix = make_mix<double, F>(g);
        double wp[F::NV];
        cons_to_prim_n<F::NF>(mix, q, wp);
        rho = density_n<F::NF>(q);
        u = wp[F::IM], v = wp[F::IM + 1], w = wp[F::IM + 2];
        const double G = mix.Gamma(q + F::IA), P = mix.Pi(q + F::IA);
        c2 = ((G + 1.0) * wp[F::IE] + P) / (G * rho);
    }
    const double c = sqrt(c2);
    double s = 0.0;
    const double vel[3] = {u, v, w};
#pragma unroll
    for (int d = 0; d < 3; ++d)
        if (g.active[d]) s = s + (fabs(vel[d]) + c) / (hw ? hw[d] : g.dx[d]);
    if (!(rho > 0.0)) bad |= 1u;
    if (!(c2 > 0.0)) bad |= 2u;
    if (!isfinite(s)) bad |= 4u;
    if (alpha_out<F>(q)) bad |= 8u;
    return s;
}

// Status bits of a state (the same bits as cfl_speed without the sound
// speed): density not positive (1), a non-finite value (4), a volume
// fraction outside [0, 1] (8).
template <class F = Fl2>
__device__ __forceinline__ unsigned state_bits(const double* q)
{
    unsigned bad = 0;
    double rho = q[0];
#pragma unroll
    for (int i = 1; i < F::NF; ++i) rho = rho + q[i];
    if (!(rho > 0.0)) bad |= 1u;
    bool fin = true;
#pragma unroll
    for (int v = 0; v < F::NV; ++v) fin = fin && isfinite(q[v]);
    if (!fin) bad |= 4u;
    if (alpha_out<F>(q)) bad |= 8u;
    return bad;
}

// What the last pass of a stage checks in the state it writes.
enum : int {
    CHK_NONE = 0,   // nothing (not the last pass of a stage, or the standalone reduction follows)
    CHK_STATE = 1,  // the status bits of state_bits (stages 1 and 2)
    CHK_CFL = 2,    // the CFL maximum and every status bit (stage 3)
};

// Widths of cell `cell` per direction (the table's width where the
// direction has unequal cells, else g.dx).
__device__ __forceinline__ void cell_widths(const Grid& g, long long cell, double hw[3])
{
    const long long pos[3] = {cell % g.n[0], (cell / g.n[0]) % g.n[1], cell / g.stride[2]};
#pragma unroll
    for (int d = 0; d < 3; ++d) hw[d] = g.nu[d] ? g.nu[d][(pos[d] + 1) * NU_K + NU_H] : g.dx[d];
}

// Running CFL maximum and validity flags of the cells a lane writes.  On
// unequal cells hw holds the widths of the cell being written: the lane's
// and the block's transverse positions are fixed for a marching sweep, so
// only the width along the sweep changes (at(c), from the direction's table
// nud; null where that direction has equal cells).
template <class F = Fl2>
struct CflAcc {
    double smax;
    unsigned bad;
    bool cfl;  // false: only the status bits, no CFL speed
    double hw[3];
    const double* nud;
    int dir;
    __device__ __forceinline__ void at(int c)
    {
        if (nud) hw[dir] = nud[(long long)(c + 1) * NU_K + NU_H];
    }
    __device__ __forceinline__ void add(const Grid& g, const double* q)
    {
        if (cfl)
            smax = fmax(smax, cfl_speed<F>(g, q, bad, g.nonuniform ? hw : nullptr));
        else
            bad |= state_bits<F>(q);
    }
};

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

// Everything an output needs: the stage state (for the stage update), the
// step's initial state (aliases out in stage 3), the partial RHS buffer (of
// the compute type) and the caller RHS or new state.
template <typename T>
struct OutArgs {
    const double* qs;
    const double* qn;
    T* racc;
    double* out;
    double dt;
};

// What a pass does with a cell's contribution of this direction: fd[v] =
// (F_{c-1/2} - F_{c+1/2}) / dx and the alpha1 source term src, added to the
// running sum as (R + fd) + src for alpha1 and R + fd otherwise.  FIRST
// (no running sum yet) and MODE (what is written) are compile-time so each
// kernel carries only its own path.
// qsc, qnc: the cell's stage state and step state when the caller holds
// them (else read from o.qs, o.qn).  acc: receives the new state of a stage
// update (CFL maximum of the result).
template <typename T, int MODE, class F = Fl2>
__device__ __forceinline__ void store_cell(const Grid& g, const OutArgs<T>& o, long long cell, const T* r,
                                           const double* qsc = nullptr, CflAcc<F>* acc = nullptr,
                                           const double* qnc = nullptr)
{
    const long long N = g.N;
    if constexpr (MODE == OUT_ACCUM) {
#pragma unroll
        for (int v = 0; v < F::NV; ++v) o.racc[v * N + cell] = r[v];
    } else if constexpr (MODE == OUT_RHS) {
#pragma unroll
        for (int v = 0; v < F::NV; ++v) o.out[v * N + cell] = (double)r[v];
    } else {
        double qo[F::NV];
#pragma unroll
        for (int v = 0; v < F::NV; ++v) {
            const double qnv = MODE == OUT_STAGE1 ? 0.0 : (qnc ? qnc[v] : o.qn[v * N + cell]);
            qo[v] = rk3_combine(MODE, qnv, qsc ? qsc[v] : o.qs[v * N + cell], o.dt, (double)r[v]);
        }
#pragma unroll
        for (int v = 0; v < F::NV; ++v) o.out[v * N + cell] = qo[v];
        if (acc) acc->add(g, qo);
    }
}

// src[a]: the volume-fraction sources alpha_a div(u) (F::NA of them).
template <typename T, bool FIRST, int MODE, class F = Fl2>
__device__ __forceinline__ void emit_cell(const Grid& g, const OutArgs<T>& o, long long cell, const T* fd,
                                          const T* src, const double* qsc = nullptr, CflAcc<F>* acc = nullptr)
{
    T r[F::NV];
#pragma unroll
    for (int v = 0; v < F::NV; ++v) r[v] = FIRST ? fd[v] : o.racc[v * g.N + cell] + fd[v];
#pragma unroll
    for (int a = 0; a < F::NA; ++a) r[F::IA + a] += src[a];
    store_cell<T, MODE, F>(g, o, cell, r, qsc, acc);
}

// Primitives of one cell in the compute type: the inversion is float64.
template <typename T, class F = Fl2>
__device__ __forceinline__ void prim_of(const MixOf<F>& mix, const double* q, T* w)
{
    double wd[F::NV];
    cons_to_prim_f<F>(mix, q, wd);
#pragma unroll
    for (int v = 0; v < F::NV; ++v) w[v] = (T)wd[v];
}

// Primitives w of a reflective or inflow ghost at position pos (outside the
// row, on the side pos names), given the primitives of the cell the index
// map loaded for it: a reflective ghost negates the normal velocity (the
// same bits as negating the momentum before the conversion), an inflow
// ghost takes the side's fixed state.
template <int DIR, typename T, class F = Fl2>
__device__ __forceinline__ void ghost_fix(const Grid& g, const MixOf<F>& mixd, int pos, int bclo, int bchi, T* w)
{
    const int side = pos < 0 ? 0 : 1;
    if ((side ? bchi : bclo) == BC_REFLECTIVE) {
        w[F::IM + DIR] = -w[F::IM + DIR];
    } else {
        double qi[F::NV];
#pragma unroll
        for (int v = 0; v < F::NV; ++v) qi[v] = g.inflow[DIR][side][v];
        prim_of<T, F>(mixd, qi, w);
    }
}

// Where the march converts the cell entering its window (see march).
constexpr int ENTER_BEFORE = 0, ENTER_AFTER = 1;

// Sink of the y and z sweeps: each lane writes its own cell (lanes are
// consecutive x, so every access is a contiguous row).  KEEPQ: the march
// hands over the cell's stage state, which it loaded four cells earlier,
// so the stage update does not read it again.
// CHK: what the pass checks in the state it writes (acc): the status bits
// (stages 1 and 2), or also the CFL wave speed of the step's new state
// (stage 3).  prefetch() loads the running sum and the step state
// of the cell the march puts next at the top of the march step, so the
// loads are in flight during its reconstruction and Riemann solve (lanes
// past the grid read the clamped column: in bounds, never stored).
// PREFETCH off (the learned passes): the loads stay where the output needs
// them, so they do not hold registers across the network evaluations.
template <typename T, bool FIRST, int MODE, bool KEEPQ = false, int CHK = CHK_NONE, bool PREFETCH = true,
          class F = Fl2>
struct GlobalSink {
    static constexpr bool keeps_q = KEEPQ;
    static constexpr int enter_at = PREFETCH ? ENTER_BEFORE : ENTER_AFTER;  // see march
    static constexpr bool NEEDQN = MODE == OUT_STAGE2 || MODE == OUT_STAGE3;
    OutArgs<T> o;
    long long base, sd;
    bool valid;
    CflAcc<F> acc;
    T rin[FIRST ? 1 : F::NV];
    double qnin[NEEDQN ? F::NV : 1];
    __device__ __forceinline__ void prefetch(const Grid& g, int c)
    {
        if constexpr (PREFETCH) load_out(g, c);
    }
    __device__ __forceinline__ void load_out(const Grid& g, int c)
    {
        const long long cell = base + (long long)c * sd;
        if constexpr (!FIRST) {
#pragma unroll
            for (int v = 0; v < F::NV; ++v) rin[v] = o.racc[v * g.N + cell];
        }
        if constexpr (NEEDQN) {
#pragma unroll
            for (int v = 0; v < F::NV; ++v) qnin[v] = o.qn[v * g.N + cell];
        }
    }
    template <class Win>
    __device__ __forceinline__ void put(const Grid& g, int c, const T* fd, const T* src, const Win&, const double* qc)
    {
        if (valid) {
            if constexpr (!PREFETCH) load_out(g, c);
            T r[F::NV];
#pragma unroll
            for (int v = 0; v < F::NV; ++v) r[v] = FIRST ? fd[v] : rin[v] + fd[v];
#pragma unroll
            for (int a = 0; a < F::NA; ++a) r[F::IA + a] += src[a];
            if constexpr (CHK == CHK_CFL) acc.at(c);
            store_cell<T, MODE, F>(g, o, base + (long long)c * sd, r, KEEPQ ? qc : nullptr, CHK ? &acc : nullptr,
                                   NEEDQN ? qnin : nullptr);
        }
    }
};

// Views of a 5-cell window: w(k, v) = primitive v of cell c-2+k.
template <typename T, int NVV = NV>
struct ArrayWindow {
    static constexpr int nv = NVV;
    const T (*W)[NVV];
    __device__ __forceinline__ T operator()(int k, int v) const { return W[k][v]; }
};

// A lane's private ring of five cells in LDS (no other lane touches its
// column, so no barriers): element (slot, v) at col[(slot * NV + v) * LANES],
// consecutive lanes in consecutive words.  s0 is the slot of cell c-2.
// Keeping the window here instead of in registers leaves the registers to
// one variable's reconstruction at a time and needs no shifting.
template <typename T, int LANES, int NVV = NV>
struct LdsWindow {
    static constexpr bool in_registers = false;
    static constexpr int nv = NVV;
    T* col;
    int s0;
    __device__ __forceinline__ int slot(int k) const
    {
        const int s = s0 + k;
        return s >= 5 ? s - 5 : s;
    }
    __device__ __forceinline__ T operator()(int k, int v) const { return col[(slot(k) * NVV + v) * LANES]; }
    __device__ __forceinline__ void store(int k, const T* w) const
    {
#pragma unroll
        for (int v = 0; v < NVV; ++v) col[(slot(k) * NVV + v) * LANES] = w[v];
    }
    __device__ __forceinline__ void advance() { s0 = s0 == 4 ? 0 : s0 + 1; }
    // the new cell takes the slot of the oldest, which becomes the newest
    __device__ __forceinline__ void push(const T* w)
    {
        store(0, w);
        advance();
    }
};

// The ring with its newest cell in registers: four LDS slots hold cells
// c-2..c+1 (s0: the slot of c-2) and cell c+2 sits in registers, so a lane
// takes 4/5 of the LDS of LdsWindow for NVV more registers (for sweeps
// whose blocks per CU the LDS bounds).
template <typename T, int LANES, int NVV>
struct LdsRegWindow {
    static constexpr bool in_registers = false;
    static constexpr int nv = NVV;
    T* col;
    int s0;
    T r4[NVV];
    __device__ __forceinline__ int slot(int k) const
    {
        const int s = s0 + k;
        return s >= 4 ? s - 4 : s;
    }
    __device__ __forceinline__ T operator()(int k, int v) const
    {
        return k == 4 ? r4[v] : col[(slot(k) * NVV + v) * LANES];
    }
    __device__ __forceinline__ void store(int k, const T* w)
    {
        if (k == 4) {
#pragma unroll
            for (int v = 0; v < NVV; ++v) r4[v] = w[v];
        } else {
#pragma unroll
            for (int v = 0; v < NVV; ++v) col[(slot(k) * NVV + v) * LANES] = w[v];
        }
    }
    // cell c+2 takes the slot of c-2 (which leaves), the new cell c+3 the registers
    __device__ __forceinline__ void push(const T* w)
    {
#pragma unroll
        for (int v = 0; v < NVV; ++v) col[(s0 * NVV + v) * LANES] = r4[v];
        s0 = s0 == 3 ? 0 : s0 + 1;
#pragma unroll
        for (int v = 0; v < NVV; ++v) r4[v] = w[v];
    }
};

// The same ring in registers (rotated by moves), for kernels whose LDS
// holds other data.
template <typename T, int NVV = NV>
struct RegWindow {
    static constexpr bool in_registers = true;
    static constexpr int nv = NVV;
    T w[5][NVV];
    __device__ __forceinline__ T operator()(int k, int v) const { return w[k][v]; }
    __device__ __forceinline__ void store(int k, const T* x)
    {
#pragma unroll
        for (int v = 0; v < NVV; ++v) w[k][v] = x[v];
    }
    // shift out the oldest cell, the new one becomes the newest
    __device__ __forceinline__ void push(const T* x)
    {
#pragma unroll
        for (int v = 0; v < NVV; ++v) {
            w[0][v] = w[1][v];
            w[1][v] = w[2][v];
            w[2][v] = w[3][v];
            w[3][v] = w[4][v];
            w[4][v] = x[v];
        }
    }
};

// Marks a variable's edge values as final where they are computed.  Without
// it the compiler sinks each variable's last multiplications (and keeps
// their operands live) down to the first use of the values, past the
// other variables' reconstructions, which nearly doubles the registers of
// the sweep kernels.  The empty asm statement emits no instruction.
template <typename T>
__device__ __forceinline__ void settle(T& a, T& b)
{
    asm volatile("" : "+v"(a), "+v"(b));
}

// Reconstruction schemes of the non-learned passes (a compile-time
// parameter of every sweep kernel).
enum : int {
    SCHEME_WENO3 = 3,   // WENO3, Jiang-Shu weights, on the middle three cells
    SCHEME_WENO5 = 5,   // WENO5, Jiang-Shu weights
    SCHEME_WENO5Z = 6,  // WENO5, WENO-Z weights (comparison form)
    SCHEME_WENO5NU = 7, // WENO5, Jiang-Shu weights, on unequal cells (not the fused x-y pass)
};

// Reconstruction of one cell's two edge states (all seven primitives) from
// its 5-cell window in the given scheme.
template <typename T, int SCHEME = SCHEME_WENO5>
__device__ __forceinline__ void recon_scheme(T a, T b, T c, T d, T e, T eps, T& left, T& right)
{
    static_assert(SCHEME == SCHEME_WENO5 || SCHEME == SCHEME_WENO3 || SCHEME == SCHEME_WENO5Z, "scheme");
    if constexpr (SCHEME == SCHEME_WENO5)
        weno5<T>(a, b, c, d, e, eps, left, right);
    else if constexpr (SCHEME == SCHEME_WENO3)
        weno3<T>(b, c, d, eps, left, right);
    else
        weno5z<T>(a, b, c, d, e, eps, left, right);
}

template <typename T, int SCHEME = 5>
struct ReconJS {
    template <class Win>
    __device__ __forceinline__ void cell_win(const Win& W, T eps, T* lft, T* rgt)
    {
#pragma unroll
        for (int v = 0; v < Win::nv; ++v) {
            recon_scheme<T, SCHEME>(W(0, v), W(1, v), W(2, v), W(3, v), W(4, v), eps, lft[v], rgt[v]);
            settle(lft[v], rgt[v]);
        }
    }
    __device__ __forceinline__ void cell(const T W[5][NV], T eps, T lft[NV], T rgt[NV])
    {
        cell_win(ArrayWindow<T>{W}, eps, lft, rgt);
    }
    __device__ __forceinline__ void count_edges(bool, bool) {}
    __device__ __forceinline__ void flush(unsigned long long*) {}
    // equal cells: no per-position data, one reciprocal width for the direction
    template <int DIR>
    __device__ __forceinline__ void bind(const Grid&) {}
    __device__ __forceinline__ void at(int) {}
    __device__ __forceinline__ T inv_width(int, T idx) const { return idx; }
};

// Unequal cells along the sweep: at(c) loads the coefficients of stencil
// position c from the direction's table (the same position on every lane of
// a marching sweep, so the loads are uniform; in the x row kernel each lane
// loads its own position once per block), the flux difference of cell c
// divides by its own width.
template <typename T>
struct ReconJS<T, SCHEME_WENO5NU> {
    const double* tab;
    NuCoef<T> K;
    template <int DIR>
    __device__ __forceinline__ void bind(const Grid& g)
    {
        tab = g.nu[DIR];
    }
    __device__ __forceinline__ void at(int c)
    {
        const double* t = tab + (long long)(c + 1) * NU_K;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                K.a[k][i] = (T)t[NU_A + 3 * k + i];
                K.b[k][i] = (T)t[NU_B + 3 * k + i];
                K.c[k][i] = (T)t[NU_C + 3 * k + i];
            }
            K.dr[k] = (T)t[NU_DR + k];
            K.dl[k] = (T)t[NU_DL + k];
        }
    }
    __device__ __forceinline__ T inv_width(int c, T) const { return (T)tab[(long long)(c + 1) * NU_K + NU_IH]; }
    template <class Win>
    __device__ __forceinline__ void cell_win(const Win& W, T eps, T* lft, T* rgt)
    {
#pragma unroll
        for (int v = 0; v < Win::nv; ++v) {
            const T st[5] = {W(0, v), W(1, v), W(2, v), W(3, v), W(4, v)};
            weno5_nu<T>(K, st, eps, lft[v], rgt[v]);
            settle(lft[v], rgt[v]);
        }
    }
    __device__ __forceinline__ void count_edges(bool, bool) {}
    __device__ __forceinline__ void flush(unsigned long long*) {}
};

// Learned weights (float32 form); the whole wave must call cell() together.
// An edge state whose weights are not finite or that is not admissible is
// replaced by the Jiang-Shu edge state of all seven variables.
// Fallbacks are counted for the edges the caller names with count_edges()
// before each cell: those a face of the launch uses, each distinct face
// once (a face two segments both solve is counted by one of them).
// PIPE: evaluate the network's two tiles in step (see mlp_logits).
template <bool PIPE = true>
struct ReconLearned {
    const MlpNet& m;  // the packed network (the block's LDS copy, or global memory)
    Mix<float> mix;
    bool valid;  // this lane owns a real cell (only those are counted)
    unsigned fallbacks;
    bool edge;  // one evaluation per edge for all variables
    bool cnt_r = true, cnt_l = true;  // count the right / left edge of the next cell
    __device__ __forceinline__ void count_edges(bool r, bool l)
    {
        cnt_r = r;
        cnt_l = l;
    }
    template <class Win>
    __device__ __forceinline__ void cell_win(const Win& W, float eps, float lft[NV], float rgt[NV])
    {
        if (edge)
            cell_edge(W, eps, lft, rgt);
        else
            cell_var(W, eps, lft, rgt);
    }

    // Shared form: one pair of network evaluations (right edge, mirrored
    // left edge) per cell on the componentwise maximum of the seven
    // variables' features; the logits correct each variable's own
    // Jiang-Shu weights.
    template <class Win>
    __device__ __forceinline__ void cell_edge(const Win& W, float eps, float lft[NV], float rgt[NV])
    {
        float f[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
        bool flat = true;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const float a = W(0, v), b = W(1, v), c = W(2, v), d = W(3, v), e = W(4, v);
            flat = flat && a == b && b == c && c == d && d == e;
            float x[5];
            edge_features(a, b, c, d, e, eps, x);
#pragma unroll
            for (int k = 0; k < 5; ++k) f[k] = fmaxf(f[k], x[k]);
        }
        if (__all(flat)) {
            // constant stencils reconstruct to their value under any convex weights
#pragma unroll
            for (int v = 0; v < NV; ++v) lft[v] = rgt[v] = W(2, v);
            return;
        }
        const float fm[5] = {f[2], f[1], f[0], f[3], f[4]};
        float zr[3], zl[3], er[3], el[3];
        mlp_logits<PIPE>(m, f, zr);
        mlp_logits<PIPE>(m, fm, zl);
        exp_logits(zr, er);
        exp_logits(zl, el);
        // the stencils are read again from the window (LDS) below rather than
        // held in registers across the network evaluations
        asm volatile("" ::: "memory");
        bool finR = isfinite(er[0] + er[1] + er[2]), finL = isfinite(el[0] + el[1] + el[2]);
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const float a = W(0, v), b = W(1, v), c = W(2, v), d = W(3, v), e = W(4, v);
            float om[3], oml[3];
            bool fr, fl;
            shared_weights(a, b, c, d, e, eps, er, el, om, oml, fr, fl);
            weno5_apply(om, oml, a, b, c, d, e, lft[v], rgt[v]);
            finR = finR && fr;
            finL = finL && fl;
        }
        finish(W, eps, finR, finL, lft, rgt);
    }

    // Fallback per edge and counting (both forms): lft/rgt hold the learned
    // edge states; an edge whose weights are not finite or whose state is
    // not admissible takes the Jiang-Shu values of all its variables (the
    // Jiang-Shu reconstruction runs only when some lane of the wave needs
    // it).
    template <class Win>
    __device__ __forceinline__ void finish(const Win& W, float eps, bool finR, bool finL, float lft[NV], float rgt[NV])
    {
        const bool okR = finR && admissible(mix, rgt);
        const bool okL = finL && admissible(mix, lft);
        if (__any(!(okR && okL))) {
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                float jl, jr;
                weno5<float>(W(0, v), W(1, v), W(2, v), W(3, v), W(4, v), eps, jl, jr);
                rgt[v] = okR ? rgt[v] : jr;
                lft[v] = okL ? lft[v] : jl;
                __builtin_amdgcn_sched_barrier(0);  // one variable at a time (registers)
            }
        }
        if (valid) fallbacks += (okR || !cnt_r ? 0u : 1u) + (okL || !cnt_l ? 0u : 1u);
    }

    template <class Win>
    __device__ __forceinline__ void cell_var(const Win& W, float eps, float lft[NV], float rgt[NV])
    {
        bool finR = true, finL = true;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const float a = W(0, v), b = W(1, v), c = W(2, v), d = W(3, v), e = W(4, v);
            // A constant stencil reconstructs to its value under any convex
            // weights: where the whole wave has one, the network is skipped.
            const bool flat = a == b && b == c && c == d && d == e;
            if (__all(flat)) {
                lft[v] = rgt[v] = c;
            } else {
                bool fr, fl;
                weno5_learned<PIPE>(m, a, b, c, d, e, eps, lft[v], rgt[v], fr, fl);
                finR = finR && fr;
                finL = finL && fl;
            }
        }
        finish(W, eps, finR, finL, lft, rgt);
    }
    __device__ __forceinline__ void cell(const float W[5][NV], float eps, float lft[NV], float rgt[NV])
    {
        cell_win(ArrayWindow<float>{W}, eps, lft, rgt);
    }
    template <int DIR>
    __device__ __forceinline__ void bind(const Grid&) {}
    __device__ __forceinline__ void at(int) {}
    __device__ __forceinline__ float inv_width(int, float idx) const { return idx; }
    // wave sum of the fallback counts, one atomic per wave
    __device__ __forceinline__ void flush(unsigned long long* counter)
    {
        unsigned long long c = fallbacks;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
        if ((threadIdx.x & 63) == 0 && c) atomicAdd(counter, c);
    }
};

template <typename T, bool LEARNED, int SCHEME = 5, bool PIPE = true>
struct ReconOf {
    using type = ReconJS<T, SCHEME>;
};
template <bool PIPE>
struct ReconOf<float, true, 5, PIPE> {
    using type = ReconLearned<PIPE>;
};

// SHARED: the block (every thread calls this) copies the packed network to
// LDS and the evaluations read it there; otherwise they read it from global
// memory (one-wave blocks, for which a 12 KB LDS copy per wave would cost
// occupancy).  Either way it holds no registers across the march.
template <typename T, bool LEARNED, int SCHEME = 5, bool SHARED = true, bool PIPE = true>
__device__ __forceinline__ typename ReconOf<T, LEARNED, SCHEME, PIPE>::type make_recon(const Grid& g,
                                                                                     const MlpNet* mlp, bool valid)
{
    if constexpr (LEARNED && !SHARED) {
        return ReconLearned<PIPE>{*mlp, Mix<float>{(float)g.G1, (float)g.G2, (float)g.P1, (float)g.P2}, valid, 0u,
                                  g.edge_weights != 0};
    } else if constexpr (LEARNED) {
        __shared__ MlpNet snet;
        const u32x4* src = &mlp->w[0][0];
        u32x4* dst = &snet.w[0][0];
        for (int i = threadIdx.x; i < MLP_WORDS * 64; i += blockDim.x) dst[i] = src[i];
        __syncthreads();
        return ReconLearned<PIPE>{snet, Mix<float>{(float)g.G1, (float)g.G2, (float)g.P1, (float)g.P2}, valid, 0u,
                                  g.edge_weights != 0};
    } else {
        (void)g;
        (void)mlp;
        (void)valid;
        return ReconJS<T, SCHEME>{};
    }
}

// The marching loop over the segment [c0, c1).  Src::load(pos, q) returns
// the conserved state of cell `pos` along the sweep (boundary map applied);
// it is called for positions c0-3, c0-2, ..., c1+2 in that order, and
// Sink::put for cells c0..c1-1 in order, the same sequence on every lane.
// W: the 5-cell window (LdsWindow or RegWindow), handed to Sink::put too,
// where W(1, .) holds the primitives of the cell being put.
template <int DIR, typename T, class F, class Src, class Sink, class Recon, class Win>
__device__ __forceinline__ void march(const Grid& g, Src& src, Sink& sink, Recon& recon, int c0, int c1, Win& W)
{
    constexpr int V = F::NV;
    const T idx = (T)g.inv_dx[DIR];
    const T eps = (T)g.eps;
    const MixOf<F> mixd = make_mix<double, F>(g);
    const auto mix = make_mix<T, F>(g);
    recon.template bind<DIR>(g);

    // window: W(k) = primitives of cell c-2+k while reconstructing cell c
    // qh (when the sink keeps the stage state): conserved cells c-1 .. c+2.
    // Register-held windows and qh need constant indices (unrolled fill);
    // an LDS ring without qh is filled by a rolled loop (smaller code).
    constexpr bool KQ = Sink::keeps_q;
    double qh[KQ ? 4 : 1][V];
    auto fill = [&](int k) {
        double qc[V];
        src.load(c0 - 3 + k, qc);
        if constexpr (KQ) {
            if (k >= 1) {
#pragma unroll
                for (int v = 0; v < V; ++v) qh[k - 1][v] = qc[v];
            }
        }
        T w[V];
        prim_of<T, F>(mixd, qc, w);
        src.finish(c0 - 3 + k, w);
        W.store(k, w);
    };
    if constexpr (KQ || Win::in_registers) {
#pragma unroll
        for (int k = 0; k < 5; ++k) fill(k);
    } else {
#pragma unroll 1
        for (int k = 0; k < 5; ++k) fill(k);
    }

    T rprev[V], Fprev[V], ufprev = T(0);
#pragma unroll
    for (int v = 0; v < V; ++v) rprev[v] = Fprev[v] = T(0);

    // faces this segment counts (learned fallbacks): c0+1/2 .. c1-1/2, and
    // c0-1/2 in the first segment unless it is the periodic image of the
    // last segment's c1-1/2
    const bool own_first = c0 == 0 && g.bc[DIR][0] != BC_PERIODIC;
    for (int c = c0 - 1; c <= c1; ++c) {
        // next cell entering the window (c+3), and what the output of cell
        // c-1 needs, fetched early
        double qnext[V];
        if (c < c1) src.load(c + 3, qnext);
        if (c > c0) sink.prefetch(g, c - 1);

        T lft[V], rgt[V];
        recon.count_edges((c >= c0 && c < c1) || (c == c0 - 1 && own_first),
                          (c > c0 && c <= c1) || (c == c0 && own_first));
        recon.at(c);
        recon.cell_win(W, eps, lft, rgt);

        // The entering cell c+3 is converted before this step's stores are
        // issued where the sink allows: vector-memory loads and stores share
        // one completion counter, so a load used after a store would wait
        // for the store as well.  ENTER_BEFORE (the y and z sweeps with
        // Jiang-Shu weights): before the output, the stage state of the
        // output cell c-1 taken out of the history before the entering
        // cell's joins it.  ENTER_AFTER (the learned passes, the fused x-y
        // pass and the LDS outputs of the marching x sweep): after the
        // output, where converting costs no registers (converting earlier in
        // the fused x-y pass took it from 247 to 256 registers with spills).
        constexpr int AT = Sink::enter_at;
        static_assert(!KQ || AT == ENTER_BEFORE, "a sink that keeps the stage state converts first");
        T wn[AT == ENTER_BEFORE ? V : 1];
        double qout[KQ ? V : 1];
        if constexpr (AT == ENTER_BEFORE) {
            if constexpr (KQ) {
#pragma unroll
                for (int v = 0; v < V; ++v) qout[v] = qh[0][v];
            }
            if (c < c1) {
                prim_of<T, F>(mixd, qnext, wn);
                src.finish_ahead(c + 3, wn);  // c + 3 >= c0 + 2 >= 2
            }
            if constexpr (KQ) {
                if (c < c1) {
#pragma unroll
                    for (int v = 0; v < V; ++v) {
                        qh[0][v] = qh[1][v];
                        qh[1][v] = qh[2][v];
                        qh[2][v] = qh[3][v];
                        qh[3][v] = qnext[v];
                    }
                }
            }
        }

        if (c >= c0) {
            T Fl[V], uf;
            hllc_f<DIR, T, F>(mix, rprev, lft, Fl, uf);
            if (c > c0) {
                // cell c-1: faces c-3/2 (Fprev) and c-1/2 (Fl)
                const T ih = recon.inv_width(c - 1, idx);
                T fd[V];
#pragma unroll
                for (int v = 0; v < V; ++v) fd[v] = (Fprev[v] - Fl[v]) * ih;
                // every volume fraction's source alpha_a div(u)
                T src_a[F::NA];
#pragma unroll
                for (int a = 0; a < F::NA; ++a) src_a[a] = W(1, F::IA + a) * ((uf - ufprev) * ih);
                sink.put(g, c - 1, fd, src_a, W, qout);
            }
#pragma unroll
            for (int v = 0; v < V; ++v) Fprev[v] = Fl[v];
            ufprev = uf;
        }
#pragma unroll
        for (int v = 0; v < V; ++v) rprev[v] = rgt[v];

        // cell c+3 enters, cell c-2 (no longer needed) leaves
        if constexpr (AT == ENTER_AFTER) {
            if (c < c1) {
                T w[V];
                prim_of<T, F>(mixd, qnext, w);
                src.finish_ahead(c + 3, w);  // c + 3 >= c0 + 2 >= 2
                W.push(w);
            }
        } else if (c < c1) {
            W.push(wn);
        }
    }
}

// Cell source for the y and z sweeps (DIR 1 or 2): straight from global
// memory; the lanes of a wave are consecutive x, so each load is a
// contiguous row.
template <int DIR, class F = Fl2>
struct GlobalSrc {
    const double* __restrict__ qs;
    const double* inf;  // device copy of this direction's inflow states [2][NVMAX] (required)
    long long base, sd, N;
    int n, bclo, bchi;
    // inflow ghosts: positions below ilo or at/above ihi; reflective ghosts:
    // below flo or at/above fhi
    int ilo = bclo == BC_INFLOW ? 0 : INT_MIN;
    int ihi = bchi == BC_INFLOW ? n : INT_MAX;
    int flo = bclo == BC_REFLECTIVE ? 0 : INT_MIN;
    int fhi = bchi == BC_REFLECTIVE ? n : INT_MAX;
    // An inflow ghost reads the side's state instead of a cell: only the
    // (wave-uniform) base pointer and stride of the same loads change.
    __device__ __forceinline__ void load(int pos, double* q) const
    {
        const bool lo = pos < ilo, hi = pos >= ihi;
        const double* p = lo ? inf : (hi ? inf + NVMAX : qs + base + (long long)map_cell(pos, n, bclo, bchi) * sd);
        const long long st = (lo || hi) ? 1 : N;
#pragma unroll
        for (int v = 0; v < F::NV; ++v) q[v] = p[v * st];
    }
    // A reflective ghost enters with its normal velocity negated; applied to
    // the primitives where the march uses them (the same bits as negating
    // the momentum before the conversion), so the load stays in flight.
    template <typename T>
    __device__ __forceinline__ void finish(int pos, T* w) const
    {
        if (pos < flo || pos >= fhi) w[F::IM + DIR] = -w[F::IM + DIR];
    }
    // the same for a position known to be >= 0 (cells entering the window
    // ahead of the march)
    template <typename T>
    __device__ __forceinline__ void finish_ahead(int pos, T* w) const
    {
        if (pos >= fhi) w[F::IM + DIR] = -w[F::IM + DIR];
    }
};

// Launch geometry of the y and z sweeps: blockIdx.x * BLOCK + threadIdx.x =
// x index, blockIdx.y = the other transverse index (z for the y sweep, y for
// the z sweep), blockIdx.z = segment along the sweep.
// qn and out alias in the third stage (the new state overwrites q in place;
// each cell's q is read only by the thread that then writes it), so neither
// is declared __restrict__.
// CFL (stage 3 only): the block's CFL maximum of the new state goes to
// partial[block] and invalid states set bits in *status, as in the
// standalone reduction.  Stages 1 and 2 set the status bits of the states
// they write (state_bits) in *status.
// Block size: the Jiang-Shu passes run one wave per block (waves do not
// cooperate, so every lane is used for any nx that is a multiple of 64);
// the learned passes run four (measured faster for them).
template <bool LEARNED>
constexpr int yz_block()
{
    return LEARNED ? 256 : 64;
}

// (The learned passes keep the occupancy hint of two waves per SIMD: without
// it the compiler schedules them for a higher occupancy they cannot reach.)
template <int DIR, typename T, bool FIRST, int MODE, bool LEARNED, bool CFL = false, int SCHEME = 5, class F = Fl2>
__global__ void __launch_bounds__(yz_block<LEARNED>(), LEARNED ? 3 : 1) sweep_yz(Grid g, const double* __restrict__ qs, const double* qn,
                                                   T* __restrict__ racc, double* out, int seg,
                                                   const double* __restrict__ dt_dev, double dt_arg,
                                                   const MlpNet* __restrict__ mlp, unsigned long long* fb,
                                                   double* __restrict__ partial, unsigned* __restrict__ status)
{
    constexpr int BLOCK = yz_block<LEARNED>();
    static_assert(DIR == 1 || DIR == 2, "y or z sweep");
    constexpr int SA = (DIR == 2) ? 1 : 2;  // slow transverse axis
    const int n = g.n[DIR];
    const int nx = g.n[0];
    const int i_raw = blockIdx.x * BLOCK + threadIdx.x;
    const bool valid = i_raw < nx;
    const int i = valid ? i_raw : nx - 1;

    const long long base = (long long)i + (long long)blockIdx.y * g.stride[SA];
    const int c0 = blockIdx.z * seg;
    const int c1 = min(c0 + seg, n);
    GlobalSrc<DIR, F> src{qs, g.inflow_dev + DIR * 2 * NVMAX, base, g.stride[DIR], g.N, n, g.bc[DIR][0], g.bc[DIR][1]};
    constexpr int CHK = (MODE == OUT_STAGE1 || MODE == OUT_STAGE2) ? CHK_STATE : (CFL ? CHK_CFL : CHK_NONE);
    // The stage updates keep the stage state from the window loads, except
    // in float64 on unequal cells: there the marching position's 33
    // coefficients already take the registers the history would need, and
    // keeping it drops the sweep to one wave per SIMD (re-reading the state
    // is faster).
    constexpr bool KEEPQ =
        MODE >= OUT_STAGE1 && !LEARNED && (SCHEME != SCHEME_WENO5NU || sizeof(T) == sizeof(float));
    CflAcc<F> acc{0.0, 0u, CHK == CHK_CFL, {g.dx[0], g.dx[1], g.dx[2]}, nullptr, DIR};
    if constexpr (CHK == CHK_CFL) {
        if (g.nonuniform) {  // widths of the lane's x position and the block's transverse position
            if (g.nu[0]) acc.hw[0] = g.nu[0][(long long)(i + 1) * NU_K + NU_H];
            if (g.nu[SA]) acc.hw[SA] = g.nu[SA][(long long)(blockIdx.y + 1) * NU_K + NU_H];
            acc.nud = g.nu[DIR];
        }
    }
    GlobalSink<T, FIRST, MODE, KEEPQ, CHK, !LEARNED, F> sink{
        OutArgs<T>{qs, qn, racc, out, dt_dev ? *dt_dev : dt_arg}, base, g.stride[DIR], valid, acc};
    auto recon = make_recon<T, LEARNED, SCHEME>(g, mlp, valid);
    // Three fluids in the accumulating passes: the window's LDS (5 x 9
    // values per lane) rather than the registers bounds the blocks per CU,
    // so its newest cell moves to registers.
    constexpr bool REG_HEAD = F::NF == 3 && !LEARNED && (MODE == OUT_ACCUM || MODE == OUT_RHS);
    using Win = typename std::conditional<REG_HEAD, LdsRegWindow<T, BLOCK, F::NV>, LdsWindow<T, BLOCK, F::NV>>::type;
    __shared__ T win[REG_HEAD ? 4 : 5][F::NV][BLOCK];
    Win W{&win[0][0][threadIdx.x], 0};
    march<DIR, T, F>(g, src, sink, recon, c0, c1, W);
    recon.flush(fb);
    if constexpr (CHK != CHK_NONE) {
        if (sink.acc.bad) atomicOr(status, sink.acc.bad);
    }
    if constexpr (CHK == CHK_CFL) {
        const unsigned blk = (blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
        block_max_to<BLOCK>(sink.acc.smax, partial + blk);
    }
}

// Marching x sweep, for rows longer than the whole-row kernel takes.  The 64
// lanes of the (one-wave) block own 64 consecutive rows (row = k * ny + j,
// x-contiguous in memory) and march along x together.  Inputs: every XCHUNK
// positions the block stages the next XCHUNK cells of all 64 rows through
// LDS with row-contiguous reads, then each lane reads its own row.  Outputs:
// each lane parks its cell's contribution in LDS and every XCHUNK cells the
// block writes them out row-contiguously (including the partial-RHS read and
// the stage update), so no global access is strided across lanes.
constexpr int XROWS = 64;
constexpr int XCHUNK = 4;

template <class F = Fl2>
struct LdsSrc {
    double (*buf)[F::NV][XROWS];  // [XCHUNK][F::NV][XROWS]
    const double* __restrict__ qs;
    const double* inf;  // device copy of the x inflow states [2][NVMAX] (required)
    long long N;
    long long row0;  // first row of the block
    long long nrows;
    int nx, bclo, bchi;
    int pstart;  // first position fetched (c0 - 3)

    __device__ __forceinline__ void load(int pos, double* q) const
    {
        const int slot = (pos - pstart) % XCHUNK;
        if (slot == 0) {
            __syncthreads();  // every lane has consumed the previous chunk
#pragma unroll 1
            for (int it = 0; it < XCHUNK; ++it) {
                const int item = threadIdx.x + it * XROWS;
                const int r = item / XCHUNK, cx = item % XCHUNK;
                const long long row = min(row0 + r, nrows - 1);
                // inflow ghosts read the side's state (base pointer and stride)
                const int pp = pos + cx;
                const bool lo = pp < ilo, hi = pp >= ihi;
                const double* p = lo ? inf : (hi ? inf + NVMAX : qs + row * nx + map_cell(pp, nx, bclo, bchi));
                const long long st = (lo || hi) ? 1 : N;
#pragma unroll
                for (int v = 0; v < F::NV; ++v) buf[cx][v][r] = p[v * st];
            }
            __syncthreads();
        }
#pragma unroll
        for (int v = 0; v < F::NV; ++v) q[v] = buf[slot][v][threadIdx.x];
    }
    int ilo = bclo == BC_INFLOW ? 0 : INT_MIN;
    int ihi = bchi == BC_INFLOW ? nx : INT_MAX;
    // every lane marches at the same x position: reflective ghosts are
    // fixed on the primitives as in GlobalSrc
    int flo = bclo == BC_REFLECTIVE ? 0 : INT_MIN;
    int fhi = bchi == BC_REFLECTIVE ? nx : INT_MAX;
    template <typename T>
    __device__ __forceinline__ void finish(int pos, T* w) const
    {
        if (pos < flo || pos >= fhi) w[F::IM] = -w[F::IM];
    }
    template <typename T>
    __device__ __forceinline__ void finish_ahead(int pos, T* w) const
    {
        if (pos >= fhi) w[F::IM] = -w[F::IM];
    }
};

template <typename T, bool FIRST, int MODE, class F = Fl2>
struct LdsSink {
    T (*buf)[F::NV + F::NA][XROWS];  // [XCHUNK][flux differences, volume-fraction sources][XROWS]
    OutArgs<T> o;
    long long row0, nrows;
    int nx, c0, c1;

    static constexpr bool keeps_q = false;
    static constexpr int enter_at = ENTER_AFTER;
    __device__ __forceinline__ void prefetch(const Grid&, int) {}
    template <class Win>
    __device__ __forceinline__ void put(const Grid& g, int c, const T* fd, const T* src, const Win&, const double*)
    {
        const int slot = (c - c0) % XCHUNK;
#pragma unroll
        for (int v = 0; v < F::NV; ++v) buf[slot][v][threadIdx.x] = fd[v];
#pragma unroll
        for (int a = 0; a < F::NA; ++a) buf[slot][F::NV + a][threadIdx.x] = src[a];
        if (slot == XCHUNK - 1 || c == c1 - 1) {
            const int p0 = c - slot, cnt = slot + 1;
            __syncthreads();
#pragma unroll 1
            for (int it = 0; it < XCHUNK; ++it) {
                const int item = threadIdx.x + it * XROWS;
                const int r = item / XCHUNK, cx = item % XCHUNK;
                if (cx < cnt && row0 + r < nrows) {
                    T f[F::NV], sa[F::NA];
#pragma unroll
                    for (int v = 0; v < F::NV; ++v) f[v] = buf[cx][v][r];
#pragma unroll
                    for (int a = 0; a < F::NA; ++a) sa[a] = buf[cx][F::NV + a][r];
                    const long long cell = (row0 + r) * nx + p0 + cx;
                    emit_cell<T, FIRST, MODE, F>(g, o, cell, f, sa);
                }
            }
            __syncthreads();  // the buffer is refilled next
        }
    }
};

// (No occupancy target: a one-wave block stages XCHUNK rows of input and
// output and the 5-cell window in LDS, about 48 KB in float64, so LDS
// rather than registers bounds the blocks per CU.  This pass serves rows
// longer than the row kernels take and x inflow sides with aliased row
// buffers.)
template <typename T, bool FIRST, int MODE, bool LEARNED, int SCHEME = 5, class F = Fl2>
__global__ void __launch_bounds__(XROWS) sweep_x_march(Grid g, const double* __restrict__ qs, const double* qn,
                                                          T* __restrict__ racc, double* out, int seg,
                                                          const double* __restrict__ dt_dev, double dt_arg,
                                                          const MlpNet* __restrict__ mlp, unsigned long long* fb)
{
    __shared__ double ibuf[XCHUNK][F::NV][XROWS];
    __shared__ T obuf[XCHUNK][F::NV + F::NA][XROWS];
    const int nx = g.n[0];
    const long long nrows = (long long)g.n[1] * g.n[2];
    const long long row0 = (long long)blockIdx.x * XROWS;
    const int c0 = blockIdx.z * seg;
    const int c1 = min(c0 + seg, nx);

    LdsSrc<F> src{ibuf, qs, g.inflow_dev, g.N, row0, nrows, nx, g.bc[0][0], g.bc[0][1], c0 - 3};
    LdsSink<T, FIRST, MODE, F> sink{obuf, OutArgs<T>{qs, qn, racc, out, dt_dev ? *dt_dev : dt_arg}, row0, nrows, nx,
                                    c0, c1};
    auto recon = make_recon<T, LEARNED, SCHEME, false>(g, mlp, row0 + threadIdx.x < nrows);
    __shared__ T win[5][F::NV][XROWS];
    LdsWindow<T, XROWS, F::NV> W{&win[0][0][threadIdx.x], 0};
    march<0, T, F>(g, src, sink, recon, c0, c1, W);
    recon.flush(fb);
}

}  // namespace mfx
