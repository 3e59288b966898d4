// mfx C ABI: context, workspace layout, launch sequencing of the per-direction
// sweeps for the right-hand side and the SSP-RK3 step, and the small kernels
// around them (primitive -> conserved, CFL reduction, state validation).
//
// Paper: arXiv 2409.10729, Sec. II-B (eq. discretization / eq. rhs).  The
// interface is declared in include/mfx.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/mfx.h"
#include "launch.h"
#include "sweep.h"
#include "xrow.h"

namespace mfx {
int mlp_pack_on_stream(const float* params, void* packed, hipStream_t st);
}

using namespace mfx;

namespace {

constexpr int UTIL_BLOCK = 256;
constexpr int CFL_BLOCKS = 1024;  // grid of the standalone CFL reduction
constexpr size_t ALIGN = 256;

thread_local std::string g_init_error;

size_t align_up(size_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }

// Fluids and variables of a descriptor (num_fluids 0 reads as 2).
int fluids_of(const mfx_grid_desc* d) { return d->num_fluids == 0 ? 2 : d->num_fluids; }
int vars_of(const mfx_grid_desc* d) { return 2 * fluids_of(d) + 3; }

// Launch-shape overrides for tuning and tests (results do not depend on
// them): MFX_SWEEP_SEG = segment length of the marching sweeps,
// MFX_XSWEEP = "march" to force the marching x sweep.
struct Overrides {
    int seg;
    int xmode;
    int fuse_xy;
    int fuse_cfl;
};

Overrides read_overrides()
{
    Overrides o{0, 0, 1, 1};
    if (const char* s = std::getenv("MFX_SWEEP_SEG")) o.seg = std::atoi(s);
    if (const char* s = std::getenv("MFX_XSWEEP")) o.xmode = std::strcmp(s, "march") == 0 ? 1 : 0;
    if (const char* s = std::getenv("MFX_FUSE_XY")) o.fuse_xy = std::atoi(s) != 0;
    if (const char* s = std::getenv("MFX_FUSE_CFL")) o.fuse_cfl = std::atoi(s) != 0;
    return o;
}

struct Layout {
    size_t q, q1, q2, r, scal, inflow, partial, bface, mlp, mlp_params, nu[3], total;
    long long n_partial;
};

// The x sweep takes whole rows when a row fits the row kernel (nx <=
// XROW_MAX and its LDS, for nv variables, fits a workgroup), else it
// marches along x.  (x_mode() below sends an inflow x side with aliased
// row buffers to the march: the row kernels write inflow ghost slots once
// per block.)
bool use_xrows(const int n[3], int mode_override, size_t elem, int nv)
{
    if (mode_override == 1) return false;
    return n[0] <= XROW_MAX && xrow_lds_bytes(n[0], elem, nv) <= 64 * 1024;
}

// x sweep mode for a descriptor: the override, or the march (1) when an x
// side is inflow and the row buffers would be aliased.
int x_mode(const mfx_grid_desc* d, int xmode_override)
{
    const size_t elem = d->precision == MFX_FP32_MIXED ? sizeof(float) : sizeof(double);
    const bool inflow_x = d->bc[0][0] == MFX_BC_INFLOW || d->bc[0][1] == MFX_BC_INFLOW;
    if (inflow_x && d->n[0] <= XROW_MAX && xrow_layout(d->n[0], elem, vars_of(d)).alias) return 1;
    return xmode_override;
}

SweepGeom sweep_geom(const int n[3], int d, int seg_override, int xmode_override, size_t elem, bool learned, int nv)
{
    int seg = seg_override > 0 ? seg_override : 64;
    SweepGeom g;
    g.lds = 0;
    g.xrows = false;
    if (d == 0 && use_xrows(n, xmode_override, elem, nv)) {
        const long long rows = (long long)n[1] * n[2];
        // about 2048 blocks, at least one row each
        const long long rpb = std::max<long long>(1, rows / 2048);
        g.grid = dim3((unsigned)((rows + rpb - 1) / rpb), 1, 1);
        g.block = 64 * ((n[0] + 63) / 64);
        g.seg = (int)rpb;
        g.lds = xrow_lds_bytes(n[0], elem, nv);
        g.xrows = true;
    } else if (d == 0) {
        // blocks of XROWS rows (y,z flattened), segments along x
        const long long rows = (long long)n[1] * n[2];
        while (seg > 16 && rows * ((n[0] + seg - 1) / seg) < 256LL * 64 * 16) seg /= 2;
        seg = std::min(seg, n[0]);
        g.grid = dim3((unsigned)((rows + XROWS - 1) / XROWS), 1, (n[0] + seg - 1) / seg);
        g.block = XROWS;
        g.seg = seg;
    } else {
        const int sa = (d == 2) ? 1 : 2;
        const long long pencils = (long long)n[0] * n[sa];
        // keep enough waves in flight: shrink segments while the pencil count is small
        while (seg > 16 && pencils * ((n[d] + seg - 1) / seg) < 256LL * 64 * 16) seg /= 2;
        seg = std::min(seg, n[d]);
        const int block = learned ? yz_block<true>() : yz_block<false>();
        g.grid = dim3((n[0] + block - 1) / block, n[sa], (n[d] + seg - 1) / seg);
        g.block = block;
        g.seg = seg;
    }
    return g;
}

Layout make_layout(const mfx_grid_desc* d, int seg_override, int xmode_override)
{
    Layout L{};
    const long long N = (long long)d->n[0] * d->n[1] * d->n[2];
    const size_t nv = (size_t)vars_of(d);
    const size_t state = align_up(sizeof(double) * nv * (size_t)N);
    const size_t elem = d->precision == MFX_FP32_MIXED ? sizeof(float) : sizeof(double);
    // per-block maxima of the CFL reduction: the standalone pass, or the
    // blocks of a y/z sweep that reduces the new state of a step
    long long np = CFL_BLOCKS;
    for (int dd = 1; dd < 3; ++dd) {
        const SweepGeom sg = sweep_geom(d->n, dd, seg_override, xmode_override, elem, false, (int)nv);
        np = std::max<long long>(np, (long long)sg.grid.x * sg.grid.y * sg.grid.z);
    }
    const long long nrows = (long long)d->n[1] * d->n[2];
    size_t off = 0;
    L.q = off;
    off += state;
    L.q1 = off;
    off += state;
    L.q2 = off;
    off += state;
    L.r = off;
    off += align_up(elem * nv * (size_t)N);
    L.scal = off;
    off += align_up(64);
    L.inflow = off;  // the inflow ghost states [3][2][NVMAX], read by the loaders
    off += align_up(sizeof(double) * 3 * 2 * NVMAX);
    L.partial = off;
    off += align_up(sizeof(double) * (size_t)np);
    L.bface = off;
    off += align_up(elem * (nv + 1) * 2 * (size_t)nrows);  // flux components and face velocity per face
    L.mlp = off;
    off += align_up(sizeof(MlpNet));
    L.mlp_params = off;
    off += align_up(sizeof(float) * MLP_PARAMS);
    for (int k = 0; k < 3; ++k) {  // per-position tables of directions with unequal cells
        L.nu[k] = off;
        if (d->faces[k]) off += align_up(sizeof(double) * NU_K * ((size_t)d->n[k] + 2));
    }
    L.total = off;
    L.n_partial = np;
    return L;
}

bool learned_weights(const mfx_grid_desc& d)
{
    return d.weights == MFX_WENO5_LEARNED || d.weights == MFX_WENO5_LEARNED_EDGE;
}

// Reconstruction scheme of the non-learned passes.
int scheme_of(const mfx_grid_desc& d)
{
    if (d.weights == MFX_WENO5_Z) return SCHEME_WENO5Z;
    return d.weno_order == 3 ? SCHEME_WENO3 : SCHEME_WENO5;
}

// Calls f with std::integral_constant<int, scheme> (one instantiation per
// scheme; NU: whether the unequal-cell scheme is one of them).
template <bool NU = true, class F>
void by_scheme(int scheme, F&& f)
{
    switch (scheme) {
    case SCHEME_WENO3: f(std::integral_constant<int, SCHEME_WENO3>{}); break;
    case SCHEME_WENO5Z: f(std::integral_constant<int, SCHEME_WENO5Z>{}); break;
    case SCHEME_WENO5NU:
        if constexpr (NU) {
            f(std::integral_constant<int, SCHEME_WENO5NU>{});
            break;
        }
        [[fallthrough]];
    default: f(std::integral_constant<int, SCHEME_WENO5>{}); break;
    }
}

// ---------------------------------------------------------------- unequal cells
//
// WENO5 coefficients on cells of unequal widths by the primitive-function
// route (Shu's construction of reconstructions on non-uniform meshes): on the
// boundaries z_0 < ... < z_m of m consecutive cells, in the coordinate xi of
// the middle cell of the five (which spans [-1/2, 1/2]), the primitive
// V(z_j) = sum_{i<j} v_i (z_{i+1} - z_i) is interpolated by the Lagrange
// polynomial P of degree m, and P' is the polynomial of degree m - 1 whose
// cell averages are the v_i.  So the coefficient of v_i in any linear
// functional of P' is (z_{i+1} - z_i) times the sum over the nodes j > i of
// that functional applied to the derivative of node j's basis polynomial.

// Derivative of the Lagrange basis polynomial of node j (nodes z[0..m]) at node z[s].
double basis_slope_at_node(const double* z, int m, int j, int s)
{
    if (j == s) {
        double acc = 0.0;
        for (int q = 0; q <= m; ++q)
            if (q != s) acc += 1.0 / (z[s] - z[q]);
        return acc;
    }
    double num = 1.0, den = 1.0;
    for (int q = 0; q <= m; ++q) {
        if (q == j) continue;
        den *= z[j] - z[q];
        if (q != s) num *= z[s] - z[q];
    }
    return num / den;
}

static_assert(NU_DL + 3 == MFX_NU_COEFS, "table layout starts with the exported coefficients");

// The MFX_NU_COEFS values of mfx_weno5_nu_coefficients for widths h[0..4].
void nu_coefficients(const double h[5], double* out)
{
    double z[6];
    z[2] = -0.5;
    z[3] = 0.5;
    z[1] = z[2] - h[1] / h[2];
    z[0] = z[1] - h[0] / h[2];
    z[4] = z[3] + h[3] / h[2];
    z[5] = z[4] + h[4] / h[2];
    double w[5];
    for (int i = 0; i < 5; ++i) w[i] = z[i + 1] - z[i];
    // candidate k, nodes z[k .. k+3]: A = P'(0), B = P''(0), C = P'''(0) / 2.
    // With node j's basis numerator prod_{q != j} (xi - z_q) = xi^3 - e1 xi^2
    // + e2 xi - e3 and denominator D = prod_{q != j} (z_j - z_q), its first,
    // second and third derivatives at 0 are e2 / D, -2 e1 / D and 6 / D.
    for (int k = 0; k < 3; ++k) {
        const double* zz = z + k;
        double fa[4] = {0.0, 0.0, 0.0, 0.0}, fb[4] = {0.0, 0.0, 0.0, 0.0}, fc[4] = {0.0, 0.0, 0.0, 0.0};
        for (int j = 1; j < 4; ++j) {
            double o[3], D = 1.0;
            int no = 0;
            for (int q = 0; q < 4; ++q) {
                if (q == j) continue;
                D *= zz[j] - zz[q];
                o[no++] = zz[q];
            }
            const double e1 = o[0] + o[1] + o[2];
            const double e2 = o[0] * o[1] + o[0] * o[2] + o[1] * o[2];
            fa[j] = e2 / D;
            fb[j] = -2.0 * e1 / D;
            fc[j] = 3.0 / D;
        }
        for (int i = 0; i < 3; ++i) {
            double sa = 0.0, sb = 0.0, sc = 0.0;
            for (int j = i + 1; j < 4; ++j) {
                sa += fa[j];
                sb += fb[j];
                sc += fc[j];
            }
            out[NU_A + 3 * k + i] = w[k + i] * sa;
            out[NU_B + 3 * k + i] = w[k + i] * sb;
            out[NU_C + 3 * k + i] = w[k + i] * sc;
        }
    }
    // Ideal weights of an edge (node s of the five cells' boundaries: 3 for
    // xi = 1/2, 2 for xi = -1/2): the five-cell value there is matched by
    // the three candidates' values; only candidate 0 holds cell c-2 and only
    // candidate 2 holds cell c+2, which fixes d_0 and d_2, and the weights
    // sum to one (every row reproduces constants).
    for (int e = 0; e < 2; ++e) {
        const int s = e == 0 ? 3 : 2;
        double g0 = 0.0;
        for (int j = 1; j <= 5; ++j) g0 += basis_slope_at_node(z, 5, j, s);
        g0 *= w[0];
        const double g4 = w[4] * basis_slope_at_node(z, 5, 5, s);
        double r0 = 0.0;
        for (int j = 1; j <= 3; ++j) r0 += basis_slope_at_node(z, 3, j, s);
        r0 *= w[0];
        const double r2 = w[4] * basis_slope_at_node(z + 2, 3, 3, s - 2);
        double* d = out + (e == 0 ? NU_DR : NU_DL);
        d[0] = g0 / r0;
        d[2] = g4 / r2;
        d[1] = 1.0 - d[0] - d[2];
    }
}

// Table of direction dir (NU_K values per stencil position -1 .. n): the
// widths of the five cells each position's stencil reaches, a ghost cell
// taking the width of the cell the boundary rule maps it to.
std::vector<double> nu_table(const mfx_grid_desc* d, int dir)
{
    const int n = d->n[dir];
    const double* xf = d->faces[dir];
    const int blo = d->bc[dir][0], bhi = d->bc[dir][1];
    auto width = [&](int i) {
        const int j = map_cell(i, n, blo, bhi);
        return xf[j + 1] - xf[j];
    };
    std::vector<double> t((size_t)NU_K * (n + 2), 0.0);
    for (int c = -1; c <= n; ++c) {
        double h[5];
        for (int o = 0; o < 5; ++o) h[o] = width(c - 2 + o);
        double* row = t.data() + (size_t)(c + 1) * NU_K;
        nu_coefficients(h, row);
        row[NU_H] = width(c);
        row[NU_IH] = 1.0 / row[NU_H];
    }
    return t;
}

bool validate(const mfx_grid_desc* d, std::string& why)
{
    if (!d) {
        why = "descriptor is NULL";
        return false;
    }
    if (d->num_fluids != 0 && (d->num_fluids < 2 || d->num_fluids > MFX_MAX_FLUIDS)) {
        why = "num_fluids must lie in [2, " + std::to_string(MFX_MAX_FLUIDS) + "] (0 reads as 2)";
        return false;
    }
    const int nf = fluids_of(d), nv = vars_of(d);
    long long N = 1;
    for (int k = 0; k < 3; ++k) {
        if (d->n[k] < 1 || d->n[k] > 65535) {
            why = "n[" + std::to_string(k) + "] must lie in [1, 65535]";
            return false;
        }
        N *= d->n[k];
        if (!(d->dx[k] > 0.0) || !std::isfinite(d->dx[k])) {
            why = "dx[" + std::to_string(k) + "] must be finite and > 0";
            return false;
        }
        for (int s = 0; s < 2; ++s) {
            if (d->bc[k][s] != MFX_BC_PERIODIC && d->bc[k][s] != MFX_BC_TRANSMISSIVE &&
                d->bc[k][s] != MFX_BC_REFLECTIVE && d->bc[k][s] != MFX_BC_INFLOW) {
                why = "bc[" + std::to_string(k) + "] holds an unknown boundary type";
                return false;
            }
            if (d->bc[k][s] == MFX_BC_INFLOW) {
                const double* q = d->inflow[k][s];
                bool ok = true;
                for (int v = 0; v < nv; ++v) ok = ok && std::isfinite(q[v]);
                double rho = 0.0, asum = 0.0;
                for (int f = 0; f < nf; ++f) {
                    ok = ok && q[f] >= 0.0;
                    rho += q[f];
                }
                for (int a = nf + 4; a < nv; ++a) {
                    ok = ok && q[a] >= 0.0 && q[a] <= 1.0;
                    asum += q[a];
                }
                ok = ok && rho > 0.0 && asum <= 1.0;
                if (!ok) {
                    why = "inflow[" + std::to_string(k) + "][" + std::to_string(s) +
                          "] must be finite, with partial densities >= 0, a positive density and volume fractions in "
                          "[0, 1] summing to at most 1";
                    return false;
                }
            }
        }
        if ((d->bc[k][0] == MFX_BC_PERIODIC) != (d->bc[k][1] == MFX_BC_PERIODIC)) {
            why = "periodic boundaries must be paired (bc[" + std::to_string(k) + "])";
            return false;
        }
        if ((d->bc[k][0] == MFX_BC_REFLECTIVE || d->bc[k][1] == MFX_BC_REFLECTIVE) && d->n[k] == 2) {
            why = "a reflective side needs n[" + std::to_string(k) + "] >= 3 (the mirror of three ghost cells)";
            return false;
        }
        if ((d->bc[k][0] >= MFX_BC_REFLECTIVE || d->bc[k][1] >= MFX_BC_REFLECTIVE) && d->n[k] == 1) {
            why = "reflective and inflow sides need an active direction (n[" + std::to_string(k) + "] > 1)";
            return false;
        }
    }
    if (N > (1LL << 31)) {
        why = "grid too large for one context (more than 2^31 cells)";
        return false;
    }
    for (int f = 0; f < nf; ++f) {
        if (!(d->gamma[f] > 1.0) || !std::isfinite(d->gamma[f])) {
            why = "gamma must be finite and > 1";
            return false;
        }
        if (!(d->pi_inf[f] >= 0.0) || !std::isfinite(d->pi_inf[f])) {
            why = "pi_inf must be finite and >= 0";
            return false;
        }
    }
    if (!(d->cfl > 0.0 && d->cfl <= 1.0)) {
        why = "cfl must lie in (0, 1]";
        return false;
    }
    if (!(d->weno_eps > 0.0) || !std::isfinite(d->weno_eps)) {
        why = "weno_eps must be finite and > 0";
        return false;
    }
    if (d->precision != MFX_FP64 && d->precision != MFX_FP32_MIXED) {
        why = "unknown precision";
        return false;
    }
    if (d->weights != MFX_WENO5_JS && d->weights != MFX_WENO5_LEARNED && d->weights != MFX_WENO5_LEARNED_EDGE &&
        d->weights != MFX_WENO5_Z) {
        why = "unknown weights mode";
        return false;
    }
    if (d->weno_order != 0 && d->weno_order != 3 && d->weno_order != 5) {
        why = "weno_order must be 3 or 5 (0 reads as 5)";
        return false;
    }
    if (d->weno_order == 3 && d->weights != MFX_WENO5_JS) {
        why = "the learned and WENO-Z weights need weno_order 5";
        return false;
    }
    if (nf != 2 && (d->weights == MFX_WENO5_LEARNED || d->weights == MFX_WENO5_LEARNED_EDGE)) {
        why = "the learned weights are defined for two fluids";
        return false;
    }
    for (int k = 0; k < 3; ++k) {
        const double* xf = d->faces[k];
        if (!xf) continue;
        const std::string nm = "faces[" + std::to_string(k) + "]";
        if (d->n[k] < 2) {
            why = nm + " needs an active direction (n > 1)";
            return false;
        }
        if (d->weights != MFX_WENO5_JS || (d->weno_order != 0 && d->weno_order != 5)) {
            why = "unequal cells take WENO5 with Jiang-Shu weights (weno_order 5, MFX_WENO5_JS)";
            return false;
        }
        for (int i = 0; i <= d->n[k]; ++i) {
            if (!std::isfinite(xf[i]) || (i > 0 && !(xf[i] > xf[i - 1]))) {
                why = nm + " must hold n + 1 finite, strictly increasing face coordinates";
                return false;
            }
        }
    }
    return true;
}

// ---------------------------------------------------------------- kernels

template <class F>
__global__ void __launch_bounds__(UTIL_BLOCK) prim_to_cons_kernel(Grid g, const double* __restrict__ w,
                                                                  double* __restrict__ q)
{
    const long long N = g.N;
    if constexpr (F::NF != 2) {
        // the model's total energy rho E = Gamma p + Pi + rho |u|^2 / 2,
        // Gamma and Pi linear in the volume fractions (Sec. II-A)
        const MixN<double, F::NF> mix = make_mix<double, F>(g);
        for (long long c = blockIdx.x * (long long)UTIL_BLOCK + threadIdx.x; c < N;
             c += (long long)gridDim.x * UTIL_BLOCK) {
            double wc[F::NV];
#pragma unroll
            for (int v = 0; v < F::NV; ++v) wc[v] = w[v * N + c];
            const double rho = density_n<F::NF>(wc);
            const double u = wc[F::IM], v = wc[F::IM + 1], ww = wc[F::IM + 2];
            const double ke = 0.5 * rho * (u * u + v * v + ww * ww);
            const double G = mix.Gamma(wc + F::IA), P = mix.Pi(wc + F::IA);
#pragma unroll
            for (int k = 0; k < F::NV; ++k) q[k * N + c] = wc[k];
            q[F::IM * N + c] = rho * u;
            q[(F::IM + 1) * N + c] = rho * v;
            q[(F::IM + 2) * N + c] = rho * ww;
            q[F::IE * N + c] = G * wc[F::IE] + P + ke;
        }
        return;
    }
    for (long long c = blockIdx.x * (long long)UTIL_BLOCK + threadIdx.x; c < N;
         c += (long long)gridDim.x * UTIL_BLOCK) {
        const double a1 = w[6 * N + c];
        const double rho = w[0 * N + c] + w[1 * N + c];
        const double u = w[2 * N + c], v = w[3 * N + c], ww = w[4 * N + c];
        const double ke = 0.5 * rho * (u * u + v * v + ww * ww);
        const double G = a1 * g.G1 + (1.0 - a1) * g.G2;
        const double P = a1 * g.P1 + (1.0 - a1) * g.P2;
        q[0 * N + c] = w[0 * N + c];
        q[1 * N + c] = w[1 * N + c];
        q[2 * N + c] = rho * u;
        q[3 * N + c] = rho * v;
        q[4 * N + c] = rho * ww;
        q[5 * N + c] = G * w[5 * N + c] + P + ke;
        q[6 * N + c] = a1;
    }
}

// CFL partial maxima over the state q, with the validity checks.
template <class F>
__global__ void __launch_bounds__(UTIL_BLOCK) cfl_partial_kernel(Grid g, const double* __restrict__ q,
                                                                 double* __restrict__ partial,
                                                                 unsigned* __restrict__ status)
{
    const long long N = g.N;
    double smax = 0.0;
    unsigned bad = 0;
    for (long long c = blockIdx.x * (long long)UTIL_BLOCK + threadIdx.x; c < N;
         c += (long long)gridDim.x * UTIL_BLOCK) {
        double qc[F::NV];
#pragma unroll
        for (int v = 0; v < F::NV; ++v) qc[v] = q[v * N + c];
        double hw[3];
        const double* hp = nullptr;
        if (g.nonuniform) {  // the cell's own widths where a direction has unequal cells
            cell_widths(g, c, hw);
            hp = hw;
        }
        smax = fmax(smax, cfl_speed<F>(g, qc, bad, hp));
    }
    if (bad) atomicOr(status, bad);
    block_max_to<UTIL_BLOCK>(smax, partial + blockIdx.x);
}

// Scalars kept on the device: [0] dt of the current state, [1] time,
// [2] step count (as double), [3] spare.
__global__ void __launch_bounds__(UTIL_BLOCK) cfl_finalize_kernel(const double* __restrict__ partial, long long np,
                                                                  double cfl, double* scal, int advance,
                                                                  double dt_arg)
{
    double m = 0.0;
    for (long long i = threadIdx.x; i < np; i += UTIL_BLOCK) m = fmax(m, partial[i]);
    __shared__ double red[UTIL_BLOCK / 64];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        double mm = red[0];
        for (int i = 1; i < UTIL_BLOCK / 64; ++i) mm = fmax(mm, red[i]);
        if (advance) {
            const double used = dt_arg > 0.0 ? dt_arg : scal[0];
            scal[1] = scal[1] + used;
            scal[2] = scal[2] + 1.0;
        }
        scal[0] = cfl / mm;
    }
}

}  // namespace

// ---------------------------------------------------------------- context

struct mfx_ctx {
    mfx_grid_desc desc;
    Grid g;
    int nv;  // variables per cell (2 * fluids + 3)
    hipStream_t stream;
    int device;
    char* ws;
    size_t ws_bytes;
    Layout L;
    double *q, *q1, *q2, *scal, *partial;
    void *r, *bface;  // compute-type buffers
    size_t elem;      // sizeof the compute type
    MlpNet* mlp;                  // packed network operands (learned weights)
    float* mlp_params;            // float32 copy of the network
    unsigned long long* fallback; // edges that fell back to Jiang-Shu
    bool has_mlp;
    unsigned* status;
    int dirs[3];
    int ndirs;
    int seg_override;
    int xmode_override;  // MFX_XSWEEP: 0 automatic, 1 marching x sweep
    bool fuse_xy;        // x and y passes as one kernel where it applies (MFX_FUSE_XY=0 disables)
    bool fuse_cfl;       // CFL reduction inside the step's last y/z sweep (MFX_FUSE_CFL=0 disables)
    bool has_state;
    std::string err;
    // kernel timing (mfx_profile): events around each sweep launch
    bool profiling;
    struct Pending {
        int kind;
        hipEvent_t a, b;
    };
    std::vector<Pending> pending;
    std::vector<hipEvent_t> pool;
    double prof_ms[MFX_PROF_KINDS];
    int64_t prof_n[MFX_PROF_KINDS];
};

namespace {

int fail(mfx_ctx* c, int code, const std::string& msg)
{
    if (c)
        c->err = msg;
    else
        g_init_error = msg;
    return code;
}

#define HIP_TRY(ctx, call)                                                                       \
    do {                                                                                         \
        hipError_t e_ = (call);                                                                  \
        if (e_ != hipSuccess) return fail((ctx), MFX_EHIP, std::string(#call ": ") + hipGetErrorString(e_)); \
    } while (0)

int launch_check(mfx_ctx* c, const char* what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(c, MFX_EHIP, std::string(what) + ": " + hipGetErrorString(e));
    return MFX_OK;
}

int set_device(mfx_ctx* c)
{
    int cur = -1;
    HIP_TRY(c, hipGetDevice(&cur));
    if (cur != c->device) HIP_TRY(c, hipSetDevice(c->device));
    return MFX_OK;
}

// Launch the sweep for direction d.
hipEvent_t take_event(mfx_ctx* c)
{
    if (!c->pool.empty()) {
        hipEvent_t e = c->pool.back();
        c->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

int launch_sweep(mfx_ctx* c, int d, const double* qs, const double* qn, double* out, int first, int mode,
                 const double* dt_dev, double dt_arg, bool cfl = false)
{
    SweepGeom sg = sweep_geom(c->g.n, d, c->seg_override, c->xmode_override, c->elem,
                              learned_weights(c->desc), vars_of(&c->desc));
    mfx_ctx::Pending pend{(d * 2 + (first ? 1 : 0)) * 5 + mode, nullptr, nullptr};
    if (c->profiling) {
        pend.a = take_event(c);
        pend.b = take_event(c);
        if (!pend.a || !pend.b) return fail(c, MFX_EHIP, "hipEventCreate failed");
        HIP_TRY(c, hipEventRecord(pend.a, c->stream));
    }
    const LaunchArgs la{&sg,      c->stream,   &c->g,      qs,        qn,       c->r,
                        out,      dt_dev,      dt_arg,     c->bface,  c->mlp,   c->fallback,
                        c->partial, c->status, cfl};
    // a direction with unequal cells takes the per-position scheme
    const int sch = c->g.nu[d] ? SCHEME_WENO5NU : scheme_of(c->desc);
    if (learned_weights(c->desc))
        launch_dispatch<float, true, SCHEME_WENO5, Fl2>(d, first != 0, mode, la);
    else if (c->g.nf == 3 && c->desc.precision == MFX_FP32_MIXED)
        by_scheme(sch, [&](auto s) { launch_dispatch<float, false, decltype(s)::value, Fl<3>>(d, first != 0, mode, la); });
    else if (c->g.nf == 3)
        by_scheme(sch, [&](auto s) { launch_dispatch<double, false, decltype(s)::value, Fl<3>>(d, first != 0, mode, la); });
    else if (c->desc.precision == MFX_FP32_MIXED)
        by_scheme(sch, [&](auto s) { launch_dispatch<float, false, decltype(s)::value, Fl2>(d, first != 0, mode, la); });
    else
        by_scheme(sch, [&](auto s) { launch_dispatch<double, false, decltype(s)::value, Fl2>(d, first != 0, mode, la); });
    int rc = launch_check(c, "sweep kernel");
    if (rc) return rc;
    if (c->profiling) {
        HIP_TRY(c, hipEventRecord(pend.b, c->stream));
        c->pending.push_back(pend);
    }
    return MFX_OK;
}

// The fused x-y pass applies when x and y are the first two active
// directions, x rows fit the row kernel, the weights are Jiang-Shu-family and
// the cells are equal along x and y.  Three fluids in float64 keep the
// separate x row and y passes: the fused pass holds its five-cell window in
// registers (90 for nine float64 variables) and would spill.
bool fused_xy(const mfx_ctx* c)
{
    if (c->g.nf == 3 && c->elem == sizeof(double)) return false;
    return c->fuse_xy && !learned_weights(c->desc) && c->ndirs >= 2 && c->dirs[0] == 0 && c->dirs[1] == 1 &&
           !c->g.nu[0] && !c->g.nu[1] && use_xrows(c->g.n, c->xmode_override, c->elem, vars_of(&c->desc));
}

// The fused pass, profiled as direction 3 (first pass).
int launch_sweep_xy(mfx_ctx* c, const double* qs, const double* qn, double* out, int mode, const double* dt_dev,
                    double dt_arg)
{
    mfx_ctx::Pending pend{(3 * 2 + 1) * 5 + mode, nullptr, nullptr};
    if (c->profiling) {
        pend.a = take_event(c);
        pend.b = take_event(c);
        if (!pend.a || !pend.b) return fail(c, MFX_EHIP, "hipEventCreate failed");
        HIP_TRY(c, hipEventRecord(pend.a, c->stream));
    }
    const XYArgs xa{&c->g, c->stream, qs, qn, c->r, out, dt_dev, dt_arg, c->bface, c->mlp, c->fallback, c->seg_override};
    const bool f32 = c->desc.precision == MFX_FP32_MIXED;
    if (c->g.nf == 3)  // (float only: see fused_xy)
        by_scheme<false>(scheme_of(c->desc), [&](auto s) { launch_xy<float, decltype(s)::value, Fl<3>>(mode, xa); });
    else if (f32)
        by_scheme<false>(scheme_of(c->desc), [&](auto s) { launch_xy<float, decltype(s)::value, Fl2>(mode, xa); });
    else
        by_scheme<false>(scheme_of(c->desc), [&](auto s) { launch_xy<double, decltype(s)::value, Fl2>(mode, xa); });
    int rc = launch_check(c, "fused x-y sweep");
    if (rc) return rc;
    if (c->profiling) {
        HIP_TRY(c, hipEventRecord(pend.b, c->stream));
        c->pending.push_back(pend);
    }
    return MFX_OK;
}

// Blocks of the last pass when that pass (a y or z sweep with Jiang-Shu
// weights writing a step's new state) also reduces the CFL speed of its
// output (on unequal cells with each cell's widths, as the standalone
// reduction); 0 when the standalone reduction is needed.
long long cfl_blocks_in_last_pass(const mfx_ctx* c)
{
    if (!c->fuse_cfl || learned_weights(c->desc)) return 0;
    const int d = c->dirs[c->ndirs - 1];
    if (d == 0 || !c->g.active[d]) return 0;
    if (fused_xy(c) && c->ndirs == 2) return 0;  // the fused x-y pass is the last
    const SweepGeom sg = sweep_geom(c->g.n, d, c->seg_override, c->xmode_override, c->elem, false, vars_of(&c->desc));
    return (long long)sg.grid.x * sg.grid.y * sg.grid.z;
}

// All direction passes of one right-hand-side evaluation; the last active
// direction applies `last_mode` with output `out` (and, with cfl, reduces
// the CFL speed of that output).
int run_passes(mfx_ctx* c, const double* qs, const double* qn, double* out, int last_mode, const double* dt_dev,
               double dt_arg, bool cfl = false)
{
    int i0 = 0;
    if (fused_xy(c)) {
        const bool last = c->ndirs == 2;
        int rc = launch_sweep_xy(c, qs, qn, last ? out : nullptr, last ? last_mode : OUT_ACCUM, dt_dev, dt_arg);
        if (rc != MFX_OK) return rc;
        i0 = 2;
    }
    for (int i = i0; i < c->ndirs; ++i) {
        const int d = c->dirs[i];
        const bool last = (i == c->ndirs - 1);
        int rc = launch_sweep(c, d, qs, qn, last ? out : nullptr, i == 0 && i0 == 0, last ? last_mode : OUT_ACCUM,
                              dt_dev, dt_arg, last && cfl);
        if (rc != MFX_OK) return rc;
    }
    return MFX_OK;
}

// CFL time step of the current state (per-block maxima, then one block),
// which also flags a non-physical state in the status word; with advance,
// t and the step count first move on by the step just taken (dt_arg, or
// the device time step when dt_arg is 0).
int standalone_cfl(mfx_ctx* c, int advance = 0, double dt_arg = 0.0)
{
    if (c->g.nf == 3)
        cfl_partial_kernel<Fl<3>><<<CFL_BLOCKS, UTIL_BLOCK, 0, c->stream>>>(c->g, c->q, c->partial, c->status);
    else
        cfl_partial_kernel<Fl2><<<CFL_BLOCKS, UTIL_BLOCK, 0, c->stream>>>(c->g, c->q, c->partial, c->status);
    int rc = launch_check(c, "cfl_partial_kernel");
    if (rc != MFX_OK) return rc;
    cfl_finalize_kernel<<<1, UTIL_BLOCK, 0, c->stream>>>(c->partial, CFL_BLOCKS, c->g.cfl, c->scal, advance, dt_arg);
    return launch_check(c, "cfl_finalize_kernel");
}

// Device-to-host copy of n bytes into host memory that may live on the
// caller's stack: the copy is waited for before returning, so no copy is
// left in flight when an error path returns early.
int read_device(mfx_ctx* c, void* host, const void* dev, size_t n)
{
    HIP_TRY(c, hipMemcpyAsync(host, dev, n, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return MFX_OK;
}

int read_status(mfx_ctx* c, unsigned* st)
{
    return read_device(c, st, c->status, sizeof(unsigned));
}

// MFX_ESTATE for a status word with an error bit (alpha1 outside [0, 1]
// alone is recorded, not an error).
int status_error(mfx_ctx* c, unsigned st)
{
    if (st & MFX_STATUS_ERRORS)
        return fail(c, MFX_ESTATE, "non-physical state flagged (status " + std::to_string(st) + ")");
    return MFX_OK;
}

// Grid constants and the active directions of a context from its
// descriptor; inflow_dev: device copy of the inflow states.
void setup_grid(const mfx_grid_desc* desc, mfx_ctx* c, const double* inflow_dev)
{
    Grid& g = c->g;
    g.N = (long long)desc->n[0] * desc->n[1] * desc->n[2];
    g.stride[0] = 1;
    g.stride[1] = desc->n[0];
    g.stride[2] = (long long)desc->n[0] * desc->n[1];
    c->ndirs = 0;
    for (int k = 0; k < 3; ++k) {
        g.n[k] = desc->n[k];
        g.dx[k] = desc->dx[k];
        g.inv_dx[k] = 1.0 / desc->dx[k];
        g.bc[k][0] = desc->bc[k][0];
        g.bc[k][1] = desc->bc[k][1];
        for (int s = 0; s < 2; ++s)
            for (int v = 0; v < NVMAX; ++v)
                g.inflow[k][s][v] = desc->bc[k][s] == MFX_BC_INFLOW && v < vars_of(desc) ? desc->inflow[k][s][v] : 0.0;
        g.active[k] = desc->n[k] > 1;
        if (g.active[k]) c->dirs[c->ndirs++] = k;
    }
    g.inflow_dev = inflow_dev;
    for (int k = 0; k < 3; ++k) g.nu[k] = nullptr;  // mfx_init_grid binds the tables of unequal cells
    g.nonuniform = 0;
    if (c->ndirs == 0) c->dirs[c->ndirs++] = 0;  // a single cell still sweeps x (all faces from ghosts)
    g.G1 = 1.0 / (desc->gamma[0] - 1.0);
    g.G2 = 1.0 / (desc->gamma[1] - 1.0);
    g.P1 = desc->gamma[0] * desc->pi_inf[0] / (desc->gamma[0] - 1.0);
    g.P2 = desc->gamma[1] * desc->pi_inf[1] / (desc->gamma[1] - 1.0);
    g.nf = fluids_of(desc);
    c->nv = vars_of(desc);
    for (int f = 0; f < MAXF; ++f) {
        g.Gn[f] = f < g.nf ? 1.0 / (desc->gamma[f] - 1.0) : 0.0;
        g.Pn[f] = f < g.nf ? desc->gamma[f] * desc->pi_inf[f] / (desc->gamma[f] - 1.0) : 0.0;
    }
    g.eps = desc->weno_eps;
    g.edge_weights = desc->weights == MFX_WENO5_LEARNED_EDGE ? 1 : 0;
    g.cfl = desc->cfl;
}

}  // namespace

// ---------------------------------------------------------------- C ABI

extern "C" {

size_t mfx_workspace_bytes(const mfx_grid_desc* desc)
{
    std::string why;
    if (!validate(desc, why)) return 0;
    const Overrides o = read_overrides();
    return make_layout(desc, o.seg, x_mode(desc, o.xmode)).total;
}

int mfx_init_grid(const mfx_grid_desc* desc, void* ws_dev, size_t ws_bytes, void* hip_stream, mfx_ctx** out)
{
    if (!out) return fail(nullptr, MFX_EINVAL, "out is NULL");
    *out = nullptr;
    std::string why;
    if (!validate(desc, why)) return fail(nullptr, MFX_EINVAL, why);
    if (learned_weights(*desc) && desc->precision != MFX_FP32_MIXED)
        return fail(nullptr, MFX_EINVAL, "learned weights run in the MFX_FP32_MIXED precision form");
    if (!ws_dev) return fail(nullptr, MFX_EINVAL, "workspace pointer is NULL");
    if (reinterpret_cast<uintptr_t>(ws_dev) % ALIGN != 0)
        return fail(nullptr, MFX_EINVAL, "workspace must be 256-byte aligned");

    const Overrides ov = read_overrides();
    const int xmode = x_mode(desc, ov.xmode);
    Layout L = make_layout(desc, ov.seg, xmode);
    if (ws_bytes < L.total)
        return fail(nullptr, MFX_ENOMEM, "workspace has " + std::to_string(ws_bytes) + " bytes, needs " +
                                             std::to_string(L.total));

    mfx_ctx* c = new (std::nothrow) mfx_ctx();
    if (!c) return fail(nullptr, MFX_ENOMEM, "host allocation of the context failed");
    c->desc = *desc;
    c->stream = reinterpret_cast<hipStream_t>(hip_stream);
    c->seg_override = ov.seg;
    c->xmode_override = xmode;
    c->fuse_xy = ov.fuse_xy != 0;
    c->fuse_cfl = ov.fuse_cfl != 0;

    if (hipGetDevice(&c->device) != hipSuccess) {
        delete c;
        return fail(nullptr, MFX_EHIP, "hipGetDevice failed");
    }
    c->ws = static_cast<char*>(ws_dev);
    c->ws_bytes = ws_bytes;
    c->L = L;
    c->q = reinterpret_cast<double*>(c->ws + L.q);
    c->q1 = reinterpret_cast<double*>(c->ws + L.q1);
    c->q2 = reinterpret_cast<double*>(c->ws + L.q2);
    c->r = c->ws + L.r;
    c->elem = desc->precision == MFX_FP32_MIXED ? sizeof(float) : sizeof(double);
    c->scal = reinterpret_cast<double*>(c->ws + L.scal);
    c->status = reinterpret_cast<unsigned*>(c->ws + L.scal + 4 * sizeof(double));
    c->partial = reinterpret_cast<double*>(c->ws + L.partial);
    c->bface = c->ws + L.bface;
    c->mlp = reinterpret_cast<MlpNet*>(c->ws + L.mlp);
    c->mlp_params = reinterpret_cast<float*>(c->ws + L.mlp_params);
    c->fallback = reinterpret_cast<unsigned long long*>(c->ws + L.scal + 40);
    c->has_mlp = false;

    setup_grid(desc, c, reinterpret_cast<const double*>(c->ws + L.inflow));

    // an error after a copy was queued waits for the stream before the
    // copy's host source (the context, the tables below) is freed
    auto abandon = [&](const char* msg) {
        (void)hipStreamSynchronize(c->stream);
        delete c;
        return fail(nullptr, MFX_EHIP, msg);
    };
    if (hipMemsetAsync(c->ws + L.scal, 0, 64, c->stream) != hipSuccess)
        return abandon("hipMemsetAsync of the scalar block failed");
    // the inflow states for the loaders (zero for other sides); the source
    // lives in the context
    if (hipMemcpyAsync(c->ws + L.inflow, &c->g.inflow[0][0][0], sizeof(double) * 3 * 2 * NVMAX, hipMemcpyHostToDevice,
                       c->stream) != hipSuccess)
        return abandon("copy of the inflow states failed");
    // per-position tables of directions with unequal cells (host copies
    // kept until the stream has taken them)
    std::vector<double> tabs[3];
    for (int k = 0; k < 3; ++k) {
        if (!desc->faces[k]) continue;
        tabs[k] = nu_table(desc, k);
        if (hipMemcpyAsync(c->ws + L.nu[k], tabs[k].data(), sizeof(double) * tabs[k].size(), hipMemcpyHostToDevice,
                           c->stream) != hipSuccess)
            return abandon("copy of the unequal-cell tables failed");
        c->g.nu[k] = reinterpret_cast<const double*>(c->ws + L.nu[k]);
        c->g.nonuniform = 1;
    }
    if (hipStreamSynchronize(c->stream) != hipSuccess)
        return abandon("hipStreamSynchronize after the table copies failed");
    for (int k = 0; k < 3; ++k) c->desc.faces[k] = nullptr;  // read here only; the caller may free them
    c->has_state = false;
    c->profiling = false;
    for (int k = 0; k < MFX_PROF_KINDS; ++k) {
        c->prof_ms[k] = 0.0;
        c->prof_n[k] = 0;
    }
    *out = c;
    return MFX_OK;
}

int mfx_weno5_nu_coefficients(const double* h, double* out)
{
    if (!h || !out) return fail(nullptr, MFX_EINVAL, "h and out must not be NULL");
    for (int i = 0; i < 5; ++i)
        if (!(h[i] > 0.0) || !std::isfinite(h[i])) return fail(nullptr, MFX_EINVAL, "widths must be finite and > 0");
    double t[NU_K];
    nu_coefficients(h, t);
    for (int i = 0; i < MFX_NU_COEFS; ++i) out[i] = t[i];
    return MFX_OK;
}

int mfx_set_state(mfx_ctx* c, const double* q_dev)
{
    if (!c) return fail(nullptr, MFX_EINVAL, "ctx is NULL");
    if (!q_dev) return fail(c, MFX_EINVAL, "q_dev is NULL");
    int rc = set_device(c);
    if (rc) return rc;
    HIP_TRY(c, hipMemcpyAsync(c->q, q_dev, sizeof(double) * c->nv * (size_t)c->g.N, hipMemcpyDeviceToDevice,
                              c->stream));
    HIP_TRY(c, hipMemsetAsync(c->ws + c->L.scal, 0, 64, c->stream));
    c->has_state = true;
    return standalone_cfl(c);
}

int mfx_set_primitive(mfx_ctx* c, const double* w_dev)
{
    if (!c) return fail(nullptr, MFX_EINVAL, "ctx is NULL");
    if (!w_dev) return fail(c, MFX_EINVAL, "w_dev is NULL");
    int rc = set_device(c);
    if (rc) return rc;
    const long long blocks = std::min<long long>((c->g.N + UTIL_BLOCK - 1) / UTIL_BLOCK, 65536);
    if (c->g.nf == 3)
        prim_to_cons_kernel<Fl<3>><<<(unsigned)blocks, UTIL_BLOCK, 0, c->stream>>>(c->g, w_dev, c->q);
    else
        prim_to_cons_kernel<Fl2><<<(unsigned)blocks, UTIL_BLOCK, 0, c->stream>>>(c->g, w_dev, c->q);
    rc = launch_check(c, "prim_to_cons_kernel");
    if (rc) return rc;
    HIP_TRY(c, hipMemsetAsync(c->ws + c->L.scal, 0, 64, c->stream));
    c->has_state = true;
    return standalone_cfl(c);
}

int mfx_get_state(mfx_ctx* c, double* q_dev_out)
{
    if (!c) return fail(nullptr, MFX_EINVAL, "ctx is NULL");
    if (!q_dev_out) return fail(c, MFX_EINVAL, "q_dev_out is NULL");
    if (!c->has_state) return fail(c, MFX_EINVAL, "no state set");
    int rc = set_device(c);
    if (rc) return rc;
    HIP_TRY(c, hipMemcpyAsync(q_dev_out, c->q, sizeof(double) * c->nv * (size_t)c->g.N, hipMemcpyDeviceToDevice,
                              c->stream));
    unsigned st = 0;
    rc = read_status(c, &st);
    if (rc) return rc;
    return status_error(c, st);
}

namespace {
int need_mlp(mfx_ctx* c)
{
    if (learned_weights(c->desc) && !c->has_mlp)
        return fail(c, MFX_EINVAL, "learned weights selected but no network set (mfx_set_mlp)");
    return MFX_OK;
}
}  // namespace

int mfx_rhs(mfx_ctx* c, double* rhs_out)
{
    if (!c) return fail(nullptr, MFX_EINVAL, "ctx is NULL");
    if (int rc = need_mlp(c)) return rc;
    if (!rhs_out) return fail(c, MFX_EINVAL, "rhs_dev_out is NULL");
    if (!c->has_state) return fail(c, MFX_EINVAL, "no state set");
    const char* o = reinterpret_cast<const char*>(rhs_out);
    if (o < c->ws + c->ws_bytes && o + sizeof(double) * c->nv * c->g.N > c->ws)
        return fail(c, MFX_EINVAL, "rhs_dev_out overlaps the workspace");
    int rc = set_device(c);
    if (rc) return rc;
    return run_passes(c, c->q, c->q, rhs_out, OUT_RHS, nullptr, 0.0);
}

int mfx_rk3_step(mfx_ctx* c, double dt, double* dt_used_host)
{
    if (!c) return fail(nullptr, MFX_EINVAL, "ctx is NULL");
    if (int rc = need_mlp(c)) return rc;
    if (!c->has_state) return fail(c, MFX_EINVAL, "no state set");
    if (!std::isfinite(dt)) return fail(c, MFX_EINVAL, "dt is not finite");
    if (!(dt > 0.0) && !(c->g.active[0] || c->g.active[1] || c->g.active[2]))
        return fail(c, MFX_EINVAL, "no active direction: the CFL time step is undefined, pass dt > 0");
    int rc = set_device(c);
    if (rc) return rc;
    const double* dt_dev = dt > 0.0 ? nullptr : c->scal;
    const double dt_arg = dt > 0.0 ? dt : 0.0;
    // the CFL time step this step uses, read before the step overwrites it
    // (the caller asked for it, so the call synchronises anyway)
    double dt_seen = 0.0;
    if (dt_used_host && !(dt > 0.0)) {
        rc = read_device(c, &dt_seen, c->scal, sizeof(double));
        if (rc) return rc;
    }
    rc = run_passes(c, c->q, c->q, c->q1, OUT_STAGE1, dt_dev, dt_arg);
    if (rc) return rc;
    rc = run_passes(c, c->q1, c->q, c->q2, OUT_STAGE2, dt_dev, dt_arg);
    if (rc) return rc;
    const long long nb = cfl_blocks_in_last_pass(c);
    rc = run_passes(c, c->q2, c->q, c->q, OUT_STAGE3, dt_dev, dt_arg, nb > 0);
    if (rc) return rc;
    // time step of the new state for the next step, and its physicality check
    if (nb > 0) {
        cfl_finalize_kernel<<<1, UTIL_BLOCK, 0, c->stream>>>(c->partial, nb, c->g.cfl, c->scal, 1, dt_arg);
        rc = launch_check(c, "cfl_finalize_kernel");
    } else {
        rc = standalone_cfl(c, 1, dt_arg);
    }
    if (rc) return rc;
    if (dt_used_host) {
        unsigned st = 0;
        rc = read_status(c, &st);
        if (rc) return rc;
        *dt_used_host = dt > 0.0 ? dt : dt_seen;
        return status_error(c, st);
    }
    return MFX_OK;
}

int mfx_set_mlp(mfx_ctx* c, const float* params_dev, int32_t n_params)
{
    if (!c) return fail(nullptr, MFX_EINVAL, "ctx is NULL");
    if (!params_dev) return fail(c, MFX_EINVAL, "params_dev is NULL");
    if (n_params != MLP_PARAMS) return fail(c, MFX_EINVAL, "the network has " + std::to_string(MLP_PARAMS) + " parameters");
    int rc = set_device(c);
    if (rc) return rc;
    HIP_TRY(c, hipMemcpyAsync(c->mlp_params, params_dev, sizeof(float) * MLP_PARAMS, hipMemcpyDeviceToDevice,
                              c->stream));
    rc = mlp_pack_on_stream(c->mlp_params, c->mlp, c->stream);
    if (rc) return fail(c, rc, "packing the network failed");
    c->has_mlp = true;
    return MFX_OK;
}

int mfx_stats(mfx_ctx* c, double* t, int64_t* step, int64_t* fallback_faces, uint32_t* status)
{
    if (!c) return fail(nullptr, MFX_EINVAL, "ctx is NULL");
    int rc = set_device(c);
    if (rc) return rc;
    double sc[4];
    unsigned st = 0;
    unsigned long long fb = 0;
    if ((rc = read_device(c, sc, c->scal, sizeof(sc))) || (rc = read_device(c, &st, c->status, sizeof(unsigned))) ||
        (rc = read_device(c, &fb, c->fallback, sizeof(fb))))
        return rc;
    if (t) *t = sc[1];
    if (step) *step = (int64_t)sc[2];
    if (fallback_faces) *fallback_faces = (int64_t)fb;
    if (status) *status = st;
    return status_error(c, st);
}

int mfx_profile(mfx_ctx* c, int enable)
{
    if (!c) return fail(nullptr, MFX_EINVAL, "ctx is NULL");
    int rc = set_device(c);
    if (rc) return rc;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    for (auto& p : c->pending) {
        c->pool.push_back(p.a);
        c->pool.push_back(p.b);
    }
    c->pending.clear();
    for (int k = 0; k < MFX_PROF_KINDS; ++k) {
        c->prof_ms[k] = 0.0;
        c->prof_n[k] = 0;
    }
    c->profiling = enable != 0;
    return MFX_OK;
}

int mfx_profile_read(mfx_ctx* c, double* ms, int64_t* counts)
{
    if (!c) return fail(nullptr, MFX_EINVAL, "ctx is NULL");
    int rc = set_device(c);
    if (rc) return rc;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    for (auto& p : c->pending) {
        float e = 0.f;
        HIP_TRY(c, hipEventElapsedTime(&e, p.a, p.b));
        c->prof_ms[p.kind] += e;
        c->prof_n[p.kind] += 1;
        c->pool.push_back(p.a);
        c->pool.push_back(p.b);
    }
    c->pending.clear();
    for (int k = 0; k < MFX_PROF_KINDS; ++k) {
        if (ms) ms[k] = c->prof_ms[k];
        if (counts) counts[k] = c->prof_n[k];
    }
    return MFX_OK;
}

void mfx_destroy(mfx_ctx* c)
{
    if (!c) return;
    for (auto& p : c->pending) {
        c->pool.push_back(p.a);
        c->pool.push_back(p.b);
    }
    for (hipEvent_t e : c->pool) (void)hipEventDestroy(e);
    delete c;
}

const char* mfx_last_error(const mfx_ctx* c) { return c ? c->err.c_str() : g_init_error.c_str(); }

}  // extern "C"

// ---------------------------------------------------------------- right-hand side without allocation
//
// mfx_rhs_static: the passes of mfx_rhs on a context built on the stack,
// with every buffer besides the caller's state and output in `scratch`.

// One copy per GPU the library runs on, held until the process ends.  In
// host code this name is only a handle: the array's device address comes
// from hipGetSymbolAddress, once per device (static_scratch below).
static __device__ __align__(256) unsigned char scratch[MFX_STATIC_SCRATCH_BYTES];

namespace {

constexpr size_t SCR_INFLOW = 0;    // inflow states [3][2][NVMAX] float64 (432 bytes)
constexpr size_t SCR_STATUS = 512;  // status word (unused by the right-hand side, kept zero)
constexpr size_t SCR_FB = 520;      // fallback counter (learned weights only; kept zero)
constexpr size_t SCR_BFACE = 768;   // x rows' boundary faces, then the partial right-hand side
constexpr int MAX_DEVICES = 64;

std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};

size_t static_bface_bytes(const mfx_grid_desc* d, size_t elem)
{
    return align_up(elem * (vars_of(d) + 1) * 2 * (size_t)d->n[1] * (size_t)d->n[2]);
}

size_t static_need(const mfx_grid_desc* d)
{
    const size_t elem = d->precision == MFX_FP32_MIXED ? sizeof(float) : sizeof(double);
    const size_t N = (size_t)d->n[0] * d->n[1] * d->n[2];
    return SCR_BFACE + static_bface_bytes(d, elem) + align_up(elem * vars_of(d) * N);
}

// Device address of `scratch` on device dev (current), looked up once per device.
int static_scratch(int dev, char** out, std::string& why)
{
    if (dev < 0 || dev >= MAX_DEVICES) {
        why = "device index " + std::to_string(dev) + " beyond the scratch table";
        return MFX_EINVAL;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            why = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
            return MFX_EHIP;
        }
        g_scratch_ptr[dev] = p;
    }
    *out = static_cast<char*>(g_scratch_ptr[dev]);
    return MFX_OK;
}

// Inflow states into the scratch (from the kernel arguments, so no copy
// call), status word and fallback counter cleared.
__global__ void __launch_bounds__(64) static_setup_kernel(Grid g, double* __restrict__ inflow,
                                                           unsigned* __restrict__ status,
                                                           unsigned long long* __restrict__ fb)
{
    const int t = threadIdx.x;
    if (t < 3 * 2 * NVMAX) inflow[t] = (&g.inflow[0][0][0])[t];
    if (t == 0) {
        *status = 0u;
        *fb = 0ull;
    }
}

int static_fail(int code, const std::string& msg)
{
    g_init_error = msg;
    return code;
}

}  // namespace

extern "C" int mfx_rhs_static(const mfx_grid_desc* desc, const double* q_dev, double* rhs_dev_out,
                              void* hip_stream)
{
    std::string why;
    if (!validate(desc, why)) return static_fail(MFX_EINVAL, why);
    if (learned_weights(*desc))
        return static_fail(MFX_EINVAL, "mfx_rhs_static takes Jiang-Shu or WENO-Z weights (a network needs a context)");
    if (desc->faces[0] || desc->faces[1] || desc->faces[2])
        return static_fail(MFX_EINVAL, "mfx_rhs_static takes uniform cells (faces all NULL): unequal cells need a context");
    if (!q_dev || !rhs_dev_out) return static_fail(MFX_EINVAL, "q_dev and rhs_dev_out must not be NULL");
    const size_t N = (size_t)desc->n[0] * desc->n[1] * desc->n[2];
    const size_t bytes = sizeof(double) * vars_of(desc) * N;
    const char* qa = reinterpret_cast<const char*>(q_dev);
    const char* ra = reinterpret_cast<const char*>(rhs_dev_out);
    if (ra < qa + bytes && qa < ra + bytes) return static_fail(MFX_EINVAL, "q_dev and rhs_dev_out overlap");
    const size_t need = static_need(desc);
    if (need > MFX_STATIC_SCRATCH_BYTES)
        return static_fail(MFX_ENOMEM, "the grid needs " + std::to_string(need) + " bytes of scratch; the static array holds " +
                                           std::to_string((size_t)MFX_STATIC_SCRATCH_BYTES));
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return static_fail(MFX_EHIP, "hipGetDevice failed");
    char* sb = nullptr;
    if (int rc = static_scratch(dev, &sb, why)) return static_fail(rc, why);

    mfx_ctx c{};  // zero-initialised; lives for this call only
    c.desc = *desc;
    c.stream = reinterpret_cast<hipStream_t>(hip_stream);
    c.device = dev;
    const Overrides ov = read_overrides();
    c.seg_override = ov.seg;
    c.xmode_override = x_mode(desc, ov.xmode);
    c.fuse_xy = ov.fuse_xy != 0;
    c.fuse_cfl = ov.fuse_cfl != 0;
    c.elem = desc->precision == MFX_FP32_MIXED ? sizeof(float) : sizeof(double);
    c.ws = sb;
    c.ws_bytes = need;
    c.status = reinterpret_cast<unsigned*>(sb + SCR_STATUS);
    c.fallback = reinterpret_cast<unsigned long long*>(sb + SCR_FB);
    c.bface = sb + SCR_BFACE;
    c.r = sb + SCR_BFACE + static_bface_bytes(desc, c.elem);
    c.has_state = true;
    setup_grid(desc, &c, reinterpret_cast<const double*>(sb + SCR_INFLOW));
    static_setup_kernel<<<1, 64, 0, c.stream>>>(c.g, reinterpret_cast<double*>(sb + SCR_INFLOW), c.status, c.fallback);
    int rc = launch_check(&c, "static_setup_kernel");
    if (rc == MFX_OK) rc = run_passes(&c, q_dev, q_dev, rhs_dev_out, OUT_RHS, nullptr, 0.0);
    if (rc != MFX_OK) return static_fail(rc, c.err);
    return MFX_OK;
}
