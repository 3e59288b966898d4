// Learned WENO weights: training-data preparation, the network's forward and
// backward passes in float32 with a deterministic two-stage gradient
// reduction, Adam, and packing of the bfloat16 operands that the sweeps use
// for inference.  The C entry points are declared in include/mfx.h.
//
// Weights omega_i = softmax(ln omega^JS_i + z_i), z the network output.
// Loss of one minibatch of n samples (stencil-normalised values, primes):
//   L = (1/n) sum_i (sum_k omega_ik p'_ik - t'_i)^2
//     + lam (1/n) sum_i sum_k (omega_ik - omega^JS_ik)^2.
#include <hip/hip_runtime.h>

#include <cmath>
#include <string>

#include "../../include/mfx.h"
#include "learned.h"
#include "physics.h"
#include "sweep.h"

using namespace mfx;

namespace {

constexpr int TB = 64;                     // samples per block in the gradient kernel
constexpr int GRAD_SLOTS = MLP_PARAMS + 1;  // parameters + loss

__device__ __forceinline__ float gelu_grad(float x)
{
    const float u = GELU_C * (x + GELU_A * x * x * x);
    const float t = tanhf(u);
    return 0.5f * (1.0f + t) + 0.5f * x * (1.0f - t * t) * GELU_C * (1.0f + 3.0f * GELU_A * x * x);
}

// GELU in its tanh form, for training (the inference kernels evaluate the
// polynomial form of learned.h, within 1.2e-4 of this one).
__device__ __forceinline__ float gelu_ref(float x)
{
    return 0.5f * x * (1.0f + tanhf(GELU_C * (x + GELU_A * x * x * x)));
}

// Right-edge stencils along x of a 1D state q[7][n] and their targets: sample
// (v, i, side) -> index ((side * 7 + v) * n + i).  side 0: cells i-2..i+2,
// target face_prim[v][i+1]; side 1: the mirrored stencil i+2..i-2 (the left
// edge of cell i), target face_prim[v][i].  Ghost cells by the x boundary map.
__global__ void __launch_bounds__(256) sample_stencils_kernel(Grid g, const double* __restrict__ q,
                                                              const double* __restrict__ face_prim,
                                                              double* __restrict__ stencil, double* __restrict__ target)
{
    const int n = g.n[0];
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const Mix<double> mix{g.G1, g.G2, g.P1, g.P2};
    double w[5][NV];
    for (int k = 0; k < 5; ++k) {
        const int c = map_cell(i - 2 + k, n, g.bc[0][0], g.bc[0][1]);
        double qc[NV];
        for (int v = 0; v < NV; ++v) qc[v] = q[(long long)v * n + c];
        cons_to_prim(mix, qc, w[k]);
    }
    for (int v = 0; v < NV; ++v) {
        const long long r = (long long)(0 * NV + v) * n + i;
        const long long l = (long long)(1 * NV + v) * n + i;
        for (int k = 0; k < 5; ++k) {
            stencil[r * 5 + k] = w[k][v];
            stencil[l * 5 + k] = w[4 - k][v];
        }
        target[r] = face_prim[(long long)v * (n + 1) + i + 1];
        target[l] = face_prim[(long long)v * (n + 1) + i];
    }
}

// Reference primitive values at the faces of a coarse grid from a state on
// a grid r times finer (same domain): coarse face i sits on fine face r*i,
// whose value is taken as the mean of the two fine cells beside it (the
// boundary cell at a domain end).  out[7][nc + 1], nc = nf / r.
__global__ void __launch_bounds__(256) face_targets_kernel(Grid g, const double* __restrict__ q, int r,
                                                           double* __restrict__ out)
{
    const int nf = g.n[0];
    const int nc = nf / r;
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i > nc) return;
    const Mix<double> mix{g.G1, g.G2, g.P1, g.P2};
    const int f = r * i;
    const int a = map_cell(f - 1, nf, g.bc[0][0], g.bc[0][1]);
    const int b = map_cell(f, nf, g.bc[0][0], g.bc[0][1]);
    double qa[NV], qb[NV], wa[NV], wb[NV];
    for (int v = 0; v < NV; ++v) {
        qa[v] = q[(long long)v * nf + a];
        qb[v] = q[(long long)v * nf + b];
    }
    cons_to_prim(mix, qa, wa);
    cons_to_prim(mix, qb, wb);
    for (int v = 0; v < NV; ++v) out[(long long)v * (nc + 1) + i] = 0.5 * (wa[v] + wb[v]);
}

// Features (float), Jiang-Shu weights, stencil-normalised candidates and
// target of n right-edge reconstructions.  Normalisation: (x - v2) / scale,
// scale = max - min of the stencil; a flat stencil (scale 0) gets zero
// candidates and target (it carries no information).
__global__ void __launch_bounds__(256) features_kernel(const double* __restrict__ st, const double* __restrict__ tg,
                                                       long long n, double eps, float* __restrict__ feat,
                                                       float* __restrict__ cand, float* __restrict__ tn,
                                                       float* __restrict__ ojs)
{
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const double a = st[i * 5 + 0], b = st[i * 5 + 1], c = st[i * 5 + 2], d = st[i * 5 + 3], e = st[i * 5 + 4];
    const double b0 = 13.0 / 12.0 * (a - 2 * b + c) * (a - 2 * b + c) + 0.25 * (a - 4 * b + 3 * c) * (a - 4 * b + 3 * c);
    const double b1 = 13.0 / 12.0 * (b - 2 * c + d) * (b - 2 * c + d) + 0.25 * (b - d) * (b - d);
    const double b2 = 13.0 / 12.0 * (c - 2 * d + e) * (c - 2 * d + e) + 0.25 * (3 * c - 4 * d + e) * (3 * c - 4 * d + e);
    const double S = b0 + b1 + b2 + eps;
    const double D = a - 4 * b + 6 * c - 4 * d + e;
    feat[i * 5 + 0] = (float)(b0 / S);
    feat[i * 5 + 1] = (float)(b1 / S);
    feat[i * 5 + 2] = (float)(b2 / S);
    feat[i * 5 + 3] = (float)(fabs(b0 - b2) / S);
    feat[i * 5 + 4] = (float)(D * D / (S + D * D));
    const double al0 = 0.1 / ((eps + b0) * (eps + b0)), al1 = 0.6 / ((eps + b1) * (eps + b1)),
                 al2 = 0.3 / ((eps + b2) * (eps + b2));
    const double sa = al0 + al1 + al2;
    ojs[i * 3 + 0] = (float)(al0 / sa);
    ojs[i * 3 + 1] = (float)(al1 / sa);
    ojs[i * 3 + 2] = (float)(al2 / sa);
    const double mx = fmax(fmax(fmax(a, b), fmax(c, d)), e), mn = fmin(fmin(fmin(a, b), fmin(c, d)), e);
    const double sc = mx - mn;
    const double inv = sc > 0.0 ? 1.0 / sc : 0.0;
    cand[i * 3 + 0] = (float)(((2 * a - 7 * b + 11 * c) / 6.0 - c) * inv);
    cand[i * 3 + 1] = (float)(((-b + 5 * c + 2 * d) / 6.0 - c) * inv);
    cand[i * 3 + 2] = (float)(((2 * c + 5 * d - e) / 6.0 - c) * inv);
    tn[i] = (float)((tg[i] - c) * inv);
}

// Shared form: one sample per (side, cell) of a 1D sample set laid out as
// mfx_mlp_sample_stencils writes it (stencil (side*7 + v)*ncell + i).
// Sample j = side*ncell + i gets the componentwise maximum of the seven
// variables' features and per variable its Jiang-Shu weights (base[j][v]),
// stencil-normalised candidates and target; a variable whose stencil is
// flat, or whose normalised target lies more than `tmax` from the stencil
// value, contributes zero candidates and target.
__global__ void __launch_bounds__(256) features_edge_kernel(const double* __restrict__ st,
                                                            const double* __restrict__ tg, long long ncell, double eps,
                                                            double tmax, float* __restrict__ feat,
                                                            float* __restrict__ cand, float* __restrict__ tn,
                                                            float* __restrict__ base)
{
    const long long j = (long long)blockIdx.x * 256 + threadIdx.x;
    if (j >= 2 * ncell) return;
    const long long side = j / ncell, i = j % ncell;
    double f[5] = {0, 0, 0, 0, 0};
    for (int v = 0; v < NV; ++v) {
        const long long s = (side * NV + v) * ncell + i;
        const double a = st[s * 5 + 0], b = st[s * 5 + 1], c = st[s * 5 + 2], d = st[s * 5 + 3], e = st[s * 5 + 4];
        const double b0 = 13.0 / 12.0 * (a - 2 * b + c) * (a - 2 * b + c) + 0.25 * (a - 4 * b + 3 * c) * (a - 4 * b + 3 * c);
        const double b1 = 13.0 / 12.0 * (b - 2 * c + d) * (b - 2 * c + d) + 0.25 * (b - d) * (b - d);
        const double b2 = 13.0 / 12.0 * (c - 2 * d + e) * (c - 2 * d + e) + 0.25 * (3 * c - 4 * d + e) * (3 * c - 4 * d + e);
        const double S = b0 + b1 + b2 + eps;
        const double D = a - 4 * b + 6 * c - 4 * d + e;
        const double x[5] = {b0 / S, b1 / S, b2 / S, fabs(b0 - b2) / S, D * D / (S + D * D)};
        for (int k = 0; k < 5; ++k) f[k] = fmax(f[k], x[k]);
        const double al0 = 0.1 / ((eps + b0) * (eps + b0)), al1 = 0.6 / ((eps + b1) * (eps + b1)),
                     al2 = 0.3 / ((eps + b2) * (eps + b2));
        const double sa = al0 + al1 + al2;
        float* bv = base + (j * NV + v) * 3;
        bv[0] = (float)(al0 / sa);
        bv[1] = (float)(al1 / sa);
        bv[2] = (float)(al2 / sa);
        const double mx = fmax(fmax(fmax(a, b), fmax(c, d)), e), mn = fmin(fmin(fmin(a, b), fmin(c, d)), e);
        const double sc = mx - mn;
        const double inv = sc > 0.0 ? 1.0 / sc : 0.0;
        double c0 = ((2 * a - 7 * b + 11 * c) / 6.0 - c) * inv, c1 = ((-b + 5 * c + 2 * d) / 6.0 - c) * inv,
               c2 = ((2 * c + 5 * d - e) / 6.0 - c) * inv, t = (tg[s] - c) * inv;
        if (!(fabs(t) <= tmax)) c0 = c1 = c2 = t = 0.0;
        float* cv = cand + (j * NV + v) * 3;
        cv[0] = (float)c0;
        cv[1] = (float)c1;
        cv[2] = (float)c2;
        tn[j * NV + v] = (float)t;
    }
    for (int k = 0; k < 5; ++k) feat[j * 5 + k] = (float)f[k];
}

// Float32 logits of one sample; h1, h2 hidden activations and a1, a2
// pre-activations returned for the backward pass.
__device__ __forceinline__ void mlp_logits_f32(const float* P, const float x[5], float a1[MLP_H], float a2[MLP_H],
                                               float h1[MLP_H], float h2[MLP_H], float zn[3])
{
    for (int i = 0; i < MLP_H; ++i) {
        float s = P[MLP_OFF_B1 + i];
        for (int k = 0; k < 5; ++k) s += P[MLP_OFF_W1 + i * 5 + k] * x[k];
        a1[i] = s;
        h1[i] = gelu_ref(s);
    }
    for (int i = 0; i < MLP_H; ++i) {
        float s = P[MLP_OFF_B2 + i];
        for (int j = 0; j < MLP_H; ++j) s += P[MLP_OFF_W2 + i * MLP_H + j] * h1[j];
        a2[i] = s;
        h2[i] = gelu_ref(s);
    }
    for (int i = 0; i < 3; ++i) {
        float s = P[MLP_OFF_B3 + i];
        for (int j = 0; j < MLP_H; ++j) s += P[MLP_OFF_W3 + i * MLP_H + j] * h2[j];
        zn[i] = s;
    }
}

// omega = softmax(zn + ln ojs).
__device__ __forceinline__ void softmax_base(const float zn[3], const float ojs[3], float om[3])
{
    const float z[3] = {zn[0] + logf(ojs[0]), zn[1] + logf(ojs[1]), zn[2] + logf(ojs[2])};
    const float zm = fmaxf(z[0], fmaxf(z[1], z[2]));
    const float e0 = expf(z[0] - zm), e1 = expf(z[1] - zm), e2 = expf(z[2] - zm);
    const float se = e0 + e1 + e2;
    om[0] = e0 / se;
    om[1] = e1 / se;
    om[2] = e2 / se;
}

__global__ void __launch_bounds__(256) forward_f32_kernel(const float* __restrict__ P, const float* __restrict__ feat,
                                                          const float* __restrict__ ojs, long long n,
                                                          float* __restrict__ omega)
{
    __shared__ float sP[MLP_PARAMS];
    for (int k = threadIdx.x; k < MLP_PARAMS; k += 256) sP[k] = P[k];
    __syncthreads();
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    float x[5], o[3], a1[MLP_H], a2[MLP_H], h1[MLP_H], h2[MLP_H], zn[3], om[3];
    for (int k = 0; k < 5; ++k) x[k] = feat[i * 5 + k];
    for (int k = 0; k < 3; ++k) o[k] = ojs[i * 3 + k];
    mlp_logits_f32(sP, x, a1, a2, h1, h2, zn);
    softmax_base(zn, o, om);
    for (int k = 0; k < 3; ++k) omega[i * 3 + k] = om[k];
}

// bfloat16 matrix-core forward, exactly as the sweeps evaluate it.  Every
// lane of every wave takes part (samples past n are computed on the last
// sample and not stored).
__global__ void __launch_bounds__(256) forward_mfma_kernel(const MlpNet* __restrict__ packed,
                                                           const float* __restrict__ feat,
                                                           const float* __restrict__ ojs, long long n,
                                                           float* __restrict__ omega)
{
    const MlpNet& m = *packed;
    const long long i_raw = (long long)blockIdx.x * 256 + threadIdx.x;
    const long long i = i_raw < n ? i_raw : n - 1;
    float x[5], lw[3], om[3];
    for (int k = 0; k < 5; ++k) x[k] = feat[i * 5 + k];
    for (int k = 0; k < 3; ++k) lw[k] = log2f(ojs[i * 3 + k]);
    mlp_omega(m, x, lw, om);
    if (i_raw < n)
        for (int k = 0; k < 3; ++k) omega[i * 3 + k] = om[k];
}

// Operand words of the matrix-core evaluation (layouts in learned.h), one
// thread per lane.
__global__ void __launch_bounds__(64) pack_kernel(const float* __restrict__ P, MlpNet* __restrict__ packed)
{
    const int l = threadIdx.x;
    const int row = l % 32, g = l / 32;
    bf16x4 a1;
    for (int i = 0; i < 4; ++i) {
        const int k = 4 * g + i;  // layer-1 K index: 0..4 features, 5 bias, 6..7 zero
        float w1 = 0.f;
        if (k < 5) w1 = P[MLP_OFF_W1 + row * 5 + k];
        else if (k == 5) w1 = P[MLP_OFF_B1 + row];
        a1[i] = bf16_bits(w1);
    }
    for (int s = 0; s < 2; ++s) {
        bf16x8 a2, a3[2];
        for (int i = 0; i < 8; ++i) {
            const int u = mlp_kslot_unit(s, g, i);
            a2[i] = bf16_bits(P[MLP_OFF_W2 + row * MLP_H + u]);
            // tile h keeps W3 in rows 4h .. 4h+2
            for (int h = 0; h < 2; ++h) {
                const int o = row - 4 * h;
                a3[h][i] = bf16_bits(o >= 0 && o < 3 ? P[MLP_OFF_W3 + o * MLP_H + u] : 0.f);
            }
        }
        packed->w[MW_A2 + s][l] = __builtin_bit_cast(u32x4, a2);
        for (int h = 0; h < 2; ++h) {
            const bf16x8 t = a3[h];  // (bit casts take whole objects, not elements)
            packed->w[MW_A3 + 2 * h + s][l] = __builtin_bit_cast(u32x4, t);
        }
    }
    for (int j = 0; j < 4; ++j) {
        float c[4];
        for (int i = 0; i < 4; ++i) {
            const int r = 4 * j + i;  // accumulator register r holds unit 8(r/4) + 4g + r%4
            c[i] = P[MLP_OFF_B2 + 8 * (r / 4) + 4 * g + (r % 4)];
        }
        packed->w[MW_C2 + j][l] = u32x4{__float_as_uint(c[0]), __float_as_uint(c[1]), __float_as_uint(c[2]),
                                        __float_as_uint(c[3])};
    }
    const u32x2 a1w = __builtin_bit_cast(u32x2, a1);
    packed->w[MW_A1][l] = u32x4{a1w[0], a1w[1], __float_as_uint(P[MLP_OFF_B3]), __float_as_uint(P[MLP_OFF_B3 + 1])};
    packed->w[MW_C3][l] = u32x4{__float_as_uint(P[MLP_OFF_B3 + 2]), 0u, 0u, 0u};
}

// Stage 1 of the gradient: each block of TB samples runs forward and
// backward per sample, parks the vectors the weight gradients need in LDS,
// then sums each parameter's gradient over its samples in a fixed order.
// NVAR variables share one sample's logits, each correcting its own
// Jiang-Shu weights (cand and ojs [n][NVAR][3], tn[n][NVAR]); the error
// term and the regulariser average over them.
template <int NVAR>
__global__ void __launch_bounds__(TB) grad_partial_kernel(const float* __restrict__ P, const float* __restrict__ feat,
                                                          const float* __restrict__ cand, const float* __restrict__ tn,
                                                          const float* __restrict__ ojs, long long n, float lam,
                                                          float inv_n, float* __restrict__ partial)
{
    __shared__ float sP[MLP_PARAMS];
    __shared__ float sx[TB][5], sh1[TB][MLP_H], sh2[TB][MLP_H], sd1[TB][MLP_H], sd2[TB][MLP_H], sdz[TB][3];
    __shared__ float sl[TB];
    const int t = threadIdx.x;
    for (int k = t; k < MLP_PARAMS; k += TB) sP[k] = P[k];
    __syncthreads();
    const long long i = (long long)blockIdx.x * TB + t;
    const bool valid = i < n;
    const long long ic = valid ? i : n - 1;
    float x[5], a1[MLP_H], a2[MLP_H], h1[MLP_H], h2[MLP_H], zn[3];
    for (int k = 0; k < 5; ++k) x[k] = feat[ic * 5 + k];
    mlp_logits_f32(sP, x, a1, a2, h1, h2, zn);
    float err = 0.f, reg = 0.f, dz[3] = {0.f, 0.f, 0.f};
    for (int v = 0; v < NVAR; ++v) {
        const long long iv = ic * NVAR + v;
        float o[3], om[3], dom[3];
        for (int k = 0; k < 3; ++k) o[k] = ojs[iv * 3 + k];
        softmax_base(zn, o, om);
        const float* c = cand + iv * 3;
        const float r = om[0] * c[0] + om[1] * c[1] + om[2] * c[2] - tn[iv];
        err += r * r;
        for (int k = 0; k < 3; ++k) {
            reg += (om[k] - o[k]) * (om[k] - o[k]);
            dom[k] = (2.f * inv_n / NVAR) * (r * c[k] + lam * (om[k] - o[k]));
        }
        // softmax backward of this variable; the variables share the logits
        const float sdo = dom[0] * om[0] + dom[1] * om[1] + dom[2] * om[2];
        for (int k = 0; k < 3; ++k) dz[k] += om[k] * (dom[k] - sdo);
    }
    if (!valid) dz[0] = dz[1] = dz[2] = 0.f;
    // dA2 = (W3^T dz) * gelu'(a2); dA1 = (W2^T dA2) * gelu'(a1)
    float d2[MLP_H];
    for (int j = 0; j < MLP_H; ++j) {
        float s = 0.f;
        for (int k = 0; k < 3; ++k) s += sP[MLP_OFF_W3 + k * MLP_H + j] * dz[k];
        d2[j] = s * gelu_grad(a2[j]);
    }
    for (int j = 0; j < MLP_H; ++j) {
        float s = 0.f;
        for (int k = 0; k < MLP_H; ++k) s += sP[MLP_OFF_W2 + k * MLP_H + j] * d2[k];
        sd1[t][j] = s * gelu_grad(a1[j]);
        sd2[t][j] = d2[j];
        sh1[t][j] = h1[j];
        sh2[t][j] = h2[j];
    }
    for (int k = 0; k < 5; ++k) sx[t][k] = x[k];
    for (int k = 0; k < 3; ++k) sdz[t][k] = dz[k];
    sl[t] = valid ? (err + lam * reg) * (1.f / NVAR) * inv_n : 0.f;
    __syncthreads();
    float* out = partial + (long long)blockIdx.x * GRAD_SLOTS;
    for (int p = t; p < GRAD_SLOTS; p += TB) {
        float s = 0.f;
        if (p < MLP_OFF_B1) {
            const int a = p / 5, k = p % 5;
            for (int q = 0; q < TB; ++q) s += sd1[q][a] * sx[q][k];
        } else if (p < MLP_OFF_W2) {
            const int a = p - MLP_OFF_B1;
            for (int q = 0; q < TB; ++q) s += sd1[q][a];
        } else if (p < MLP_OFF_B2) {
            const int a = (p - MLP_OFF_W2) / MLP_H, k = (p - MLP_OFF_W2) % MLP_H;
            for (int q = 0; q < TB; ++q) s += sd2[q][a] * sh1[q][k];
        } else if (p < MLP_OFF_W3) {
            const int a = p - MLP_OFF_B2;
            for (int q = 0; q < TB; ++q) s += sd2[q][a];
        } else if (p < MLP_OFF_B3) {
            const int a = (p - MLP_OFF_W3) / MLP_H, k = (p - MLP_OFF_W3) % MLP_H;
            for (int q = 0; q < TB; ++q) s += sdz[q][a] * sh2[q][k];
        } else if (p < MLP_PARAMS) {
            const int a = p - MLP_OFF_B3;
            for (int q = 0; q < TB; ++q) s += sdz[q][a];
        } else {
            for (int q = 0; q < TB; ++q) s += sl[q];
        }
        out[p] = s;
    }
}

// Stage 2: sum the block partials of each slot in block order.
__global__ void __launch_bounds__(256) grad_reduce_kernel(const float* __restrict__ partial, long long nblk,
                                                          float* __restrict__ grad, float* __restrict__ loss)
{
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= GRAD_SLOTS) return;
    float s = 0.f;
    for (long long b = 0; b < nblk; ++b) s += partial[b * GRAD_SLOTS + p];
    if (p < MLP_PARAMS)
        grad[p] = s;
    else if (loss)
        *loss = s;
}

__global__ void __launch_bounds__(256) adam_kernel(float* __restrict__ P, float* __restrict__ m, float* __restrict__ v,
                                                   const float* __restrict__ g, float lr, float b1, float b2, float eps,
                                                   float c1, float c2)
{
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= MLP_PARAMS) return;
    const float gi = g[p];
    const float mi = b1 * m[p] + (1.f - b1) * gi;
    const float vi = b2 * v[p] + (1.f - b2) * gi * gi;
    m[p] = mi;
    v[p] = vi;
    P[p] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

thread_local std::string g_mlp_error;

int err(int code, const std::string& msg)
{
    g_mlp_error = msg;
    return code;
}

int check_launch(const char* what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return err(MFX_EHIP, std::string(what) + ": " + hipGetErrorString(e));
    return MFX_OK;
}

unsigned blocks_for(long long n, int per) { return (unsigned)((n + per - 1) / per); }

}  // namespace

// Exposed to mfx.hip (same library).
namespace mfx {
int mlp_pack_on_stream(const float* params, void* packed, hipStream_t st)
{
    pack_kernel<<<1, 64, 0, st>>>(params, static_cast<MlpNet*>(packed));
    return check_launch("pack_kernel");
}
}  // namespace mfx

extern "C" {

const char* mfx_mlp_last_error(void) { return g_mlp_error.c_str(); }

size_t mfx_mlp_packed_bytes(void) { return sizeof(MlpNet); }

int mfx_mlp_sample_stencils(const mfx_grid_desc* desc, const double* q_dev, const double* face_prim_dev,
                            double* stencil_out, double* target_out, void* stream)
{
    if (!desc || !q_dev || !face_prim_dev || !stencil_out || !target_out) return err(MFX_EINVAL, "NULL argument");
    if (desc->n[1] != 1 || desc->n[2] != 1 || desc->n[0] < 1) return err(MFX_EINVAL, "sampling needs a 1D grid (n = nx,1,1)");
    if (desc->num_fluids != 0 && desc->num_fluids != 2) return err(MFX_EINVAL, "the learned weights are for two fluids");
    if (desc->bc[0][0] >= MFX_BC_REFLECTIVE || desc->bc[0][1] >= MFX_BC_REFLECTIVE)
        return err(MFX_EINVAL, "sampling takes periodic or transmissive ends");
    if (desc->faces[0] || desc->faces[1] || desc->faces[2]) return err(MFX_EINVAL, "sampling takes uniform cells");
    Grid g{};
    g.n[0] = desc->n[0];
    g.n[1] = g.n[2] = 1;
    g.bc[0][0] = desc->bc[0][0];
    g.bc[0][1] = desc->bc[0][1];
    g.G1 = 1.0 / (desc->gamma[0] - 1.0);
    g.G2 = 1.0 / (desc->gamma[1] - 1.0);
    g.P1 = desc->gamma[0] * desc->pi_inf[0] / (desc->gamma[0] - 1.0);
    g.P2 = desc->gamma[1] * desc->pi_inf[1] / (desc->gamma[1] - 1.0);
    sample_stencils_kernel<<<blocks_for(g.n[0], 256), 256, 0, (hipStream_t)stream>>>(g, q_dev, face_prim_dev,
                                                                                       stencil_out, target_out);
    return check_launch("sample_stencils_kernel");
}

int mfx_mlp_face_targets(const mfx_grid_desc* fine_desc, const double* q_fine_dev, int32_t refine, double* face_prim_out,
                         void* stream)
{
    if (!fine_desc || !q_fine_dev || !face_prim_out) return err(MFX_EINVAL, "NULL argument");
    if (fine_desc->n[1] != 1 || fine_desc->n[2] != 1) return err(MFX_EINVAL, "face targets need a 1D grid");
    if (fine_desc->num_fluids != 0 && fine_desc->num_fluids != 2)
        return err(MFX_EINVAL, "the learned weights are for two fluids");
    if (refine < 1 || fine_desc->n[0] % refine != 0) return err(MFX_EINVAL, "refine must divide nx of the fine grid");
    if (fine_desc->bc[0][0] >= MFX_BC_REFLECTIVE || fine_desc->bc[0][1] >= MFX_BC_REFLECTIVE)
        return err(MFX_EINVAL, "face targets take periodic or transmissive ends");
    if (fine_desc->faces[0] || fine_desc->faces[1] || fine_desc->faces[2])
        return err(MFX_EINVAL, "face targets take uniform cells");
    Grid g{};
    g.n[0] = fine_desc->n[0];
    g.n[1] = g.n[2] = 1;
    g.bc[0][0] = fine_desc->bc[0][0];
    g.bc[0][1] = fine_desc->bc[0][1];
    g.G1 = 1.0 / (fine_desc->gamma[0] - 1.0);
    g.G2 = 1.0 / (fine_desc->gamma[1] - 1.0);
    g.P1 = fine_desc->gamma[0] * fine_desc->pi_inf[0] / (fine_desc->gamma[0] - 1.0);
    g.P2 = fine_desc->gamma[1] * fine_desc->pi_inf[1] / (fine_desc->gamma[1] - 1.0);
    const int nc = g.n[0] / refine;
    face_targets_kernel<<<blocks_for(nc + 1, 256), 256, 0, (hipStream_t)stream>>>(g, q_fine_dev, refine, face_prim_out);
    return check_launch("face_targets_kernel");
}

int mfx_mlp_features(const double* stencils, const double* targets, int64_t n, double eps, float* feat, float* cand,
                     float* tnorm, float* omega_js, void* stream)
{
    if (n < 0 || (n > 0 && (!stencils || !targets || !feat || !cand || !tnorm || !omega_js)))
        return err(MFX_EINVAL, "bad arguments");
    if (!(eps > 0.0)) return err(MFX_EINVAL, "eps must be > 0");
    if (n == 0) return MFX_OK;
    features_kernel<<<blocks_for(n, 256), 256, 0, (hipStream_t)stream>>>(stencils, targets, n, eps, feat, cand, tnorm,
                                                                          omega_js);
    return check_launch("features_kernel");
}

int mfx_mlp_features_edge(const double* stencils, const double* targets, int64_t ncell, double eps, double tmax,
                          float* feat, float* cand, float* tnorm, float* omega_base, void* stream)
{
    if (ncell < 0 || (ncell > 0 && (!stencils || !targets || !feat || !cand || !tnorm || !omega_base)))
        return err(MFX_EINVAL, "bad arguments");
    if (!(eps > 0.0) || !(tmax > 0.0)) return err(MFX_EINVAL, "eps and tmax must be > 0");
    if (ncell == 0) return MFX_OK;
    features_edge_kernel<<<blocks_for(2 * ncell, 256), 256, 0, (hipStream_t)stream>>>(stencils, targets, ncell, eps,
                                                                                      tmax, feat, cand, tnorm,
                                                                                      omega_base);
    return check_launch("features_edge_kernel");
}

int mfx_mlp_pack(const float* params, void* packed, void* stream)
{
    if (!params || !packed) return err(MFX_EINVAL, "NULL argument");
    return mlp_pack_on_stream(params, packed, (hipStream_t)stream);
}

int mfx_mlp_forward(const float* params, const void* packed, const float* feat, const float* omega_js, int64_t n,
                    float* omega, void* stream)
{
    if (n < 0 || (n > 0 && (!feat || !omega_js || !omega))) return err(MFX_EINVAL, "bad arguments");
    if (!params == !packed) return err(MFX_EINVAL, "pass exactly one of params (float32) or packed (bfloat16 matrix cores)");
    if (n == 0) return MFX_OK;
    if (params)
        forward_f32_kernel<<<blocks_for(n, 256), 256, 0, (hipStream_t)stream>>>(params, feat, omega_js, n, omega);
    else
        forward_mfma_kernel<<<blocks_for(n, 256), 256, 0, (hipStream_t)stream>>>(
            static_cast<const MlpNet*>(packed), feat, omega_js, n, omega);
    return check_launch("mlp forward");
}

size_t mfx_mlp_grad_workspace(int64_t n)
{
    if (n <= 0) return 0;
    return sizeof(float) * (size_t)blocks_for(n, TB) * GRAD_SLOTS;
}

int mfx_mlp_loss_grad(const float* params, const float* feat, const float* cand, const float* tnorm,
                      const float* omega_js, int64_t n, int32_t nvar, float lambda, void* ws, size_t ws_bytes,
                      float* grad_out, float* loss_out, void* stream)
{
    if (n <= 0 || !params || !feat || !cand || !tnorm || !omega_js || !grad_out) return err(MFX_EINVAL, "bad arguments");
    if (nvar != 1 && nvar != NV) return err(MFX_EINVAL, "nvar must be 1 or 7");
    if (!ws || ws_bytes < mfx_mlp_grad_workspace(n)) return err(MFX_ENOMEM, "gradient workspace too small");
    const unsigned nb = blocks_for(n, TB);
    float* partial = static_cast<float*>(ws);
    if (nvar == 1)
        grad_partial_kernel<1><<<nb, TB, 0, (hipStream_t)stream>>>(params, feat, cand, tnorm, omega_js, n, lambda,
                                                                   1.0f / (float)n, partial);
    else
        grad_partial_kernel<NV><<<nb, TB, 0, (hipStream_t)stream>>>(params, feat, cand, tnorm, omega_js, n, lambda,
                                                                    1.0f / (float)n, partial);
    int rc = check_launch("grad_partial_kernel");
    if (rc) return rc;
    grad_reduce_kernel<<<blocks_for(GRAD_SLOTS, 256), 256, 0, (hipStream_t)stream>>>(partial, nb, grad_out, loss_out);
    return check_launch("grad_reduce_kernel");
}

int mfx_mlp_adam(float* params, float* m, float* v, const float* grad, int64_t step, float lr, void* stream)
{
    if (!params || !m || !v || !grad || step < 1 || !(lr > 0.f)) return err(MFX_EINVAL, "bad arguments");
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
    adam_kernel<<<blocks_for(MLP_PARAMS, 256), 256, 0, (hipStream_t)stream>>>(params, m, v, grad, lr, b1, b2, 1e-8f,
                                                                              c1, c2);
    return check_launch("adam_kernel");
}

}  // extern "C"
