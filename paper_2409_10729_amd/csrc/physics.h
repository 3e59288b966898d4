// Device-side physics of the five-equation model: mixture stiffened-gas EOS,
// WENO5 face reconstruction and the HLLC flux.  Templated on the arithmetic
// type T (double for the FP64 path, float for the mixed-precision bulk).
//
// Paper: arXiv 2409.10729, Sec. II-A (model; EOS rho E = Gamma p + Pi with
// mixture Gamma = 1/(gamma-1), Pi = gamma pi_inf/(gamma-1)) and Sec. II-B
// (HLLC after Toro from WENO5 states after Shu).
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

namespace mfx {

constexpr int NV = 7;  // alpha1 rho1, alpha2 rho2, rho u, rho v, rho w, rho E, alpha1
constexpr int MAXF = 3;               // fluids the kernels are built for
constexpr int NVMAX = 2 * MAXF + 3;   // variables of the largest model

// Per-fluid constants of the mixture rules, linear in alpha1:
//   Gamma(a) = a G1 + (1 - a) G2,  Pi(a) = a P1 + (1 - a) P2
// with G_i = 1/(gamma_i - 1) and P_i = gamma_i pi_i / (gamma_i - 1).
template <typename T>
struct Mix {
    T G1, G2, P1, P2;
    __device__ __forceinline__ T Gamma(T a) const { return a * G1 + (T(1) - a) * G2; }
    __device__ __forceinline__ T Pi(T a) const { return a * P1 + (T(1) - a) * P2; }
};

// The same rules for NF > 2 fluids (Sec. II-A's model with one continuity
// and one volume-fraction equation per component), linear in the volume
// fractions a[0 .. NF-2]; the last fluid takes 1 minus their sum:
//   Gamma = sum_i a_i G_i + (1 - sum_i a_i) G_NF, likewise Pi.
template <typename T, int NF>
struct MixN {
    T G[NF], P[NF];
    __device__ __forceinline__ T lin(const T* c, const T* a) const
    {
        T m = a[0] * c[0], s = a[0];
#pragma unroll
        for (int i = 1; i < NF - 1; ++i) {
            m = m + a[i] * c[i];
            s = s + a[i];
        }
        return m + (T(1) - s) * c[NF - 1];
    }
    __device__ __forceinline__ T Gamma(const T* a) const { return lin(G, a); }
    __device__ __forceinline__ T Pi(const T* a) const { return lin(P, a); }
};

// Variable layout of the NF-fluid model: partial densities 0 .. NF-1,
// momentum (velocity) NF .. NF+2, energy (pressure) NF+3, volume fractions
// NF+4 .. 2 NF+2 (fluids 1 .. NF-1).  Two fluids: the seven variables above.
template <int NF_>
struct Fl {
    static constexpr int NF = NF_;
    static constexpr int NV = 2 * NF + 3;
    static constexpr int IM = NF;      // x momentum / velocity
    static constexpr int IE = NF + 3;  // energy / pressure
    static constexpr int IA = NF + 4;  // first volume fraction
    static constexpr int NA = NF - 1;  // volume fractions carried
};
using Fl2 = Fl<2>;

// Conserved -> primitive for one cell, always in float64 and without
// contraction, in the operation order of the plain definition
//   u = (rho u) (1/rho), p = (rho E - rho |u|^2 / 2 - Pi) / Gamma.
// In water at 1e5 Pa the subtraction cancels about four digits
// (Pi ~ 7.8e8), so the pressure carries ~1e-7 Pa of rounding noise that
// every later stage inherits; fixing the order makes that noise the same
// as in any other implementation of the definition.
__device__ __forceinline__ void cons_to_prim(const Mix<double>& mix, const double q[NV], double w[NV])
{
#pragma clang fp contract(off)
    const double rho = q[0] + q[1];
    const double ir = 1.0 / rho;
    const double u = q[2] * ir, v = q[3] * ir, ww = q[4] * ir;
    const double ke = 0.5 * rho * (u * u + v * v + ww * ww);
    const double a1 = q[6];
    const double G = a1 * mix.G1 + (1.0 - a1) * mix.G2;
    const double P = a1 * mix.P1 + (1.0 - a1) * mix.P2;
    w[0] = q[0];
    w[1] = q[1];
    w[2] = u;
    w[3] = v;
    w[4] = ww;
    w[5] = (q[5] - ke - P) / G;
    w[6] = a1;
}

// WENO5 with Jiang-Shu weights for cell c from w_{c-2..c+2} = a..e: both
// edge values from one set of smoothness indicators.  right is the value at
// c+1/2 (linear weights 1/10, 6/10, 3/10 on the stencils {c-2..c},
// {c-1..c+1}, {c..c+2}), left the value at c-1/2 (weights 3/10, 6/10, 1/10).
//
// The weights alpha_k = d_k / (eps + beta_k)^2 are scaled by the product of
// the three (eps + beta)^2 so each edge needs one division:
//   value = sum_k d_k t_k p_k / sum_k d_k t_k,  t_0 = s1 s2, t_1 = s0 s2, t_2 = s0 s1.
// In float64 the products stay far from overflow for physical data
// (beta <= 1e20 gives t <= 1e80).
// Quotient for the reconstruction and Riemann steps (not the conserved ->
// primitive inversion, the stage update or the CFL reduction, which keep
// IEEE division).  Denominators here are nonzero and in the normal range.
// double: the hardware reciprocal refined by two Newton steps, times the
// numerator (within about 1.5 ulp of the rounded quotient; 6 instructions
// against 10 for the IEEE sequence).  float: numerator times the hardware
// reciprocal (1 ulp), which the float form's accuracy bound absorbs.
template <typename T>
__device__ __forceinline__ T qdiv(T a, T b);
template <>
__device__ __forceinline__ double qdiv<double>(double a, double b)
{
    double r = __builtin_amdgcn_rcp(b);
    double e = fma(-b, r, 1.0);
    r = fma(r, e, r);
    e = fma(-b, r, 1.0);
    r = fma(r, e, r);
    return a * r;
}
template <>
__device__ __forceinline__ float qdiv<float>(float a, float b)
{
    return a * __builtin_amdgcn_rcpf(b);
}

// Square root of a sound speed squared in the float form.
template <typename T>
__device__ __forceinline__ T qsqrt(T x);
template <>
__device__ __forceinline__ float qsqrt<float>(float x)
{
    return sqrtf(x);
}

template <typename T>
__device__ __forceinline__ void weno5_js(T a, T b, T c, T d, T e, T eps, T& left, T& right)
{
    // beta_k = (13/12) q_k^2 + (1/4) h_k^2 with the factors taken into the
    // differences (sqrt(13/12) q_k and h_k / 2), so each eps + beta_k is two
    // fused multiply-adds
    const T c13 = T(1.0408329997330663);  // sqrt(13/12)
    const T q0 = c13 * (a - T(2) * b + c), h0 = T(0.5) * a - T(2) * b + T(1.5) * c;
    const T q1 = c13 * (b - T(2) * c + d), h1 = T(0.5) * (b - d);
    const T q2 = c13 * (c - T(2) * d + e), h2 = T(1.5) * c - T(2) * d + T(0.5) * e;
    T s0 = fma(q0, q0, fma(h0, h0, eps));
    T s1 = fma(q1, q1, fma(h1, h1, eps));
    T s2 = fma(q2, q2, fma(h2, h2, eps));
    s0 *= s0;
    s1 *= s1;
    s2 *= s2;
    const T t0 = s1 * s2, t1 = s0 * s2, t2 = s0 * s1;

    // six times the candidate values
    const T r0 = T(2) * a - T(7) * b + T(11) * c;
    const T r1 = -b + T(5) * c + T(2) * d;
    const T r2 = T(2) * c + T(5) * d - e;
    const T l0 = -a + T(5) * b + T(2) * c;
    const T l1 = T(2) * b + T(5) * c - d;
    const T l2 = T(11) * c - T(7) * d + T(2) * e;

    // linear weights times ten (1, 6, 3 and 3, 6, 1: exact, and the common
    // factor cancels in each quotient)
    const T u0 = T(3) * t0, u1 = T(6) * t1, u2 = T(3) * t2;
    // one refined reciprocal of Dr Dl serves both quotients (the weights'
    // products stay far inside the float64 range: (eps + beta)^2 products up
    // to ~1e90 for pressure jumps of 1e11, down to ~1e-24 on flat data);
    // the candidates' factor 6 is applied once, to the reciprocal
    const T Nr = t0 * r0 + u1 * r1 + u2 * r2, Dr = t0 + u1 + u2;
    const T Nl = u0 * l0 + u1 * l1 + t2 * l2, Dl = u0 + u1 + t2;
    const T inv = qdiv(T(1.0 / 6.0), Dr * Dl);
    right = Nr * (Dl * inv);
    left = Nl * (Dr * inv);
}

// Same weights in the overflow-free ratio form for float32, where the
// product form overflows for pressure jumps of 1e9:
//   alpha_k ~ d_k ((eps + beta_min) / (eps + beta_k))^2.
__device__ __forceinline__ void weno5_js_ratio(float a, float b, float c, float d, float e, float eps,
                                               float& left, float& right)
{
    // indicators as in weno5_js (factors taken into the differences)
    const float c13 = 1.04083300f;  // sqrt(13/12)
    const float q0 = c13 * (a - 2.f * b + c), h0 = 0.5f * a - 2.f * b + 1.5f * c;
    const float q1 = c13 * (b - 2.f * c + d), h1 = 0.5f * (b - d);
    const float q2 = c13 * (c - 2.f * d + e), h2 = 1.5f * c - 2.f * d + 0.5f * e;
    const float s0 = fmaf(q0, q0, fmaf(h0, h0, eps));
    const float s1 = fmaf(q1, q1, fmaf(h1, h1, eps));
    const float s2 = fmaf(q2, q2, fmaf(h2, h2, eps));
    const float smin = fminf(s0, fminf(s1, s2));
    float x0 = qdiv(smin, s0), x1 = qdiv(smin, s1), x2 = qdiv(smin, s2);
    x0 *= x0;
    x1 *= x1;
    x2 *= x2;
    const float r0 = 2.f * a - 7.f * b + 11.f * c;
    const float r1 = -b + 5.f * c + 2.f * d;
    const float r2 = 2.f * c + 5.f * d - e;
    const float l0 = -a + 5.f * b + 2.f * c;
    const float l1 = 2.f * b + 5.f * c - d;
    const float l2 = 11.f * c - 7.f * d + 2.f * e;
    // linear weights times ten, as in weno5_js
    const float u0 = 3.f * x0, u1 = 6.f * x1, u2 = 3.f * x2;
    right = qdiv(x0 * r0 + u1 * r1 + u2 * r2, 6.f * (x0 + u1 + u2));
    left = qdiv(u0 * l0 + u1 * l1 + x2 * l2, 6.f * (u0 + u1 + x2));
}

// WENO5 in the compute type: the product form in float64, the ratio form
// in float32.
template <typename T>
__device__ __forceinline__ void weno5(T a, T b, T c, T d, T e, T eps, T& left, T& right);
template <>
__device__ __forceinline__ void weno5<double>(double a, double b, double c, double d, double e, double eps,
                                              double& left, double& right)
{
    weno5_js<double>(a, b, c, d, e, eps, left, right);
}
template <>
__device__ __forceinline__ void weno5<float>(float a, float b, float c, float d, float e, float eps, float& left,
                                             float& right)
{
    weno5_js_ratio(a, b, c, d, e, eps, left, right);
}

// WENO5 with WENO-Z weights (Borges, Carmona, Costa & Don, J. Comput. Phys.
// 227, 2008; exponent 1), a comparison form for the learned weights: the
// same candidates and indicators as Jiang-Shu, weights
// alpha_k = d_k (1 + tau / (beta_k + eps)) with tau = |beta_0 - beta_2|.
// float64: alpha_k scaled by the product of the three (beta + eps), one
// division per edge: alpha_k ~ d_k (e_k + tau) prod_{j != k} e_j.
__device__ __forceinline__ void weno5z_prod(double a, double b, double c, double d, double e, double eps,
                                            double& left, double& right)
{
    const double k13 = 13.0 / 12.0;
    const double q0 = a - 2.0 * b + c, h0 = a - 4.0 * b + 3.0 * c;
    const double q1 = b - 2.0 * c + d, h1 = b - d;
    const double q2 = c - 2.0 * d + e, h2 = 3.0 * c - 4.0 * d + e;
    const double b0 = k13 * q0 * q0 + 0.25 * h0 * h0;
    const double b1 = k13 * q1 * q1 + 0.25 * h1 * h1;
    const double b2 = k13 * q2 * q2 + 0.25 * h2 * h2;
    const double tau = fabs(b0 - b2);
    const double e0 = b0 + eps, e1 = b1 + eps, e2 = b2 + eps;
    const double g0 = (e0 + tau) * (e1 * e2), g1 = (e1 + tau) * (e0 * e2), g2 = (e2 + tau) * (e0 * e1);
    // six times the candidate values
    const double r0 = 2.0 * a - 7.0 * b + 11.0 * c;
    const double r1 = -b + 5.0 * c + 2.0 * d;
    const double r2 = 2.0 * c + 5.0 * d - e;
    const double l0 = -a + 5.0 * b + 2.0 * c;
    const double l1 = 2.0 * b + 5.0 * c - d;
    const double l2 = 11.0 * c - 7.0 * d + 2.0 * e;
    const double wr0 = 0.1 * g0, wr1 = 0.6 * g1, wr2 = 0.3 * g2;
    const double wl0 = 0.3 * g0, wl1 = 0.6 * g1, wl2 = 0.1 * g2;
    right = qdiv(wr0 * r0 + wr1 * r1 + wr2 * r2, 6.0 * (wr0 + wr1 + wr2));
    left = qdiv(wl0 * l0 + wl1 * l1 + wl2 * l2, 6.0 * (wl0 + wl1 + wl2));
}

// float32: the weights as defined (three reciprocal quotients), which cannot
// overflow: 1 <= 1 + tau / (beta + eps) <= 1 + tau / eps.
__device__ __forceinline__ void weno5z_direct(float a, float b, float c, float d, float e, float eps, float& left,
                                              float& right)
{
    const float k13 = 13.0f / 12.0f;
    const float q0 = a - 2.f * b + c, h0 = a - 4.f * b + 3.f * c;
    const float q1 = b - 2.f * c + d, h1 = b - d;
    const float q2 = c - 2.f * d + e, h2 = 3.f * c - 4.f * d + e;
    const float b0 = k13 * q0 * q0 + 0.25f * h0 * h0;
    const float b1 = k13 * q1 * q1 + 0.25f * h1 * h1;
    const float b2 = k13 * q2 * q2 + 0.25f * h2 * h2;
    const float tau = fabsf(b0 - b2);
    const float z0 = 1.f + qdiv(tau, b0 + eps), z1 = 1.f + qdiv(tau, b1 + eps), z2 = 1.f + qdiv(tau, b2 + eps);
    const float r0 = 2.f * a - 7.f * b + 11.f * c;
    const float r1 = -b + 5.f * c + 2.f * d;
    const float r2 = 2.f * c + 5.f * d - e;
    const float l0 = -a + 5.f * b + 2.f * c;
    const float l1 = 2.f * b + 5.f * c - d;
    const float l2 = 11.f * c - 7.f * d + 2.f * e;
    const float wr0 = 0.1f * z0, wr1 = 0.6f * z1, wr2 = 0.3f * z2;
    const float wl0 = 0.3f * z0, wl1 = 0.6f * z1, wl2 = 0.1f * z2;
    right = qdiv(wr0 * r0 + wr1 * r1 + wr2 * r2, 6.f * (wr0 + wr1 + wr2));
    left = qdiv(wl0 * l0 + wl1 * l1 + wl2 * l2, 6.f * (wl0 + wl1 + wl2));
}

template <typename T>
__device__ __forceinline__ void weno5z(T a, T b, T c, T d, T e, T eps, T& left, T& right);
template <>
__device__ __forceinline__ void weno5z<double>(double a, double b, double c, double d, double e, double eps,
                                               double& left, double& right)
{
    weno5z_prod(a, b, c, d, e, eps, left, right);
}
template <>
__device__ __forceinline__ void weno5z<float>(float a, float b, float c, float d, float e, float eps, float& left,
                                              float& right)
{
    weno5z_direct(a, b, c, d, e, eps, left, right);
}

// WENO3 with Jiang-Shu weights (the third-order reconstruction named
// beside WENO5 in Sec. II-B) for cell c from w_{c-1..c+1} = a, b, c:
// candidates on {c-1, c} and {c, c+1}; right edge (c+1/2) with linear
// weights 1/3, 2/3 and candidates (3b - a)/2, (b + c)/2; left edge (c-1/2)
// with 2/3, 1/3 and (a + b)/2, (3b - c)/2; indicators (b - a)^2, (c - b)^2.
// float64: weights scaled by the product of the two (eps + beta)^2, one
// division per edge.
__device__ __forceinline__ void weno3_js(double a, double b, double c, double eps, double& left, double& right)
{
    const double d0 = b - a, d1 = c - b;
    double s0 = eps + d0 * d0, s1 = eps + d1 * d1;
    s0 *= s0;
    s1 *= s1;
    // right: (s1 (3b - a) + 2 s0 (b + c)) / (2 (s1 + 2 s0))
    right = qdiv(s1 * (3.0 * b - a) + 2.0 * s0 * (b + c), 2.0 * (s1 + 2.0 * s0));
    // left: (2 s1 (a + b) + s0 (3b - c)) / (2 (2 s1 + s0))
    left = qdiv(2.0 * s1 * (a + b) + s0 * (3.0 * b - c), 2.0 * (2.0 * s1 + s0));
}

// float32: the ratio form, alpha_k ~ d_k ((eps + beta_min) / (eps + beta_k))^2.
__device__ __forceinline__ void weno3_ratio(float a, float b, float c, float eps, float& left, float& right)
{
    const float d0 = b - a, d1 = c - b;
    const float s0 = eps + d0 * d0, s1 = eps + d1 * d1;
    const float m = fminf(s0, s1);
    float x0 = qdiv(m, s0), x1 = qdiv(m, s1);
    x0 *= x0;
    x1 *= x1;
    right = qdiv(x0 * (3.f * b - a) + 2.f * x1 * (b + c), 2.f * (x0 + 2.f * x1));
    left = qdiv(2.f * x0 * (a + b) + x1 * (3.f * b - c), 2.f * (2.f * x0 + x1));
}

template <typename T>
__device__ __forceinline__ void weno3(T a, T b, T c, T eps, T& left, T& right);
template <>
__device__ __forceinline__ void weno3<double>(double a, double b, double c, double eps, double& left, double& right)
{
    weno3_js(a, b, c, eps, left, right);
}
template <>
__device__ __forceinline__ void weno3<float>(float a, float b, float c, float eps, float& left, float& right)
{
    weno3_ratio(a, b, c, eps, left, right);
}

// WENO5 with Jiang-Shu weights on cells of unequal widths (a direction of the
// structured mesh refined locally by a hyperbolic tangent, Sec. III-A), for
// cell c from w_{c-2..c+2} = v[0..4].  In the cell's own coordinate
// xi = (x - x_c) / h_c (the cell spans [-1/2, 1/2]) candidate k (cells
// c-2+k .. c+k) is the quadratic A_k + B_k xi + C_k xi^2 whose averages over
// its three cells are their values; A, B, C are linear in those values, with
// coefficients that depend only on the widths (NuCoef, one set per stencil
// position, computed on the host).  Indicator beta_k = B_k^2 + 13/3 C_k^2
// (h_c times the integral of p'^2 plus h_c^3 times that of p''^2 over the
// cell); the ideal weights of each edge (dr at xi = 1/2, dl at xi = -1/2)
// combine the three candidates into the quartic through all five averages.
// On equal widths this is weno5_js up to rounding.
template <typename T>
struct NuCoef {
    T a[3][3], b[3][3], c[3][3];  // [candidate][value of cell c-2+k+i]
    T dr[3], dl[3];
};

// float64: the weights scaled by the product of the three (eps + beta)^2 as
// in weno5_js; float32: the ratio form of weno5_js_ratio.
template <typename T>
__device__ __forceinline__ void weno5_nu(const NuCoef<T>& K, const T v[5], T eps, T& left, T& right)
{
    T pr[3], pl[3], s[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const T A = K.a[k][0] * v[k] + K.a[k][1] * v[k + 1] + K.a[k][2] * v[k + 2];
        const T B = K.b[k][0] * v[k] + K.b[k][1] * v[k + 1] + K.b[k][2] * v[k + 2];
        const T C = K.c[k][0] * v[k] + K.c[k][1] * v[k + 1] + K.c[k][2] * v[k + 2];
        s[k] = eps + (B * B + T(13.0 / 3.0) * (C * C));
        pr[k] = A + T(0.5) * B + T(0.25) * C;
        pl[k] = A - T(0.5) * B + T(0.25) * C;
    }
    T t[3];
    if constexpr (sizeof(T) == sizeof(double)) {
        const T s0 = s[0] * s[0], s1 = s[1] * s[1], s2 = s[2] * s[2];
        t[0] = s1 * s2;
        t[1] = s0 * s2;
        t[2] = s0 * s1;
    } else {
        const T m = fminf(s[0], fminf(s[1], s[2]));
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const T x = qdiv(m, s[k]);
            t[k] = x * x;
        }
    }
    const T wr0 = K.dr[0] * t[0], wr1 = K.dr[1] * t[1], wr2 = K.dr[2] * t[2];
    const T wl0 = K.dl[0] * t[0], wl1 = K.dl[1] * t[1], wl2 = K.dl[2] * t[2];
    right = qdiv(wr0 * pr[0] + wr1 * pr[1] + wr2 * pr[2], wr0 + wr1 + wr2);
    left = qdiv(wl0 * pl[0] + wl1 * pl[1] + wl2 * pl[2], wl0 + wl1 + wl2);
}

// FP64 HLLC in the plain definition's operation order, without contraction
// and with IEEE division and square root.  The star-state flux
// F = F_K + s (U*_K - U_K) subtracts energies of size Pi (7.8e8 in water)
// and multiplies the difference by a wave speed of ~1.6e3, which amplifies
// rounding in U* about a thousand-fold; evaluated exactly as the definition
// states, that amplified noise is the same in every implementation of it.
template <int DIR>
__device__ __forceinline__ void hllc_fp64(const Mix<double>& mix, const double wl[NV], const double wr[NV],
                                          double F[NV], double& uf)
{
#pragma clang fp contract(off)
    const double rl = wl[0] + wl[1], rr = wr[0] + wr[1];
    const double pl = wl[5], pr = wr[5];
    const double unl = wl[2 + DIR], unr = wr[2 + DIR];
    // mixture rules written out (Mix's members may be contracted)
    const double Gl = wl[6] * mix.G1 + (1.0 - wl[6]) * mix.G2, Gr = wr[6] * mix.G1 + (1.0 - wr[6]) * mix.G2;
    const double Pl = wl[6] * mix.P1 + (1.0 - wl[6]) * mix.P2, Pr = wr[6] * mix.P1 + (1.0 - wr[6]) * mix.P2;
    const double El = Gl * pl + Pl + 0.5 * rl * (wl[2] * wl[2] + wl[3] * wl[3] + wl[4] * wl[4]);
    const double Er = Gr * pr + Pr + 0.5 * rr * (wr[2] * wr[2] + wr[3] * wr[3] + wr[4] * wr[4]);
    const double cl = sqrt(((Gl + 1.0) * pl + Pl) / (Gl * rl));
    const double cr = sqrt(((Gr + 1.0) * pr + Pr) / (Gr * rr));

    const double SL = fmin(unl - cl, unr - cr);
    const double SR = fmax(unl + cl, unr + cr);
    const double Ss = (pr - pl + rl * unl * (SL - unl) - rr * unr * (SR - unr)) / (rl * (SL - unl) - rr * (SR - unr));

    const bool left = Ss >= 0.0;
    double w[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) w[v] = left ? wl[v] : wr[v];
    const double rho = left ? rl : rr;
    const double p = left ? pl : pr;
    const double un = left ? unl : unr;
    const double E = left ? El : Er;
    const double S = left ? SL : SR;
    const double s = left ? fmin(0.0, SL) : fmax(0.0, SR);

    double U[NV], Us[NV], Fk[NV];
    U[0] = w[0];
    U[1] = w[1];
    U[2] = rho * w[2];
    U[3] = rho * w[3];
    U[4] = rho * w[4];
    U[5] = E;
    U[6] = w[6];
#pragma unroll
    for (int v = 0; v < NV; ++v) Fk[v] = U[v] * un;
    Fk[2 + DIR] = Fk[2 + DIR] + p;
    Fk[5] = (E + p) * un;

    // one quotient for xi and the star energy's pressure term, whose
    // xi (S* - u) p / (S - u) equals (S* - u) p / (S - S*)
    const double inv = 1.0 / (S - Ss);
    const double xi = (S - un) * inv;
    Us[0] = xi * w[0];
    Us[1] = xi * w[1];
    Us[2] = xi * (rho * w[2]);
    Us[3] = xi * (rho * w[3]);
    Us[4] = xi * (rho * w[4]);
    Us[2 + DIR] = xi * (rho * Ss);
    Us[5] = xi * (E + (Ss - un) * (rho * Ss)) + (Ss - un) * (p * inv);
    Us[6] = xi * w[6];
#pragma unroll
    for (int v = 0; v < NV; ++v) F[v] = Fk[v] + s * (Us[v] - U[v]);
    uf = un + s * (xi - 1.0);
}

// The same flux in the float form: contraction allowed, reciprocal quotients.
template <int DIR, typename T>
__device__ __forceinline__ void hllc_fast(const Mix<T>& mix, const T wl[NV], const T wr[NV], T F[NV], T& uf)
{
    const T rl = wl[0] + wl[1], rr = wr[0] + wr[1];
    const T pl = wl[5], pr = wr[5];
    const T unl = wl[2 + DIR], unr = wr[2 + DIR];
    const T Gl = mix.Gamma(wl[6]), Gr = mix.Gamma(wr[6]);
    const T Pl = mix.Pi(wl[6]), Pr = mix.Pi(wr[6]);
    const T El = Gl * pl + Pl + T(0.5) * rl * (wl[2] * wl[2] + wl[3] * wl[3] + wl[4] * wl[4]);
    const T Er = Gr * pr + Pr + T(0.5) * rr * (wr[2] * wr[2] + wr[3] * wr[3] + wr[4] * wr[4]);
    const T cl = qsqrt(qdiv((Gl + T(1)) * pl + Pl, Gl * rl));
    const T cr = qsqrt(qdiv((Gr + T(1)) * pr + Pr, Gr * rr));

    const T SL = fmin(unl - cl, unr - cr);
    const T SR = fmax(unl + cl, unr + cr);
    const T ml = rl * (SL - unl), mr = rr * (SR - unr);
    const T Ss = qdiv(pr - pl + ml * unl - mr * unr, ml - mr);

    const bool left = Ss >= T(0);
    T w[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) w[v] = left ? wl[v] : wr[v];
    const T rho = left ? rl : rr;
    const T p = left ? pl : pr;
    const T un = left ? unl : unr;
    const T E = left ? El : Er;
    const T S = left ? SL : SR;
    const T s = left ? fmin(T(0), SL) : fmax(T(0), SR);

    const T inv = qdiv(T(1), S - Ss);  // as in the float64 flux: one quotient
    const T xi = (S - un) * inv;

    T U[NV], Us[NV];
    U[0] = w[0];
    U[1] = w[1];
    U[2] = rho * w[2];
    U[3] = rho * w[3];
    U[4] = rho * w[4];
    U[5] = E;
    U[6] = w[6];
#pragma unroll
    for (int v = 0; v < NV; ++v) Us[v] = xi * U[v];
    Us[2 + DIR] = xi * (rho * Ss);
    Us[5] = xi * (E + (Ss - un) * (rho * Ss)) + (Ss - un) * (p * inv);

    T Fk[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) Fk[v] = U[v] * un;
    Fk[2 + DIR] += p;
    Fk[5] = (E + p) * un;
#pragma unroll
    for (int v = 0; v < NV; ++v) F[v] = Fk[v] + s * (Us[v] - U[v]);
    uf = un + s * (xi - T(1));
}

// HLLC flux across a face normal to direction DIR (Toro 2009, Sec. 10.4),
// Davis wave-speed estimates, extended to the five-equation model: each
// partial density and alpha1 are scaled by xi = (S_K - u_K)/(S_K - S*) in
// the star state.  Also returns the face velocity u_f used for div(u) in
// the alpha1 source; the side of the contact is chosen by S* >= 0 (ties go
// left), and only that side's star state is formed.
template <int DIR, typename T>
__device__ __forceinline__ void hllc(const Mix<T>& mix, const T wl[NV], const T wr[NV], T F[NV], T& uf)
{
    if constexpr (sizeof(T) == sizeof(double))
        hllc_fp64<DIR>(mix, wl, wr, F, uf);
    else
        hllc_fast<DIR, T>(mix, wl, wr, F, uf);
}

// ---- the NF-fluid model (NF > 2): the same definitions with every partial
// density and volume fraction (two fluids use the functions above)

template <class F>
using MixOf = typename std::conditional<F::NF == 2, Mix<double>, MixN<double, F::NF>>::type;

template <int NF>
__device__ __forceinline__ double density_n(const double* x)
{
    double rho = x[0];
#pragma unroll
    for (int i = 1; i < NF; ++i) rho = rho + x[i];
    return rho;
}

// Conserved -> primitive, float64, plain operation order, no contraction.
template <int NF>
__device__ __forceinline__ void cons_to_prim_n(const MixN<double, NF>& mix, const double* q, double* w)
{
#pragma clang fp contract(off)
    using F = Fl<NF>;
    const double rho = density_n<NF>(q);
    const double ir = 1.0 / rho;
    const double u = q[F::IM] * ir, v = q[F::IM + 1] * ir, ww = q[F::IM + 2] * ir;
    const double ke = 0.5 * rho * (u * u + v * v + ww * ww);
    double m = q[F::IA] * mix.G[0], s = q[F::IA];
    double mp = q[F::IA] * mix.P[0];
#pragma unroll
    for (int i = 1; i < NF - 1; ++i) {
        m = m + q[F::IA + i] * mix.G[i];
        mp = mp + q[F::IA + i] * mix.P[i];
        s = s + q[F::IA + i];
    }
    const double G = m + (1.0 - s) * mix.G[NF - 1];
    const double P = mp + (1.0 - s) * mix.P[NF - 1];
#pragma unroll
    for (int i = 0; i < F::NV; ++i) w[i] = q[i];
    w[F::IM] = u;
    w[F::IM + 1] = v;
    w[F::IM + 2] = ww;
    w[F::IE] = (q[F::IE] - ke - P) / G;
}

// HLLC of the NF-fluid model: every partial density and volume fraction is
// scaled by xi in the star state.  float64: the plain definition's operation
// order, no contraction, IEEE division and square root (as hllc_fp64).
template <int DIR, int NF>
__device__ __forceinline__ void hllc_fp64_n(const MixN<double, NF>& mix, const double* wl, const double* wr, double* F,
                                            double& uf)
{
#pragma clang fp contract(off)
    using L = Fl<NF>;
    const double rl = density_n<NF>(wl), rr = density_n<NF>(wr);
    const double pl = wl[L::IE], pr = wr[L::IE];
    const double unl = wl[L::IM + DIR], unr = wr[L::IM + DIR];
    double Gl = wl[L::IA] * mix.G[0], Gr = wr[L::IA] * mix.G[0], Pl = wl[L::IA] * mix.P[0], Pr = wr[L::IA] * mix.P[0];
    double sl = wl[L::IA], sr = wr[L::IA];
#pragma unroll
    for (int i = 1; i < NF - 1; ++i) {
        Gl = Gl + wl[L::IA + i] * mix.G[i];
        Gr = Gr + wr[L::IA + i] * mix.G[i];
        Pl = Pl + wl[L::IA + i] * mix.P[i];
        Pr = Pr + wr[L::IA + i] * mix.P[i];
        sl = sl + wl[L::IA + i];
        sr = sr + wr[L::IA + i];
    }
    Gl = Gl + (1.0 - sl) * mix.G[NF - 1];
    Gr = Gr + (1.0 - sr) * mix.G[NF - 1];
    Pl = Pl + (1.0 - sl) * mix.P[NF - 1];
    Pr = Pr + (1.0 - sr) * mix.P[NF - 1];
    const int m = L::IM;
    const double El = Gl * pl + Pl + 0.5 * rl * (wl[m] * wl[m] + wl[m + 1] * wl[m + 1] + wl[m + 2] * wl[m + 2]);
    const double Er = Gr * pr + Pr + 0.5 * rr * (wr[m] * wr[m] + wr[m + 1] * wr[m + 1] + wr[m + 2] * wr[m + 2]);
    const double cl = sqrt(((Gl + 1.0) * pl + Pl) / (Gl * rl));
    const double cr = sqrt(((Gr + 1.0) * pr + Pr) / (Gr * rr));

    const double SL = fmin(unl - cl, unr - cr);
    const double SR = fmax(unl + cl, unr + cr);
    const double Ss = (pr - pl + rl * unl * (SL - unl) - rr * unr * (SR - unr)) / (rl * (SL - unl) - rr * (SR - unr));

    const bool left = Ss >= 0.0;
    double w[L::NV];
#pragma unroll
    for (int v = 0; v < L::NV; ++v) w[v] = left ? wl[v] : wr[v];
    const double rho = left ? rl : rr;
    const double p = left ? pl : pr;
    const double un = left ? unl : unr;
    const double E = left ? El : Er;
    const double S = left ? SL : SR;
    const double s = left ? fmin(0.0, SL) : fmax(0.0, SR);

    double U[L::NV], Us[L::NV], Fk[L::NV];
#pragma unroll
    for (int v = 0; v < L::NV; ++v) U[v] = w[v];
    U[m] = rho * w[m];
    U[m + 1] = rho * w[m + 1];
    U[m + 2] = rho * w[m + 2];
    U[L::IE] = E;
#pragma unroll
    for (int v = 0; v < L::NV; ++v) Fk[v] = U[v] * un;
    Fk[m + DIR] = Fk[m + DIR] + p;
    Fk[L::IE] = (E + p) * un;

    // one quotient for xi and the star energy's pressure term, whose
    // xi (S* - u) p / (S - u) equals (S* - u) p / (S - S*)
    const double inv = 1.0 / (S - Ss);
    const double xi = (S - un) * inv;
#pragma unroll
    for (int v = 0; v < L::NV; ++v) Us[v] = xi * w[v];
    Us[m] = xi * (rho * w[m]);
    Us[m + 1] = xi * (rho * w[m + 1]);
    Us[m + 2] = xi * (rho * w[m + 2]);
    Us[m + DIR] = xi * (rho * Ss);
    Us[L::IE] = xi * (E + (Ss - un) * (rho * Ss)) + (Ss - un) * (p * inv);
#pragma unroll
    for (int v = 0; v < L::NV; ++v) F[v] = Fk[v] + s * (Us[v] - U[v]);
    uf = un + s * (xi - 1.0);
}

// The same flux in the float form (contraction allowed, reciprocal quotients).
template <int DIR, typename T, int NF>
__device__ __forceinline__ void hllc_fast_n(const MixN<T, NF>& mix, const T* wl, const T* wr, T* F, T& uf)
{
    using L = Fl<NF>;
    T rl = wl[0], rr = wr[0];
#pragma unroll
    for (int i = 1; i < NF; ++i) {
        rl += wl[i];
        rr += wr[i];
    }
    const T pl = wl[L::IE], pr = wr[L::IE];
    const T unl = wl[L::IM + DIR], unr = wr[L::IM + DIR];
    const T Gl = mix.Gamma(wl + L::IA), Gr = mix.Gamma(wr + L::IA);
    const T Pl = mix.Pi(wl + L::IA), Pr = mix.Pi(wr + L::IA);
    const int m = L::IM;
    const T El = Gl * pl + Pl + T(0.5) * rl * (wl[m] * wl[m] + wl[m + 1] * wl[m + 1] + wl[m + 2] * wl[m + 2]);
    const T Er = Gr * pr + Pr + T(0.5) * rr * (wr[m] * wr[m] + wr[m + 1] * wr[m + 1] + wr[m + 2] * wr[m + 2]);
    const T cl = qsqrt(qdiv((Gl + T(1)) * pl + Pl, Gl * rl));
    const T cr = qsqrt(qdiv((Gr + T(1)) * pr + Pr, Gr * rr));

    const T SL = fmin(unl - cl, unr - cr);
    const T SR = fmax(unl + cl, unr + cr);
    const T ml = rl * (SL - unl), mr = rr * (SR - unr);
    const T Ss = qdiv(pr - pl + ml * unl - mr * unr, ml - mr);

    const bool left = Ss >= T(0);
    T w[L::NV];
#pragma unroll
    for (int v = 0; v < L::NV; ++v) w[v] = left ? wl[v] : wr[v];
    const T rho = left ? rl : rr;
    const T p = left ? pl : pr;
    const T un = left ? unl : unr;
    const T E = left ? El : Er;
    const T S = left ? SL : SR;
    const T s = left ? fmin(T(0), SL) : fmax(T(0), SR);

    const T inv = qdiv(T(1), S - Ss);  // as in the float64 flux: one quotient
    const T xi = (S - un) * inv;

    T U[L::NV], Us[L::NV];
#pragma unroll
    for (int v = 0; v < L::NV; ++v) U[v] = w[v];
    U[m] = rho * w[m];
    U[m + 1] = rho * w[m + 1];
    U[m + 2] = rho * w[m + 2];
    U[L::IE] = E;
#pragma unroll
    for (int v = 0; v < L::NV; ++v) Us[v] = xi * U[v];
    Us[m + DIR] = xi * (rho * Ss);
    Us[L::IE] = xi * (E + (Ss - un) * (rho * Ss)) + (Ss - un) * (p * inv);

    T Fk[L::NV];
#pragma unroll
    for (int v = 0; v < L::NV; ++v) Fk[v] = U[v] * un;
    Fk[m + DIR] += p;
    Fk[L::IE] = (E + p) * un;
#pragma unroll
    for (int v = 0; v < L::NV; ++v) F[v] = Fk[v] + s * (Us[v] - U[v]);
    uf = un + s * (xi - T(1));
}

// Model-generic entry points: two fluids take the functions above, more
// fluids the _n forms.
template <class F>
__device__ __forceinline__ void cons_to_prim_f(const MixOf<F>& mix, const double* q, double* w)
{
    if constexpr (F::NF == 2)
        cons_to_prim(mix, q, w);
    else
        cons_to_prim_n<F::NF>(mix, q, w);
}

template <int DIR, typename T, class F>
__device__ __forceinline__ void hllc_f(const typename std::conditional<F::NF == 2, Mix<T>, MixN<T, F::NF>>::type& mix,
                                       const T* wl, const T* wr, T* Fo, T& uf)
{
    if constexpr (F::NF == 2) {
        hllc<DIR, T>(mix, wl, wr, Fo, uf);
    } else if constexpr (sizeof(T) == sizeof(double)) {
        hllc_fp64_n<DIR, F::NF>(mix, wl, wr, Fo, uf);
    } else {
        hllc_fast_n<DIR, T, F::NF>(mix, wl, wr, Fo, uf);
    }
}

}  // namespace mfx
