// Learned WENO weights: a 5-32-32-3 MLP (GELU) maps scale-free smoothness
// features of a 5-cell stencil to three logits z that correct the Jiang-Shu
// weights of the WENO5 candidates (the reconstruction of arXiv 2409.10729,
// Sec. II-B): omega = softmax(log omega_JS + z).  A zero output layer gives
// Jiang-Shu exactly.  Evaluated inside the sweeps on the matrix cores:
// bfloat16 operands, float32 accumulation.
//
// Formulation on v_mfma_f32_32x32x8_bf16 (one wave, 32 samples per tile):
// each layer computes H^T = W * X^T with the weights as the A operand (rows =
// output units) and the activations as the B operand (columns = samples).
// The accumulator of one layer holds, in lane l, unit 8(r/4) + 4(l/32) + r%4
// of sample l%32 in register r, which is exactly the B-operand layout of the
// next layer's K-step r/4; so the three layers chain in registers with no
// data exchange.  Layer 1 takes the 5 features plus a constant 1 (bias) as
// its K = 8; layers 2 and 3 start from the bias in the accumulator.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mfx {

constexpr int MLP_H = 32;
constexpr int MLP_PARAMS = MLP_H * 5 + MLP_H + MLP_H * MLP_H + MLP_H + 3 * MLP_H + 3;  // 1347
constexpr int MLP_OFF_W1 = 0, MLP_OFF_B1 = 160, MLP_OFF_W2 = 192, MLP_OFF_B2 = 1216, MLP_OFF_W3 = 1248,
              MLP_OFF_B3 = 1344;
constexpr float GELU_C = 0.7978845608028654f;  // sqrt(2/pi)
constexpr float GELU_A = 0.044715f;

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// Per-lane slice of the network in MFMA operand layout (packed once by
// mlp_pack_kernel).  152 bytes per lane, 64 lanes.
struct MlpLane {
    bf16x4 a1;     // layer 1: row l%32, k = 4(l/32)..+3 of [W1 | b1 | 0 0]
    bf16x4 a2[4];  // layer 2: row l%32, k = 8s + 4(l/32) + i
    bf16x4 a3[4];  // layer 3: rows >= 3 are zero
    f32x16 c2;     // layer-2 bias in accumulator layout
    float c3[4];   // layer-3 bias for registers 0..2 (zero for lanes >= 32)
};

__device__ __forceinline__ short bf16_bits(float x) { return __builtin_bit_cast(short, (__bf16)x); }

// GELU, tanh form: 0.5 x (1 + tanh(y)), y = c (x + a x^3), written as
// x - x / (1 + e^{2y}) (exact identity; saturates correctly at +-inf: the
// hardware reciprocal of +inf is 0).  Its result is rounded to bfloat16, so
// the 1-ulp hardware exponential and reciprocal are ample.
__device__ __forceinline__ float gelu(float x)
{
    const float y2 = 2.0f * GELU_C * x * (1.0f + GELU_A * x * x);
    const float e = __expf(y2);
    return x - x * __builtin_amdgcn_rcpf(1.0f + e);
}

__device__ __forceinline__ f32x16 mlp_layers(const MlpLane& m, bf16x4 b1)
{
    f32x16 acc = {};
    acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(m.a1, b1, acc, 0, 0, 0);
    bf16x4 b2[4];
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int i = 0; i < 4; ++i) b2[s][i] = bf16_bits(gelu(acc[4 * s + i]));
    f32x16 acc2 = m.c2;
#pragma unroll
    for (int s = 0; s < 4; ++s) acc2 = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(m.a2[s], b2[s], acc2, 0, 0, 0);
    bf16x4 b3[4];
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int i = 0; i < 4; ++i) b3[s][i] = bf16_bits(gelu(acc2[4 * s + i]));
    f32x16 acc3 = {};
    acc3[0] = m.c3[0];
    acc3[1] = m.c3[1];
    acc3[2] = m.c3[2];
#pragma unroll
    for (int s = 0; s < 4; ++s) acc3 = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(m.a3[s], b3[s], acc3, 0, 0, 0);
    return acc3;
}

// Per-wave LDS slot for one variable's samples: the two edge samples (side 0
// right edge, side 1 mirrored = left edge) of each of the 64 lanes.
struct LearnedLds {
    short feat[2][64][8];  // bfloat16 features 0..4, constant 1 (bias), 0, 0
    float z[2][64][4];     // network outputs (logits)
};

// Jiang-Shu smoothness indicators of the stencil a..e and its fourth
// difference D.
__device__ __forceinline__ void weno_betas(float a, float b, float c, float d, float e, float& b0, float& b1,
                                           float& b2, float& D)
{
    const float k13 = 13.0f / 12.0f;
    const float q0 = a - 2.f * b + c, h0 = a - 4.f * b + 3.f * c;
    const float q1 = b - 2.f * c + d, h1 = b - d;
    const float q2 = c - 2.f * d + e, h2 = 3.f * c - 4.f * d + e;
    b0 = k13 * q0 * q0 + 0.25f * h0 * h0;
    b1 = k13 * q1 * q1 + 0.25f * h1 * h1;
    b2 = k13 * q2 * q2 + 0.25f * h2 * h2;
    D = a - 4.f * b + 6.f * c - 4.f * d + e;
}

// Features of the stencil a..e reconstructed at its right edge: the
// Jiang-Shu indicators over their sum S (with eps), |beta0 - beta2| / S, and
// D^2 / (S + D^2) with D the fourth difference.  All in [0, 1].
// nlb_k = -2 log2(eps + beta_k): with log2 of the linear weight added, the
// log2 of the unnormalised Jiang-Shu weight d_k / (eps + beta_k)^2 (a common
// offset cancels in the softmax, so no normalisation and no overflow).
__device__ __forceinline__ void weno_features(float a, float b, float c, float d, float e, float eps, float x[5],
                                              float nlb[3])
{
    float b0, b1, b2, D;
    weno_betas(a, b, c, d, e, b0, b1, b2, D);
    const float S = b0 + b1 + b2 + eps;
    const float iS = __builtin_amdgcn_rcpf(S);  // features go to bfloat16: 1 ulp is ample
    x[0] = b0 * iS;
    x[1] = b1 * iS;
    x[2] = b2 * iS;
    x[3] = fabsf(b0 - b2) * iS;
    x[4] = D * D * __builtin_amdgcn_rcpf(S + D * D);
    nlb[0] = -2.0f * log2f(eps + b0);
    nlb[1] = -2.0f * log2f(eps + b1);
    nlb[2] = -2.0f * log2f(eps + b2);
}

// Shared form, per variable: the features (as above) and the normalised
// Jiang-Shu weights of the right edge (o) and of the mirrored left edge
// (om, in the mirrored candidates' order), in the overflow-free ratio form
// d_k (min_j s_j / s_k)^2, s_k = eps + beta_k.
__device__ __forceinline__ void edge_stats(float a, float b, float c, float d, float e, float eps, float x[5],
                                           float o[3], float om[3])
{
    float b0, b1, b2, D;
    weno_betas(a, b, c, d, e, b0, b1, b2, D);
    const float S = b0 + b1 + b2 + eps;
    const float iS = __builtin_amdgcn_rcpf(S);
    x[0] = b0 * iS;
    x[1] = b1 * iS;
    x[2] = b2 * iS;
    x[3] = fabsf(b0 - b2) * iS;
    x[4] = D * D * __builtin_amdgcn_rcpf(S + D * D);
    const float s0 = eps + b0, s1 = eps + b1, s2 = eps + b2;
    const float smin = fminf(s0, fminf(s1, s2));
    float q0 = smin * __builtin_amdgcn_rcpf(s0), q1 = smin * __builtin_amdgcn_rcpf(s1),
          q2 = smin * __builtin_amdgcn_rcpf(s2);
    q0 *= q0;
    q1 *= q1;
    q2 *= q2;
    const float ir = __builtin_amdgcn_rcpf(0.1f * q0 + 0.6f * q1 + 0.3f * q2);
    o[0] = 0.1f * q0 * ir;
    o[1] = 0.6f * q1 * ir;
    o[2] = 0.3f * q2 * ir;
    const float im = __builtin_amdgcn_rcpf(0.1f * q2 + 0.6f * q1 + 0.3f * q0);
    om[0] = 0.1f * q2 * im;
    om[1] = 0.6f * q1 * im;
    om[2] = 0.3f * q0 * im;
}

// Both edge values of the stencil a..e with the right edge's weights om
// and the mirrored left edge's weights oml.
__device__ __forceinline__ void weno5_apply(const float om[3], const float oml[3], float a, float b, float c, float d,
                                            float e, float& left, float& right)
{
    const float r0 = 2.f * a - 7.f * b + 11.f * c, r1 = -b + 5.f * c + 2.f * d, r2 = 2.f * c + 5.f * d - e;
    const float l0 = 2.f * e - 7.f * d + 11.f * c, l1 = -d + 5.f * c + 2.f * b, l2 = 2.f * c + 5.f * b - a;
    right = (om[0] * r0 + om[1] * r1 + om[2] * r2) * (1.0f / 6.0f);
    left = (oml[0] * l0 + oml[1] * l1 + oml[2] * l2) * (1.0f / 6.0f);
}

constexpr float LOG2_D0 = -3.321928094887362f;  // log2(0.1)
constexpr float LOG2_D1 = -0.736965594166206f;  // log2(0.6)
constexpr float LOG2_D2 = -1.736965594166206f;  // log2(0.3)

// omega_k = softmax(z_k + ln w_k) with the log-weights given in base 2.
__device__ __forceinline__ void softmax3(const float z[3], const float lw[3], float om[3])
{
    constexpr float LOG2E = 1.4426950408889634f;
    const float l0 = z[0] * LOG2E + lw[0], l1 = z[1] * LOG2E + lw[1], l2 = z[2] * LOG2E + lw[2];
    const float lm = fmaxf(l0, fmaxf(l1, l2));
    const float e0 = exp2f(l0 - lm), e1 = exp2f(l1 - lm), e2 = exp2f(l2 - lm);
    const float inv = __builtin_amdgcn_rcpf(e0 + e1 + e2);
    om[0] = e0 * inv;
    om[1] = e1 * inv;
    om[2] = e2 * inv;
}

// Orders this wave's LDS writes before reads of them by its other lanes.
// The slot is private to the wave and LDS instructions of one wave execute
// in order, so only the compiler must be kept from moving accesses across.
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Learned weights of 2 samples per lane (x0: side 0, x1: side 1) for the
// whole wave, which must call this together.  The wave stages its 128
// samples in its own LDS slot and runs them as four 32-sample tiles on the
// matrix cores.
__device__ __forceinline__ void mlp_omega_pair(const MlpLane& m, LearnedLds* L, const float x0[5], const float x1[5],
                                               const float lw0[3], const float lw1[3], float om0[3], float om1[3])
{
    const int lane = threadIdx.x & 63;
    const short one = bf16_bits(1.0f);
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        L->feat[0][lane][k] = bf16_bits(x0[k]);
        L->feat[1][lane][k] = bf16_bits(x1[k]);
    }
    L->feat[0][lane][5] = one;
    L->feat[1][lane][5] = one;
    L->feat[0][lane][6] = L->feat[0][lane][7] = 0;
    L->feat[1][lane][6] = L->feat[1][lane][7] = 0;
    wave_lds_sync();
#pragma unroll 1
    for (int t = 0; t < 4; ++t) {
        const int side = t >> 1, half = t & 1;
        const bf16x4 b = *reinterpret_cast<const bf16x4*>(&L->feat[side][32 * half + (lane & 31)][4 * (lane >> 5)]);
        const f32x16 z = mlp_layers(m, b);
        if (lane < 32) {
            L->z[side][32 * half + lane][0] = z[0];
            L->z[side][32 * half + lane][1] = z[1];
            L->z[side][32 * half + lane][2] = z[2];
        }
    }
    wave_lds_sync();
    const float z0[3] = {L->z[0][lane][0], L->z[0][lane][1], L->z[0][lane][2]};
    const float z1[3] = {L->z[1][lane][0], L->z[1][lane][1], L->z[1][lane][2]};
    softmax3(z0, lw0, om0);
    softmax3(z1, lw1, om1);
}

// One sample per lane (stand-alone inference): the second side is unused.
__device__ __forceinline__ void mlp_omega(const MlpLane& m, LearnedLds* L, const float f[5], const float lw[3],
                                          float om[3])
{
    float dummy[3];
    mlp_omega_pair(m, L, f, f, lw, lw, om, dummy);
}

// Both edge values of one cell with learned weights (right edge: features
// as computed; left edge: the mirrored stencil, i.e. features with beta0 and
// beta2 swapped, weights applied to the mirrored candidates).
__device__ __forceinline__ void weno5_learned(const MlpLane& m, LearnedLds* L, float a, float b, float c, float d,
                                              float e, float eps, float& left, float& right, bool& finite_r,
                                              bool& finite_l)
{
    float x[5], xm[5], nlb[3], om[3], oml[3];
    weno_features(a, b, c, d, e, eps, x, nlb);
    xm[0] = x[2];
    xm[1] = x[1];
    xm[2] = x[0];
    xm[3] = x[3];
    xm[4] = x[4];
    // mirrored stencil: indicators reversed, linear weights (0.1, 0.6, 0.3) kept
    const float lw[3] = {LOG2_D0 + nlb[0], LOG2_D1 + nlb[1], LOG2_D2 + nlb[2]};
    const float lwm[3] = {LOG2_D0 + nlb[2], LOG2_D1 + nlb[1], LOG2_D2 + nlb[0]};
    mlp_omega_pair(m, L, x, xm, lw, lwm, om, oml);
    weno5_apply(om, oml, a, b, c, d, e, left, right);
    finite_r = isfinite(om[0] + om[1] + om[2]);
    finite_l = isfinite(oml[0] + oml[1] + oml[2]);
}

// A face state is admissible if its partial densities are non-negative,
// alpha1 lies in [0, 1] and the squared sound speed is positive.
template <typename M>
__device__ __forceinline__ bool admissible(const M& mix, const float w[7])
{
    const float G = mix.Gamma(w[6]), P = mix.Pi(w[6]);
    bool ok = w[0] >= 0.f && w[1] >= 0.f && w[6] >= 0.f && w[6] <= 1.f && (G + 1.f) * w[5] + P > 0.f;
#pragma unroll
    for (int v = 0; v < 7; ++v) ok = ok && isfinite(w[v]);
    return ok;
}

}  // namespace mfx
