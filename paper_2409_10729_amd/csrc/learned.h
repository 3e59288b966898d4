// Learned WENO weights: a 5-32-32-3 MLP (GELU) maps scale-free smoothness
// features of a 5-cell stencil to three logits z that correct the Jiang-Shu
// weights of the WENO5 candidates (the reconstruction of arXiv 2409.10729,
// Sec. II-B): omega = softmax(log omega_JS + z).  A zero output layer gives
// Jiang-Shu exactly.  Evaluated inside the sweeps on the matrix cores:
// bfloat16 operands, float32 accumulation.
//
// One wave evaluates 64 samples, one per lane, as two 32-sample tiles (tile
// h holds the samples of lanes 32h .. 32h+31).  Each layer computes
// H^T = W * X^T with the weights as the A operand (rows = output units) and
// the activations as the B operand (columns = samples):
//   layer 1 on v_mfma_f32_32x32x8_bf16 (K = 5 features, a constant 1 for the
//     bias, two zeros): lane l supplies k = 4(l/32) .. +3 of sample l%32 of
//     its tile; the lanes of the other half hold those values, so one
//     v_permlane32_swap per dword builds both tiles' operands from each
//     lane's own features;
//   layers 2 and 3 on v_mfma_f32_32x32x16_bf16 (K = 32 hidden units in two
//     K-steps): the accumulator of a layer holds, in lane l and register r,
//     unit 8(r/4) + 4(l/32) + r%4 of sample l%32; K-step s takes registers
//     8s .. 8s+7 as its k-slots 8(l/32) .. +7, so the next layer's weights
//     are packed with their input units permuted the same way and the layers
//     chain in registers;
//   layer 3 of tile h keeps its three outputs in rows 4h .. 4h+2, which land
//     in registers 0..2 of the lanes that own the tile's samples: both tiles
//     accumulate into one register block and every lane reads its own logits.
// No LDS and no wave synchronisation: the caller needs only uniform control
// flow across the wave.
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
typedef short bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16v8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16v4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// Input unit that k-slot i of K-step s feeds in lane half g (layers 2, 3).
__host__ __device__ constexpr int mlp_kslot_unit(int s, int g, int i) { return 8 * (2 * s + i / 4) + 4 * g + i % 4; }

// The network in matrix-core operand layout (packed once by the pack
// kernel): MLP_WORDS 16-byte words per lane, stored word-major (word w of
// lane l at w[w][l]), so a wave reads one word of all its lanes as one
// contiguous kilobyte (no LDS bank conflicts, coalesced in global memory).
constexpr int MW_A2 = 0;  // 2 words: layer-2 A operand, K-steps 0, 1 (row l%32, k-slots 8(l/32)..+7)
constexpr int MW_A3 = 2;  // 4 words: layer-3 A operand of tile h, K-step s, at MW_A3 + 2h + s
                          //          (rows 4h..4h+2 hold W3, other rows zero)
constexpr int MW_C2 = 6;  // 4 words: layer-2 bias in accumulator layout (registers 4j..4j+3 in word j)
constexpr int MW_A1 = 10; // 1 word: layer-1 A operand (row l%32, k = 4(l/32)..+3 of [W1 | b1 | 0 0]) in
                          //         dwords 0-1, layer-3 bias 0 and 1 in dwords 2-3
constexpr int MW_C3 = 11; // 1 word: layer-3 bias 2 in dword 0, then zeros
constexpr int MLP_WORDS = 12;

// (a plain vector type: bit casts to and from HIP's uint4 struct are not
// reliable)
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned u32x2 __attribute__((ext_vector_type(2)));

struct MlpNet {
    u32x4 w[MLP_WORDS][64];
};

__device__ __forceinline__ short bf16_bits(float x) { return __builtin_bit_cast(short, (__bf16)x); }

// GELU as the inference evaluates it: the tanh form of GELU,
// 0.5 x (1 + tanh(sqrt(2/pi) (x + 0.044715 x^3))), equals max(x, 0) - h(|x|)
// with h(a) = 0.5 a (1 - tanh(sqrt(2/pi) (a + 0.044715 a^3))) a bump that
// vanishes quickly; h is replaced by t Q(t), t = min(|x|, 3.75), Q the
// degree-6 polynomial below (a minimax fit; within 1.2e-4 of the tanh form
// for every x, about 1/30 of a bfloat16 step at 1, and the result is
// rounded to bfloat16).  Nine instructions, no transcendental functions.
constexpr float GELU_T = 3.75f;
constexpr float GELU_Q[7] = {0.497150153f,   -0.375513077f, -0.0665387958f, 0.157749414f,
                             -0.0645674914f, 0.0113088572f, -0.00075154379f};

__device__ __forceinline__ float gelu(float x)
{
    // min(|x|, T) and max(x, 0) as medians of three (one v_med3_f32 each;
    // min/max of a matrix-core result would first be quieted, one more
    // instruction each); the median with the largest float equals max(x, 0)
    // for every finite x
    const float t = __builtin_amdgcn_fmed3f(fabsf(x), 0.0f, GELU_T);
    const float relu = __builtin_amdgcn_fmed3f(x, 0.0f, 3.40282347e38f);
    float q = GELU_Q[6];
#pragma unroll
    for (int k = 5; k >= 0; --k) q = __builtin_fmaf(q, t, GELU_Q[k]);
    return __builtin_fmaf(-q, t, relu);
}

// bfloat16 (nearest, ties to even) of GELU of eight accumulator registers.
__device__ __forceinline__ bf16x8 gelu8(const f32x16& acc, int r0)
{
    bf16v8 b;
#pragma unroll
    for (int i = 0; i < 8; ++i) b[i] = (__bf16)gelu(acc[r0 + i]);
    return __builtin_bit_cast(bf16x8, b);
}

// Logits z of the lane's own sample x[0..4] (features in [0, 1]); the whole
// wave calls this together.  net: the packed network (LDS or global).
// PIPE: the two tiles in step (each tile's activations on the vector units
// while the other tile's matrix-core operation runs; about 14 more
// registers), else one tile after the other.
template <bool PIPE = true>
__device__ __forceinline__ void mlp_logits(const MlpNet& net, const float x[5], float z[3])
{
    // one evaluation at a time: the scheduler would otherwise interleave the
    // matrix-core chains of many samples and run out of registers
    __builtin_amdgcn_sched_barrier(0);
    const int lane = threadIdx.x & 63;
    auto word = [&](int w) { return net.w[w][lane]; };
    // layer-1 operands of both tiles from the lanes' own features
    bf16v4 lo4 = {(__bf16)x[0], (__bf16)x[1], (__bf16)x[2], (__bf16)x[3]};
    bf16v4 hi4 = {(__bf16)x[4], (__bf16)1.0f, (__bf16)0.0f, (__bf16)0.0f};
    const u32x2 lo = __builtin_bit_cast(u32x2, lo4), hi = __builtin_bit_cast(u32x2, hi4);
    const auto s0 = __builtin_amdgcn_permlane32_swap(lo[0], hi[0], false, false);
    const auto s1 = __builtin_amdgcn_permlane32_swap(lo[1], hi[1], false, false);
    const u32x2 t0 = {s0[0], s1[0]}, t1 = {s0[1], s1[1]};
    const bf16x4 b1[2] = {__builtin_bit_cast(bf16x4, t0), __builtin_bit_cast(bf16x4, t1)};
    const u32x4 w10 = word(MW_A1);
    const u32x2 a1w = {w10[0], w10[1]};
    const bf16x4 a1 = __builtin_bit_cast(bf16x4, a1w);
    f32x16 c2;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const u32x4 cw = word(MW_C2 + j);
#pragma unroll
        for (int i = 0; i < 4; ++i) c2[4 * j + i] = __uint_as_float(cw[i]);
    }
    const bf16v8 a2[2] = {__builtin_bit_cast(bf16v8, word(MW_A2)), __builtin_bit_cast(bf16v8, word(MW_A2 + 1))};
    auto layer2 = [&](const f32x16& acc1) {
        f32x16 acc2 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a2[0], __builtin_bit_cast(bf16v8, gelu8(acc1, 0)), c2, 0,
                                                              0, 0);
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a2[1], __builtin_bit_cast(bf16v8, gelu8(acc1, 8)), acc2, 0, 0,
                                                       0);
    };
    auto layer3 = [&](const f32x16& acc2, int h, const f32x16& acc) {
        f32x16 acc3 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16v8, word(MW_A3 + 2 * h)),
                                                              __builtin_bit_cast(bf16v8, gelu8(acc2, 0)), acc, 0, 0, 0);
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16v8, word(MW_A3 + 2 * h + 1)),
                                                       __builtin_bit_cast(bf16v8, gelu8(acc2, 8)), acc3, 0, 0, 0);
    };
    const f32x16 zero = {};
    f32x16 acc3;
    if constexpr (PIPE) {
        const f32x16 acc1_0 = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a1, b1[0], zero, 0, 0, 0);
        const f32x16 acc1_1 = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a1, b1[1], zero, 0, 0, 0);
        const f32x16 acc2_0 = layer2(acc1_0);
        const f32x16 acc2_1 = layer2(acc1_1);
        acc3 = layer3(acc2_0, 0, zero);
        acc3 = layer3(acc2_1, 1, acc3);
    } else {
        acc3 = layer3(layer2(__builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a1, b1[0], zero, 0, 0, 0)), 0, zero);
        acc3 = layer3(layer2(__builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a1, b1[1], zero, 0, 0, 0)), 1, acc3);
    }
    const u32x4 w11 = word(MW_C3);
    z[0] = acc3[0] + __uint_as_float(w10[2]);
    z[1] = acc3[1] + __uint_as_float(w10[3]);
    z[2] = acc3[2] + __uint_as_float(w11[0]);
    __builtin_amdgcn_sched_barrier(0);
}

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

// Features of the stencil a..e (as weno_features) and its indicators.
__device__ __forceinline__ void edge_features(float a, float b, float c, float d, float e, float eps, float x[5])
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
}

// Shared form, per variable: the learned weights of the right edge (om)
// and of the mirrored left edge (oml, in the mirrored candidates' order)
// from the edge's exponentiated logits er, el (each exp(z - max z)):
// omega_k proportional to omega_JS,k exp(z_k), with the Jiang-Shu weights
// in the overflow-free ratio form d_k (min_j s_j / s_k)^2, s_k = eps +
// beta_k (their normalisation cancels).  fin_r, fin_l: the weights are
// finite.
__device__ __forceinline__ void shared_weights(float a, float b, float c, float d, float e, float eps,
                                               const float er[3], const float el[3], float om[3], float oml[3],
                                               bool& fin_r, bool& fin_l)
{
    float b0, b1, b2, D;
    weno_betas(a, b, c, d, e, b0, b1, b2, D);
    const float s0 = eps + b0, s1 = eps + b1, s2 = eps + b2;
    const float smin = fminf(s0, fminf(s1, s2));
    float q0 = smin * __builtin_amdgcn_rcpf(s0), q1 = smin * __builtin_amdgcn_rcpf(s1),
          q2 = smin * __builtin_amdgcn_rcpf(s2);
    q0 *= q0;
    q1 *= q1;
    q2 *= q2;
    const float r0 = 0.1f * q0 * er[0], r1 = 0.6f * q1 * er[1], r2 = 0.3f * q2 * er[2];
    const float ir = __builtin_amdgcn_rcpf(r0 + r1 + r2);
    om[0] = r0 * ir;
    om[1] = r1 * ir;
    om[2] = r2 * ir;
    const float m0 = 0.1f * q2 * el[0], m1 = 0.6f * q1 * el[1], m2 = 0.3f * q0 * el[2];
    const float im = __builtin_amdgcn_rcpf(m0 + m1 + m2);
    oml[0] = m0 * im;
    oml[1] = m1 * im;
    oml[2] = m2 * im;
    fin_r = isfinite(ir);
    fin_l = isfinite(im);
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

// exp(z_k - max z) of three logits (finite logits give values in (0, 1],
// the largest exactly 1; a non-finite logit makes them NaN).
__device__ __forceinline__ void exp_logits(const float z[3], float ez[3])
{
    constexpr float LOG2E = 1.4426950408889634f;
    const float zm = fmaxf(z[0], fmaxf(z[1], z[2]));
    ez[0] = exp2f((z[0] - zm) * LOG2E);
    ez[1] = exp2f((z[1] - zm) * LOG2E);
    ez[2] = exp2f((z[2] - zm) * LOG2E);
}

// Learned weights of the lane's own sample (the whole wave calls this
// together): omega = softmax(z + ln omega_JS), lw the base-2 log-weights.
template <bool PIPE = true>
__device__ __forceinline__ void mlp_omega(const MlpNet& m, const float x[5], const float lw[3], float om[3])
{
    float z[3];
    mlp_logits<PIPE>(m, x, z);
    softmax3(z, lw, om);
}

// Both edge values of one cell with learned weights (right edge: features
// as computed; left edge: the mirrored stencil, i.e. features with beta0 and
// beta2 swapped, weights applied to the mirrored candidates).
template <bool PIPE = true>
__device__ __forceinline__ void weno5_learned(const MlpNet& m, float a, float b, float c, float d, float e,
                                              float eps, float& left, float& right, bool& finite_r, bool& finite_l)
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
    mlp_omega<PIPE>(m, x, lw, om);
    mlp_omega<PIPE>(m, xm, lwm, oml);
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
