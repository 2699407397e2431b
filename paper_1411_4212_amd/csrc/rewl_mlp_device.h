// rewl_mlp_device.h -- learned proposal on the device: the 4-64-64-12 MLP
// evaluated with BF16 MFMA (FP32 accumulation) for up to 16 inputs per
// wavefront, and the von Mises-Fisher mixture it parameterises.
//
// The proposal is an extension, not part of the paper: a mixture
//   q(s|x) = eps/(4 pi) + (1 - eps) sum_c alpha_c f(s; mu_c, kappa_c),
//   f(s; mu, k) = k / (2 pi (1 - e^{-2k})) exp(k (mu.s - 1)),
// from outputs (v_c, a_c), c = 0..2: kappa_c = clip(|v_c|, 1e-3, 1e3),
// mu_c = v_c/|v_c|, alpha = softmax(a).  The Wang-Landau acceptance then
// carries the ratio q(S_i|x)/q(S'|x), which keeps the walk exact.
//
// MFMA orientation.  v_mfma_f32_16x16x32_bf16 multiplies A (16x32) by B
// (32x16): lane l supplies A[l%16][8(l/16)+j] and B[8(l/16)+j][l%16],
// j < 8, and receives D[4(l/16)+j][l%16], j < 4.  Each layer is computed as
// (weights) x (activations^T): weights are the A operand (16 output
// features per call), the 16 inputs are the columns.  A layer's output then
// sits in lane l as features 4(l/16)..+3 of each 16-feature block for input
// l%16, which is exactly a B operand of the next layer once that layer's
// weight columns are permuted to match: for K-step t, slot (g = l/16, j)
// holds feature 32t + 4g + j (j < 4) or 32t + 16 + 4g + (j - 4) (j >= 4).
// The permutation is applied when the weights are packed, so activations
// never move between lanes.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rewl {
namespace mlp {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kIn = 4, kH = 64, kOut = 12;
constexpr int kParams = kH * kIn + kH + kH * kH + kH + kOut * kH + kOut;   // 5260
constexpr float kEps = 0.05f;
constexpr float kKmin = 1e-3f, kKmax = 1e3f;

// Offsets of the FP32 master parameters (same order as the FP64 reference).
constexpr int oW1 = 0, oB1 = oW1 + kH * kIn, oW2 = oB1 + kH, oB2 = oW2 + kH * kH,
              oW3 = oB2 + kH, oB3 = oW3 + kOut * kH;

// One lane's share of the packed network (368 bytes).
struct Lane {
    bf16x8 A1[4];        // layer 1, output blocks 0..3 (K padded from 4 to 32)
    bf16x8 A2[4][2];     // layer 2, output blocks 0..3, K-steps 0..1
    bf16x8 A3[2];        // layer 3 (12 outputs padded to 16), K-steps 0..1
    float b1[16];        // bias of the features this lane receives, [block][j]
    float b2[16];
    float b3[4];
};

// Feature held in K-slot (g, j) of K-step t (see the orientation note).
__host__ __device__ inline int kslot_feature(int t, int g, int j)
{
    return 32 * t + (j < 4 ? 4 * g + j : 16 + 4 * g + (j - 4));
}

__device__ __forceinline__ f32x4 mfma(const bf16x8 &a, const bf16x8 &b, const f32x4 &c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Forward pass for the 16 inputs whose layer-1 B operand `xb` the lanes hold
// (lane l < 16 carries input l's four features in slots 0..3).  Returns the
// four outputs this lane receives: outputs 4(l/16)..+3 of input l%16.
__device__ __forceinline__ f32x4 forward(const Lane &W, const bf16x8 &xb)
{
    const f32x4 zero = {0.f, 0.f, 0.f, 0.f};
    float a1[4][4];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const f32x4 d = mfma(W.A1[b], xb, zero);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const float z = d[j] + W.b1[4 * b + j];
            a1[b][j] = z > 0.f ? z : 0.f;
        }
    }
    bf16x8 h1[2];
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int j = 0; j < 8; ++j) h1[t][j] = (__bf16)a1[2 * t + (j >> 2)][j & 3];
    float a2[4][4];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        f32x4 d = mfma(W.A2[b][0], h1[0], zero);
        d = mfma(W.A2[b][1], h1[1], d);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const float z = d[j] + W.b2[4 * b + j];
            a2[b][j] = z > 0.f ? z : 0.f;
        }
    }
    bf16x8 h2[2];
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int j = 0; j < 8; ++j) h2[t][j] = (__bf16)a2[2 * t + (j >> 2)][j & 3];
    f32x4 o = mfma(W.A3[0], h2[0], zero);
    o = mfma(W.A3[1], h2[1], o);
#pragma unroll
    for (int j = 0; j < 4; ++j) o[j] += W.b3[j];
    return o;
}

// Layer-1 B operand of lane l for inputs given per lane (lanes l < 16 use
// their own x; other lanes supply zeros).
__device__ __forceinline__ bf16x8 input_operand(float x0, float x1, float x2, float x3, bool active)
{
    bf16x8 v;
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = (__bf16)0.f;
    if (active) {
        v[0] = (__bf16)x0;
        v[1] = (__bf16)x1;
        v[2] = (__bf16)x2;
        v[3] = (__bf16)x3;
    }
    return v;
}

// Mixture parameters of one input (evaluated by the lane that holds it).
// Scalar members only, so that the compiler keeps them in registers.
struct Comp {
    float mx, my, mz;   // mean direction
    float k;            // concentration
    float lnn;          // ln(alpha) + ln(kappa / (2 pi (1 - e^{-2 kappa})))
    float alpha;
};
struct Mix {
    Comp c0, c1, c2;
};

__device__ __forceinline__ Comp component(float vx, float vy, float vz, float alpha)
{
    Comp c;
    const float r = __builtin_sqrtf(__builtin_fmaf(vx, vx, __builtin_fmaf(vy, vy, vz * vz)));
    const float k = fminf(fmaxf(r, kKmin), kKmax);
    const bool ok = r > 0.f;
    const float ir = ok ? 1.f / r : 0.f;
    c.mx = vx * ir;
    c.my = vy * ir;
    c.mz = ok ? vz * ir : 1.f;
    c.k = k;
    c.alpha = alpha;
    c.lnn = __logf(alpha) + __logf(k) - 1.8378770664093453f /* ln 2 pi */ - __logf(-expm1f(-2.f * k));
    return c;
}

__device__ __forceinline__ Mix mixture(const float o[12])
{
    const float amax = fmaxf(o[3], fmaxf(o[7], o[11]));
    const float e0 = __expf(o[3] - amax), e1 = __expf(o[7] - amax), e2 = __expf(o[11] - amax);
    const float ies = 1.f / (e0 + e1 + e2);
    Mix m;
    m.c0 = component(o[0], o[1], o[2], e0 * ies);
    m.c1 = component(o[4], o[5], o[6], e1 * ies);
    m.c2 = component(o[8], o[9], o[10], e2 * ies);
    return m;
}

__device__ __forceinline__ float comp_density(const Comp c, float sx, float sy, float sz)
{
    const float w = __builtin_fmaf(c.mx, sx, __builtin_fmaf(c.my, sy, c.mz * sz));
    return __expf(c.lnn + c.k * (w - 1.f));
}

// ln q(s | mixture).
__device__ __forceinline__ float log_q(const Mix m, float sx, float sy, float sz)
{
    const float t = comp_density(m.c0, sx, sy, sz) + comp_density(m.c1, sx, sy, sz) +
                    comp_density(m.c2, sx, sy, sz);
    return __logf(kEps * 0.07957747154594767f /* 1/(4 pi) */ + (1.f - kEps) * t);
}

// Draw s ~ q: the given uniform direction with probability eps, else
// component c ~ alpha, w = mu.s from the inverse CDF, azimuth 2 pi u_phi
// about mu in the basis (e1, e2) built from the axis least aligned with mu.
__device__ __forceinline__ void sample(const Mix m, float u_mix, float u_w, float u_phi, float ux,
                                       float uy, float uz, float &sx, float &sy, float &sz)
{
    if (u_mix < kEps) {
        sx = ux;
        sy = uy;
        sz = uz;
        return;
    }
    const float um = (u_mix - kEps) / (1.f - kEps);
    const bool s0 = um < m.c0.alpha;
    const bool s1 = !s0 && um < m.c0.alpha + m.c1.alpha;
    const float k = s0 ? m.c0.k : (s1 ? m.c1.k : m.c2.k);
    const float mx = s0 ? m.c0.mx : (s1 ? m.c1.mx : m.c2.mx);
    const float my = s0 ? m.c0.my : (s1 ? m.c1.my : m.c2.my);
    const float mz = s0 ? m.c0.mz : (s1 ? m.c1.mz : m.c2.mz);
    float w = 1.f + __logf(u_w + (1.f - u_w) * __expf(-2.f * k)) / k;
    w = fminf(fmaxf(w, -1.f), 1.f);
    // e1: the coordinate axis least aligned with mu, orthogonalised
    const float ax = fabsf(mx), ay = fabsf(my), az = fabsf(mz);
    const bool px = ax <= ay && ax <= az;
    const bool py = !px && ay <= az;
    const float tx = px ? 1.f : 0.f, ty = py ? 1.f : 0.f, tz = (!px && !py) ? 1.f : 0.f;
    const float d = tx * mx + ty * my + tz * mz;
    float e1x = tx - d * mx, e1y = ty - d * my, e1z = tz - d * mz;
    const float inv = 1.f / __builtin_sqrtf(e1x * e1x + e1y * e1y + e1z * e1z);
    e1x *= inv;
    e1y *= inv;
    e1z *= inv;
    const float e2x = my * e1z - mz * e1y, e2y = mz * e1x - mx * e1z, e2z = mx * e1y - my * e1x;
    float sp, cp;
    __sincosf(6.283185307179586f * u_phi, &sp, &cp);
    const float rt = __builtin_sqrtf(fmaxf(1.f - w * w, 0.f));
    sx = w * mx + rt * (cp * e1x + sp * e2x);
    sy = w * my + rt * (cp * e1y + sp * e2y);
    sz = w * mz + rt * (cp * e1z + sp * e2z);
}

// Gather the 12 outputs of input l%16 into the lane l < 16 that owns it
// (components 1 and 2 live 16 and 32 lanes higher).
__device__ __forceinline__ void gather_outputs(const f32x4 &o, float out[12])
{
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        out[j] = o[j];
        out[4 + j] = __shfl_down(o[j], 16, 64);
        out[8 + j] = __shfl_down(o[j], 32, 64);
    }
}

}  // namespace mlp
}  // namespace rewl
