// rewl_device.h -- device-side building blocks of the REWL kernels (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rewl_internal.h"

namespace rewl {
namespace dev {

struct U4 {
    uint32_t x, y, z, w;
};

// Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32->64
// multiplications with Weyl-sequence key bumps.  Pure integer VALU work.
__device__ __forceinline__ U4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                     uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
        const uint32_t lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
        const uint32_t n0 = hi1 ^ c1 ^ k0;
        const uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return U4{c0, c1, c2, c3};
}

__device__ __forceinline__ U4 draw(uint32_t seed, uint32_t stream, uint64_t n, uint32_t word2,
                                   uint32_t tag)
{
    return philox((uint32_t)n, (uint32_t)(n >> 32), word2, tag, seed, stream);
}

// 53-bit uniform on [0,1) from two words.
__device__ __forceinline__ double u53(uint32_t a, uint32_t b)
{
    return ((double)(a >> 5) * 67108864.0 + (double)(b >> 6)) * (1.0 / 9007199254740992.0);
}

// Uniform site on 0..N-1: high word of w*N.
__device__ __forceinline__ int pick_site(uint32_t w, int N)
{
    return (int)__umulhi(w, (uint32_t)N);
}

// Uniform direction on S^2 by Marsaglia's rejection (two tries per Philox
// block, blocks numbered by the third counter word; +z after 64 blocks).
__device__ __forceinline__ void sphere_d(uint32_t seed, uint32_t stream, uint64_t n, uint32_t tag,
                                         double &ox, double &oy, double &oz)
{
    for (uint32_t blk = 0; blk < 64; ++blk) {
        const U4 r = draw(seed, stream, n, blk, tag);
        double v1 = (double)(int32_t)r.x * (1.0 / 2147483648.0);
        double v2 = (double)(int32_t)r.y * (1.0 / 2147483648.0);
        double s = v1 * v1 + v2 * v2;
        if (s < 1.0) {
            const double q = sqrt(1.0 - s);
            ox = (2.0 * v1) * q;
            oy = (2.0 * v2) * q;
            oz = 1.0 - 2.0 * s;
            return;
        }
        v1 = (double)(int32_t)r.z * (1.0 / 2147483648.0);
        v2 = (double)(int32_t)r.w * (1.0 / 2147483648.0);
        s = v1 * v1 + v2 * v2;
        if (s < 1.0) {
            const double q = sqrt(1.0 - s);
            ox = (2.0 * v1) * q;
            oy = (2.0 * v2) * q;
            oz = 1.0 - 2.0 * s;
            return;
        }
    }
    ox = 0.0;
    oy = 0.0;
    oz = 1.0;
}

// The same draw in FP32 arithmetic (FP32 proposal mode).
__device__ __forceinline__ void sphere_f(uint32_t seed, uint32_t stream, uint64_t n, uint32_t tag,
                                         float &ox, float &oy, float &oz)
{
    for (uint32_t blk = 0; blk < 64; ++blk) {
        const U4 r = draw(seed, stream, n, blk, tag);
        float v1 = (float)(int32_t)r.x * (1.0f / 2147483648.0f);
        float v2 = (float)(int32_t)r.y * (1.0f / 2147483648.0f);
        float s = __builtin_fmaf(v1, v1, v2 * v2);
        if (s < 1.0f) {
            const float q = 2.0f * __builtin_sqrtf(1.0f - s);
            ox = v1 * q;
            oy = v2 * q;
            oz = __builtin_fmaf(-2.0f, s, 1.0f);
            return;
        }
        v1 = (float)(int32_t)r.z * (1.0f / 2147483648.0f);
        v2 = (float)(int32_t)r.w * (1.0f / 2147483648.0f);
        s = __builtin_fmaf(v1, v1, v2 * v2);
        if (s < 1.0f) {
            const float q = 2.0f * __builtin_sqrtf(1.0f - s);
            ox = v1 * q;
            oy = v2 * q;
            oz = __builtin_fmaf(-2.0f, s, 1.0f);
            return;
        }
    }
    ox = 0.0f;
    oy = 0.0f;
    oz = 1.0f;
}

// e^x for x <= 0 with a fixed sequence of IEEE operations (no contraction):
// x = k ln2 + r (ln 2 in a 32-bit head plus tail), e^r by its degree-13
// Taylor polynomial in Horner form, times 2^k built from the exponent bits.
__device__ __forceinline__ double exp_det(double x)
{
    if (x > 0.0) x = 0.0;
    if (x < -700.0) return 0.0;
    const double ln2_hi = 0x1.62e42ff000000p-1;
    const double ln2_lo = -0x1.718432a1b0e26p-35;
    const double inv_ln2 = 0x1.71547652b82fep+0;
    const double kd = floor(x * inv_ln2 + 0.5);
    const double r = (x - kd * ln2_hi) - kd * ln2_lo;
    double p = 1.0 / 6227020800.0;
    p = p * r + 1.0 / 479001600.0;
    p = p * r + 1.0 / 39916800.0;
    p = p * r + 1.0 / 3628800.0;
    p = p * r + 1.0 / 362880.0;
    p = p * r + 1.0 / 40320.0;
    p = p * r + 1.0 / 5040.0;
    p = p * r + 1.0 / 720.0;
    p = p * r + 1.0 / 120.0;
    p = p * r + 1.0 / 24.0;
    p = p * r + 1.0 / 6.0;
    p = p * r + 0.5;
    p = p * r + 1.0;
    p = p * r + 1.0;
    const int k = (int)kd;
    const double scale = __longlong_as_double((long long)(k + 1023) << 52);
    return p * scale;
}

// Orders this wavefront's LDS accesses across lanes (a walker is one
// wavefront and owns its LDS region, so no workgroup barrier is needed).
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// ---------------------------------------------------------------- wave sums
template <int CTRL>
__device__ __forceinline__ float dpp_f(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}

template <int CTRL>
__device__ __forceinline__ double dpp_d(double v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ float readlane_f(float v, int l)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

__device__ __forceinline__ double readlane_d(double v, int l)
{
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
    return __hiloint2double(hi, lo);
}

// Sum over the 64 lanes, result uniform.  Within each row of 16 lanes:
// swap neighbours, swap pairs, rotate by 4, rotate by 8 (every lane then
// holds its row sum); the four row sums are read out and added.
__device__ __forceinline__ float wave_sum_f(float v)
{
    v += dpp_f<0xB1>(v);    // quad_perm [1,0,3,2]
    v += dpp_f<0x4E>(v);    // quad_perm [2,3,0,1]
    v += dpp_f<0x124>(v);   // row_ror:4
    v += dpp_f<0x128>(v);   // row_ror:8
    return (readlane_f(v, 0) + readlane_f(v, 16)) + (readlane_f(v, 32) + readlane_f(v, 48));
}

__device__ __forceinline__ double wave_sum_d(double v)
{
    v += dpp_d<0xB1>(v);
    v += dpp_d<0x4E>(v);
    v += dpp_d<0x124>(v);
    v += dpp_d<0x128>(v);
    return (readlane_d(v, 0) + readlane_d(v, 16)) + (readlane_d(v, 32) + readlane_d(v, 48));
}

__device__ __forceinline__ int wave_sum_i(int v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        const uint32_t w = (uint32_t)__shfl_xor((int)v, o, 64);
        v = w < v ? w : v;
    }
    return v;
}

// q = floor(a / d) and a - q d for 0 <= a < 2^22 and 1 <= d < 2^10, from a
// float reciprocal estimate corrected by one step.
__device__ __forceinline__ int divmod_small(int a, int d, float inv_d, int &rem)
{
    int q = (int)((float)a * inv_d);
    int r = a - q * d;
    if (r < 0) { q -= 1; r += d; }
    if (r >= d) { q += 1; r -= d; }
    rem = r;
    return q;
}

// Index of the neighbour of `site` reached through bcc slot `sl`.
__device__ __forceinline__ int bcc_neighbour(int site, int L, float invL, const BccSlot &sl)
{
    int x, y, z;
    int q = divmod_small(site, L, invL, x);
    q = divmod_small(q, L, invL, y);
    const int s = divmod_small(q, L, invL, z);
    // selects rather than an indexed load of the slot (keeps it in registers)
    int nx = x + (s ? sl.d[1][0] : sl.d[0][0]);
    int ny = y + (s ? sl.d[1][1] : sl.d[0][1]);
    int nz = z + (s ? sl.d[1][2] : sl.d[0][2]);
    nx += nx < 0 ? L : 0;
    nx -= nx >= L ? L : 0;
    ny += ny < 0 ? L : 0;
    ny -= ny >= L ? L : 0;
    nz += nz < 0 ? L : 0;
    nz -= nz >= L ? L : 0;
    const int t = s ^ (int)sl.flip;
    return ((t * L + nz) * L + ny) * L + nx;
}

}  // namespace dev
}  // namespace rewl
