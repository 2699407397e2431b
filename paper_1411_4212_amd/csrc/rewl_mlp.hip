// rewl_mlp.hip -- training and evaluation kernels of the learned proposal
// (an extension: the paper's trial move is a uniform new direction).
//
//  * mlp_pack_kernel       FP32 master parameters -> per-lane BF16 MFMA layout
//  * mlp_eval_kernel       ln q(s|x) and a draw from q(.|x), BF16 MFMA forward
//  * mlp_grad_kernel       per-block mean-NLL gradient, FP32, deterministic
//  * mlp_reduce_kernel     fixed-order sum of the block partials
//  * mlp_adam_kernel       Adam step on the FP32 master parameters
// Training records are 8 floats: x0..x3 (features), s0..s2 (spin), pad.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>
#include <string>
#include <vector>

#include "rewl_device.h"
#include "rewl_internal.h"
#include "rewl_mlp_device.h"

namespace rewl {
namespace mlp {

constexpr int kRec = 8;           // floats per training record
constexpr int kTB = 64;           // samples per gradient block (one wavefront)
constexpr int kSt = kTB + 1;      // LDS row stride of [feature][sample] arrays (no bank conflicts)

__global__ void __launch_bounds__(64) mlp_pack_kernel(const float *__restrict__ P, Lane *__restrict__ out)
{
    const int l = threadIdx.x;
    const int r = l & 15, g = l >> 4;
    Lane L;
    for (int b = 0; b < 4; ++b)
        for (int j = 0; j < 8; ++j)
            L.A1[b][j] = (__bf16)((g == 0 && j < kIn) ? P[oW1 + (16 * b + r) * kIn + j] : 0.f);
    for (int b = 0; b < 4; ++b)
        for (int t = 0; t < 2; ++t)
            for (int j = 0; j < 8; ++j)
                L.A2[b][t][j] = (__bf16)P[oW2 + (16 * b + r) * kH + kslot_feature(t, g, j)];
    for (int t = 0; t < 2; ++t)
        for (int j = 0; j < 8; ++j)
            L.A3[t][j] = (__bf16)(r < kOut ? P[oW3 + r * kH + kslot_feature(t, g, j)] : 0.f);
    for (int b = 0; b < 4; ++b)
        for (int j = 0; j < 4; ++j) {
            L.b1[4 * b + j] = P[oB1 + 16 * b + 4 * g + j];
            L.b2[4 * b + j] = P[oB2 + 16 * b + 4 * g + j];
        }
    for (int j = 0; j < 4; ++j) L.b3[j] = (4 * g + j < kOut) ? P[oB3 + 4 * g + j] : 0.f;
    out[l] = L;
}

// One wavefront evaluates 16 inputs per step.
__global__ void __launch_bounds__(64) mlp_eval_kernel(const Lane *__restrict__ W, const float *__restrict__ x,
                                                      const float *__restrict__ s, const float *__restrict__ u,
                                                      const float *__restrict__ ud, float *__restrict__ lnq_s,
                                                      float *__restrict__ samp, float *__restrict__ lnq_samp,
                                                      int64_t n)
{
    const int l = threadIdx.x;
    const Lane Wl = W[l];
    for (int64_t base = (int64_t)blockIdx.x * 16; base < n; base += (int64_t)gridDim.x * 16) {
        const int64_t i = base + l;
        const bool mine = l < 16 && i < n;
        float x0 = 0.f, x1 = 0.f, x2 = 0.f, x3 = 0.f;
        if (mine) {
            x0 = x[4 * i];
            x1 = x[4 * i + 1];
            x2 = x[4 * i + 2];
            x3 = x[4 * i + 3];
        }
        const f32x4 o = forward(Wl, input_operand(x0, x1, x2, x3, l < 16));
        float out[12];
        gather_outputs(o, out);
        if (mine) {
            const Mix m = mixture(out);
            lnq_s[i] = log_q(m, s[3 * i], s[3 * i + 1], s[3 * i + 2]);
            float sx, sy, sz;
            sample(m, u[3 * i], u[3 * i + 1], u[3 * i + 2], ud[3 * i], ud[3 * i + 1], ud[3 * i + 2], sx, sy, sz);
            samp[3 * i] = sx;
            samp[3 * i + 1] = sy;
            samp[3 * i + 2] = sz;
            lnq_samp[i] = log_q(m, sx, sy, sz);
        }
    }
}

// dL/d(outputs) of the per-sample loss -ln q(s|x) (FP32).
__device__ void nll_output_grad(const float out[12], float sx, float sy, float sz, float d_out[12],
                                float &loss)
{
    float amax = fmaxf(out[3], fmaxf(out[7], out[11]));
    float e[3], es = 0.f;
    for (int c = 0; c < 3; ++c) {
        e[c] = expf(out[4 * c + 3] - amax);
        es += e[c];
    }
    float alpha[3], f[3], k[3], r[3], w[3], mu[3][3];
    float F = 0.f;
    for (int c = 0; c < 3; ++c) {
        const float vx = out[4 * c], vy = out[4 * c + 1], vz = out[4 * c + 2];
        r[c] = sqrtf(vx * vx + vy * vy + vz * vz);
        k[c] = fminf(fmaxf(r[c], kKmin), kKmax);
        const float ir = r[c] > 0.f ? 1.f / r[c] : 0.f;
        mu[c][0] = vx * ir;
        mu[c][1] = vy * ir;
        mu[c][2] = r[c] > 0.f ? vz * ir : 1.f;
        w[c] = mu[c][0] * sx + mu[c][1] * sy + mu[c][2] * sz;
        alpha[c] = e[c] / es;
        f[c] = expf(logf(k[c]) - 1.8378770664093453f - logf(-expm1f(-2.f * k[c])) + k[c] * (w[c] - 1.f));
        F += alpha[c] * f[c];
    }
    const float Q = kEps * 0.07957747154594767f + (1.f - kEps) * F;
    loss = -logf(Q);
    const float coef = -(1.f - kEps) / Q;
    for (int c = 0; c < 3; ++c) {
        d_out[4 * c + 3] = coef * alpha[c] * (f[c] - F);
        const bool inside = r[c] > kKmin && r[c] < kKmax;
        const float e2 = expf(-2.f * k[c]);
        const float dk = inside ? (1.f / k[c] - 2.f * e2 / (-expm1f(-2.f * k[c])) + (w[c] - 1.f)) : 0.f;
        const float ir = r[c] > 0.f ? 1.f / r[c] : 0.f;
        const float pf = coef * alpha[c] * f[c];
        const float s3[3] = {sx, sy, sz};
        for (int d = 0; d < 3; ++d) {
            const float dmu = (s3[d] - w[c] * mu[c][d]) * ir;
            d_out[4 * c + d] = pf * (k[c] * dmu + dk * mu[c][d]);
        }
    }
}

// Gradient of the mean NLL over the samples of this block: forward and
// backward per sample (one lane each), then the weight gradients as
// fixed-order sums over the block's samples.  Writes one partial gradient
// per block (scaled by `scale`) and the block's loss sum.
__global__ void __launch_bounds__(64) mlp_grad_kernel(const float *__restrict__ P, const float *__restrict__ rec,
                                                      int64_t n, int32_t count, int32_t random_pick,
                                                      uint32_t seed, uint64_t step, float scale,
                                                      float *__restrict__ partial, float *__restrict__ loss_partial)
{
    extern __shared__ __align__(16) float sm[];
    float *Ps = sm;                          // kParams
    float *X = Ps + kParams;                 // [4][kSt]   feature-major: X[k*kSt + s]
    float *A1 = X + kSt * kIn;               // [64][kSt]
    float *A2 = A1 + kSt * kH;
    float *Do = A2 + kSt * kH;               // [12][kSt]
    float *D2 = Do + kSt * kOut;             // [64][kSt]
    float *D1 = D2 + kSt * kH;               // [64][kSt]
    const int t = threadIdx.x;
    for (int i = t; i < kParams; i += kTB) Ps[i] = P[i];
    __syncthreads();

    const int pos = blockIdx.x * kTB + t;
    const bool valid = pos < count;
    int64_t idx = 0;
    if (valid) {
        if (random_pick) {
            const dev::U4 r = dev::draw(seed, 0x7EA1u, step, (uint32_t)pos, 8u);
            idx = (int64_t)(((uint64_t)r.x * (uint64_t)n) >> 32);   // n < 2^32
        } else {
            idx = pos;
        }
    }
    float x[kIn], s3[3];
    for (int k = 0; k < kIn; ++k) x[k] = valid ? rec[idx * kRec + k] : 0.f;
    for (int k = 0; k < 3; ++k) s3[k] = valid ? rec[idx * kRec + 4 + k] : 0.f;
    if (!valid) s3[2] = 1.f;
    for (int k = 0; k < kIn; ++k) X[k * kSt + t] = valid ? x[k] : 0.f;
    // forward
    for (int i = 0; i < kH; ++i) {
        float z = Ps[oB1 + i];
        for (int k = 0; k < kIn; ++k) z = fmaf(Ps[oW1 + i * kIn + k], x[k], z);
        A1[i * kSt + t] = z > 0.f ? z : 0.f;
    }
    for (int i = 0; i < kH; ++i) {
        float z = Ps[oB2 + i];
        for (int k = 0; k < kH; ++k) z = fmaf(Ps[oW2 + i * kH + k], A1[k * kSt + t], z);
        A2[i * kSt + t] = z > 0.f ? z : 0.f;
    }
    float out[kOut];
    for (int o = 0; o < kOut; ++o) {
        float z = Ps[oB3 + o];
        for (int k = 0; k < kH; ++k) z = fmaf(Ps[oW3 + o * kH + k], A2[k * kSt + t], z);
        out[o] = z;
    }
    float dout[kOut], loss = 0.f;
    nll_output_grad(out, s3[0], s3[1], s3[2], dout, loss);
    for (int o = 0; o < kOut; ++o) Do[o * kSt + t] = valid ? dout[o] : 0.f;
    // backward through the layers (per sample)
    for (int k = 0; k < kH; ++k) {
        float d = 0.f;
        for (int o = 0; o < kOut; ++o) d = fmaf(Ps[oW3 + o * kH + k], Do[o * kSt + t], d);
        D2[k * kSt + t] = A2[k * kSt + t] > 0.f ? d : 0.f;
    }
    for (int k = 0; k < kH; ++k) {
        float d = 0.f;
        for (int i = 0; i < kH; ++i) d = fmaf(Ps[oW2 + i * kH + k], D2[i * kSt + t], d);
        D1[k * kSt + t] = A1[k * kSt + t] > 0.f ? d : 0.f;
    }
    __syncthreads();
    // weight gradients: sums over the block's samples in sample order
    float *G = partial + (size_t)blockIdx.x * kParams;
    {
        const int i = t;   // hidden unit i (64 lanes)
        for (int k = 0; k < kIn; ++k) {
            float a = 0.f;
            for (int s = 0; s < kTB; ++s) a = fmaf(D1[i * kSt + s], X[k * kSt + s], a);
            G[oW1 + i * kIn + k] = a * scale;
        }
        float b1 = 0.f, b2 = 0.f;
        for (int s = 0; s < kTB; ++s) {
            b1 += D1[i * kSt + s];
            b2 += D2[i * kSt + s];
        }
        G[oB1 + i] = b1 * scale;
        G[oB2 + i] = b2 * scale;
        for (int k = 0; k < kH; ++k) {
            float a = 0.f;
            for (int s = 0; s < kTB; ++s) a = fmaf(D2[i * kSt + s], A1[k * kSt + s], a);
            G[oW2 + i * kH + k] = a * scale;
        }
        const int k = t;   // hidden unit k of layer 2 feeds W3[:, k]
        for (int o = 0; o < kOut; ++o) {
            float a = 0.f;
            for (int s = 0; s < kTB; ++s) a = fmaf(Do[o * kSt + s], A2[k * kSt + s], a);
            G[oW3 + o * kH + k] = a * scale;
        }
        if (t < kOut) {
            float b = 0.f;
            for (int s = 0; s < kTB; ++s) b += Do[t * kSt + s];
            G[oB3 + t] = b * scale;
        }
    }
    // block loss (fixed order)
    __syncthreads();
    Do[t] = valid ? loss : 0.f;
    __syncthreads();
    if (t == 0) {
        float a = 0.f;
        for (int s = 0; s < kTB; ++s) a += Do[s];
        loss_partial[blockIdx.x] = a;
    }
}

__global__ void mlp_reduce_kernel(const float *__restrict__ partial, int nblocks, float *__restrict__ grad,
                                  const float *__restrict__ loss_partial, float *__restrict__ loss_out)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < kParams) {
        float a = 0.f;
        for (int b = 0; b < nblocks; ++b) a += partial[(size_t)b * kParams + p];
        grad[p] = a;
    }
    if (p == 0 && loss_out) {
        float a = 0.f;
        for (int b = 0; b < nblocks; ++b) a += loss_partial[b];
        *loss_out += a;
    }
}

__global__ void mlp_adam_kernel(float *__restrict__ P, const float *__restrict__ g, float *__restrict__ m,
                                float *__restrict__ v, float lr, float c1, float c2)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kParams) return;
    const float b1 = 0.9f, b2 = 0.999f, e = 1e-8f;
    const float gi = g[p];
    const float mi = b1 * m[p] + (1.f - b1) * gi;
    const float vi = b2 * v[p] + (1.f - b2) * gi * gi;
    m[p] = mi;
    v[p] = vi;
    P[p] -= lr * (mi / c1) / (sqrtf(vi / c2) + e);
}

__global__ void fill_zero_kernel(float *p, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.f;
}

constexpr size_t kGradLds = sizeof(float) * (kParams + kSt * (kIn + kH + kH + kOut + kH + kH));

}  // namespace mlp
}  // namespace rewl

using namespace rewl;
using namespace rewl::mlp;

namespace {
rewl_status mfail(rewl_status c, const char *m) { return rewl::report_error(c, m); }
constexpr size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

// workspace: m, v, grad (kParams each), loss slot, partials, loss partials
struct Ws {
    float *m, *v, *g, *loss, *partial, *lossp;
};
Ws carve(void *w, int nblocks)
{
    unsigned char *p = (unsigned char *)w;
    Ws s;
    size_t o = 0;
    s.m = (float *)(p + o);
    o = al256(o + sizeof(float) * kParams);
    s.v = (float *)(p + o);
    o = al256(o + sizeof(float) * kParams);
    s.g = (float *)(p + o);
    o = al256(o + sizeof(float) * kParams);
    s.loss = (float *)(p + o);
    o = al256(o + sizeof(float));
    s.partial = (float *)(p + o);
    o = al256(o + sizeof(float) * kParams * (size_t)nblocks);
    s.lossp = (float *)(p + o);
    return s;
}
constexpr size_t ws_bytes(int nblocks)
{
    return al256(sizeof(float) * kParams) * 3 + 256 + al256(sizeof(float) * kParams * (size_t)nblocks) +
           al256(sizeof(float) * (size_t)nblocks);
}

rewl_status grad_step(const float *rec, int64_t n, int32_t count, int32_t random_pick, uint32_t seed,
                      uint64_t step, const float *P, const Ws &w, float *grad_out, bool add_loss,
                      hipStream_t s)
{
    const int nblocks = (count + kTB - 1) / kTB;
    hipLaunchKernelGGL(mlp_grad_kernel, dim3(nblocks), dim3(kTB), kGradLds, s, P, rec, n, count, random_pick,
                       seed, step, 1.0f / (float)count, w.partial, w.lossp);
    hipLaunchKernelGGL(mlp_reduce_kernel, dim3((kParams + 255) / 256), dim3(256), 0, s, w.partial, nblocks,
                       grad_out, w.lossp, add_loss ? w.loss : nullptr);
    return hipGetLastError() == hipSuccess ? REWL_OK : mfail(REWL_EDEVICE, "mlp kernel launch failed");
}
// Workspace of rewl_mlp_train_static: a file-scope device array, one copy per
// GPU, sized for minibatches of up to kStaticMaxBatch records.  Host code
// never uses the array's name as an address: each device's address comes
// from hipGetSymbolAddress, taken once per device with that device current.
constexpr int kStaticMaxBatch = 8192;
constexpr size_t kStaticScratchBytes = ws_bytes((kStaticMaxBatch + kTB - 1) / kTB);
constexpr int kMaxDevices = 64;
__device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

rewl_status static_scratch(void **out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) return mfail(REWL_EDEVICE, "no current device");
    if (dev >= kMaxDevices) return mfail(REWL_EUNSUPPORTED, "device index beyond the static workspace table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p)
            return mfail(REWL_EDEVICE, "hipGetSymbolAddress of the static workspace failed");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return REWL_OK;
}
}  // namespace

namespace rewl {
int launch_mlp_pack(const float *dev_params, void *dev_packed, hipStream_t s)
{
    hipLaunchKernelGGL(mlp_pack_kernel, dim3(1), dim3(64), 0, s, dev_params, (Lane *)dev_packed);
    return hipGetLastError() == hipSuccess ? REWL_OK : REWL_EDEVICE;
}
}  // namespace rewl

extern "C" {

int32_t rewl_mlp_param_count(void) { return kParams; }

size_t rewl_mlp_packed_bytes(void) { return sizeof(Lane) * 64; }

rewl_status rewl_mlp_workspace_bytes(int64_t max_batch, size_t *bytes)
{
    if (max_batch < 1 || !bytes) return mfail(REWL_EINVAL, "bad arguments");
    *bytes = ws_bytes((int)((max_batch + kTB - 1) / kTB));
    return REWL_OK;
}

rewl_status rewl_mlp_pack(const float *dev_params, void *dev_packed, void *hip_stream)
{
    if (!dev_params || !dev_packed) return mfail(REWL_EINVAL, "null pointer");
    return launch_mlp_pack(dev_params, dev_packed, (hipStream_t)hip_stream) == REWL_OK
               ? REWL_OK : mfail(REWL_EDEVICE, "pack launch failed");
}

rewl_status rewl_mlp_eval(const void *dev_packed, const float *dev_x, const float *dev_s, const float *dev_u,
                          const float *dev_udir, float *dev_lnq_s, float *dev_sample, float *dev_lnq_sample,
                          int64_t n, void *hip_stream)
{
    if (!dev_packed || !dev_x || !dev_s || !dev_u || !dev_udir || !dev_lnq_s || !dev_sample || !dev_lnq_sample)
        return mfail(REWL_EINVAL, "null pointer");
    if (n < 0) return mfail(REWL_EINVAL, "negative count");
    if (n == 0) return REWL_OK;
    const int64_t blocks = std::min<int64_t>((n + 15) / 16, 4096);
    hipLaunchKernelGGL(mlp_eval_kernel, dim3((unsigned)blocks), dim3(64), 0, (hipStream_t)hip_stream,
                       (const Lane *)dev_packed, dev_x, dev_s, dev_u, dev_udir, dev_lnq_s, dev_sample,
                       dev_lnq_sample, n);
    return hipGetLastError() == hipSuccess ? REWL_OK : mfail(REWL_EDEVICE, "eval launch failed");
}

rewl_status rewl_mlp_loss_grad(const float *dev_records, int64_t n, const float *dev_params, float *dev_grad,
                               double *loss_out, void *dev_workspace, void *hip_stream)
{
    if (!dev_records || !dev_params || !dev_grad || !loss_out || !dev_workspace) return mfail(REWL_EINVAL, "null pointer");
    if (n < 1 || n > (1 << 24)) return mfail(REWL_EINVAL, "n out of range");
    hipStream_t s = (hipStream_t)hip_stream;
    const int nblocks = (int)((n + kTB - 1) / kTB);
    Ws w = carve(dev_workspace, nblocks);
    hipLaunchKernelGGL(fill_zero_kernel, dim3(1), dim3(64), 0, s, w.loss, 1);
    rewl_status st = grad_step(dev_records, n, (int32_t)n, 0, 0, 0, dev_params, w, dev_grad, true, s);
    if (st) return st;
    float l = 0.f;
    if (hipMemcpyAsync(&l, w.loss, sizeof l, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return mfail(REWL_EDEVICE, "loss read-back failed");
    *loss_out = (double)l / (double)n;
    return REWL_OK;
}

rewl_status rewl_mlp_train(const float *dev_records, int64_t n, int32_t epochs, int32_t batch, float lr,
                           uint64_t seed, float *dev_params, void *dev_workspace, float *loss_per_epoch,
                           void *hip_stream)
{
    if (!dev_records || !dev_params || !dev_workspace) return mfail(REWL_EINVAL, "null pointer");
    if (n < 1 || epochs < 0 || batch < 1 || batch > (1 << 20) || !(lr > 0.f)) return mfail(REWL_EINVAL, "bad arguments");
    hipStream_t s = (hipStream_t)hip_stream;
    const int nblocks = (batch + kTB - 1) / kTB;
    Ws w = carve(dev_workspace, nblocks);
    hipLaunchKernelGGL(fill_zero_kernel, dim3((kParams + 255) / 256), dim3(256), 0, s, w.m, kParams);
    hipLaunchKernelGGL(fill_zero_kernel, dim3((kParams + 255) / 256), dim3(256), 0, s, w.v, kParams);
    const int64_t steps_per_epoch = std::max<int64_t>(1, n / batch);
    uint64_t step = 0;
    double b1t = 1.0, b2t = 1.0;
    for (int e = 0; e < epochs; ++e) {
        hipLaunchKernelGGL(fill_zero_kernel, dim3(1), dim3(64), 0, s, w.loss, 1);
        for (int64_t k = 0; k < steps_per_epoch; ++k) {
            rewl_status st = grad_step(dev_records, n, batch, 1, (uint32_t)seed, step, dev_params, w, w.g, true, s);
            if (st) return st;
            ++step;
            b1t *= 0.9;
            b2t *= 0.999;
            hipLaunchKernelGGL(mlp_adam_kernel, dim3((kParams + 255) / 256), dim3(256), 0, s, dev_params, w.g,
                               w.m, w.v, lr, (float)(1.0 - b1t), (float)(1.0 - b2t));
        }
        if (loss_per_epoch) {
            float l = 0.f;
            if (hipMemcpyAsync(&l, w.loss, sizeof l, hipMemcpyDeviceToHost, s) != hipSuccess ||
                hipStreamSynchronize(s) != hipSuccess)
                return mfail(REWL_EDEVICE, "loss read-back failed");
            loss_per_epoch[e] = l / (float)(steps_per_epoch * batch);
        }
    }
    if (hipGetLastError() != hipSuccess) return mfail(REWL_EDEVICE, "training launch failed");
    return REWL_OK;
}

rewl_status rewl_mlp_train_static(const float *dev_records, int64_t n, int32_t epochs, int32_t batch, float lr,
                                  uint64_t seed, float *dev_params, float *loss_per_epoch, void *hip_stream)
{
    if (batch > kStaticMaxBatch) return mfail(REWL_ERANGE, "batch above 8192 records, the static workspace's limit");
    void *ws = nullptr;
    rewl_status st = static_scratch(&ws);
    if (st) return st;
    // Adam moments and the loss slot are cleared by fill kernels inside the
    // call; the gradient partials are overwritten before they are read
    return rewl_mlp_train(dev_records, n, epochs, batch, lr, seed, dev_params, ws, loss_per_epoch, hip_stream);
}

}  // extern "C"
