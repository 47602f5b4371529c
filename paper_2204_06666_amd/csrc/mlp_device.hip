// Learned parameter predictor: a fully connected network 32 -> 64 -> 64 -> 3
// (ReLU, ReLU, linear) in binary32, with forward, backward (mean squared
// error) and Adam kernels.  It maps the sparsity features of a matrix to the
// preprocessing parameters (partition size, ELL width, rows per wave) that
// the paper fixes by rule (Eq. 1) or leaves to the user.
//
// Mapping onto a 64-lane wavefront: lane j owns hidden unit j of both hidden
// layers, one sample at a time.  A layer's input is broadcast from the lane
// that holds it (readlane), so a layer is 32 or 64 fused multiply-adds per
// lane with the weights in LDS, laid out so that the 64 lanes read 64
// consecutive words (no bank conflicts).  The backward pass accumulates the
// gradient of one parameter row per lane in registers over the wave's
// samples; waves, then workgroups, are summed in a fixed order, so results
// are bitwise reproducible.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>

#include "internal.h"

using namespace ehyb;

namespace {

constexpr int kIn = EHYB_MLP_IN, kHid = EHYB_MLP_HIDDEN, kOut = EHYB_MLP_OUT;
// parameter layout: W1 [kHid][kIn], b1 [kHid], W2 [kHid][kHid], b2 [kHid], W3 [kOut][kHid], b3 [kOut]
constexpr int oW1 = 0, oB1 = oW1 + kHid * kIn, oW2 = oB1 + kHid, oB2 = oW2 + kHid * kHid, oW3 = oB2 + kHid,
              oB3 = oW3 + kOut * kHid, kParams = oB3 + kOut;
static_assert(kParams == EHYB_MLP_PARAMS, "parameter count");
static_assert(kHid == 64, "one hidden unit per lane of a wave64");
constexpr int kWaves = 4, kThreads = kWaves * 64;
constexpr int kMaxBlocks = 256;

struct Weights {
    float w1t[kIn][kHid];   // w1t[k][j] = W1[j][k]
    float w2t[kHid][kHid];  // w2t[i][j] = W2[j][i]   (forward: lane j reads row i)
    float w2[kHid][kHid];   // w2[j][i]  = W2[j][i]   (backward: lane i reads row j)
    float w3[kOut][kHid];
};
union MlpLds {
    Weights w;
    float acc[kParams + 1];  // block sum of the gradients (+ loss), after the samples
};

__device__ __forceinline__ float bcast(float v, int lane) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), lane));
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ void load_weights(const float* __restrict__ p, Weights& w, bool backward) {
    for (int t = threadIdx.x; t < kHid * kIn; t += kThreads) w.w1t[t % kIn][t / kIn] = p[oW1 + t];
    for (int t = threadIdx.x; t < kHid * kHid; t += kThreads) {
        const float v = p[oW2 + t];
        w.w2t[t % kHid][t / kHid] = v;
        if (backward) w.w2[t / kHid][t % kHid] = v;
    }
    for (int t = threadIdx.x; t < kOut * kHid; t += kThreads) w.w3[t / kHid][t % kHid] = p[oW3 + t];
}

struct Fwd {
    float z1, h1, z2, h2, y[kOut], x;  // per lane: unit `lane` of each layer; x = input `lane % kIn`
};

__device__ __forceinline__ void forward(const Weights& w, const float* __restrict__ p, const float* __restrict__ xb,
                                        int lane, Fwd& f) {
    f.x = xb[lane % kIn];
    float z1 = p[oB1 + lane];
#pragma unroll
    for (int k = 0; k < kIn; ++k) z1 = fmaf(w.w1t[k][lane], bcast(f.x, k), z1);
    f.z1 = z1;
    f.h1 = fmaxf(z1, 0.0f);
    float z2 = p[oB2 + lane];
#pragma unroll
    for (int i = 0; i < kHid; ++i) z2 = fmaf(w.w2t[i][lane], bcast(f.h1, i), z2);
    f.z2 = z2;
    f.h2 = fmaxf(z2, 0.0f);
#pragma unroll
    for (int o = 0; o < kOut; ++o) f.y[o] = wave_sum(w.w3[o][lane] * f.h2) + p[oB3 + o];
}

__global__ void __launch_bounds__(kThreads) mlp_forward_kernel(const float* __restrict__ p, int batch,
                                                               const float* __restrict__ X, float* __restrict__ Y) {
    __shared__ MlpLds lds;
    load_weights(p, lds.w, false);
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int gw = __builtin_amdgcn_readfirstlane(blockIdx.x * kWaves + (threadIdx.x >> 6));
    for (int b = gw; b < batch; b += gridDim.x * kWaves) {
        Fwd f;
        forward(lds.w, p, X + (size_t)b * kIn, lane, f);
        if (lane < kOut) Y[(size_t)b * kOut + lane] = lane == 0 ? f.y[0] : (lane == 1 ? f.y[1] : f.y[2]);
    }
}

// Loss = sum over samples and outputs of (y - t)^2, divided by batch * kOut.
// Each workgroup writes its gradient sum (parameter layout) and its share of
// the loss to partial[blockIdx.x][0 .. kParams].
__global__ void __launch_bounds__(kThreads) mlp_grad_kernel(const float* __restrict__ p, int batch,
                                                            const float* __restrict__ X, const float* __restrict__ T,
                                                            float* __restrict__ partial) {
    __shared__ MlpLds lds;
    load_weights(p, lds.w, true);
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int gw = __builtin_amdgcn_readfirstlane(blockIdx.x * kWaves + wave);
    const float scale = 2.0f / ((float)batch * (float)kOut);
    float gw1[kIn], gw2[kHid], gw3[kOut], gb3[kOut];
    float gb1 = 0.0f, gb2 = 0.0f, loss = 0.0f;
#pragma unroll
    for (int k = 0; k < kIn; ++k) gw1[k] = 0.0f;
#pragma unroll
    for (int i = 0; i < kHid; ++i) gw2[i] = 0.0f;
#pragma unroll
    for (int o = 0; o < kOut; ++o) gw3[o] = gb3[o] = 0.0f;
    for (int b = gw; b < batch; b += gridDim.x * kWaves) {
        Fwd f;
        forward(lds.w, p, X + (size_t)b * kIn, lane, f);
        float dh2 = 0.0f;
#pragma unroll
        for (int o = 0; o < kOut; ++o) {
            const float e = f.y[o] - T[(size_t)b * kOut + o];
            loss = fmaf(e, e, loss);
            const float dy = scale * e;
            gw3[o] = fmaf(dy, f.h2, gw3[o]);
            gb3[o] += dy;
            dh2 = fmaf(lds.w.w3[o][lane], dy, dh2);
        }
        const float dz2 = f.z2 > 0.0f ? dh2 : 0.0f;
        gb2 += dz2;
        float dh1 = 0.0f;
#pragma unroll
        for (int i = 0; i < kHid; ++i) gw2[i] = fmaf(dz2, bcast(f.h1, i), gw2[i]);
#pragma unroll
        for (int j = 0; j < kHid; ++j) dh1 = fmaf(lds.w.w2[j][lane], bcast(dz2, j), dh1);
        const float dz1 = f.z1 > 0.0f ? dh1 : 0.0f;
        gb1 += dz1;
#pragma unroll
        for (int k = 0; k < kIn; ++k) gw1[k] = fmaf(dz1, bcast(f.x, k), gw1[k]);
    }
    __syncthreads();  // weights no longer needed: the LDS becomes the block sum
    for (int w = 0; w < kWaves; ++w) {
        if (wave == w) {
            float* a = lds.acc;
            const bool first = w == 0;
#pragma unroll
            for (int k = 0; k < kIn; ++k) {
                float& d = a[oW1 + lane * kIn + k];
                d = first ? gw1[k] : d + gw1[k];
            }
            a[oB1 + lane] = first ? gb1 : a[oB1 + lane] + gb1;
#pragma unroll
            for (int i = 0; i < kHid; ++i) {
                float& d = a[oW2 + lane * kHid + i];
                d = first ? gw2[i] : d + gw2[i];
            }
            a[oB2 + lane] = first ? gb2 : a[oB2 + lane] + gb2;
#pragma unroll
            for (int o = 0; o < kOut; ++o) {
                float& d = a[oW3 + o * kHid + lane];
                d = first ? gw3[o] : d + gw3[o];
            }
            if (lane == 0) {
#pragma unroll
                for (int o = 0; o < kOut; ++o) a[oB3 + o] = first ? gb3[o] : a[oB3 + o] + gb3[o];
                a[kParams] = first ? loss : a[kParams] + loss;
            }
        }
        __syncthreads();
    }
    float* out = partial + (size_t)blockIdx.x * (kParams + 1);
    for (int t = threadIdx.x; t < kParams + 1; t += kThreads) out[t] = lds.acc[t];
}

// grad[t] = sum over blocks of partial[.][t] (block order), loss likewise, / (batch kOut).
__global__ void __launch_bounds__(256) mlp_reduce_kernel(const float* __restrict__ partial, int nblocks, int batch,
                                                         float* __restrict__ grad, float* __restrict__ loss) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t > kParams) return;
    float s = 0.0f;
    for (int b = 0; b < nblocks; ++b) s += partial[(size_t)b * (kParams + 1) + t];
    if (t < kParams) grad[t] = s;
    else if (loss) *loss = s / ((float)batch * (float)kOut);
}

// Adam (Kingma and Ba): m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
// p -= lr (m c1) / (sqrt(v c2) + eps) with the bias corrections c1, c2.
__global__ void __launch_bounds__(256) mlp_adam_kernel(float* __restrict__ p, const float* __restrict__ g,
                                                       float* __restrict__ m, float* __restrict__ v, float lr,
                                                       float b1, float b2, float eps, float c1, float c2) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= kParams) return;
    const float gt = g[t];
    const float mt = fmaf(b1, m[t], (1.0f - b1) * gt);
    const float vt = fmaf(b2, v[t], (1.0f - b2) * gt * gt);
    m[t] = mt;
    v[t] = vt;
    p[t] -= lr * (mt * c1) / (sqrtf(vt * c2) + eps);
}

int grad_blocks(int batch) { return std::max(1, std::min(kMaxBlocks, (batch + kWaves - 1) / kWaves)); }

// The workspace of ehyb_mlp_grad_noalloc: one row of partial sums per
// workgroup of the gradient kernel, for its largest grid (any batch), in a
// file-scope device array that each device holds until the process ends.
constexpr size_t kScratchFloats = (size_t)kMaxBlocks * (kParams + 1);
__device__ __align__(256) float scratch[kScratchFloats];

// Device address of `scratch` on each device, looked up once per device (the
// array's name in host code is a host-side stand-in, not a device address).
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float* g_scratch_ptr[kMaxDevices] = {};

ehyb_status scratch_for_current_device(float** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(EHYB_EDEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return fail(EHYB_EUNSUPPORTED, "device index above 63");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(EHYB_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = static_cast<float*>(ptr);
    }
    *out = g_scratch_ptr[dev];
    return EHYB_OK;
}

}  // namespace

extern "C" {

ehyb_status ehyb_mlp_forward(const float* params, int32_t batch, const float* X, float* Y, void* stream) {
    if (batch < 0) return fail(EHYB_EINVAL, "batch must be >= 0");
    if (batch == 0) return ok();
    if (!params || !X || !Y) return fail(EHYB_EINVAL, "null pointer");
    const int nb = std::max(1, std::min(1024, (batch + kWaves - 1) / kWaves));
    hipLaunchKernelGGL(mlp_forward_kernel, dim3(nb), dim3(kThreads), 0, (hipStream_t)stream, params, batch, X, Y);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? ok() : fail(EHYB_EDEVICE, std::string("mlp forward launch: ") + hipGetErrorString(e));
}

ehyb_status ehyb_mlp_workspace_bytes(int32_t batch, size_t* bytes) {
    if (!bytes || batch < 1) return fail(EHYB_EINVAL, "batch must be >= 1");
    *bytes = (size_t)grad_blocks(batch) * (kParams + 1) * sizeof(float);
    return ok();
}

ehyb_status ehyb_mlp_grad(const float* params, int32_t batch, const float* X, const float* T, float* grad,
                          float* loss, void* workspace, size_t workspace_bytes, void* stream) {
    if (batch < 1) return fail(EHYB_EINVAL, "batch must be >= 1");
    if (!params || !X || !T || !grad || !workspace) return fail(EHYB_EINVAL, "null pointer");
    const int nb = grad_blocks(batch);
    if (workspace_bytes < (size_t)nb * (kParams + 1) * sizeof(float))
        return fail(EHYB_EINVAL, "workspace smaller than ehyb_mlp_workspace_bytes");
    hipStream_t s = (hipStream_t)stream;
    float* part = (float*)workspace;
    hipLaunchKernelGGL(mlp_grad_kernel, dim3(nb), dim3(kThreads), 0, s, params, batch, X, T, part);
    hipLaunchKernelGGL(mlp_reduce_kernel, dim3((kParams + 1 + 255) / 256), dim3(256), 0, s, part, nb, batch, grad,
                       loss);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? ok() : fail(EHYB_EDEVICE, std::string("mlp grad launch: ") + hipGetErrorString(e));
}

ehyb_status ehyb_mlp_grad_noalloc(const float* params, int32_t batch, const float* X, const float* T, float* grad,
                                  float* loss, void* stream) {
    if (batch < 1) return fail(EHYB_EINVAL, "batch must be >= 1");
    if (!params || !X || !T || !grad) return fail(EHYB_EINVAL, "null pointer");
    const int nb = grad_blocks(batch);
    if ((size_t)nb * (kParams + 1) > kScratchFloats)
        return fail(EHYB_EUNSUPPORTED, "gradient workspace larger than the library's static scratch");
    float* part = nullptr;
    const ehyb_status st = scratch_for_current_device(&part);
    if (st != EHYB_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    // every workgroup writes its whole row of partial sums before the reduction
    // reads it: nothing in the scratch needs clearing between calls
    hipLaunchKernelGGL(mlp_grad_kernel, dim3(nb), dim3(kThreads), 0, s, params, batch, X, T, part);
    hipLaunchKernelGGL(mlp_reduce_kernel, dim3((kParams + 1 + 255) / 256), dim3(256), 0, s, part, nb, batch, grad,
                       loss);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? ok() : fail(EHYB_EDEVICE, std::string("mlp grad launch: ") + hipGetErrorString(e));
}

ehyb_status ehyb_mlp_adam(float* params, const float* grad, float* m, float* v, int32_t step, float lr,
                          float beta1, float beta2, float eps, void* stream) {
    if (!params || !grad || !m || !v) return fail(EHYB_EINVAL, "null pointer");
    if (step < 1 || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f))
        return fail(EHYB_EINVAL, "need step >= 1, beta1 and beta2 in [0, 1), eps > 0");
    const float c1 = (float)(1.0 / (1.0 - std::pow((double)beta1, (double)step)));
    const float c2 = (float)(1.0 / (1.0 - std::pow((double)beta2, (double)step)));
    hipLaunchKernelGGL(mlp_adam_kernel, dim3((kParams + 255) / 256), dim3(256), 0, (hipStream_t)stream, params, grad,
                       m, v, lr, beta1, beta2, eps, c1, c2);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? ok() : fail(EHYB_EDEVICE, std::string("mlp adam launch: ") + hipGetErrorString(e));
}

}  // extern "C"
