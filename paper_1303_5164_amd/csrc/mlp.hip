// The surrogate network that ranks candidate co-schedules: fully connected
// 16 -> 64 -> 64 -> 1 with ReLU, trained with mean-squared error and Adam.
// Parameters are one fp32 array, row-major W1 [16][64], b1 [64], W2 [64][64],
// b2 [64], W3 [64], b3 [1] (5313 values).
//
// Kernels (all launched by the entry points at the end of this file):
//   mlp_forward     one thread per sample; parameters staged in LDS; writes
//                   the prediction and, for training, z1 and z2 (pre-ReLU).
//   mlp_backward    one thread per sample: dy = 2 (y - t) / B, dz2, dz1.
//   mlp_grad_adam   one thread per parameter: its gradient summed over the
//                   batch in sample order (deterministic), then one Adam
//                   step (bias-corrected), or the raw gradient when asked.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <string>

#include "kernelet.h"

namespace {

constexpr int kIn = 16, kH = 64;
constexpr int kW1 = 0, kB1 = kIn * kH, kW2 = kB1 + kH, kB2 = kW2 + kH * kH, kW3 = kB2 + kH,
              kB3 = kW3 + kH, kN = kB3 + 1;
static_assert(kN == 5313, "parameter count");

__global__ __launch_bounds__(256) void mlp_forward(const float* __restrict__ params,
                                                   const float* __restrict__ x,
                                                   const int32_t* __restrict__ idx, uint32_t n,
                                                   float* __restrict__ y, float* __restrict__ z1,
                                                   float* __restrict__ z2) {
    __shared__ float p[kN];
    for (int i = threadIdx.x; i < kN; i += blockDim.x) p[i] = params[i];
    __syncthreads();
    const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const uint32_t row = idx ? (uint32_t)idx[s] : s;
    float xin[kIn];
#pragma unroll
    for (int i = 0; i < kIn; ++i) xin[i] = x[(size_t)row * kIn + i];
    float h1[kH];
#pragma unroll 4
    for (int j = 0; j < kH; ++j) {
        float a = p[kB1 + j];
#pragma unroll
        for (int i = 0; i < kIn; ++i) a = __builtin_fmaf(xin[i], p[kW1 + i * kH + j], a);
        if (z1) z1[(size_t)s * kH + j] = a;
        h1[j] = a > 0.f ? a : 0.f;
    }
    float out = p[kB3];
    for (int j = 0; j < kH; ++j) {
        float a = p[kB2 + j];
#pragma unroll 8
        for (int i = 0; i < kH; ++i) a = __builtin_fmaf(h1[i], p[kW2 + i * kH + j], a);
        if (z2) z2[(size_t)s * kH + j] = a;
        out = __builtin_fmaf(a > 0.f ? a : 0.f, p[kW3 + j], out);
    }
    y[s] = out;
}

// dz2 = dy * W3 (z2 > 0); dz1 = (W2 dz2) (z1 > 0); dy = 2 (y - t) / B
__global__ __launch_bounds__(256) void mlp_backward(const float* __restrict__ params,
                                                    const float* __restrict__ t,
                                                    const int32_t* __restrict__ idx, uint32_t n,
                                                    const float* __restrict__ y,
                                                    const float* __restrict__ z1,
                                                    const float* __restrict__ z2,
                                                    float* __restrict__ dy,
                                                    float* __restrict__ dz1,
                                                    float* __restrict__ dz2) {
    __shared__ float p[kN];
    for (int i = threadIdx.x; i < kN; i += blockDim.x) p[i] = params[i];
    __syncthreads();
    const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const uint32_t row = idx ? (uint32_t)idx[s] : s;
    const float g = 2.0f * (y[s] - t[row]) / (float)n;
    dy[s] = g;
    float d2[kH];
#pragma unroll 8
    for (int j = 0; j < kH; ++j) {
        d2[j] = z2[(size_t)s * kH + j] > 0.f ? g * p[kW3 + j] : 0.f;
        dz2[(size_t)s * kH + j] = d2[j];
    }
    for (int i = 0; i < kH; ++i) {
        float a = 0.f;
#pragma unroll 8
        for (int j = 0; j < kH; ++j) a = __builtin_fmaf(p[kW2 + i * kH + j], d2[j], a);
        dz1[(size_t)s * kH + i] = z1[(size_t)s * kH + i] > 0.f ? a : 0.f;
    }
}

__global__ __launch_bounds__(256) void mlp_grad_adam(
    float* __restrict__ params, float* __restrict__ m, float* __restrict__ v,
    float* __restrict__ grad_out, const float* __restrict__ x, const int32_t* __restrict__ idx,
    uint32_t n, const float* __restrict__ z1, const float* __restrict__ z2,
    const float* __restrict__ dy, const float* __restrict__ dz1, const float* __restrict__ dz2,
    float lr, float beta1, float beta2, float eps, float c1, float c2) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= kN) return;
    float g = 0.f;
    if (k < kB1) {                      // dW1[i][j] = sum_s x[s][i] dz1[s][j]
        const int i = k / kH, j = k % kH;
        for (uint32_t s = 0; s < n; ++s) {
            const uint32_t row = idx ? (uint32_t)idx[s] : s;
            g = __builtin_fmaf(x[(size_t)row * kIn + i], dz1[(size_t)s * kH + j], g);
        }
    } else if (k < kW2) {               // db1[j]
        const int j = k - kB1;
        for (uint32_t s = 0; s < n; ++s) g += dz1[(size_t)s * kH + j];
    } else if (k < kB2) {               // dW2[i][j] = sum_s relu(z1[s][i]) dz2[s][j]
        const int i = (k - kW2) / kH, j = (k - kW2) % kH;
        for (uint32_t s = 0; s < n; ++s) {
            const float h = z1[(size_t)s * kH + i];
            if (h > 0.f) g = __builtin_fmaf(h, dz2[(size_t)s * kH + j], g);
        }
    } else if (k < kW3) {               // db2[j]
        const int j = k - kB2;
        for (uint32_t s = 0; s < n; ++s) g += dz2[(size_t)s * kH + j];
    } else if (k < kB3) {               // dW3[j] = sum_s relu(z2[s][j]) dy[s]
        const int j = k - kW3;
        for (uint32_t s = 0; s < n; ++s) {
            const float h = z2[(size_t)s * kH + j];
            if (h > 0.f) g = __builtin_fmaf(h, dy[s], g);
        }
    } else {                            // db3
        for (uint32_t s = 0; s < n; ++s) g += dy[s];
    }
    if (grad_out) grad_out[k] = g;
    if (!m) return;
    const float mk = beta1 * m[k] + (1.f - beta1) * g;
    const float vk = beta2 * v[k] + (1.f - beta2) * g * g;
    m[k] = mk;
    v[k] = vk;
    params[k] -= lr * (mk / c1) / (sqrtf(vk / c2) + eps);
}

}  // namespace

namespace kl {
void set_error(const std::string& msg);
}

#define KL_HIPC(call)                                                                   \
    do {                                                                                \
        hipError_t e_ = (call);                                                         \
        if (e_ != hipSuccess) {                                                         \
            kl::set_error(std::string(#call) + ": " + hipGetErrorString(e_));           \
            return KL_EHIP;                                                             \
        }                                                                               \
    } while (0)

extern "C" uint64_t kernelet_mlp_workspace_floats(uint32_t batch) {
    return (uint64_t)batch * (4 * kH + 2);
}

extern "C" kl_status kernelet_mlp_forward(const float* params, const float* x, uint32_t n,
                                          float* y, void* stream) {
    if (!params || !x || !y || n == 0) {
        kl::set_error("kernelet_mlp_forward: null pointer or n == 0");
        return KL_EINVAL;
    }
    hipStream_t st = (hipStream_t)stream;
    mlp_forward<<<(n + 255) / 256, 256, 0, st>>>(params, x, nullptr, n, y, nullptr, nullptr);
    KL_HIPC(hipGetLastError());
    return KL_OK;
}

// One step over the samples idx[0..batch): gradient of the mean-squared error,
// then Adam (when m and v are given) at step `step` (>= 1).
extern "C" kl_status kernelet_mlp_train_step(float* params, float* m, float* v,
                                             const float* x, const float* t,
                                             const int32_t* idx, uint32_t batch,
                                             uint32_t step, float lr, float* grad_out,
                                             float* workspace, void* stream) {
    if (!params || !x || !t || batch == 0 || !workspace || ((m == nullptr) != (v == nullptr)) ||
        (m && step == 0) || (!m && !grad_out)) {
        kl::set_error("kernelet_mlp_train_step: bad arguments");
        return KL_EINVAL;
    }
    hipStream_t st = (hipStream_t)stream;
    float* ws = workspace;
    float* y = ws;
    float* dy = y + batch;
    float* z1 = dy + batch;
    float* z2 = z1 + (size_t)batch * kH;
    float* dz1 = z2 + (size_t)batch * kH;
    float* dz2 = dz1 + (size_t)batch * kH;
    const unsigned g = (batch + 255) / 256;
    mlp_forward<<<g, 256, 0, st>>>(params, x, idx, batch, y, z1, z2);
    KL_HIPC(hipGetLastError());
    mlp_backward<<<g, 256, 0, st>>>(params, t, idx, batch, y, z1, z2, dy, dz1, dz2);
    KL_HIPC(hipGetLastError());
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float c1 = m ? 1.f - powf(b1, (float)step) : 1.f;
    const float c2 = m ? 1.f - powf(b2, (float)step) : 1.f;
    mlp_grad_adam<<<(kN + 255) / 256, 256, 0, st>>>(params, m, v, grad_out, x, idx, batch, z1,
                                                     z2, dy, dz1, dz2, lr, b1, b2, eps, c1, c2);
    KL_HIPC(hipGetLastError());
    return KL_OK;
}

// ------------------------------------------------- training without allocation
// The training step's workspace held in a file-scope device array, for
// callers that cannot allocate device memory.  Each device the library runs
// on holds its own copy until the process ends; host code reaches it only
// through the address hipGetSymbolAddress returns for the current device.
namespace {

constexpr uint32_t kNoAllocMaxBatch = 4096;
constexpr size_t kScratchFloats = (size_t)kNoAllocMaxBatch * (4 * kH + 2);
static __device__ __align__(256) float scratch[kScratchFloats];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float* g_scratch_ptr[kMaxDevices] = {};

// The current device's copy of `scratch` (looked up once per device, with
// that device current).  Null, with the error set, on failure.
float* scratch_for_current_device() {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        kl::set_error(std::string("kernelet_mlp_train_step_noalloc: hipGetDevice: ") +
                      (e != hipSuccess ? hipGetErrorString(e) : "device index out of range"));
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            kl::set_error(std::string("kernelet_mlp_train_step_noalloc: hipGetSymbolAddress: ") +
                          hipGetErrorString(e));
            return nullptr;
        }
        g_scratch_ptr[dev] = (float*)p;
    }
    return g_scratch_ptr[dev];
}

}  // namespace

extern "C" uint32_t kernelet_mlp_noalloc_max_batch(void) { return kNoAllocMaxBatch; }

extern "C" kl_status kernelet_mlp_train_step_noalloc(float* params, float* m, float* v,
                                                     const float* x, const float* t,
                                                     const int32_t* idx, uint32_t batch,
                                                     uint32_t step, float lr, float* grad_out,
                                                     void* stream) {
    if (batch > kNoAllocMaxBatch) {
        kl::set_error("kernelet_mlp_train_step_noalloc: batch " + std::to_string(batch) +
                      " exceeds the maximum of " + std::to_string(kNoAllocMaxBatch) +
                      " samples its static workspace holds");
        return KL_EINVAL;
    }
    float* ws = scratch_for_current_device();
    if (!ws) return KL_EHIP;
    // every workspace value the step reads is written by the same step
    // before it is read, so the previous call's contents need no clearing
    return kernelet_mlp_train_step(params, m, v, x, t, idx, batch, step, lr, grad_out, ws,
                                   stream);
}
