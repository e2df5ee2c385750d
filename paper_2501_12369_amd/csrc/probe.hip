// probe.hip -- calibration kernels for the measured ceilings that the
// benchmark reports beside the published peaks: a streaming copy and a
// write-only fill (HBM), and chains of fused multiply-adds in FP32 and FP64
// (vector ALU, built like every kernel here without packed FP32).  They
// compute nothing of the method.
#include "common.h"

namespace darb {

namespace {

constexpr int kProbeThreads = 256;
constexpr int kChains = 8;  // independent FMA chains per lane (hides the FMA latency)

constexpr int kUnroll = 4;  // float4 per lane per round, all loads issued before the stores
constexpr int kRound = kProbeThreads * kUnroll;

__global__ __launch_bounds__(kProbeThreads) void k_probe_copy(const float4 *src, float4 *dst, int64_t n4) {
    for (int64_t b = (int64_t)blockIdx.x * kRound; b < n4; b += (int64_t)gridDim.x * kRound) {
        float4 v[kUnroll];
#pragma unroll
        for (int k = 0; k < kUnroll; k++) {
            const int64_t i = b + k * kProbeThreads + threadIdx.x;
            if (i < n4) v[k] = src[i];
        }
#pragma unroll
        for (int k = 0; k < kUnroll; k++) {
            const int64_t i = b + k * kProbeThreads + threadIdx.x;
            if (i < n4) dst[i] = v[k];
        }
    }
}

__global__ __launch_bounds__(kProbeThreads) void k_probe_fill(float4 *dst, int64_t n4, float v) {
    for (int64_t b = (int64_t)blockIdx.x * kRound; b < n4; b += (int64_t)gridDim.x * kRound) {
#pragma unroll
        for (int k = 0; k < kUnroll; k++) {
            const int64_t i = b + k * kProbeThreads + threadIdx.x;
            if (i < n4) dst[i] = make_float4(v, v, v, v);
        }
    }
}

// Each lane runs kChains independent chains a <- a * x + y for `iters`
// rounds and stores their sum (so that nothing is dead code): 2 kChains iters
// flops per lane.
template <typename T>
__global__ __launch_bounds__(kProbeThreads) void k_probe_fma(T *out, int64_t threads, int iters, T x, T y) {
    const int64_t i = (int64_t)blockIdx.x * kProbeThreads + threadIdx.x;
    if (i >= threads) return;
    T a[kChains];
#pragma unroll
    for (int k = 0; k < kChains; k++) a[k] = (T)(i + k) * (T)1e-9;
    for (int r = 0; r < iters; r++) {
#pragma unroll
        for (int k = 0; k < kChains; k++) a[k] = fma(a[k], x, y);
    }
    T s = 0;
#pragma unroll
    for (int k = 0; k < kChains; k++) s += a[k];
    out[i] = s;
}

// one round of kRound float4 per workgroup, at most 2^20 workgroups (then each loops)
unsigned probe_grid(int64_t n4) {
    const int64_t b = (n4 + kRound - 1) / kRound;
    return (unsigned)std::min<int64_t>(std::max<int64_t>(b, 1), (int64_t)1 << 20);
}

}  // namespace

int probe_fma_chains() { return kChains; }

hipError_t launch_probe_copy(const float *src, float *dst, int64_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_probe_copy, dim3(probe_grid(n / 4)), dim3(kProbeThreads), 0, s,
                       reinterpret_cast<const float4 *>(src), reinterpret_cast<float4 *>(dst), n / 4);
    return hipGetLastError();
}

hipError_t launch_probe_fill(float *dst, int64_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_probe_fill, dim3(probe_grid(n / 4)), dim3(kProbeThreads), 0, s,
                       reinterpret_cast<float4 *>(dst), n / 4, 0.0f);
    return hipGetLastError();
}

hipError_t launch_probe_fma32(float *out, int64_t threads, int iters, hipStream_t s) {
    if (threads == 0) return hipSuccess;
    const unsigned grid = (unsigned)((threads + kProbeThreads - 1) / kProbeThreads);
    hipLaunchKernelGGL(k_probe_fma<float>, dim3(grid), dim3(kProbeThreads), 0, s, out, threads, iters, 0.999f, 1e-3f);
    return hipGetLastError();
}

hipError_t launch_probe_fma64(double *out, int64_t threads, int iters, hipStream_t s) {
    if (threads == 0) return hipSuccess;
    const unsigned grid = (unsigned)((threads + kProbeThreads - 1) / kProbeThreads);
    hipLaunchKernelGGL(k_probe_fma<double>, dim3(grid), dim3(kProbeThreads), 0, s, out, threads, iters, 0.999,
                       1e-3);
    return hipGetLastError();
}

}  // namespace darb
