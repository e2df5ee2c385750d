// loss.hip -- per-pixel image loss of a rendered view and its gradient (the
// photometric term that feeds the raster backward).  One pass over the
// image: every element writes its gradient and adds its loss to a per-thread
// sum; the grid size depends only on the image size, and the partial sums are
// combined in a fixed order, so the loss value is reproducible bit for bit.
// HBM-bound (reads 2 x 12 B, writes 12 B per pixel).
#include <algorithm>

#include "common.h"

namespace darb {

namespace {

constexpr int kLossThreads = 256;

// Sum of a workgroup's values in a fixed order: DPP within each wave, then the
// four wave sums in wave order.
__device__ __forceinline__ float block_sum(float v, float *lds) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    v = wave_sum_to_lane63(v);
    if (lane == 63) lds[w] = v;
    __syncthreads();
    float t = 0.0f;
    if (threadIdx.x == 0)
        for (int k = 0; k < kLossThreads / 64; k++) t += lds[k];
    return t;
}

template <int LOSS>
__global__ __launch_bounds__(kLossThreads) void k_image_loss(const float *__restrict__ img,
                                                             const float *__restrict__ tgt, size_t count, float scale,
                                                             float *__restrict__ dL, float *__restrict__ partials) {
    __shared__ float lds[kLossThreads / 64];
    float acc = 0.0f;
    const size_t stride = (size_t)gridDim.x * kLossThreads;
    for (size_t i = (size_t)blockIdx.x * kLossThreads + threadIdx.x; i < count; i += stride) {
        const float a = img[i], b = tgt[i];
        if (dL) dL[i] = loss_grad<LOSS>(a, b, scale);
        acc += loss_value<LOSS>(a, b);
    }
    if (partials) {
        const float t = block_sum(acc, lds);
        if (threadIdx.x == 0) partials[blockIdx.x] = t;
    }
}

__global__ __launch_bounds__(kLossThreads) void k_loss_final(const float *partials, int nb, float scale, float *out) {
    __shared__ float lds[kLossThreads / 64];
    float acc = 0.0f;
    for (int i = threadIdx.x; i < nb; i += kLossThreads) acc += partials[i];
    const float t = block_sum(acc, lds);
    if (threadIdx.x == 0) out[0] = t * scale;
}

}  // namespace

hipError_t launch_image_loss(int loss, const float *image, const float *target, int width, int height, float scale,
                             float *dL_dimage, float *loss_dev, float *partials, hipStream_t s) {
    const size_t count = (size_t)3 * width * height;
    const unsigned nb = (unsigned)std::min<size_t>((count + kLossThreads - 1) / kLossThreads, kLossBlocks);
    float *parts = loss_dev ? partials : nullptr;
    if (loss == DARB_LOSS_L1)
        hipLaunchKernelGGL(k_image_loss<DARB_LOSS_L1>, dim3(nb), dim3(kLossThreads), 0, s, image, target, count, scale,
                           dL_dimage, parts);
    else
        hipLaunchKernelGGL(k_image_loss<DARB_LOSS_L2>, dim3(nb), dim3(kLossThreads), 0, s, image, target, count, scale,
                           dL_dimage, parts);
    if (loss_dev)
        hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(kLossThreads), 0, s, partials, (int)nb, scale, loss_dev);
    return hipGetLastError();
}

}  // namespace darb
