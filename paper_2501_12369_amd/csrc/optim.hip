// optim.hip -- the steps after the backward in a training iteration: one Adam
// step over several parameter tensors in one launch, and the per-splat
// densification statistics.  Both are elementwise and HBM-bound (Adam: 16 B
// read + 12 B written per value; statistics: 12 B read + 12 B read-modify-write
// per splat).
#include "common.h"

namespace darb {

namespace {

// Work item -> (group, element): groups are laid end to end in units of 256.
__global__ __launch_bounds__(256) void k_adam(AdamGroups G, float beta1, float beta2, float eps, float bc1,
                                              float bc2_sqrt) {
    int gi = 0;
    int64_t base = 0;
    const int64_t blk = blockIdx.x;
    for (int k = 0; k < G.ng; k++) {  // uniform: find the group of this block
        const int64_t nb = (G.g[k].n + 255) / 256;
        if (blk < base + nb) {
            gi = k;
            break;
        }
        base += nb;
    }
    const darb_adam_group &g = G.g[gi];
    const int64_t i = (blk - base) * 256 + threadIdx.x;
    if (i >= g.n) return;
    const float gr = g.grad[i];
    const float m = fmaf(beta1, g.m[i], (1.0f - beta1) * gr);
    const float v = fmaf(beta2, g.v[i], (1.0f - beta2) * (gr * gr));
    g.m[i] = m;
    g.v[i] = v;
    const float denom = sqrtf(v) / bc2_sqrt + eps;
    g.param[i] = g.param[i] - (g.lr / bc1) * (m / denom);
}

__global__ __launch_bounds__(256) void k_densify_stats(darb_grads2d g2, const int32_t *radius, int n,
                                                       float *grad_accum, int32_t *count, int32_t *max_radius) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const int r = radius[i];
    if (r <= 0) return;
    const float2 gxy = reinterpret_cast<const float2 *>(g2.xy)[i];
    grad_accum[i] += sqrtf(fmaf(gxy.x, gxy.x, gxy.y * gxy.y));
    count[i] += 1;
    if (max_radius) max_radius[i] = max(max_radius[i], r);
}

}  // namespace

hipError_t launch_adam(const AdamGroups &groups, float beta1, float beta2, float eps, float bc1, float bc2_sqrt,
                       hipStream_t s) {
    int64_t blocks = 0;
    for (int k = 0; k < groups.ng; k++) blocks += (groups.g[k].n + 255) / 256;
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_adam, dim3((unsigned)blocks), dim3(256), 0, s, groups, beta1, beta2, eps, bc1, bc2_sqrt);
    return hipGetLastError();
}

hipError_t launch_densify_stats(const darb_grads2d &g2d, const int32_t *radius, int n, float *grad_accum,
                                int32_t *count, int32_t *max_radius, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_densify_stats, dim3((n + 255) / 256), dim3(256), 0, s, g2d, radius, n, grad_accum, count,
                       max_radius);
    return hipGetLastError();
}

}  // namespace darb
