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

// ---------------------------------------------------------------------------
// L1 + D-SSIM (the training loss of the Backpropagation section: (1 - lambda)
// L1 + lambda (1 - SSIM)).  SSIM per channel with an 11x11 Gaussian window
// (sigma 1.5, separable, zero padding), C1 = 0.01^2, C2 = 0.03^2, averaged over
// the 3 W H values.  Forward: per 16x16 tile and channel, the five window sums
// (x, y, x^2, y^2, x y) by two LDS passes; SSIM and its partials with respect
// to mu_x, sigma_x^2 and sigma_xy go to three maps.  Backward: the window is
// symmetric, so the adjoint is the same zero-padded filter over those maps:
//   d sum_p SSIM_p / dx_q = (G * M)_q + 2 x_q (G * B)_q + y_q (G * C)_q,
//   M = A - 2 B mu_x - C mu_y,  A = dS/dmu_x,  B = dS/dsigma_x^2,  C = dS/dsigma_xy.
// ---------------------------------------------------------------------------

namespace darb {

namespace {

constexpr int kSsimR = 5;                      // window radius (11 taps)
constexpr int kSsimT = 16;                     // output tile
constexpr int kSsimH = kSsimT + 2 * kSsimR;    // 26: tile with halo

struct SsimWin {
    float g[2 * kSsimR + 1];
};

// Sum and its L1 partner over a 256-thread block in a fixed order.
__device__ __forceinline__ void block_sum2(float a, float b, float *lds, float &ta, float &tb) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    a = wave_sum_to_lane63(a);
    b = wave_sum_to_lane63(b);
    if (lane == 63) {
        lds[w] = a;
        lds[4 + w] = b;
    }
    __syncthreads();
    ta = tb = 0.0f;
    if (threadIdx.x == 0)
        for (int k = 0; k < 4; k++) {
            ta += lds[k];
            tb += lds[4 + k];
        }
}

__global__ __launch_bounds__(256) void k_ssim_fwd(const float *__restrict__ img, const float *__restrict__ tgt,
                                                  int W, int H, SsimWin win, float *__restrict__ maps,
                                                  float *__restrict__ partials) {
    __shared__ float sx[kSsimH][kSsimH], sy[kSsimH][kSsimH];
    __shared__ float hs[5][kSsimH][kSsimT];
    __shared__ float red[8];
    const int ch = blockIdx.z;
    const size_t plane = (size_t)W * H;
    const float *X = img + ch * plane, *Y = tgt + ch * plane;
    const int x0 = blockIdx.x * kSsimT - kSsimR, y0 = blockIdx.y * kSsimT - kSsimR;
    for (int k = threadIdx.x; k < kSsimH * kSsimH; k += 256) {
        const int r = k / kSsimH, c = k % kSsimH;
        const int gx = x0 + c, gy = y0 + r;
        const bool in = gx >= 0 && gx < W && gy >= 0 && gy < H;
        sx[r][c] = in ? X[(size_t)gy * W + gx] : 0.0f;
        sy[r][c] = in ? Y[(size_t)gy * W + gx] : 0.0f;
    }
    __syncthreads();
    // horizontal pass: 26 rows x 16 output columns
    for (int k = threadIdx.x; k < kSsimH * kSsimT; k += 256) {
        const int r = k / kSsimT, c = k % kSsimT;
        float a = 0.f, b = 0.f, aa = 0.f, bb = 0.f, ab = 0.f;
#pragma unroll
        for (int t = 0; t <= 2 * kSsimR; t++) {
            const float u = sx[r][c + t], v = sy[r][c + t], w = win.g[t];
            a = fmaf(w, u, a);
            b = fmaf(w, v, b);
            aa = fmaf(w, u * u, aa);
            bb = fmaf(w, v * v, bb);
            ab = fmaf(w, u * v, ab);
        }
        hs[0][r][c] = a;
        hs[1][r][c] = b;
        hs[2][r][c] = aa;
        hs[3][r][c] = bb;
        hs[4][r][c] = ab;
    }
    __syncthreads();
    const int tc = threadIdx.x % kSsimT, tr = threadIdx.x / kSsimT;
    float s[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int t = 0; t <= 2 * kSsimR; t++)
#pragma unroll
        for (int q = 0; q < 5; q++) s[q] = fmaf(win.g[t], hs[q][tr + t][tc], s[q]);
    const int px = blockIdx.x * kSsimT + tc, py = blockIdx.y * kSsimT + tr;
    float ssim = 0.0f, l1 = 0.0f;
    if (px < W && py < H) {
        const float C1 = 0.01f * 0.01f, C2 = 0.03f * 0.03f;
        const float mx = s[0], my = s[1];
        const float vx = s[2] - mx * mx, vy = s[3] - my * my, cxy = s[4] - mx * my;
        const float n1 = 2.0f * mx * my + C1, n2 = 2.0f * cxy + C2;
        const float d1 = mx * mx + my * my + C1, d2 = vx + vy + C2;
        const float id1 = 1.0f / d1, id2 = 1.0f / d2;
        ssim = n1 * n2 * id1 * id2;
        // partials of S = n1 n2 / (d1 d2)
        const float A = (2.0f * my * n2 * id1 * id2) - (2.0f * mx * ssim * id1);  // dS/dmu_x
        const float B = -ssim * id2;                                              // dS/dsigma_x^2
        const float C = 2.0f * n1 * id1 * id2;                                    // dS/dsigma_xy
        const size_t p = (size_t)py * W + px;
        maps[(0 * 3 + ch) * plane + p] = A - 2.0f * B * mx - C * my;
        maps[(1 * 3 + ch) * plane + p] = B;
        maps[(2 * 3 + ch) * plane + p] = C;
        l1 = fabsf(sx[tr + kSsimR][tc + kSsimR] - sy[tr + kSsimR][tc + kSsimR]);
    }
    if (partials) {
        float ta, tb;
        block_sum2(ssim, l1, red, ta, tb);
        const int blk = (blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
        if (threadIdx.x == 0) {
            partials[2 * blk] = ta;
            partials[2 * blk + 1] = tb;
        }
    }
}

__global__ __launch_bounds__(256) void k_ssim_bwd(const float *__restrict__ img, const float *__restrict__ tgt,
                                                  int W, int H, SsimWin win, const float *__restrict__ maps,
                                                  float lambda, float scale, float *__restrict__ dL) {
    __shared__ float sm[3][kSsimH][kSsimH];
    __shared__ float hs[3][kSsimH][kSsimT];
    const int ch = blockIdx.z;
    const size_t plane = (size_t)W * H;
    const int x0 = blockIdx.x * kSsimT - kSsimR, y0 = blockIdx.y * kSsimT - kSsimR;
    for (int k = threadIdx.x; k < kSsimH * kSsimH; k += 256) {
        const int r = k / kSsimH, c = k % kSsimH;
        const int gx = x0 + c, gy = y0 + r;
        const bool in = gx >= 0 && gx < W && gy >= 0 && gy < H;
        const size_t p = (size_t)gy * W + gx;
#pragma unroll
        for (int q = 0; q < 3; q++) sm[q][r][c] = in ? maps[(q * 3 + ch) * plane + p] : 0.0f;
    }
    __syncthreads();
    for (int k = threadIdx.x; k < kSsimH * kSsimT; k += 256) {
        const int r = k / kSsimT, c = k % kSsimT;
        float a[3] = {0.f, 0.f, 0.f};
#pragma unroll
        for (int t = 0; t <= 2 * kSsimR; t++)
#pragma unroll
            for (int q = 0; q < 3; q++) a[q] = fmaf(win.g[t], sm[q][r][c + t], a[q]);
#pragma unroll
        for (int q = 0; q < 3; q++) hs[q][r][c] = a[q];
    }
    __syncthreads();
    const int tc = threadIdx.x % kSsimT, tr = threadIdx.x / kSsimT;
    const int px = blockIdx.x * kSsimT + tc, py = blockIdx.y * kSsimT + tr;
    if (px >= W || py >= H) return;
    float a[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int t = 0; t <= 2 * kSsimR; t++)
#pragma unroll
        for (int q = 0; q < 3; q++) a[q] = fmaf(win.g[t], hs[q][tr + t][tc], a[q]);
    const size_t p = ch * plane + (size_t)py * W + px;
    const float x = img[p], y = tgt[p];
    const float dssim = a[0] + 2.0f * x * a[1] + y * a[2];
    const float d = x - y;
    const float gl1 = d > 0.0f ? 1.0f : (d < 0.0f ? -1.0f : 0.0f);
    dL[p] = scale * ((1.0f - lambda) * gl1 - lambda * dssim);
}

// loss = (1 - lambda) * sum|x - y| * scale + lambda * (1 - sum SSIM * scale), sums in block order
__global__ __launch_bounds__(256) void k_ssim_final(const float *partials, int nb, float lambda, float scale,
                                                    float *out) {
    __shared__ float red[8];
    float s = 0.f, l = 0.f;
    for (int i = threadIdx.x; i < nb; i += 256) {
        s += partials[2 * i];
        l += partials[2 * i + 1];
    }
    float ts, tl;
    block_sum2(s, l, red, ts, tl);
    if (threadIdx.x == 0) out[0] = (1.0f - lambda) * tl * scale + lambda * (1.0f - ts * scale);
}

SsimWin ssim_window() {
    SsimWin w;
    double g[2 * kSsimR + 1], sum = 0.0;
    for (int i = 0; i <= 2 * kSsimR; i++) {
        const double d = i - kSsimR;
        g[i] = exp(-d * d / (2.0 * 1.5 * 1.5));
        sum += g[i];
    }
    for (int i = 0; i <= 2 * kSsimR; i++) w.g[i] = (float)(g[i] / sum);
    return w;
}

}  // namespace

size_t ssim_workspace(int width, int height) {
    const size_t maps = (size_t)9 * width * height * 4;
    const size_t nb = (size_t)((width + kSsimT - 1) / kSsimT) * ((height + kSsimT - 1) / kSsimT) * 3;
    return ((maps + 255) & ~(size_t)255) + nb * 8;
}

hipError_t launch_ssim_loss(const float *image, const float *target, int width, int height, float lambda, float scale,
                            float *dL_dimage, float *loss_dev, void *ws, hipStream_t s) {
    const SsimWin win = ssim_window();
    float *maps = static_cast<float *>(ws);
    float *partials = reinterpret_cast<float *>(static_cast<char *>(ws) +
                                                (((size_t)9 * width * height * 4 + 255) & ~(size_t)255));
    dim3 grid((width + kSsimT - 1) / kSsimT, (height + kSsimT - 1) / kSsimT, 3);
    hipLaunchKernelGGL(k_ssim_fwd, grid, dim3(256), 0, s, image, target, width, height, win, maps,
                       loss_dev ? partials : nullptr);
    if (loss_dev)
        hipLaunchKernelGGL(k_ssim_final, dim3(1), dim3(256), 0, s, partials, (int)(grid.x * grid.y * grid.z), lambda,
                           scale, loss_dev);
    hipLaunchKernelGGL(k_ssim_bwd, grid, dim3(256), 0, s, image, target, width, height, win, maps, lambda, scale,
                       dL_dimage);
    return hipGetLastError();
}

}  // namespace darb
