// raster.hip -- per-tile DARBF compositing, forward and backward.
//
// One wavefront per 16x16 tile; lane l owns the four pixels of column l % 16
// in rows l/16, l/16 + 4, l/16 + 8, l/16 + 12.  The tile's instance list is
// consumed in batches of 64: lane l gathers the projected record of the
// batch's l-th instance, then the wave walks the batch with the record of
// instance s broadcast to scalar registers (v_readlane), so every pixel test
// reads its splat operands from SGPRs.  A ballot over the lanes' "done" bits
// ends the tile early once every pixel has saturated.
//
// Forward (DARB-Splatting section, alpha blending; per-kernel forward
// listings): E = d^T Q d with d = mu' - p, alpha = min(alpha_max, o F(E)),
// skip if E outside [0, e_max] or alpha < alpha_min, stop if T(1 - alpha) <
// t_min.  Writes the image and the checkpoint (final T, last position).
//
// Backward (per-kernel backward listings): walks each tile's list from the
// largest checkpointed position down, recomputing alpha with the same device
// function, T <- T / (1 - alpha), and accumulating the per-splat partial
// gradients of its four pixels in registers; per splat the wave sums the nine
// partials with DPP row reductions and one lane issues nine float atomics.
#include "common.h"

namespace darb {

namespace {

constexpr int kPix = 4;  // pixels per lane

struct Rec {
    float x, y, a, b, c, o, r, g, bl;
    uint32_t id;
    int hit;  // the footprint's bounding box meets this tile's pixels
};

// Record of instance j (zeros when `in` is false or the stored index is out of
// range; a zero-opacity record never passes the alpha test).  `hit` is false
// when the ellipse E <= e_max, grown by one pixel, misses the tile's pixel
// range: for |dx| > sqrt(e_max / Q_xx^-1) every E exceeds e_max by a relative
// margin far above FP32 rounding, so skipping such a splat changes nothing.
__device__ __forceinline__ Rec load_rec(const darb_projected &p, const uint32_t *vals, uint32_t j, bool in, int n,
                                        float e_max, float xlo, float ylo) {
    Rec R;
    R.x = R.y = R.a = R.b = R.c = R.o = R.r = R.g = R.bl = 0.0f;
    R.id = kNone;
    R.hit = 0;
    uint32_t id = in ? vals[j] : kNone;
    if (id < (uint32_t)n) {
        float2 xy = reinterpret_cast<const float2 *>(p.xy)[id];
        float4 co = reinterpret_cast<const float4 *>(p.conic_o)[id];
        R.x = xy.x;
        R.y = xy.y;
        R.a = co.x;
        R.b = co.y;
        R.c = co.z;
        R.o = co.w;
        R.r = p.rgb[3 * id];
        R.g = p.rgb[3 * id + 1];
        R.bl = p.rgb[3 * id + 2];
        R.id = id;
        // half-extents of {E <= e_max}: sqrt(e_max * Sigma'_xx), sqrt(e_max * Sigma'_yy), Sigma' = Q^-1
        float det = fmaf(co.x, co.z, -(co.y * co.y));
        float hx = sqrtf(e_max * co.z / det) + 1.0f;
        float hy = sqrtf(e_max * co.x / det) + 1.0f;
        bool ok = (det > 0.0f) ? ((xy.x + hx >= xlo) & (xy.x - hx <= xlo + (kTile - 1)) & (xy.y + hy >= ylo) &
                                  (xy.y - hy <= ylo + (kTile - 1)))
                               : true;
        R.hit = ok ? 1 : 0;
    }
    return R;
}

template <int KIND>
__global__ __launch_bounds__(64) void k_raster_fwd(darb_projected p, const uint32_t *__restrict__ vals,
                                                   const uint32_t *__restrict__ ranges, const int32_t *overflow, int n,
                                                   int W, int H, int gx, KParams kp, ROpts o, float *__restrict__ image,
                                                   float *__restrict__ final_T, uint32_t *__restrict__ last,
                                                   uint32_t *__restrict__ n_contrib) {
    if (overflow && *overflow) return;
    const int tile = blockIdx.x;
    const int tx = tile % gx, ty = tile / gx;
    const int lane = threadIdx.x;
    const int ix = tx * kTile + (lane & 15);
    const int iy0 = ty * kTile + (lane >> 4);
    const float px = (float)ix;
    float py[kPix];
    bool done[kPix];
    float T[kPix], C0[kPix], C1[kPix], C2[kPix];
    uint32_t lst[kPix], cnt[kPix];
#pragma unroll
    for (int k = 0; k < kPix; k++) {
        int iy = iy0 + 4 * k;
        py[k] = (float)iy;
        done[k] = !(ix < W && iy < H);
        T[k] = 1.0f;
        C0[k] = C1[k] = C2[k] = 0.0f;
        lst[k] = kNone;
        cnt[k] = 0;
    }
    const uint32_t start = ranges[2 * tile], end = ranges[2 * tile + 1];
    for (uint32_t base = start; base < end; base += 64) {
        bool alldone = done[0] & done[1] & done[2] & done[3];
        if (__ballot(!alldone) == 0) break;
        uint32_t j = base + lane;
        Rec R = load_rec(p, vals, j, j < end, n, kp.e_max, (float)(tx * kTile), (float)(ty * kTile));
        int nb = (int)min(64u, end - base);
        for (int s = 0; s < nb; s++) {
            if (!readlane_i(R.hit, s)) continue;  // footprint misses this tile (uniform)
            float sx = readlane_f(R.x, s), sy = readlane_f(R.y, s);
            float sa = readlane_f(R.a, s), sb = readlane_f(R.b, s), sc = readlane_f(R.c, s);
            float so = readlane_f(R.o, s);
            float sr = readlane_f(R.r, s), sg = readlane_f(R.g, s), sbl = readlane_f(R.bl, s);
            uint32_t pos = base + s;
#pragma unroll
            for (int k = 0; k < kPix; k++) {
                Pair q = eval_pair<KIND>(sx, sy, sa, sb, sc, so, px, py[k], kp, o.alpha_min, o.alpha_max);
                bool ok = q.ok & !done[k];
                float Tn = T[k] * (1.0f - q.alpha);
                bool stop = ok & (Tn < o.t_min);
                ok = ok & !stop;
                done[k] = done[k] | stop;
                float aT = ok ? q.alpha * T[k] : 0.0f;
                C0[k] = fmaf(aT, sr, C0[k]);
                C1[k] = fmaf(aT, sg, C1[k]);
                C2[k] = fmaf(aT, sbl, C2[k]);
                T[k] = ok ? Tn : T[k];
                lst[k] = ok ? pos : lst[k];
                cnt[k] += ok ? 1u : 0u;
            }
        }
    }
    const size_t plane = (size_t)W * H;
#pragma unroll
    for (int k = 0; k < kPix; k++) {
        int iy = iy0 + 4 * k;
        if (ix < W && iy < H) {
            size_t pidx = (size_t)iy * W + ix;
            image[pidx] = fmaf(T[k], o.bg0, C0[k]);
            image[plane + pidx] = fmaf(T[k], o.bg1, C1[k]);
            image[2 * plane + pidx] = fmaf(T[k], o.bg2, C2[k]);
            final_T[pidx] = T[k];
            last[pidx] = lst[k];
            if (n_contrib) n_contrib[pidx] = cnt[k];
        }
    }
}

template <int KIND>
__global__ __launch_bounds__(64) void k_raster_bwd(darb_projected p, const uint32_t *__restrict__ vals,
                                                   const uint32_t *__restrict__ ranges, const int32_t *overflow, int n,
                                                   int W, int H, int gx, KParams kp, ROpts o,
                                                   const float *__restrict__ dL_dimg,
                                                   const float *__restrict__ final_T,
                                                   const uint32_t *__restrict__ last, darb_grads2d g2) {
    if (overflow && *overflow) return;
    const int tile = blockIdx.x;
    const int tx = tile % gx, ty = tile / gx;
    const int lane = threadIdx.x;
    const int ix = tx * kTile + (lane & 15);
    const int iy0 = ty * kTile + (lane >> 4);
    const float px = (float)ix;
    const size_t plane = (size_t)W * H;
    float py[kPix], T[kPix], S0[kPix], S1[kPix], S2[kPix], G0[kPix], G1[kPix], G2[kPix];
    uint32_t lp[kPix];  // last position + 1 (0 = no contributor or no pixel)
    uint32_t maxl = 0;
#pragma unroll
    for (int k = 0; k < kPix; k++) {
        int iy = iy0 + 4 * k;
        py[k] = (float)iy;
        lp[k] = 0;
        T[k] = 0.0f;
        S0[k] = S1[k] = S2[k] = G0[k] = G1[k] = G2[k] = 0.0f;
        if (ix < W && iy < H) {
            size_t pidx = (size_t)iy * W + ix;
            uint32_t l = last[pidx];
            if (l != kNone) {
                lp[k] = l + 1;
                T[k] = final_T[pidx];
                S0[k] = T[k] * o.bg0;
                S1[k] = T[k] * o.bg1;
                S2[k] = T[k] * o.bg2;
                G0[k] = dL_dimg[pidx];
                G1[k] = dL_dimg[plane + pidx];
                G2[k] = dL_dimg[2 * plane + pidx];
            }
        }
        maxl = max(maxl, lp[k]);
    }
    // wave maximum of the end positions
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) maxl = max(maxl, (uint32_t)__shfl_xor((int)maxl, off, 64));
    const uint32_t start = ranges[2 * tile], end = ranges[2 * tile + 1];
    maxl = min(maxl, end);  // a checkpoint always points inside its tile's range
    if (maxl == 0 || maxl <= start) return;
    // walk positions maxl-1 down to start in batches of 64
    for (uint32_t hi = maxl; hi > start;) {
        uint32_t cntb = min(64u, hi - start);
        uint32_t j = hi - 1 - lane;
        Rec R = load_rec(p, vals, j, (uint32_t)lane < cntb, n, kp.e_max, (float)(tx * kTile), (float)(ty * kTile));
        for (int s = 0; s < (int)cntb; s++) {
            if (!readlane_i(R.hit, s)) continue;  // footprint misses this tile (uniform)
            float sx = readlane_f(R.x, s), sy = readlane_f(R.y, s);
            float sa = readlane_f(R.a, s), sb = readlane_f(R.b, s), sc = readlane_f(R.c, s);
            float so = readlane_f(R.o, s);
            float sr = readlane_f(R.r, s), sg = readlane_f(R.g, s), sbl = readlane_f(R.bl, s);
            uint32_t pos1 = hi - (uint32_t)s;  // position + 1
            float gxy0 = 0.f, gxy1 = 0.f, gca = 0.f, gcb = 0.f, gcc = 0.f, gop = 0.f, gr = 0.f, gg = 0.f, gbl = 0.f;
            bool any = false;
#pragma unroll
            for (int k = 0; k < kPix; k++) {
                Pair q = eval_pair<KIND>(sx, sy, sa, sb, sc, so, px, py[k], kp, o.alpha_min, o.alpha_max);
                bool ok = q.ok & (pos1 <= lp[k]);
                any |= ok;
                float inv = __builtin_amdgcn_rcpf(1.0f - q.alpha);
                float Tb = T[k] * inv;
                float da = G0[k] * fmaf(sr, Tb, -S0[k] * inv);
                da = fmaf(G1[k], fmaf(sg, Tb, -S1[k] * inv), da);
                da = fmaf(G2[k], fmaf(sbl, Tb, -S2[k] * inv), da);
                float aT = q.alpha * Tb;
                float dE = so * profile_deriv<KIND>(q.E, q.w, kp) * da;
                float dE2 = 2.0f * dE;
                gr += ok ? aT * G0[k] : 0.0f;
                gg += ok ? aT * G1[k] : 0.0f;
                gbl += ok ? aT * G2[k] : 0.0f;
                gop += ok ? q.w * da : 0.0f;
                gxy0 += ok ? dE2 * q.q0 : 0.0f;
                gxy1 += ok ? dE2 * q.q1 : 0.0f;
                gca += ok ? dE * (q.dx * q.dx) : 0.0f;
                gcb += ok ? dE2 * (q.dx * q.dy) : 0.0f;
                gcc += ok ? dE * (q.dy * q.dy) : 0.0f;
                S0[k] = ok ? fmaf(aT, sr, S0[k]) : S0[k];
                S1[k] = ok ? fmaf(aT, sg, S1[k]) : S1[k];
                S2[k] = ok ? fmaf(aT, sbl, S2[k]) : S2[k];
                T[k] = ok ? Tb : T[k];
            }
            if (__ballot(any) != 0) {
                gxy0 = wave_sum_to_lane63(gxy0);
                gxy1 = wave_sum_to_lane63(gxy1);
                gca = wave_sum_to_lane63(gca);
                gcb = wave_sum_to_lane63(gcb);
                gcc = wave_sum_to_lane63(gcc);
                gop = wave_sum_to_lane63(gop);
                gr = wave_sum_to_lane63(gr);
                gg = wave_sum_to_lane63(gg);
                gbl = wave_sum_to_lane63(gbl);
                uint32_t id = (uint32_t)readlane_i((int)R.id, s);
                if (lane == 63 && id < (uint32_t)n) {
                    atomicAdd(&g2.xy[2 * id], gxy0);
                    atomicAdd(&g2.xy[2 * id + 1], gxy1);
                    atomicAdd(&g2.conic[3 * id], gca);
                    atomicAdd(&g2.conic[3 * id + 1], gcb);
                    atomicAdd(&g2.conic[3 * id + 2], gcc);
                    atomicAdd(&g2.opacity[id], gop);
                    atomicAdd(&g2.rgb[3 * id], gr);
                    atomicAdd(&g2.rgb[3 * id + 1], gg);
                    atomicAdd(&g2.rgb[3 * id + 2], gbl);
                }
            }
        }
        hi -= cntb;
    }
}

__global__ __launch_bounds__(256) void k_zero(float *a, size_t n) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) a[i] = 0.0f;
}

hipError_t zero(float *a, size_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    size_t blocks = std::min<size_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_zero, dim3((unsigned)blocks), dim3(256), 0, s, a, n);
    return hipGetLastError();
}

}  // namespace

#define DARB_KIND_SWITCH(kind, F, ...)                     \
    switch (kind) {                                        \
    case DARB_GAUSS: F<DARB_GAUSS> __VA_ARGS__; break;     \
    case DARB_HALF_COS: F<DARB_HALF_COS> __VA_ARGS__; break; \
    case DARB_RAISED_COS: F<DARB_RAISED_COS> __VA_ARGS__; break; \
    case DARB_SINC: F<DARB_SINC> __VA_ARGS__; break;       \
    case DARB_IMQ: F<DARB_IMQ> __VA_ARGS__; break;         \
    case DARB_IMQ_SQRT: F<DARB_IMQ_SQRT> __VA_ARGS__; break; \
    default: F<DARB_PARABOLA> __VA_ARGS__; break;          \
    }

template <int KIND>
static void fwd_launch(dim3 g, hipStream_t s, const darb_projected &p, const uint32_t *vals, const uint32_t *ranges,
                       const int32_t *ov, int n, int W, int H, int gx, const KParams &kp, const ROpts &o, float *image,
                       float *fT, uint32_t *last, uint32_t *nc) {
    hipLaunchKernelGGL(k_raster_fwd<KIND>, g, dim3(64), 0, s, p, vals, ranges, ov, n, W, H, gx, kp, o, image, fT, last,
                       nc);
}

template <int KIND>
static void bwd_launch(dim3 g, hipStream_t s, const darb_projected &p, const uint32_t *vals, const uint32_t *ranges,
                       const int32_t *ov, int n, int W, int H, int gx, const KParams &kp, const ROpts &o,
                       const float *dl, const float *fT, const uint32_t *last, const darb_grads2d &g2) {
    hipLaunchKernelGGL(k_raster_bwd<KIND>, g, dim3(64), 0, s, p, vals, ranges, ov, n, W, H, gx, kp, o, dl, fT, last,
                       g2);
}

hipError_t launch_raster_fwd(int kind, const darb_projected &p, int n, const uint32_t *vals, const uint32_t *ranges,
                             const int32_t *overflow, int width, int height, const KParams &kp, const ROpts &o,
                             float *image, float *final_T, uint32_t *last, uint32_t *n_contrib, hipStream_t s) {
    int gx = (width + kTile - 1) / kTile, gy = (height + kTile - 1) / kTile;
    dim3 g(gx * gy);
    DARB_KIND_SWITCH(kind, fwd_launch, (g, s, p, vals, ranges, overflow, n, width, height, gx, kp, o, image, final_T,
                                        last, n_contrib))
    return hipGetLastError();
}

hipError_t launch_raster_bwd(int kind, const darb_projected &p, int n, const uint32_t *vals, const uint32_t *ranges,
                             const int32_t *overflow, int width, int height, const KParams &kp, const ROpts &o,
                             const float *dL_dimage, const float *final_T, const uint32_t *last,
                             const darb_grads2d &g2d, hipStream_t s) {
    hipError_t e;
    if ((e = zero(g2d.xy, (size_t)n * 2, s)) != hipSuccess) return e;
    if ((e = zero(g2d.conic, (size_t)n * 3, s)) != hipSuccess) return e;
    if ((e = zero(g2d.opacity, (size_t)n, s)) != hipSuccess) return e;
    if ((e = zero(g2d.rgb, (size_t)n * 3, s)) != hipSuccess) return e;
    int gx = (width + kTile - 1) / kTile, gy = (height + kTile - 1) / kTile;
    dim3 g(gx * gy);
    DARB_KIND_SWITCH(kind, bwd_launch, (g, s, p, vals, ranges, overflow, n, width, height, gx, kp, o, dL_dimage,
                                        final_T, last, g2d))
    return hipGetLastError();
}

}  // namespace darb
