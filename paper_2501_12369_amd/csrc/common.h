// common.h -- device helpers shared by the libdarb kernels (gfx950, wave64).
//
// The library is compiled with -ffp-contract=off: every fused multiply-add is
// written explicitly with fmaf, so the forward and the backward raster kernels
// evaluate alpha with bit-identical arithmetic (the backward recovers the
// transmittance by dividing by (1 - alpha) and must see the same alpha).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "darb.h"

namespace darb {

constexpr int kTile = 16;
constexpr int kWave = 64;
constexpr uint32_t kNone = 0xFFFFFFFFu;
constexpr int kMaxTiles = 16384;
constexpr int kMaxSuperTiles = 1024;  // 8x8-tile groups used by the binning

// Per-launch constants of a DARBF (host-derived from darb_kernel).
struct KParams {
    float inv_xi;   // 1/xi
    float inv_xi2;  // 1/xi^2 (profiles of sqrt(E)/xi written as series in E/xi^2)
    float exp2_c;   // -log2(e)/xi  (Gaussian: exp(-E/xi) = exp2(E * exp2_c))
    float e_max;
    float psi;
    float rfac;       // binning radius in units of sqrt(lambda_max): 3, or sqrt(e_max) beyond E = 9
    float beta_half;  // beta / 2 of the modified kinds
    int family;       // modified kinds: 0 Gaussian, 1 half-cosine, 2 raised cosine, 3 sinc
};

struct ROpts {
    float alpha_min, alpha_max, t_min;
    float bg0, bg1, bg2;
};

// ---------------------------------------------------------------------------
// Profiles F(E) and dF/dE.  Trigonometric profiles are evaluated as truncated
// Taylor series in the squared argument (Horner form, explicit FMA); on the
// supports used (E/xi <= pi/2, or (sqrt(E)/xi)^2 <= pi^2) the truncation error
// stays below 1e-9 and the FP32 rounding dominates.  Values for E outside the
// support are never consumed (callers select on the support test).
// ---------------------------------------------------------------------------

// cos x as a series in u = x^2, valid for x in [0, pi/2]: sum_k (-1)^k u^k / (2k)!
__device__ __forceinline__ float cos_series_half(float u) {
    // sum_{k=0}^{7} (-1)^k u^k / (2k)!
    float p = -1.1470745597729725e-11f;  // -1/14!
    p = fmaf(p, u, 2.08767569878681e-09f);  // +1/12!
    p = fmaf(p, u, -2.755731922398589e-07f);  // -1/10!
    p = fmaf(p, u, 2.48015873015873e-05f);  // +1/8!
    p = fmaf(p, u, -0.001388888888888889f);  // -1/6!
    p = fmaf(p, u, 0.041666666666666664f);  // +1/4!
    p = fmaf(p, u, -0.5f);  // -1/2!
    return fmaf(p, u, 1.0f);  // +1/0!
}

// sin x / x as a series in u = x^2, valid for x in [0, pi/2]: sum_k (-1)^k u^k / (2k+1)!
__device__ __forceinline__ float sinc_series_half(float u) {
    // sum_{k=0}^{7} (-1)^k u^k / (2k+1)!
    float p = -7.647163731819816e-13f;  // -1/15!
    p = fmaf(p, u, 1.6059043836821613e-10f);  // +1/13!
    p = fmaf(p, u, -2.505210838544172e-08f);  // -1/11!
    p = fmaf(p, u, 2.7557319223985893e-06f);  // +1/9!
    p = fmaf(p, u, -0.0001984126984126984f);  // -1/7!
    p = fmaf(p, u, 0.008333333333333333f);  // +1/5!
    p = fmaf(p, u, -0.16666666666666666f);  // -1/3!
    return fmaf(p, u, 1.0f);  // +1/1!
}

// cos x, sin x / x and (x cos x - sin x) / x^3 as series in v = x^2, valid for x in [0, pi].
__device__ __forceinline__ float cos_series_full(float v) {
    // sum_{k=0}^{12} (-1)^k v^k / (2k)!
    float p = 1.6117375710961184e-24f;  // +1/24!
    p = fmaf(p, v, -8.896791392450574e-22f);  // -1/22!
    p = fmaf(p, v, 4.110317623312165e-19f);  // +1/20!
    p = fmaf(p, v, -1.5619206968586225e-16f);  // -1/18!
    p = fmaf(p, v, 4.779477332387385e-14f);  // +1/16!
    p = fmaf(p, v, -1.1470745597729725e-11f);  // -1/14!
    p = fmaf(p, v, 2.08767569878681e-09f);  // +1/12!
    p = fmaf(p, v, -2.755731922398589e-07f);  // -1/10!
    p = fmaf(p, v, 2.48015873015873e-05f);  // +1/8!
    p = fmaf(p, v, -0.001388888888888889f);  // -1/6!
    p = fmaf(p, v, 0.041666666666666664f);  // +1/4!
    p = fmaf(p, v, -0.5f);  // -1/2!
    return fmaf(p, v, 1.0f);  // +1/0!
}

__device__ __forceinline__ float sinc_series_full(float v) {
    // sum_{k=0}^{12} (-1)^k v^k / (2k+1)!
    float p = 6.446950284384474e-26f;  // +1/25!
    p = fmaf(p, v, -3.868170170630684e-23f);  // -1/23!
    p = fmaf(p, v, 1.9572941063391263e-20f);  // +1/21!
    p = fmaf(p, v, -8.22063524662433e-18f);  // -1/19!
    p = fmaf(p, v, 2.8114572543455206e-15f);  // +1/17!
    p = fmaf(p, v, -7.647163731819816e-13f);  // -1/15!
    p = fmaf(p, v, 1.6059043836821613e-10f);  // +1/13!
    p = fmaf(p, v, -2.505210838544172e-08f);  // -1/11!
    p = fmaf(p, v, 2.7557319223985893e-06f);  // +1/9!
    p = fmaf(p, v, -0.0001984126984126984f);  // -1/7!
    p = fmaf(p, v, 0.008333333333333333f);  // +1/5!
    p = fmaf(p, v, -0.16666666666666666f);  // -1/3!
    return fmaf(p, v, 1.0f);  // +1/1!
}

__device__ __forceinline__ float sincd_series_full(float v) {
    // (x cos x - sin x) / x^3 = sum_{j=0}^{11} (-1)^(j+1) (2j+2) / (2j+3)! v^j
    float p = 1.5472680682522736e-24f;  // +24/25!
    p = fmaf(p, v, -8.509974375387505e-22f);  // -22/23!
    p = fmaf(p, v, 3.9145882126782523e-19f);  // +20/21!
    p = fmaf(p, v, -1.4797143443923793e-16f);  // -18/19!
    p = fmaf(p, v, 4.498331606952833e-14f);  // +16/17!
    p = fmaf(p, v, -1.0706029224547743e-11f);  // -14/15!
    p = fmaf(p, v, 1.9270852604185937e-09f);  // +12/13!
    p = fmaf(p, v, -2.505210838544172e-07f);  // -10/11!
    p = fmaf(p, v, 2.2045855379188714e-05f);  // +8/9!
    p = fmaf(p, v, -0.0011904761904761906f);  // -6/7!
    p = fmaf(p, v, 0.03333333333333333f);  // +4/5!
    return fmaf(p, v, -0.3333333333333333f);  // -2/3!
}

// Modified forms (Table 1, generic roll-off beta): u = E^(beta/2) / xi, one
// template instantiation for the four families (kp.family is uniform per launch,
// so the selection is a scalar branch).  sin/cos come from the device math
// library: u may exceed the Taylor ranges above (several pulses).
__device__ __forceinline__ float modified_u(float E, const KParams &kp) {
    return E > 0.0f ? exp2f(kp.beta_half * log2f(E)) * kp.inv_xi : 0.0f;
}

__device__ __forceinline__ float modified_value(float u, const KParams &kp) {
    switch (kp.family) {
    case 0: return exp2f(-1.4426950408889634f * u);
    case 1: return cosf(u);
    case 2: return fmaf(0.5f, cosf(u), 0.5f);
    default: return u < 1e-3f ? fmaf(-u * u, 0.16666666666666666f, 1.0f) : fabsf(sinf(u)) / u;
    }
}

// dF/dE of the modified forms: dF/du * du/dE, du/dE = (beta/2) u / E (E > 0);
// at E = 0: 1/xi dF/du(0) for beta = 2, else 0.
__device__ __forceinline__ float modified_deriv(float E, float u, float w, const KParams &kp) {
    float dF;
    switch (kp.family) {
    case 0: dF = -w; break;
    case 1: dF = -sinf(u); break;
    case 2: dF = -0.5f * sinf(u); break;
    default: {
        float s, c;
        sincosf(u, &s, &c);
        const float g = u < 1e-3f ? -u * 0.3333333333333333f : (u * c - s) / (u * u);
        dF = (u < 1e-3f || s >= 0.0f) ? g : -g;
    }
    }
    const float du = E > 0.0f ? kp.beta_half * u / E : (kp.beta_half == 1.0f ? kp.inv_xi : 0.0f);
    // at E = 0 with beta = 2, dF/du(0) = -1 (Gaussian) or 0 (the trigonometric families)
    return dF * du;
}

template <int KIND>
__device__ __forceinline__ float profile(float E, const KParams &kp) {
    if constexpr (KIND >= DARB_GAUSS_BETA) {
        return modified_value(modified_u(E, kp), kp);
    } else if constexpr (KIND == DARB_GAUSS) {
        return __builtin_amdgcn_exp2f(E * kp.exp2_c);
    } else if constexpr (KIND == DARB_HALF_COS) {
        float x = E * kp.inv_xi;
        return cos_series_half(x * x);
    } else if constexpr (KIND == DARB_RAISED_COS) {
        return fmaf(0.5f, cos_series_full(E * kp.inv_xi2), 0.5f);
    } else if constexpr (KIND == DARB_SINC) {
        return sinc_series_full(E * kp.inv_xi2);
    } else if constexpr (KIND == DARB_IMQ) {
        return __builtin_amdgcn_rcpf(fmaf(E, kp.inv_xi, 1.0f));
    } else if constexpr (KIND == DARB_IMQ_SQRT) {
        return __builtin_amdgcn_rsqf(fmaf(E, kp.inv_xi, 1.0f));
    } else {
        return fmaf(-E, kp.inv_xi, 1.0f);
    }
}

// dF/dE given E and the profile value w = F(E).
template <int KIND>
__device__ __forceinline__ float profile_deriv(float E, float w, const KParams &kp) {
    if constexpr (KIND >= DARB_GAUSS_BETA) {
        return modified_deriv(E, modified_u(E, kp), w, kp);
    } else if constexpr (KIND == DARB_GAUSS) {
        return -w * kp.inv_xi;
    } else if constexpr (KIND == DARB_HALF_COS) {
        float x = E * kp.inv_xi;
        return -(x * sinc_series_half(x * x)) * kp.inv_xi;
    } else if constexpr (KIND == DARB_RAISED_COS) {
        return -0.25f * sinc_series_full(E * kp.inv_xi2) * kp.inv_xi2;
    } else if constexpr (KIND == DARB_SINC) {
        return 0.5f * sincd_series_full(E * kp.inv_xi2) * kp.inv_xi2;
    } else if constexpr (KIND == DARB_IMQ) {
        return -(w * w) * kp.inv_xi;
    } else if constexpr (KIND == DARB_IMQ_SQRT) {
        return -0.5f * (w * w * w) * kp.inv_xi;
    } else {
        return -kp.inv_xi;
    }
}

// One (pixel, splat) pair: offsets, Q d, E, profile, alpha, and the decision.
// The conic arrives as its upper-triangular factor, Q = L^T L with
// L = [[l00, l01], [0, l11]], so E = |L d|^2 is a sum of two squares: no
// cancellation for needle-like footprints, where a dx^2 + 2 b dx dy + c dy^2
// loses ~1e-3 in FP32 along the needle.  Q d = L^T (L d) feeds the gradients.
// Shared verbatim by the forward and the backward raster kernels.
struct Pair {
    float dx, dy, q0, q1, E, w, alpha;
    bool ok;
};

template <int KIND>
__device__ __forceinline__ Pair eval_pair(float sx, float sy, float l00, float l01, float l11, float o, float px,
                                          float py, const KParams &kp, float amin, float amax) {
    Pair p;
    p.dx = sx - px;
    p.dy = sy - py;
    const float t0 = fmaf(l00, p.dx, l01 * p.dy);
    const float t1 = l11 * p.dy;
    p.E = fmaf(t0, t0, t1 * t1);
    p.q0 = l00 * t0;
    p.q1 = fmaf(l01, t0, l11 * t1);
    bool inside = (p.E >= 0.0f) & (p.E <= kp.e_max);
    // outside the support the profile value is never used: every consumer
    // selects on `ok`, so no clamp of E is needed here
    p.w = profile<KIND>(p.E, kp);
    p.alpha = fminf(amax, o * p.w);
    p.ok = inside & (p.alpha >= amin);
    return p;
}

// ---------------------------------------------------------------------------
// Wavefront helpers (wave64).
// ---------------------------------------------------------------------------

__device__ __forceinline__ float readlane_f(float v, int lane) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

__device__ __forceinline__ int readlane_i(int v, int lane) { return __builtin_amdgcn_readlane(v, lane); }

// Sum over the 64 lanes with DPP row operations; the total lands in lane 63.
__device__ __forceinline__ float wave_sum_to_lane63(float v) {
    // within rows of 16: shr 1, 2, 4 (bound_ctrl=false keeps lanes without a source unchanged... use adds of zero)
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x111, 0xf, 0xf, false));  // row_shr:1
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x112, 0xf, 0xf, false));  // row_shr:2
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x114, 0xf, 0xf, false));  // row_shr:4
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x118, 0xf, 0xf, false));  // row_shr:8
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x142, 0xa, 0xf, false));  // row_bcast:15
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x143, 0xc, 0xf, false));  // row_bcast:31
    return v;
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

// Inclusive prefix sum over the 64 lanes (u32), via LDS-free shuffles.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        uint32_t t = __shfl_up(v, off, 64);
        if (lane >= off) v += t;
    }
    return v;
}

// ---------------------------------------------------------------------------
// Image losses whose gradient is per pixel (shared by the loss kernel and the
// fused forward+backward raster kernel, so both produce the same bits).
// scale = 1 / (3 W H): the loss is the mean over the three colour planes.
// ---------------------------------------------------------------------------

template <int LOSS>
__device__ __forceinline__ float loss_value(float img, float tgt) {
    float d = img - tgt;
    if constexpr (LOSS == DARB_LOSS_L1) return fabsf(d);
    else return d * d;
}

template <int LOSS>
__device__ __forceinline__ float loss_grad(float img, float tgt, float scale) {
    float d = img - tgt;
    if constexpr (LOSS == DARB_LOSS_L1) return d > 0.0f ? scale : (d < 0.0f ? -scale : 0.0f);
    else return (2.0f * scale) * d;
}

// ---------------------------------------------------------------------------
// Internal launchers (implemented per stage).
// ---------------------------------------------------------------------------

struct Cam {
    float R[9];  // R_cw
    float t[3];  // t_cw
    float campos[3];
    float fx, fy, cx, cy;
    int width, height;
    float near_z;
    double lim_x, lim_y;  // limits of |t_x/t_z|, |t_y/t_z| in J (FP64, as the projection); <= 0: no clamp
    float dilation;
};

constexpr int kMaxViews = DARB_MAX_VIEWS;

// One view as the raster kernels see it (device pointers; nullable where the
// entry point allows it).  item0 is the first work item (tile) of the view in a
// launch over several views; key0 = view index * n keys the deterministic
// reduction.
struct RView {
    darb_projected p;
    const uint32_t *vals, *ranges;
    const int32_t *overflow;
    float *image, *final_T;
    uint32_t *last, *n_contrib;
    const float *dL;      // upstream gradient [3][H][W] (backward from a checkpoint)
    const float *target;  // target image [3][H][W] (fused forward+backward)
    darb_grads2d g2;      // backward: the 2D gradients; forward: the buffers to clear when zero_n > 0
    int zero_n;           // forward: splat count of g2 to clear (0: none)
    float loss_scale;     // 1 / (3 W H)
    int W, H, gx;
    uint32_t item0, key0;
};

struct RViews {
    RView v[kMaxViews];
    int nv;
};

struct Cams {
    Cam c[kMaxViews];
    int nv;
    const darb_camera *dev;  // nullable: cameras read from device memory (c[] then only sizes the grid)
};

struct Projs {
    darb_projected p[kMaxViews];
};

// Per view: the 2D gradients, and the forward's colour checkpoint (dcolor,
// clamped; null when not kept).
struct G2s {
    darb_grads2d g[kMaxViews];
    const float *dcolor[kMaxViews];
    const uint8_t *clamped[kMaxViews];
};

// cam_dev (nullable): camera read from device memory instead of `cam`
// (whose width/height still size the tile grid)
hipError_t launch_preprocess(const Cam &cam, const darb_camera *cam_dev, const KParams &kp, int n,
                             const darb_splats &in, const darb_projected &out, hipStream_t s);
// parts: 1 the geometry (xy, depth, radius, conic_o), 2 the colour (rgb,
// clamped, dcolor; reads the geometry part's radius), 3 both in one kernel.
hipError_t launch_preprocess_parts(const Cam &cam, const KParams &kp, int n, const darb_splats &in,
                                   const darb_projected &out, int parts, hipStream_t s);
// ckpt (nullable): the forward's records of this view; its dcolor and clamped,
// when both set, replace the SH coefficients in the colour part of the chain
hipError_t launch_preprocess_bwd(const Cam &cam, const KParams &kp, int n, const darb_splats &in,
                                 const darb_projected *ckpt, const darb_grads2d &g2d, const darb_grads3d &g3d,
                                 bool accumulate, hipStream_t s);
hipError_t launch_preprocess_multi(const Cams &cams, const KParams &kp, int n, const darb_splats &in,
                                   const Projs &outs, hipStream_t s);
hipError_t launch_preprocess_bwd_multi(const Cams &cams, const KParams &kp, int n, const darb_splats &in,
                                       const G2s &g2, const darb_grads3d &g3d, hipStream_t s);

size_t binsort_workspace(int n, int width, int height, int64_t k_capacity);
int binsort_super_tiles(int width, int height);
hipError_t launch_bin_sort(const darb_projected &p, int n, int width, int height, int64_t k_capacity, void *ws,
                           uint64_t *keys, uint32_t *vals, uint32_t *ranges, int64_t *k_dev, int32_t *overflow_dev,
                           hipStream_t s);

// Device-count exclusive scan and stable LSD radix sort of (u32 key, u32 value)
// pairs (8-bit digits over the low `bits` key bits), shared by the binning and
// the deterministic gradient reduction.  `skip` must point at a device int
// (nonzero: every kernel returns at once).
size_t scan_parts_words(uint32_t max_count);
size_t radix_hist_words(uint32_t max_count);
hipError_t scan_u32(uint32_t *data, const uint32_t *count_dev, uint32_t max_count, uint32_t *parts,
                    uint32_t *total_out, const int32_t *skip, hipStream_t s);
// Sorted pairs end in (kA, vA) when the pass count ceil(bits/8) is even, else in (kB, vB).
// hist holds radix_hist_words(max_count) words.
hipError_t radix_sort_pairs(uint32_t *kA, uint32_t *vA, uint32_t *kB, uint32_t *vB, const uint32_t *count_dev,
                            uint32_t max_count, int bits, uint32_t *hist, const int32_t *skip, hipStream_t s);

// Raster launchers take one view (nv == 1) or several; `items` = tiles summed
// over the views.  Deterministic backward: `det_ws` of det_workspace() bytes.
hipError_t launch_raster_fwd(int kind, const RViews &V, uint32_t items, int n, const KParams &kp, const ROpts &o,
                             hipStream_t s);
size_t det_workspace(uint32_t items, uint64_t capacity);
// g2_zeroed: every view's 2D gradients are known to be zero (cleared by the
// forward), so the backward does not clear them first.
hipError_t launch_raster_bwd(int kind, const RViews &V, uint32_t items, int n, const KParams &kp, const ROpts &o,
                             void *det_ws, uint64_t det_capacity, bool g2_zeroed, hipStream_t s);
hipError_t launch_raster_fwdbwd(int kind, int loss, const RViews &V, uint32_t items, int n, const KParams &kp,
                                const ROpts &o, hipStream_t s);

constexpr uint32_t kLossBlocks = 1024;  // partial sums of the image loss (fixed, so the total is reproducible)
hipError_t launch_image_loss(int loss, const float *image, const float *target, int width, int height, float scale,
                             float *dL_dimage, float *loss_dev, float *partials, hipStream_t s);
size_t ssim_workspace(int width, int height);
hipError_t launch_ssim_loss(const float *image, const float *target, int width, int height, float lambda, float scale,
                            float *dL_dimage, float *loss_dev, void *ws, hipStream_t s);

constexpr int kMaxAdamGroups = 8;
struct AdamGroups {
    darb_adam_group g[kMaxAdamGroups];
    int ng;
};
hipError_t launch_adam(const AdamGroups &groups, float beta1, float beta2, float eps, float bc1, float bc2_sqrt,
                       hipStream_t s);
hipError_t launch_densify_stats(const darb_grads2d &g2d, const int32_t *radius, int n, float *grad_accum,
                                int32_t *count, int32_t *max_radius, hipStream_t s);

}  // namespace darb
