// api.hip -- the extern "C" entry points of libdarb: host-side argument
// validation, derivation of the per-launch constants, dispatch to the stage
// launchers.  Nothing here allocates device memory.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>

#include "common.h"

// Calibration probes (probe.hip): copy and fill of n floats (n a multiple of 4,
// 16-byte aligned), FMA chains over `threads` lanes (probe_fma_chains() chains
// of `iters` FMAs each per lane).
namespace darb {
int probe_fma_chains();
hipError_t launch_probe_copy(const float *src, float *dst, int64_t n, hipStream_t s);
hipError_t launch_probe_fill(float *dst, int64_t n, hipStream_t s);
hipError_t launch_probe_fma32(float *out, int64_t threads, int iters, hipStream_t s);
hipError_t launch_probe_fma64(double *out, int64_t threads, int iters, hipStream_t s);
// 1D signal reconstruction (fit1d.hip)
int fit1d_max_components();
int fit1d_max_samples();
hipError_t launch_fit1d(int kind, const KParams &kp, int batch, int n, int m, const float *x, const float *target,
                        float *params, float *adam_m, float *adam_v, int steps, int step0, const float lr[3],
                        float beta1, float beta2, float eps, float *loss, hipStream_t s);
// psi calibration (psi.hip)
size_t psi_workspace(int m, int n);
hipError_t launch_psi_calibrate(int kind, const KParams &kp, int m, const double *sigma, int n, float margin, void *ws,
                                double *cov2, double *fit, hipStream_t s);
}  // namespace darb

namespace {

thread_local char g_err[512] = "";

darb_status fail(darb_status st, const char *fmt, const char *what) {
    snprintf(g_err, sizeof(g_err), fmt, what);
    return st;
}

bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

#define REQUIRE_PTR(p)                                                                          \
    do {                                                                                        \
        if (!(p)) return fail(DARB_ERR_INVALID_ARG, "null pointer: %s", #p);                    \
        if (!aligned16(p)) return fail(DARB_ERR_INVALID_ARG, "pointer not 16-byte aligned: %s", #p); \
    } while (0)

#define OPT_PTR(p)                                                                              \
    do {                                                                                        \
        if ((p) && !aligned16(p)) return fail(DARB_ERR_INVALID_ARG, "pointer not 16-byte aligned: %s", #p); \
    } while (0)

darb_status hip_status(hipError_t e, const char *where) {
    if (e == hipSuccess) return DARB_OK;
    snprintf(g_err, sizeof(g_err), "%s: %s", where, hipGetErrorString(e));
    return DARB_ERR_HIP;
}

darb_status check_kernel(const darb_kernel *k, darb::KParams *kp) {
    if (!k) return fail(DARB_ERR_INVALID_ARG, "null pointer: %s", "kernel");
    if (k->kind < DARB_GAUSS || k->kind > DARB_SINC_BETA) return fail(DARB_ERR_INVALID_ARG, "%s", "unknown kernel kind");
    if (!(k->xi > 0.0f) || !isfinite(k->xi)) return fail(DARB_ERR_INVALID_ARG, "%s", "kernel xi must be > 0");
    if (!(k->psi > 0.0f) || !isfinite(k->psi)) return fail(DARB_ERR_INVALID_ARG, "%s", "kernel psi must be > 0");
    const bool modified = k->kind >= DARB_GAUSS_BETA;
    if (modified) {
        if (!(k->beta > 0.0f) || !(k->beta <= 8.0f))
            return fail(DARB_ERR_INVALID_ARG, "%s", "modified kernel beta must be in (0, 8]");
        if (!(k->e_max > 0.0f) || !(k->e_max <= 1024.0f))
            return fail(DARB_ERR_INVALID_ARG, "%s", "modified kernel e_max must be in (0, 1024]");
    } else {
        if (!(k->e_max > 0.0f) || !(k->e_max <= 9.0f))
            return fail(DARB_ERR_INVALID_ARG, "%s", "kernel e_max must be in (0, 9] for kinds 0..6");
        // the series of the trigonometric profiles cover the main lobe only
        const double xi = k->xi, em = k->e_max, tol = 1.0 + 1e-6;
        if (k->kind == DARB_HALF_COS && em / xi > 0.5 * M_PI * tol)
            return fail(DARB_ERR_INVALID_ARG, "%s", "half-cosine support beyond E/xi = pi/2 (use DARB_HALF_COS_BETA)");
        if ((k->kind == DARB_RAISED_COS || k->kind == DARB_SINC) && sqrt(em) / xi > M_PI * tol)
            return fail(DARB_ERR_INVALID_ARG, "%s", "support beyond sqrt(E)/xi = pi (use the modified kinds)");
    }
    kp->inv_xi = 1.0f / k->xi;
    kp->inv_xi2 = kp->inv_xi * kp->inv_xi;
    kp->exp2_c = (float)(-1.4426950408889634 / (double)k->xi);
    kp->e_max = k->e_max;
    kp->psi = k->psi;
    kp->rfac = k->e_max > 9.0f ? sqrtf(k->e_max) : 3.0f;
    kp->beta_half = modified ? 0.5f * k->beta : 0.0f;
    kp->family = modified ? k->kind - DARB_GAUSS_BETA : 0;
    return DARB_OK;
}

darb_status check_camera(const darb_camera *c, darb::Cam *cam) {
    if (!c) return fail(DARB_ERR_INVALID_ARG, "null pointer: %s", "camera");
    if (c->width <= 0 || c->height <= 0) return fail(DARB_ERR_INVALID_ARG, "%s", "camera width/height must be > 0");
    if (!(c->fx > 0.0f) || !(c->fy > 0.0f)) return fail(DARB_ERR_INVALID_ARG, "%s", "camera fx/fy must be > 0");
    if (!(c->near_z > 0.0f)) return fail(DARB_ERR_INVALID_ARG, "%s", "camera near_z must be > 0");
    if (!(c->dilation >= 0.0f)) return fail(DARB_ERR_INVALID_ARG, "%s", "camera dilation must be >= 0");
    for (int r = 0; r < 3; r++) {
        for (int k = 0; k < 3; k++) cam->R[r * 3 + k] = c->viewmat[r * 4 + k];
        cam->t[r] = c->viewmat[r * 4 + 3];
        cam->campos[r] = c->campos[r];
    }
    cam->fx = c->fx;
    cam->fy = c->fy;
    cam->cx = c->cx;
    cam->cy = c->cy;
    cam->width = c->width;
    cam->height = c->height;
    cam->near_z = c->near_z;
    if (c->jac_clamp > 0.0f) {
        cam->lim_x = (double)c->jac_clamp * (0.5 * (double)c->width) / (double)c->fx;
        cam->lim_y = (double)c->jac_clamp * (0.5 * (double)c->height) / (double)c->fy;
    } else {
        cam->lim_x = cam->lim_y = 0.0;
    }
    cam->dilation = c->dilation;
    return DARB_OK;
}

darb_status check_opts(const darb_raster_opts *o, darb::ROpts *ro) {
    if (!o) return fail(DARB_ERR_INVALID_ARG, "null pointer: %s", "opts");
    if (!(o->alpha_min >= 0.0f) || !(o->alpha_max > 0.0f) || !(o->alpha_max < 1.0f) || !(o->alpha_min <= o->alpha_max))
        return fail(DARB_ERR_INVALID_ARG, "%s", "opts need 0 <= alpha_min <= alpha_max < 1");
    if (!(o->t_min >= 0.0f) || !(o->t_min < 1.0f)) return fail(DARB_ERR_INVALID_ARG, "%s", "opts t_min must be in [0, 1)");
    *ro = darb::ROpts{o->alpha_min, o->alpha_max, o->t_min, o->bg[0], o->bg[1], o->bg[2]};
    return DARB_OK;
}

darb_status check_n(int64_t n) {
    if (n < 0) return fail(DARB_ERR_INVALID_ARG, "%s", "n must be >= 0");
    if (n > 0x7FFFFFFFll) return fail(DARB_ERR_UNSUPPORTED, "%s", "n must be < 2^31");
    return DARB_OK;
}

darb_status check_size(int32_t width, int32_t height) {
    if (width <= 0 || height <= 0) return fail(DARB_ERR_INVALID_ARG, "%s", "width/height must be > 0");
    int64_t gx = (width + darb::kTile - 1) / darb::kTile, gy = (height + darb::kTile - 1) / darb::kTile;
    if (gx * gy > darb::kMaxTiles) return fail(DARB_ERR_UNSUPPORTED, "%s", "more than 16384 tiles");
    if (darb::binsort_super_tiles(width, height) > darb::kMaxSuperTiles)
        return fail(DARB_ERR_UNSUPPORTED, "%s", "more than 1024 groups of 8x8 tiles (extreme aspect ratio)");
    return DARB_OK;
}

darb_status check_splats(const darb_splats *in, int64_t n) {
    if (!in) return fail(DARB_ERR_INVALID_ARG, "null pointer: %s", "splats");
    if (in->sh_degree < 0 || in->sh_degree > 3) return fail(DARB_ERR_INVALID_ARG, "%s", "sh_degree must be 0..3");
    if (n == 0) return DARB_OK;
    REQUIRE_PTR(in->means);
    REQUIRE_PTR(in->scales);
    REQUIRE_PTR(in->quats);
    REQUIRE_PTR(in->opacity);
    REQUIRE_PTR(in->sh);
    return DARB_OK;
}

darb_status check_projected(const darb_projected *p, int64_t n, bool need_all) {
    if (!p) return fail(DARB_ERR_INVALID_ARG, "null pointer: %s", "projected");
    if (n == 0) return DARB_OK;
    REQUIRE_PTR(p->xy);
    REQUIRE_PTR(p->depth);
    REQUIRE_PTR(p->radius);
    REQUIRE_PTR(p->extent);
    if (need_all) {
        REQUIRE_PTR(p->conic_o);
        REQUIRE_PTR(p->rgb);
        REQUIRE_PTR(p->clamped);
    }
    return DARB_OK;
}

darb_status check_g2d(const darb_grads2d *g, int64_t n) {
    if (!g) return fail(DARB_ERR_INVALID_ARG, "null pointer: %s", "grads2d");
    if (n == 0) return DARB_OK;
    REQUIRE_PTR(g->xy);
    REQUIRE_PTR(g->conic);
    REQUIRE_PTR(g->opacity);
    REQUIRE_PTR(g->rgb);
    return DARB_OK;
}

darb_status check_g3d(const darb_grads3d *g, int64_t n) {
    if (!g) return fail(DARB_ERR_INVALID_ARG, "null pointer: %s", "grads3d");
    if (n == 0) return DARB_OK;
    REQUIRE_PTR(g->means);
    REQUIRE_PTR(g->scales);
    REQUIRE_PTR(g->quats);
    REQUIRE_PTR(g->opacity);
    REQUIRE_PTR(g->sh);
    return DARB_OK;
}

darb::RView make_rview(const darb_projected &p, const uint32_t *vals, const uint32_t *ranges,
                        const int32_t *overflow, int width, int height) {
    darb::RView v{};
    v.p = p;
    v.vals = vals;
    v.ranges = ranges;
    v.overflow = overflow;
    v.W = width;
    v.H = height;
    v.gx = (width + darb::kTile - 1) / darb::kTile;
    v.loss_scale = 1.0f / (float)(3.0 * (double)width * (double)height);
    return v;
}

uint32_t tile_count(int width, int height) {
    return (uint32_t)(((width + darb::kTile - 1) / darb::kTile) * ((height + darb::kTile - 1) / darb::kTile));
}

#define TRY(x)                                  \
    do {                                        \
        darb_status _st = (x);                  \
        if (_st != DARB_OK) return _st;         \
    } while (0)


enum ViewNeed : unsigned {
    kNeedProj = 1u,      // projected splats (all fields)
    kNeedList = 2u,      // vals, ranges
    kNeedFwdOut = 4u,    // image, final_T, last
    kNeedImage = 8u,     // image only (final_T, last optional)
    kNeedBwdIn = 16u,    // final_T, last, dL_dimage
    kNeedTarget = 32u,   // target
    kNeedG2 = 64u,       // grads2d
};

// Validates views[0..nv) for what a call needs and builds the device view table.
darb_status check_views(const darb_view *views, int32_t nv, int64_t n, unsigned need, darb::RViews *rv,
                        darb::Cams *cams, uint32_t *items, uint64_t *cap_total) {
    if (!views) return fail(DARB_ERR_INVALID_ARG, "null pointer: %s", "views");
    if (nv < 1 || nv > DARB_MAX_VIEWS) return fail(DARB_ERR_INVALID_ARG, "%s", "nv must be in [1, DARB_MAX_VIEWS]");
    uint32_t it = 0;
    uint64_t cap = 0;
    if (rv) *rv = darb::RViews{};
    if (cams) *cams = darb::Cams{};
    for (int v = 0; v < nv; v++) {
        const darb_view &V = views[v];
        darb::Cam c;
        TRY(check_camera(&V.cam, &c));
        TRY(check_size(V.cam.width, V.cam.height));
        if (need & kNeedProj) TRY(check_projected(&V.proj, n, true));
        if (need & kNeedList) {
            if (n > 0) REQUIRE_PTR(V.vals);
            REQUIRE_PTR(V.ranges);
            OPT_PTR(V.overflow_dev);
            if (V.k_capacity < 0) return fail(DARB_ERR_INVALID_ARG, "%s", "view k_capacity must be >= 0");
            cap += (uint64_t)V.k_capacity;
        }
        if (need & kNeedFwdOut) {
            REQUIRE_PTR(V.image);
            REQUIRE_PTR(V.final_T);
            REQUIRE_PTR(V.last);
            OPT_PTR(V.n_contrib);
        }
        if (need & kNeedImage) {
            REQUIRE_PTR(V.image);
            OPT_PTR(V.final_T);
            OPT_PTR(V.last);
            OPT_PTR(V.n_contrib);
        }
        if (need & kNeedBwdIn) {
            REQUIRE_PTR(V.final_T);
            REQUIRE_PTR(V.last);
            REQUIRE_PTR(V.dL_dimage);
        }
        if (need & kNeedTarget) REQUIRE_PTR(V.target);
        if (need & kNeedG2) TRY(check_g2d(&V.grads2d, n));
        if (rv) {
            darb::RView r = make_rview(V.proj, V.vals, V.ranges, V.overflow_dev, V.cam.width, V.cam.height);
            r.image = V.image;
            r.final_T = V.final_T;
            r.last = V.last;
            r.n_contrib = V.n_contrib;
            r.dL = V.dL_dimage;
            r.target = V.target;
            r.g2 = V.grads2d;
            r.item0 = it;
            r.key0 = (uint32_t)((uint64_t)v * (uint64_t)n);
            rv->v[v] = r;
        }
        if (cams) cams->c[v] = c;
        it += tile_count(V.cam.width, V.cam.height);
    }
    if (rv) rv->nv = nv;
    if (cams) {
        cams->nv = nv;
        cams->dev = nullptr;
    }
    if (items) *items = it;
    if (cap_total) *cap_total = cap;
    return DARB_OK;
}

darb_status check_det(int64_t n, int32_t nv, uint64_t cap) {
    if ((uint64_t)nv * (uint64_t)n >= 0xFFFFFFFFull)
        return fail(DARB_ERR_UNSUPPORTED, "%s", "deterministic mode needs nv * n < 2^32 - 1");
    if (cap >= 0xFFFFFFFFull) return fail(DARB_ERR_UNSUPPORTED, "%s", "deterministic mode needs capacity < 2^32 - 1");
    return DARB_OK;
}

}  // namespace

extern "C" {

int32_t darb_version(void) { return DARB_ABI_VERSION; }

const char *darb_status_string(int32_t st) {
    switch (st) {
    case DARB_OK: return "ok";
    case DARB_ERR_INVALID_ARG: return "invalid argument";
    case DARB_ERR_CAPACITY: return "instance capacity exceeded";
    case DARB_ERR_HIP: return "HIP runtime error";
    case DARB_ERR_UNSUPPORTED: return "unsupported";
    default: return "unknown status";
    }
}

const char *darb_last_error(void) { return g_err; }

darb_status darb_preprocess(const darb_camera *cam, const darb_kernel *kernel, int64_t n, const darb_splats *in,
                            const darb_projected *out, void *stream) {
    darb::Cam c;
    darb::KParams kp;
    TRY(check_n(n));
    TRY(check_camera(cam, &c));
    TRY(check_kernel(kernel, &kp));
    TRY(check_size(cam->width, cam->height));
    TRY(check_splats(in, n));
    TRY(check_projected(out, n, true));
    g_err[0] = 0;
    return hip_status(darb::launch_preprocess(c, nullptr, kp, (int)n, *in, *out, (hipStream_t)stream),
                      "darb_preprocess");
}

darb_status darb_preprocess_parts(const darb_camera *cam, const darb_kernel *kernel, int64_t n, const darb_splats *in,
                                  const darb_projected *out, int32_t parts, void *stream) {
    if (parts < DARB_PRE_GEOMETRY || parts > (DARB_PRE_GEOMETRY | DARB_PRE_COLOUR)) {
        snprintf(g_err, sizeof(g_err), "parts must be 1, 2 or 3 (got %d)", (int)parts);
        return DARB_ERR_INVALID_ARG;
    }
    darb::Cam c;
    darb::KParams kp;
    TRY(check_n(n));
    TRY(check_camera(cam, &c));
    TRY(check_kernel(kernel, &kp));
    TRY(check_size(cam->width, cam->height));
    TRY(check_splats(in, n));
    TRY(check_projected(out, n, true));
    g_err[0] = 0;
    return hip_status(darb::launch_preprocess_parts(c, kp, (int)n, *in, *out, (int)parts, (hipStream_t)stream),
                      "darb_preprocess_parts");
}

darb_status darb_preprocess_cam_dev(const darb_camera *cam_dev, int32_t width, int32_t height,
                                    const darb_kernel *kernel, int64_t n, const darb_splats *in,
                                    const darb_projected *out, void *stream) {
    darb::KParams kp;
    TRY(check_n(n));
    REQUIRE_PTR(cam_dev);
    TRY(check_kernel(kernel, &kp));
    TRY(check_size(width, height));
    TRY(check_splats(in, n));
    TRY(check_projected(out, n, true));
    darb::Cam c{};
    c.width = width;
    c.height = height;
    g_err[0] = 0;
    return hip_status(darb::launch_preprocess(c, cam_dev, kp, (int)n, *in, *out, (hipStream_t)stream),
                      "darb_preprocess_cam_dev");
}

size_t darb_bin_sort_workspace(int64_t n, int32_t width, int32_t height, int64_t k_capacity) {
    if (n < 0 || n > 0x7FFFFFFFll || width <= 0 || height <= 0) return 0;
    if (k_capacity < 0 || k_capacity >= 0xFFFFFFFFll) return 0;
    int64_t gx = (width + darb::kTile - 1) / darb::kTile, gy = (height + darb::kTile - 1) / darb::kTile;
    if (gx * gy > darb::kMaxTiles || darb::binsort_super_tiles(width, height) > darb::kMaxSuperTiles) return 0;
    return darb::binsort_workspace((int)n, width, height, k_capacity);
}

namespace {

// The call behind darb_bin_sort and darb_bin_sort_noalloc: argument checks,
// the launches on `ws`, the optional blocking readback of K.
darb_status bin_sort_impl(const char *who, const darb_projected *proj, int64_t n, int32_t width, int32_t height,
                          int64_t k_capacity, void *ws, size_t ws_bytes, uint64_t *keys, uint32_t *vals,
                          uint32_t *ranges, int64_t *k_dev, int32_t *overflow_dev, int64_t *k_host, hipStream_t s) {
    g_err[0] = 0;
    TRY(hip_status(darb::launch_bin_sort(*proj, (int)n, width, height, k_capacity, ws, keys, vals, ranges, k_dev,
                                         overflow_dev, s),
                   who));
    if (k_host) {
        TRY(hip_status(hipMemcpyAsync(k_host, k_dev, sizeof(int64_t), hipMemcpyDeviceToHost, s), "darb_bin_sort readback"));
        TRY(hip_status(hipStreamSynchronize(s), "darb_bin_sort sync"));
        if (*k_host > k_capacity) {
            snprintf(g_err, sizeof(g_err), "instance count %lld exceeds capacity %lld", (long long)*k_host,
                     (long long)k_capacity);
            return DARB_ERR_CAPACITY;
        }
    }
    (void)ws_bytes;
    return DARB_OK;
}

darb_status check_bin_sort_args(const darb_projected *proj, int64_t n, int32_t width, int32_t height,
                                int64_t k_capacity, uint32_t *vals, uint32_t *ranges, int64_t *k_dev,
                                int32_t *overflow_dev, uint64_t *keys) {
    TRY(check_n(n));
    TRY(check_size(width, height));
    TRY(check_projected(proj, n, false));
    if (k_capacity < 0) return fail(DARB_ERR_INVALID_ARG, "%s", "k_capacity must be >= 0");
    if (k_capacity >= 0xFFFFFFFFll) return fail(DARB_ERR_UNSUPPORTED, "%s", "k_capacity must be < 2^32 - 1");
    REQUIRE_PTR(ranges);
    REQUIRE_PTR(k_dev);
    REQUIRE_PTR(overflow_dev);
    OPT_PTR(keys);
    if (k_capacity > 0) REQUIRE_PTR(vals);
    return DARB_OK;
}

// Scratch of darb_bin_sort_noalloc: a file-scope device array, one copy per
// GPU, allocated with the library's code object.  In host code `scratch` is a
// host-side stand-in for the symbol, not a device address: the device address
// of each GPU's copy comes from hipGetSymbolAddress, taken once per device with
// that device current, and only that address is handed to kernels.
static __device__ __align__(256) unsigned char scratch[DARB_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_dev[kMaxDevices] = {};

darb_status scratch_address(void **out) {
    int dev = -1;
    TRY(hip_status(hipGetDevice(&dev), "darb_bin_sort_noalloc: hipGetDevice"));
    if (dev < 0 || dev >= kMaxDevices) return fail(DARB_ERR_UNSUPPORTED, "%s", "device ordinal beyond 63");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        TRY(hip_status(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "darb_bin_sort_noalloc: hipGetSymbolAddress"));
        if (!p) return fail(DARB_ERR_HIP, "%s", "darb_bin_sort_noalloc: null scratch address");
        g_scratch_dev[dev] = p;
    }
    *out = g_scratch_dev[dev];
    return DARB_OK;
}

}  // namespace

darb_status darb_bin_sort(const darb_projected *proj, int64_t n, int32_t width, int32_t height, int64_t k_capacity,
                          void *ws, size_t ws_bytes, uint64_t *keys, uint32_t *vals, uint32_t *ranges, int64_t *k_dev,
                          int32_t *overflow_dev, int64_t *k_host, void *stream) {
    TRY(check_bin_sort_args(proj, n, width, height, k_capacity, vals, ranges, k_dev, overflow_dev, keys));
    REQUIRE_PTR(ws);
    size_t need = darb::binsort_workspace((int)n, width, height, k_capacity);
    if (ws_bytes < need) {
        snprintf(g_err, sizeof(g_err), "workspace too small: %zu < %zu bytes", ws_bytes, need);
        return DARB_ERR_INVALID_ARG;
    }
    return bin_sort_impl("darb_bin_sort", proj, n, width, height, k_capacity, ws, ws_bytes, keys, vals, ranges, k_dev,
                         overflow_dev, k_host, (hipStream_t)stream);
}

darb_status darb_bin_sort_noalloc(const darb_projected *proj, int64_t n, int32_t width, int32_t height,
                                  int64_t k_capacity, uint64_t *keys, uint32_t *vals, uint32_t *ranges, int64_t *k_dev,
                                  int32_t *overflow_dev, int64_t *k_host, void *stream) {
    TRY(check_bin_sort_args(proj, n, width, height, k_capacity, vals, ranges, k_dev, overflow_dev, keys));
    const size_t need = darb::binsort_workspace((int)n, width, height, k_capacity);
    if (need > (size_t)DARB_NOALLOC_SCRATCH_BYTES) {
        snprintf(g_err, sizeof(g_err),
                 "darb_bin_sort_noalloc: n = %lld and k_capacity = %lld need %zu bytes of scratch, more than the "
                 "library's %llu (use darb_bin_sort with a workspace)",
                 (long long)n, (long long)k_capacity, need, (unsigned long long)DARB_NOALLOC_SCRATCH_BYTES);
        return DARB_ERR_UNSUPPORTED;
    }
    void *ws = nullptr;
    TRY(scratch_address(&ws));
    return bin_sort_impl("darb_bin_sort_noalloc", proj, n, width, height, k_capacity, ws,
                         (size_t)DARB_NOALLOC_SCRATCH_BYTES, keys, vals, ranges, k_dev, overflow_dev, k_host,
                         (hipStream_t)stream);
}

darb_status darb_raster_fwd(const darb_projected *proj, int64_t n, const uint32_t *vals, const uint32_t *ranges,
                            const int32_t *overflow_dev, int32_t width, int32_t height, const darb_kernel *kernel,
                            const darb_raster_opts *opts, float *image, float *final_T, uint32_t *last,
                            uint32_t *n_contrib, const darb_grads2d *zero_g2d, void *stream) {
    darb::KParams kp;
    darb::ROpts ro;
    TRY(check_n(n));
    TRY(check_size(width, height));
    TRY(check_kernel(kernel, &kp));
    TRY(check_opts(opts, &ro));
    TRY(check_projected(proj, n, true));
    if (n > 0) REQUIRE_PTR(vals);
    REQUIRE_PTR(ranges);
    OPT_PTR(overflow_dev);
    REQUIRE_PTR(image);
    REQUIRE_PTR(final_T);
    REQUIRE_PTR(last);
    OPT_PTR(n_contrib);
    if (zero_g2d) TRY(check_g2d(zero_g2d, n));
    g_err[0] = 0;
    darb::RViews rv{};
    rv.nv = 1;
    rv.v[0] = make_rview(*proj, vals, ranges, overflow_dev, width, height);
    rv.v[0].image = image;
    rv.v[0].final_T = final_T;
    rv.v[0].last = last;
    rv.v[0].n_contrib = n_contrib;
    if (zero_g2d && n > 0) {
        rv.v[0].g2 = *zero_g2d;
        rv.v[0].zero_n = (int)n;
    }
    return hip_status(darb::launch_raster_fwd(kernel->kind, rv, tile_count(width, height), (int)n, kp, ro,
                                              (hipStream_t)stream),
                      "darb_raster_fwd");
}

darb_status darb_preprocess_bwd(const darb_camera *cam, const darb_kernel *kernel, int64_t n, const darb_splats *in,
                                const darb_projected *proj, const darb_grads2d *g2d, const darb_grads3d *g3d,
                                int32_t accumulate, void *stream) {
    darb::Cam c;
    darb::KParams kp;
    TRY(check_n(n));
    TRY(check_camera(cam, &c));
    TRY(check_kernel(kernel, &kp));
    TRY(check_size(cam->width, cam->height));
    TRY(check_splats(in, n));
    TRY(check_g2d(g2d, n));
    TRY(check_g3d(g3d, n));
    g_err[0] = 0;
    return hip_status(darb::launch_preprocess_bwd(c, kp, (int)n, *in, proj, *g2d, *g3d, accumulate != 0,
                                                  (hipStream_t)stream),
                      "darb_preprocess_bwd");
}

darb_status darb_raster_bwd(const darb_projected *proj, int64_t n, const uint32_t *vals, const uint32_t *ranges,
                            const int32_t *overflow_dev, int32_t width, int32_t height, const darb_kernel *kernel,
                            const darb_raster_opts *opts, const float *dL_dimage, const float *final_T,
                            const uint32_t *last, const darb_grads2d *g2d, int32_t g2d_zeroed,
                            const darb_camera *cam, const darb_splats *in, const darb_grads3d *g3d,
                            int32_t deterministic, int64_t k_capacity, void *ws, size_t ws_bytes, void *stream) {
    darb::KParams kp;
    darb::ROpts ro;
    darb::Cam c;
    TRY(check_n(n));
    TRY(check_size(width, height));
    TRY(check_kernel(kernel, &kp));
    TRY(check_opts(opts, &ro));
    TRY(check_projected(proj, n, true));
    if (n > 0) REQUIRE_PTR(vals);
    REQUIRE_PTR(ranges);
    OPT_PTR(overflow_dev);
    REQUIRE_PTR(dL_dimage);
    REQUIRE_PTR(final_T);
    REQUIRE_PTR(last);
    TRY(check_g2d(g2d, n));
    if (g3d) {
        TRY(check_camera(cam, &c));
        if (cam->width != width || cam->height != height)
            return fail(DARB_ERR_INVALID_ARG, "%s", "camera size differs from the raster size");
        TRY(check_splats(in, n));
        TRY(check_g3d(g3d, n));
    }
    const uint32_t items = tile_count(width, height);
    if (deterministic) {
        if (k_capacity < 0) return fail(DARB_ERR_INVALID_ARG, "%s", "k_capacity must be >= 0");
        TRY(check_det(n, 1, (uint64_t)k_capacity));
        REQUIRE_PTR(ws);
        size_t need = darb::det_workspace(items, (uint64_t)k_capacity);
        if (ws_bytes < need) {
            snprintf(g_err, sizeof(g_err), "workspace too small: %zu < %zu bytes", ws_bytes, need);
            return DARB_ERR_INVALID_ARG;
        }
    }
    g_err[0] = 0;
    hipStream_t s = (hipStream_t)stream;
    darb::RViews rv{};
    rv.nv = 1;
    rv.v[0] = make_rview(*proj, vals, ranges, overflow_dev, width, height);
    rv.v[0].final_T = const_cast<float *>(final_T);
    rv.v[0].last = const_cast<uint32_t *>(last);
    rv.v[0].dL = dL_dimage;
    rv.v[0].g2 = *g2d;
    TRY(hip_status(darb::launch_raster_bwd(kernel->kind, rv, items, (int)n, kp, ro, deterministic ? ws : nullptr,
                                           deterministic ? (uint64_t)k_capacity : 0, g2d_zeroed != 0, s),
                   "darb_raster_bwd"));
    if (g3d)
        TRY(hip_status(darb::launch_preprocess_bwd(c, kp, (int)n, *in, proj, *g2d, *g3d, false, s),
                       "darb_raster_bwd chain"));
    return DARB_OK;
}

size_t darb_raster_bwd_workspace(int64_t n, int32_t width, int32_t height, int64_t k_capacity) {
    if (n < 0 || n > 0x7FFFFFFFll || width <= 0 || height <= 0) return 0;
    if (k_capacity < 0 || k_capacity >= 0xFFFFFFFFll || (uint64_t)n >= 0xFFFFFFFFull) return 0;
    int64_t gx = (width + darb::kTile - 1) / darb::kTile, gy = (height + darb::kTile - 1) / darb::kTile;
    if (gx * gy > darb::kMaxTiles) return 0;
    return darb::det_workspace((uint32_t)(gx * gy), (uint64_t)k_capacity);
}

darb_status darb_image_loss(const float *image, const float *target, int32_t width, int32_t height, int32_t loss_kind,
                            float *dL_dimage, float *loss_dev, void *ws, size_t ws_bytes, void *stream) {
    if (width <= 0 || height <= 0) return fail(DARB_ERR_INVALID_ARG, "%s", "width/height must be > 0");
    if (loss_kind != DARB_LOSS_L1 && loss_kind != DARB_LOSS_L2)
        return fail(DARB_ERR_INVALID_ARG, "%s", "unknown loss kind");
    REQUIRE_PTR(image);
    REQUIRE_PTR(target);
    OPT_PTR(dL_dimage);
    OPT_PTR(loss_dev);
    if (loss_dev) {
        REQUIRE_PTR(ws);
        if (ws_bytes < DARB_LOSS_WS_BYTES)
            return fail(DARB_ERR_INVALID_ARG, "%s", "workspace smaller than DARB_LOSS_WS_BYTES");
    }
    g_err[0] = 0;
    const darb::RView r = make_rview(darb_projected{}, nullptr, nullptr, nullptr, width, height);
    return hip_status(darb::launch_image_loss(loss_kind, image, target, width, height, r.loss_scale, dL_dimage,
                                              loss_dev, static_cast<float *>(ws), (hipStream_t)stream),
                      "darb_image_loss");
}

size_t darb_ssim_loss_workspace(int32_t width, int32_t height) {
    if (width <= 0 || height <= 0) return 0;
    if ((int64_t)width * height > ((int64_t)1 << 31)) return 0;
    return darb::ssim_workspace(width, height);
}

darb_status darb_ssim_loss(const float *image, const float *target, int32_t width, int32_t height, float lambda,
                           float *dL_dimage, float *loss_dev, void *ws, size_t ws_bytes, void *stream) {
    if (width <= 0 || height <= 0) return fail(DARB_ERR_INVALID_ARG, "%s", "width/height must be > 0");
    if ((int64_t)width * height > ((int64_t)1 << 31)) return fail(DARB_ERR_UNSUPPORTED, "%s", "image too large");
    if (!(lambda >= 0.0f) || !(lambda <= 1.0f)) return fail(DARB_ERR_INVALID_ARG, "%s", "lambda must be in [0, 1]");
    REQUIRE_PTR(image);
    REQUIRE_PTR(target);
    REQUIRE_PTR(dL_dimage);
    OPT_PTR(loss_dev);
    REQUIRE_PTR(ws);
    const size_t need = darb::ssim_workspace(width, height);
    if (ws_bytes < need) {
        snprintf(g_err, sizeof(g_err), "workspace too small: %zu < %zu bytes", ws_bytes, need);
        return DARB_ERR_INVALID_ARG;
    }
    g_err[0] = 0;
    const darb::RView r = make_rview(darb_projected{}, nullptr, nullptr, nullptr, width, height);
    return hip_status(darb::launch_ssim_loss(image, target, width, height, lambda, r.loss_scale, dL_dimage, loss_dev,
                                             ws, (hipStream_t)stream),
                      "darb_ssim_loss");
}

darb_status darb_adam(const darb_adam_group *groups, int32_t n_groups, int32_t step, float beta1, float beta2,
                      float eps, void *stream) {
    if (!groups) return fail(DARB_ERR_INVALID_ARG, "null pointer: %s", "groups");
    if (n_groups < 1 || n_groups > DARB_MAX_ADAM_GROUPS)
        return fail(DARB_ERR_INVALID_ARG, "%s", "n_groups must be in [1, DARB_MAX_ADAM_GROUPS]");
    if (step < 1) return fail(DARB_ERR_INVALID_ARG, "%s", "step must be >= 1");
    if (!(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f))
        return fail(DARB_ERR_INVALID_ARG, "%s", "need 0 <= beta1, beta2 < 1 and eps > 0");
    darb::AdamGroups G{};
    int64_t blocks = 0;
    for (int k = 0; k < n_groups; k++) {
        const darb_adam_group &g = groups[k];
        if (g.n < 0) return fail(DARB_ERR_INVALID_ARG, "%s", "group n must be >= 0");
        if (g.n > 0) {
            REQUIRE_PTR(g.param);
            REQUIRE_PTR(g.grad);
            REQUIRE_PTR(g.m);
            REQUIRE_PTR(g.v);
        }
        if (!isfinite(g.lr)) return fail(DARB_ERR_INVALID_ARG, "%s", "group lr must be finite");
        G.g[k] = g;
        blocks += (g.n + 255) / 256;
    }
    if (blocks > 0x7FFFFFFFll) return fail(DARB_ERR_UNSUPPORTED, "%s", "too many values");
    G.ng = n_groups;
    const double bc1 = 1.0 - pow((double)beta1, (double)step);
    const double bc2 = 1.0 - pow((double)beta2, (double)step);
    g_err[0] = 0;
    return hip_status(darb::launch_adam(G, beta1, beta2, eps, (float)bc1, (float)sqrt(bc2), (hipStream_t)stream),
                      "darb_adam");
}

darb_status darb_densify_stats(const darb_grads2d *g2d, const int32_t *radius, int64_t n, float *grad_accum,
                               int32_t *count, int32_t *max_radius, void *stream) {
    TRY(check_n(n));
    if (!g2d) return fail(DARB_ERR_INVALID_ARG, "null pointer: %s", "grads2d");
    if (n > 0) {
        REQUIRE_PTR(g2d->xy);
        REQUIRE_PTR(radius);
        REQUIRE_PTR(grad_accum);
        REQUIRE_PTR(count);
        OPT_PTR(max_radius);
    }
    g_err[0] = 0;
    return hip_status(darb::launch_densify_stats(*g2d, radius, (int)n, grad_accum, count, max_radius,
                                                 (hipStream_t)stream),
                      "darb_densify_stats");
}

darb_status darb_probe_copy(const float *src, float *dst, int64_t n, void *stream) {
    TRY(check_n(n));
    if (n % 4 != 0) return fail(DARB_ERR_INVALID_ARG, "%s", "n must be a multiple of 4");
    if (n > 0) {
        REQUIRE_PTR(src);
        REQUIRE_PTR(dst);
    }
    g_err[0] = 0;
    return hip_status(darb::launch_probe_copy(src, dst, n, (hipStream_t)stream), "darb_probe_copy");
}

darb_status darb_probe_fill(float *dst, int64_t n, void *stream) {
    TRY(check_n(n));
    if (n % 4 != 0) return fail(DARB_ERR_INVALID_ARG, "%s", "n must be a multiple of 4");
    if (n > 0) REQUIRE_PTR(dst);
    g_err[0] = 0;
    return hip_status(darb::launch_probe_fill(dst, n, (hipStream_t)stream), "darb_probe_fill");
}

darb_status darb_probe_fma(void *out, int64_t threads, int32_t iters, int32_t fp64, int32_t *chains, void *stream) {
    TRY(check_n(threads));
    if (iters < 0) return fail(DARB_ERR_INVALID_ARG, "%s", "iters must be >= 0");
    if (threads > 0) REQUIRE_PTR(out);
    if (chains) *chains = darb::probe_fma_chains();
    g_err[0] = 0;
    if (fp64)
        return hip_status(darb::launch_probe_fma64(static_cast<double *>(out), threads, (int)iters,
                                                   (hipStream_t)stream),
                          "darb_probe_fma");
    return hip_status(darb::launch_probe_fma32(static_cast<float *>(out), threads, (int)iters, (hipStream_t)stream),
                      "darb_probe_fma");
}

darb_status darb_preprocess_multi(const darb_view *views, int32_t nv, const darb_kernel *kernel, int64_t n,
                                  const darb_splats *in, void *stream) {
    darb::KParams kp;
    darb::Cams cams;
    TRY(check_n(n));
    TRY(check_kernel(kernel, &kp));
    TRY(check_splats(in, n));
    TRY(check_views(views, nv, n, kNeedProj, nullptr, &cams, nullptr, nullptr));
    darb::Projs outs{};
    for (int v = 0; v < nv; v++) outs.p[v] = views[v].proj;
    g_err[0] = 0;
    return hip_status(darb::launch_preprocess_multi(cams, kp, (int)n, *in, outs, (hipStream_t)stream),
                      "darb_preprocess_multi");
}

darb_status darb_preprocess_multi_cam_dev(const darb_view *views, int32_t nv, const darb_camera *cams_dev,
                                          const darb_kernel *kernel, int64_t n, const darb_splats *in, void *stream) {
    darb::KParams kp;
    darb::Cams cams;
    TRY(check_n(n));
    TRY(check_kernel(kernel, &kp));
    TRY(check_splats(in, n));
    TRY(check_views(views, nv, n, kNeedProj, nullptr, &cams, nullptr, nullptr));
    REQUIRE_PTR(cams_dev);
    cams.dev = cams_dev;
    darb::Projs outs{};
    for (int v = 0; v < nv; v++) outs.p[v] = views[v].proj;
    g_err[0] = 0;
    return hip_status(darb::launch_preprocess_multi(cams, kp, (int)n, *in, outs, (hipStream_t)stream),
                      "darb_preprocess_multi_cam_dev");
}

darb_status darb_raster_fwd_multi(const darb_view *views, int32_t nv, int64_t n, const darb_kernel *kernel,
                                  const darb_raster_opts *opts, void *stream) {
    darb::KParams kp;
    darb::ROpts ro;
    darb::RViews rv;
    uint32_t items;
    TRY(check_n(n));
    TRY(check_kernel(kernel, &kp));
    TRY(check_opts(opts, &ro));
    TRY(check_views(views, nv, n, kNeedProj | kNeedList | kNeedFwdOut, &rv, nullptr, &items, nullptr));
    g_err[0] = 0;
    return hip_status(darb::launch_raster_fwd(kernel->kind, rv, items, (int)n, kp, ro, (hipStream_t)stream),
                      "darb_raster_fwd_multi");
}

size_t darb_raster_bwd_multi_workspace(const darb_view *views, int32_t nv, int64_t n) {
    uint32_t items;
    uint64_t cap;
    if (n < 0 || n > 0x7FFFFFFFll) return 0;
    if (check_views(views, nv, n, kNeedList, nullptr, nullptr, &items, &cap) != DARB_OK) return 0;
    if (check_det(n, nv, cap) != DARB_OK) return 0;
    return darb::det_workspace(items, cap);
}

darb_status darb_raster_bwd_multi(const darb_view *views, int32_t nv, int64_t n, const darb_kernel *kernel,
                                  const darb_raster_opts *opts, int32_t deterministic, void *ws, size_t ws_bytes,
                                  void *stream) {
    darb::KParams kp;
    darb::ROpts ro;
    darb::RViews rv;
    uint32_t items;
    uint64_t cap;
    TRY(check_n(n));
    TRY(check_kernel(kernel, &kp));
    TRY(check_opts(opts, &ro));
    TRY(check_views(views, nv, n, kNeedProj | kNeedList | kNeedBwdIn | kNeedG2, &rv, nullptr, &items, &cap));
    if (deterministic) {
        TRY(check_det(n, nv, cap));
        REQUIRE_PTR(ws);
        size_t need = darb::det_workspace(items, cap);
        if (ws_bytes < need) {
            snprintf(g_err, sizeof(g_err), "workspace too small: %zu < %zu bytes", ws_bytes, need);
            return DARB_ERR_INVALID_ARG;
        }
    }
    g_err[0] = 0;
    return hip_status(darb::launch_raster_bwd(kernel->kind, rv, items, (int)n, kp, ro, deterministic ? ws : nullptr,
                                              deterministic ? cap : 0, false, (hipStream_t)stream),
                      "darb_raster_bwd_multi");
}

darb_status darb_raster_fwdbwd_multi(const darb_view *views, int32_t nv, int64_t n, const darb_kernel *kernel,
                                     const darb_raster_opts *opts, int32_t loss_kind, void *stream) {
    darb::KParams kp;
    darb::ROpts ro;
    darb::RViews rv;
    uint32_t items;
    TRY(check_n(n));
    TRY(check_kernel(kernel, &kp));
    TRY(check_opts(opts, &ro));
    if (loss_kind != DARB_LOSS_L1 && loss_kind != DARB_LOSS_L2)
        return fail(DARB_ERR_INVALID_ARG, "%s", "unknown loss kind");
    TRY(check_views(views, nv, n, kNeedProj | kNeedList | kNeedImage | kNeedTarget | kNeedG2, &rv, nullptr, &items,
                    nullptr));
    g_err[0] = 0;
    return hip_status(darb::launch_raster_fwdbwd(kernel->kind, loss_kind, rv, items, (int)n, kp, ro,
                                                 (hipStream_t)stream),
                      "darb_raster_fwdbwd_multi");
}

darb_status darb_preprocess_bwd_multi(const darb_view *views, int32_t nv, const darb_kernel *kernel, int64_t n,
                                      const darb_splats *in, const darb_grads3d *g3d, void *stream) {
    darb::KParams kp;
    darb::Cams cams;
    TRY(check_n(n));
    TRY(check_kernel(kernel, &kp));
    TRY(check_splats(in, n));
    TRY(check_g3d(g3d, n));
    TRY(check_views(views, nv, n, kNeedG2, nullptr, &cams, nullptr, nullptr));
    darb::G2s g2{};
    for (int v = 0; v < nv; v++) {
        g2.g[v] = views[v].grads2d;
        g2.dcolor[v] = views[v].proj.dcolor;
        g2.clamped[v] = views[v].proj.clamped;
    }
    g_err[0] = 0;
    return hip_status(darb::launch_preprocess_bwd_multi(cams, kp, (int)n, *in, g2, *g3d, (hipStream_t)stream),
                      "darb_preprocess_bwd_multi");
}

}  // extern "C"

darb_status darb_fit1d(const darb_kernel *kernel, int32_t batch, int32_t n_comp, int32_t m, const float *x,
                       const float *target, float *params, float *adam_m, float *adam_v, int32_t steps, int32_t step0,
                       const float *lr, float beta1, float beta2, float eps, float *loss, void *stream) {
    darb::KParams kp;
    TRY(check_kernel(kernel, &kp));
    if (batch < 0) return fail(DARB_ERR_INVALID_ARG, "%s", "batch must be >= 0");
    if (n_comp < 1 || n_comp > darb::fit1d_max_components())
        return fail(DARB_ERR_UNSUPPORTED, "%s", "n_comp must be in [1, 64]");
    if (m < 1 || m > darb::fit1d_max_samples()) return fail(DARB_ERR_UNSUPPORTED, "%s", "m must be in [1, 4096]");
    if (steps < 0 || step0 < 0) return fail(DARB_ERR_INVALID_ARG, "%s", "steps and step0 must be >= 0");
    if (!lr) return fail(DARB_ERR_INVALID_ARG, "null pointer: %s", "lr");
    if (!(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps >= 0.0f))
        return fail(DARB_ERR_INVALID_ARG, "%s", "Adam needs 0 <= beta1, beta2 < 1 and eps >= 0");
    if (batch == 0 || steps == 0) return DARB_OK;
    REQUIRE_PTR(x);
    REQUIRE_PTR(target);
    REQUIRE_PTR(params);
    REQUIRE_PTR(adam_m);
    REQUIRE_PTR(adam_v);
    OPT_PTR(loss);
    g_err[0] = 0;
    return hip_status(darb::launch_fit1d(kernel->kind, kp, batch, n_comp, m, x, target, params, adam_m, adam_v, steps,
                                         step0, lr, beta1, beta2, eps, loss, (hipStream_t)stream),
                      "darb_fit1d");
}

size_t darb_psi_calibrate_workspace(int32_t m, int32_t grid_n) {
    if (m < 0 || m > 65535 || grid_n < 5 || grid_n > 2049 || (grid_n & 1) == 0) return 0;
    return darb::psi_workspace(m, grid_n);
}

darb_status darb_psi_calibrate(const darb_kernel *kernel, int32_t m, const double *sigma, int32_t grid_n, void *ws,
                               size_t ws_bytes, double *cov2, double *fit, void *stream) {
    darb::KParams kp;
    TRY(check_kernel(kernel, &kp));
    if (m < 0 || m > 65535) return fail(DARB_ERR_INVALID_ARG, "%s", "m must be in [0, 65535]");
    if (grid_n < 5 || grid_n > 2049 || (grid_n & 1) == 0)
        return fail(DARB_ERR_INVALID_ARG, "%s", "grid_n must be odd, in [5, 2049] (Simpson's rule)");
    if (fit && m < 6) return fail(DARB_ERR_INVALID_ARG, "%s", "the 6-input fit needs m >= 6 samples");
    if (m == 0) return DARB_OK;
    REQUIRE_PTR(sigma);
    REQUIRE_PTR(ws);
    REQUIRE_PTR(cov2);
    OPT_PTR(fit);
    const size_t need = darb::psi_workspace(m, grid_n);
    if (ws_bytes < need) {
        snprintf(g_err, sizeof(g_err), "workspace too small: %zu < %zu bytes", ws_bytes, need);
        return DARB_ERR_INVALID_ARG;
    }
    g_err[0] = 0;
    const float margin = 1.0f + 2.0f / (float)(grid_n - 1);
    return hip_status(darb::launch_psi_calibrate(kernel->kind, kp, m, sigma, grid_n, margin, ws, cov2, fit,
                                                 (hipStream_t)stream),
                      "darb_psi_calibrate");
}

