/*
 * darb.h -- C ABI of libdarb, an MI355X (gfx950) implementation of the
 * differentiable tile rasterizer of DARB-Splatting (arXiv 2501.12369):
 * anisotropic splats whose footprint is a decaying anisotropic radial basis
 * function (DARBF) F of the squared Mahalanobis distance E = d_M^2.
 *
 * Conventions shared by every call
 * --------------------------------
 * - Every buffer is a DEVICE pointer owned by the caller; the library never
 *   allocates device memory.  Scratch space comes in through a workspace
 *   argument whose size a *_workspace query returns.
 * - Every call is asynchronous on `stream` (a hipStream_t passed as void*;
 *   NULL = the null stream) unless stated otherwise.  Arguments are validated
 *   on the host before anything is enqueued; on an error nothing is enqueued.
 * - Every device pointer must be 16-byte aligned.
 * - Counts are int64_t; indices into the sorted instance list are uint32_t, so
 *   the number of (tile, splat) instances must stay below 2^32.
 * - Errors: a darb_status code; darb_last_error() returns a message for the
 *   last failing call on the calling thread.  No C++ exception crosses the ABI.
 * - Thread safety: no global mutable state besides the per-thread error text;
 *   calls on different streams may run concurrently.
 * - Geometry: camera frame x right, y down, z forward; pixel (i, j) (column i,
 *   row j) is evaluated at image coordinates (i, j).  Images are planar
 *   [3][H][W] FP32; per-pixel buffers are [H][W].
 * - The 2D footprint is rasterised on 16x16-pixel tiles.
 */
#ifndef DARB_H
#define DARB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#if defined(__GNUC__) || defined(__clang__)
#define DARB_API __attribute__((visibility("default")))
#else
#define DARB_API
#endif

#define DARB_ABI_VERSION 7
#define DARB_TILE 16
#define DARB_MAX_VIEWS 16       /* views per multi-view call */
#define DARB_LOSS_WS_BYTES 4096 /* workspace of darb_image_loss */

typedef enum {
    DARB_OK = 0,
    DARB_ERR_INVALID_ARG = 1, /* null/misaligned pointer, negative count, bad size, unknown kind */
    DARB_ERR_CAPACITY = 2,    /* instance count exceeds the capacity (only reported by a blocking call) */
    DARB_ERR_HIP = 3,         /* a HIP runtime call failed; darb_last_error() names it */
    DARB_ERR_UNSUPPORTED = 4  /* valid request outside what the library implements */
} darb_status;

/* Kernel profiles F(E), E = d_M^2 (Table 1 and the per-kernel supplementary
 * sections).  xi is the scaling factor of Table 2. */
typedef enum {
    DARB_GAUSS = 0,      /* exp(-E/xi)                  (modified Gaussian, beta = 2; xi = 2)       */
    DARB_HALF_COS = 1,   /* cos(E/xi), E/xi <= pi/2     (half-cosine squared; xi = 18/pi)          */
    DARB_RAISED_COS = 2, /* 0.5 + 0.5 cos(sqrt(E)/xi)   (raised cosine, beta = 1; xi = 2.5/pi)      */
    DARB_SINC = 3,       /* |sin u|/u, u = sqrt(E)/xi   (modular sinc, beta = 1; xi = 3/pi)         */
    DARB_IMQ = 4,        /* 1/(E/xi + 1)                (inverse quadric of the supplementary code) */
    DARB_IMQ_SQRT = 5,   /* 1/sqrt(E/xi + 1)            (inverse multiquadric of Table 1)           */
    DARB_PARABOLA = 6,   /* 1 - E/xi                    (parabola; xi = 9)                          */
    /* Table 1's modified forms with a generic roll-off beta (darb_kernel.beta > 0):
     * u = d_M^beta / xi = E^(beta/2) / xi; the support e_max is the caller's
     * domain limit, E <= (xi U)^(2/beta) for u <= U (U = pi/2 for one
     * half-cosine lobe, n pi for n raised-cosine pulses, (n+1) pi/2 for n sinc
     * pulses).  dF/dE at E = 0 is 1/xi dF/du(0) for beta = 2 and 0 otherwise. */
    DARB_GAUSS_BETA = 7,      /* exp(-u)                                                    */
    DARB_HALF_COS_BETA = 8,   /* cos(u)                                                     */
    DARB_RAISED_COS_BETA = 9, /* 0.5 + 0.5 cos(u)                                           */
    DARB_SINC_BETA = 10       /* |sin u| / u (1 at u = 0)                                   */
} darb_kernel_kind;

/* Image losses with a per-pixel gradient, each the mean over the 3 W H values
 * of a view (the photometric L1 term of the 3DGS objective the paper trains
 * with, and the squared error). */
typedef enum {
    DARB_LOSS_L1 = 0, /* mean |I - I_target|;  dL/dI = sign(I - I_target) / (3 W H), 0 where equal */
    DARB_LOSS_L2 = 1  /* mean (I - I_target)^2; dL/dI = 2 (I - I_target) / (3 W H) */
} darb_loss_kind;

/* A DARBF: profile, scale, correction factor and support.
 * psi multiplies the projected 2x2 covariance (Eq. of the 2x2 covariance
 * projection; Table 2).  A pixel is inside the footprint iff 0 <= E <= e_max
 * (boundaries of DARBFs: one main lobe, or n pulses).  The radius is
 * 3 sqrt(lambda_max) (DARB-Splatting section), widened to
 * sqrt(e_max lambda_max) when e_max > 9; the tile box uses the same factor.
 * The fixed kinds 0..6 require 0 < e_max <= 9 and, for the trigonometric
 * ones, a support inside the main
 * lobe (E/xi <= pi/2 for DARB_HALF_COS, sqrt(E)/xi <= pi for DARB_RAISED_COS
 * and DARB_SINC); the modified kinds 7..10 take 0 < beta <= 8 and
 * 0 < e_max <= 1024 and ignore nothing else.  beta is ignored by kinds 0..6. */
typedef struct {
    int32_t kind; /* darb_kernel_kind */
    float xi;
    float psi;
    float e_max;
    float beta; /* roll-off of the modified kinds */
} darb_kernel;

/* Pinhole camera.  viewmat: world -> camera, row-major 4x4 (rotation R_cw in
 * the upper 3x3, translation t_cw in the last column).  campos: camera centre
 * in world coordinates (used for the SH view direction).  A splat with camera
 * depth t_z <= near_z is culled.  jac_clamp limits |t_x/t_z| to
 * jac_clamp * (width/2) / fx (and likewise y) inside the projection Jacobian;
 * <= 0 disables the clamp.  dilation is added to the diagonal of the 2D
 * covariance after the psi scaling. */
typedef struct {
    float viewmat[16];
    float campos[3];
    float fx, fy, cx, cy;
    int32_t width, height;
    float near_z;
    float jac_clamp;
    float dilation;
} darb_camera;

/* Compositing options (front-to-back alpha blending): alpha = min(alpha_max,
 * opacity * F(E)); a pair with alpha < alpha_min is skipped; a pixel stops
 * (without blending the splat) when the transmittance would fall below t_min;
 * the background colour bg is blended with the final transmittance. */
typedef struct {
    float alpha_min; /* 1/255 */
    float alpha_max; /* 0.99  */
    float t_min;     /* 1e-4  */
    float bg[3];
} darb_raster_opts;

/* Splat parameters (the 3DGS parameterisation kept by the paper, DARB
 * Representation), structure-of-arrays, FP32, read-only:
 *   means    [3][n]                 world position
 *   scales   [3][n]                 positive (already activated) axis scales
 *   quats    [4][n]                 (w, x, y, z), any nonzero norm
 *   opacity  [n]                    in (0, 1) (already activated)
 *   sh       [(deg+1)^2][3][n]      real SH coefficients per colour channel */
typedef struct {
    const float *means;
    const float *scales;
    const float *quats;
    const float *opacity;
    const float *sh;
    int32_t sh_degree; /* 0..3 */
} darb_splats;

/* Projected splats (preprocess output, binning/raster input):
 *   xy       [n][2]   projected mean mu' in pixels
 *   depth    [n]      camera-space t_z
 *   radius   [n]      ceil(3 sqrt(lambda_max)) in pixels; 0 = culled (other fields undefined)
 *   extent   [n][2]   int32 (rx, ry): half-width and half-height of the tile box, the
 *                     bounding box of the ellipse d^T Sigma'^-1 d <= 9 (the support
 *                     E <= 9; sqrt(e_max) in place of 3 for a support beyond E = 9):
 *                     ceil(3 sqrt(Sigma'_xx)), ceil(3 sqrt(Sigma'_yy)) <= radius; 0 = culled.
 *                     A splat is culled when this box misses the tile grid.
 *   conic_o  [n][4]   (l00, l01, l11, opacity): the conic Q = [[a, b], [b, c]] (inverse 2D
 *                     covariance) as its factor Q = L^T L, L = [[l00, l01], [0, l11]]
 *                     (l00, l11 > 0), so that E = |L d|^2 is a sum of squares
 *   rgb      [n][3]   colour after the SH evaluation and the clamp at 0
 *   clamped  [n]      bit c set when channel c was clamped at 0
 *   dcolor   [9][n]   nullable: d colour / d u, u the unit view direction from the camera
 *                     centre (plane 3 c + k holds d colour_c / d u_k, before the clamp;
 *                     zeros for culled splats).  darb_preprocess writes it when non-null;
 *                     with it darb_preprocess_bwd reads neither the SH coefficients nor
 *                     recomputes the colour (a checkpoint of the forward).              */
typedef struct {
    float *xy;
    float *depth;
    int32_t *radius;
    int32_t *extent;
    float *conic_o;
    float *rgb;
    uint8_t *clamped;
    float *dcolor;
} darb_projected;

/* Gradients with respect to the projected quantities (raster backward output):
 *   xy [n][2], conic [n][3] (d/da, d/db with b the single off-diagonal scalar,
 *   d/dc), opacity [n], rgb [n][3]. */
typedef struct {
    float *xy;
    float *conic;
    float *opacity;
    float *rgb;
} darb_grads2d;

/* Gradients with respect to the splat parameters, same layouts as darb_splats. */
typedef struct {
    float *means;
    float *scales;
    float *quats;
    float *opacity;
    float *sh;
} darb_grads3d;

/* One view of a multi-view call: its camera, its own projected splats and
 * sorted instance list (from darb_preprocess_multi and darb_bin_sort), and its
 * per-view images and gradient buffers.  Fields a call does not use may be
 * NULL; each call lists what it reads and writes.  width/height come from cam. */
typedef struct {
    darb_camera cam;
    darb_projected proj;         /* [n] per view */
    int64_t k_capacity;          /* capacity of vals (as given to darb_bin_sort) */
    const uint32_t *vals;        /* sorted instance list */
    const uint32_t *ranges;      /* [tiles][2] */
    const int32_t *overflow_dev; /* nullable: nonzero flag = this view is skipped */
    float *image;                /* [3][H][W] */
    float *final_T;              /* [H][W] checkpoint */
    uint32_t *last;              /* [H][W] checkpoint */
    uint32_t *n_contrib;         /* [H][W] nullable */
    const float *dL_dimage;      /* [3][H][W] upstream gradient (darb_raster_bwd_multi) */
    const float *target;         /* [3][H][W] target image (darb_raster_fwdbwd_multi) */
    darb_grads2d grads2d;        /* [n] per-view gradients w.r.t. the projected splats */
} darb_view;

DARB_API int32_t darb_version(void);
DARB_API const char *darb_status_string(int32_t status);
DARB_API const char *darb_last_error(void);

/*
 * darb_preprocess -- per-splat projection (DARB Projection; Eq. of the 2x2
 * covariance projection; bounding radius of the DARBF boundaries section).
 * For each splat: q/|q| -> R; Sigma = R diag(s^2) R^T; t = R_cw mu + t_cw
 * (cull t_z <= near_z); affine Jacobian J at t; Sigma'_2x2 = psi [J R_cw Sigma
 * R_cw^T J^T]_2x2 + dilation I (cull det <= 0); Q = Sigma'_2x2^-1;
 * mu' = (fx t_x/t_z + cx, fy t_y/t_z + cy); radius = ceil(3 sqrt(lambda_max));
 * tile box half-extents ceil(3 sqrt(Sigma'_xx)), ceil(3 sqrt(Sigma'_yy)) (the
 * bounding box of the support ellipse, inside the radius square); cull when
 * the tile box covers no tile; rgb = max(0, sum SH * Y(dir) + 0.5)
 * with dir = (mu - campos)/|mu - campos|.  `in` fields are read; every `out`
 * field is written.  n = 0 is a no-op.
 */
DARB_API darb_status darb_preprocess(const darb_camera *cam, const darb_kernel *kernel, int64_t n, const darb_splats *in,
                            const darb_projected *out, void *stream);

/*
 * darb_preprocess_parts -- darb_preprocess split in two launches with the same
 * arithmetic (together they write the same bits):
 *   DARB_PRE_GEOMETRY  reads means, scales, quats, opacity; writes xy, depth,
 *                      radius, extent and conic_o (what darb_bin_sort reads);
 *   DARB_PRE_COLOUR    reads radius (written by the geometry part for the same
 *                      camera and splats: a splat is kept iff radius > 0), means
 *                      and sh; writes rgb, clamped and dcolor (when non-null).
 * The colour part is not an input of darb_bin_sort, so a caller may run it on a
 * second stream (after the geometry part, by an event) while the binning runs,
 * and join before darb_raster_fwd.  parts = 3 is darb_preprocess; any other
 * value is DARB_ERR_INVALID_ARG.
 */
#define DARB_PRE_GEOMETRY 1
#define DARB_PRE_COLOUR 2
DARB_API darb_status darb_preprocess_parts(const darb_camera *cam, const darb_kernel *kernel, int64_t n,
                                           const darb_splats *in, const darb_projected *out, int32_t parts,
                                           void *stream);

/*
 * darb_preprocess_cam_dev -- darb_preprocess with the camera read from DEVICE
 * memory (one darb_camera at cam_dev), so that a captured graph of the render
 * can be replayed for a new pose after the caller rewrites that buffer.
 * width/height size the tile grid (use the camera's).  The camera values are
 * not validated on the host: non-positive fx, fy or near_z cull every splat.
 */
DARB_API darb_status darb_preprocess_cam_dev(const darb_camera *cam_dev, int32_t width, int32_t height,
                                             const darb_kernel *kernel, int64_t n, const darb_splats *in,
                                             const darb_projected *out, void *stream);

/*
 * darb_bin_sort_workspace -- bytes of device workspace darb_bin_sort needs for
 * n splats, a width x height image and an instance capacity k_capacity (the
 * workspace holds an intermediate list bounded by the instance count).
 * Returns 0 for invalid or unsupported sizes.
 */
DARB_API size_t darb_bin_sort_workspace(int64_t n, int32_t width, int32_t height, int64_t k_capacity);

/*
 * darb_bin_sort -- tile binning and depth sort ("tile-based rasterization"
 * with the bounding box, DARBF boundaries section).  Every splat with
 * extent (rx, ry) > 0 is duplicated into every 16x16 tile of its box
 *   x in [clamp(floor((u - rx)/16)), clamp(floor((u + rx)/16) + 1)),  same for y with ry,
 * (FP32, clamped to the tile grid); each instance has key (tile << 32) |
 * bits(depth) and value = splat index.  Instances are ordered by (key, index):
 * per tile, front to back, equal depths by index -- a unique order.
 *   keys      [k_capacity] u64, nullable (the raster stages do not need keys)
 *   vals      [k_capacity] u32 splat indices in sorted order
 *   ranges    [tiles][2]  u32: ranges[t] = (#instances with tile < t, #instances with tile <= t)
 *   k_dev     [2] int64 device: K, the number of instances, and N_v, the number of
 *             splats with extent > 0 whose box covers a tile (always written)
 *   overflow_dev [1] int32 device: 1 when K > k_capacity, else 0 (always written);
 *             with overflow set keys, vals and ranges are not written and the
 *             raster calls given the same flag do nothing
 *   k_host    nullable host pointer: when given, the call blocks on `stream`
 *             and stores K there (not capturable in a graph); it then returns
 *             DARB_ERR_CAPACITY on overflow
 *   ws/ws_bytes  workspace of at least darb_bin_sort_workspace(n, width, height, k_capacity) bytes
 * tiles = ceil(width/16) * ceil(height/16) must be <= 16384, and the number of
 * 8x8-tile groups ceil(tiles_x/8) * ceil(tiles_y/8) <= 1024.
 * Splats with extent > 0 must have a finite positive depth.
 */
DARB_API darb_status darb_bin_sort(const darb_projected *proj, int64_t n, int32_t width, int32_t height, int64_t k_capacity,
                          void *ws, size_t ws_bytes, uint64_t *keys, uint32_t *vals, uint32_t *ranges, int64_t *k_dev,
                          int32_t *overflow_dev, int64_t *k_host, void *stream);

/*
 * darb_bin_sort_noalloc -- darb_bin_sort for callers that cannot allocate
 * device memory or own a workspace: code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation.  Same arguments, results
 * and errors as darb_bin_sort, without ws/ws_bytes: the call runs the same
 * kernels on the library's own scratch, a device array of
 * DARB_NOALLOC_SCRATCH_BYTES bytes in the library's code object (one copy on
 * every GPU the library runs on, held until the process ends).  It calls no
 * allocating routine.
 *   Limit: darb_bin_sort_workspace(n, width, height, k_capacity) must not
 *   exceed DARB_NOALLOC_SCRATCH_BYTES; larger sizes return DARB_ERR_UNSUPPORTED
 *   with the sizes in darb_status_string's message.
 *   Sharing: every call on one GPU uses that GPU's one scratch array.  Calls
 *   that overlap on one GPU (several streams, several host threads) race and
 *   give wrong results; order them on one stream or with events.  The scratch
 *   keeps the last call's contents; every call initialises what it reads.
 *   The first call on each device looks up the array's device address
 *   (hipGetSymbolAddress); make it outside graph capture.
 */
#define DARB_NOALLOC_SCRATCH_BYTES (256ull << 20)
DARB_API darb_status darb_bin_sort_noalloc(const darb_projected *proj, int64_t n, int32_t width, int32_t height,
                                           int64_t k_capacity, uint64_t *keys, uint32_t *vals, uint32_t *ranges,
                                           int64_t *k_dev, int32_t *overflow_dev, int64_t *k_host, void *stream);

/*
 * darb_fit1d -- the 1D signal-reconstruction experiment (Assessing DARBFs
 * through 1D Simulations; the extended 1D results) for `batch` independent
 * problems in one launch.  Problem b approximates target[b][0..m) sampled at
 * x[0..m) by f(x) = sum_k a_k F(E_k(x)), E_k(x) = ((x - mu_k) / sigma_k)^2,
 * each term zero beyond E > e_max of `kernel` (psi is not used), and runs
 * `steps` Adam steps on L = (1/m) sum_j (f(x_j) - target[b][j])^2 over
 * (mu_k, log sigma_k, a_k).
 *   params  [batch][3][n_comp] in/out: mu, log sigma, amplitude
 *   adam_m, adam_v [batch][3][n_comp] in/out: first and second moments
 *   step0   steps taken before (bias corrections 1 - beta^(step0 + s + 1))
 *   lr      HOST array of 3 learning rates (mu, log sigma, amplitude)
 *   loss    nullable [batch][steps] out: L before each step
 * 1 <= n_comp <= 64, 1 <= m <= 4096.  FP32.
 */
DARB_API darb_status darb_fit1d(const darb_kernel *kernel, int32_t batch, int32_t n_comp, int32_t m, const float *x,
                                const float *target, float *params, float *adam_m, float *adam_v, int32_t steps,
                                int32_t step0, const float *lr, float beta1, float beta2, float eps, float *loss,
                                void *stream);

/*
 * darb_psi_calibrate_workspace -- bytes of workspace of darb_psi_calibrate
 * (24 m grid_n); 0 for unsupported sizes.
 */
DARB_API size_t darb_psi_calibrate_workspace(int32_t m, int32_t grid_n);

/*
 * darb_psi_calibrate -- the correction-factor experiment (Mathematical
 * Expressions of Monte Carlo Experiments; the psi regression of the extended
 * results) for the DARBF `kernel`: for each of m 3D covariances the kernel
 * F(E), E = p^T Sigma^-1 p, restricted to E <= e_max, is sampled on a grid of
 * grid_n^3 points over the box that holds its support (half-extent
 * (1 + 2/(grid_n-1)) sqrt(e_max Sigma_aa) on axis a), summed along z with
 * Simpson's rule (weights 1, 4, 2, ..., 4, 1), and the weighted covariance of
 * the resulting 2D density is taken (the paper's normalisation by the maximum
 * does not change it).
 *   sigma  [m][6] FP64 device: (a, b, c, d, e, f) = (xx, xy, xz, yy, yz, zz) of
 *          each symmetric positive definite Sigma
 *   cov2   [m][3] FP64 device out: (a', b', d') = (xx, xy, yy) of each 2D density
 *   fit    nullable [19] FP64 device out (needs m >= 6): the least-squares linear
 *          map (a, b, c, d, e, f) -> (a', b', d') without intercept, row r at
 *          fit[6 r .. 6 r + 5] (r = 0, 1, 2 for a', b', d'), and fit[18] = the
 *          scalar psi minimising sum |Sigma'_2x2 - psi Sigma_2x2|_F^2
 *   ws     darb_psi_calibrate_workspace(m, grid_n) bytes
 * grid_n must be odd, 5..2049; m <= 65535.  FP32 profile values, FP64 sums.
 */
DARB_API darb_status darb_psi_calibrate(const darb_kernel *kernel, int32_t m, const double *sigma, int32_t grid_n,
                                        void *ws, size_t ws_bytes, double *cov2, double *fit, void *stream);

/*
 * darb_raster_fwd -- per-pixel DARBF evaluation and front-to-back alpha
 * compositing (DARB-Splatting section: footprint and alpha blending; the
 * per-kernel forward listings).  For each pixel p of the tile, for the tile's
 * instances in order: d = mu' - p, E = d^T Q d; skip unless 0 <= E <= e_max;
 * alpha = min(alpha_max, o F(E)); skip if alpha < alpha_min; T' = T (1 - alpha);
 * stop if T' < t_min; C += alpha T rgb; T = T'.
 *   image     [3][H][W]  C + T bg
 *   final_T   [H][W]     transmittance after the last blended splat (checkpoint)
 *   last      [H][W]     u32 position in `vals` of the last blended instance,
 *                        0xFFFFFFFF when none (checkpoint)
 *   n_contrib [H][W]     nullable: number of blended splats
 *   zero_g2d  nullable: 2D-gradient buffers of the n splats ([n] layouts of
 *             darb_grads2d) that the call also sets to zero, from the same
 *             launch (the clearing stores use the memory bandwidth the
 *             compositing leaves idle); a following darb_raster_bwd into them
 *             can then pass g2d_zeroed = 1.  They must not alias the other
 *             arguments.
 *   overflow_dev nullable: when it points at a nonzero flag the kernel writes
 *             nothing but the zeros of zero_g2d
 */
DARB_API darb_status darb_raster_fwd(const darb_projected *proj, int64_t n, const uint32_t *vals, const uint32_t *ranges,
                            const int32_t *overflow_dev, int32_t width, int32_t height, const darb_kernel *kernel,
                            const darb_raster_opts *opts, float *image, float *final_T, uint32_t *last,
                            uint32_t *n_contrib, const darb_grads2d *zero_g2d, void *stream);

/*
 * darb_raster_bwd -- reverse-order compositing gradients (Backpropagation
 * and Error Calculation; the per-kernel backward listings) from the
 * checkpoint of darb_raster_fwd: each pixel walks its list back from `last`,
 * recomputing alpha exactly as the forward did and recovering the
 * transmittance by division by (1 - alpha).  Per pair:
 *   dL/drgb += alpha T G;  dL/dalpha = G . (rgb T - S / (1 - alpha)), S = colour behind + T_final bg;
 *   dL/do += F(E) dL/dalpha  (passed straight through the alpha_max clamp);
 *   dL/dE = o F'(E) dL/dalpha;  dL/dmu' += 2 dL/dE Q d;  dL/d(a,b,c) += dL/dE (dx^2, 2 dx dy, dy^2).
 * Per (tile, splat) the partial sums are reduced across the wavefront.  Then:
 *   deterministic = 0: one set of float atomic adds per (tile, splat) (summation
 *                      order, and so the last bits, may vary between runs);
 *   deterministic = 1: two passes: every (tile, splat) partial is stored, the
 *                      partials are sorted by splat (stable) and each splat's
 *                      are summed in tile order -- bit-reproducible.  Needs
 *                      k_capacity (the capacity of vals given to darb_bin_sort)
 *                      and ws of darb_raster_bwd_workspace() bytes; otherwise
 *                      k_capacity is ignored and ws may be NULL.
 * g2d is zeroed by the call first, unless g2d_zeroed is nonzero: the caller
 * then guarantees that every element of g2d is zero already (for instance
 * cleared by darb_raster_fwd's zero_g2d on the same stream).
 *   dL_dimage [3][H][W]
 *   g2d       required output
 *   cam, in, g3d: when g3d is non-null the call continues with the chain of
 *             darb_preprocess_bwd (cam and in then required; proj passed on, so its
 *             dcolor is used when set) and overwrites g3d.
 */
DARB_API darb_status darb_raster_bwd(const darb_projected *proj, int64_t n, const uint32_t *vals, const uint32_t *ranges,
                            const int32_t *overflow_dev, int32_t width, int32_t height, const darb_kernel *kernel,
                            const darb_raster_opts *opts, const float *dL_dimage, const float *final_T,
                            const uint32_t *last, const darb_grads2d *g2d, int32_t g2d_zeroed,
                            const darb_camera *cam, const darb_splats *in, const darb_grads3d *g3d,
                            int32_t deterministic, int64_t k_capacity, void *ws, size_t ws_bytes, void *stream);

/*
 * darb_raster_bwd_workspace -- bytes of workspace of the deterministic
 * darb_raster_bwd for n splats, a width x height image and the instance
 * capacity k_capacity of its list (the stored partials are bounded by the
 * instance count).  Returns 0 for invalid or unsupported sizes.
 */
DARB_API size_t darb_raster_bwd_workspace(int64_t n, int32_t width, int32_t height, int64_t k_capacity);

/*
 * darb_preprocess_bwd -- chain rule through darb_preprocess (psi enters the
 * 2D covariance gradient for every kernel): conic -> 2D covariance -> psi ->
 * J R_cw Sigma R_cw^T J^T -> Sigma -> scale and rotation -> quaternion
 * (through the normalisation); the mean through mu', through J (zero across
 * an active Jacobian clamp) and through the SH view direction; SH
 * coefficients (zero for clamped channels); opacity passed through.
 * proj nullable: the records darb_preprocess wrote for the same camera and
 * splats; when proj->dcolor and proj->clamped are set, the colour part of the
 * chain uses them (the SH coefficients are not read) and the splats with
 * proj->radius 0 (culled by that forward) get zero gradients without reading
 * their inputs; else it recomputes the colour from the SH coefficients.  Both
 * give the same gradients up to FP32 rounding.
 * accumulate = 0: g3d is overwritten for every splat (zeros for culled splats);
 * accumulate = 1: the gradients are added to g3d (several views in turn).
 */
DARB_API darb_status darb_preprocess_bwd(const darb_camera *cam, const darb_kernel *kernel, int64_t n, const darb_splats *in,
                                const darb_projected *proj, const darb_grads2d *g2d, const darb_grads3d *g3d,
                                int32_t accumulate, void *stream);

/*
 * darb_image_loss -- per-pixel image loss of a rendered view against a target
 * (the photometric term that drives the backward pass):
 *   loss_dev  nullable [1]: the loss value (mean over 3 W H), summed in a fixed
 *             order (reproducible); needs ws of DARB_LOSS_WS_BYTES bytes
 *   dL_dimage nullable [3][H][W]: the gradient of that loss
 * image and target are [3][H][W].
 */
DARB_API darb_status darb_image_loss(const float *image, const float *target, int32_t width, int32_t height,
                                     int32_t loss_kind, float *dL_dimage, float *loss_dev, void *ws, size_t ws_bytes,
                                     void *stream);

/*
 * darb_ssim_loss -- the training loss of the Backpropagation section,
 * (1 - lambda) L1 + lambda (1 - SSIM), over a rendered view and its target:
 * L1 and SSIM are means over the 3 W H values; SSIM per channel with an 11x11
 * Gaussian window (sigma 1.5, zero padding), C1 = 0.01^2, C2 = 0.03^2.
 *   dL_dimage required [3][H][W]: the gradient of the loss
 *   loss_dev  nullable [1]: the loss value, summed in a fixed order (reproducible)
 *   ws        darb_ssim_loss_workspace(width, height) bytes
 */
DARB_API size_t darb_ssim_loss_workspace(int32_t width, int32_t height);
DARB_API darb_status darb_ssim_loss(const float *image, const float *target, int32_t width, int32_t height,
                                    float lambda, float *dL_dimage, float *loss_dev, void *ws, size_t ws_bytes,
                                    void *stream);

/*
 * darb_adam -- one Adam step over up to DARB_MAX_ADAM_GROUPS parameter tensors
 * in one launch (the optimiser of the training the paper keeps from 3DGS):
 *   m = beta1 m + (1 - beta1) g;  v = beta2 v + (1 - beta2) g^2;
 *   p -= lr / (1 - beta1^step) * m / (sqrt(v) / sqrt(1 - beta2^step) + eps)
 * step >= 1 counts the steps taken, this one included.  param, m, v are
 * updated in place; grad is read.
 */
#define DARB_MAX_ADAM_GROUPS 8
typedef struct {
    float *param;
    const float *grad;
    float *m;
    float *v;
    int64_t n;
    float lr;
} darb_adam_group;
DARB_API darb_status darb_adam(const darb_adam_group *groups, int32_t n_groups, int32_t step, float beta1, float beta2,
                               float eps, void *stream);

/*
 * darb_densify_stats -- statistics the 3DGS densification reads after each
 * backward: for every splat with radius > 0 in this view,
 *   grad_accum += |dL/dmu'| (the 2D mean gradient norm, pixels),  count += 1,
 *   max_radius = max(max_radius, radius)   (max_radius nullable).
 */
DARB_API darb_status darb_densify_stats(const darb_grads2d *g2d, const int32_t *radius, int64_t n, float *grad_accum,
                                        int32_t *count, int32_t *max_radius, void *stream);

/*
 * Multi-view calls: nv views (1 <= nv <= DARB_MAX_VIEWS) of the same n splats
 * in one launch per stage (a training step over several views, or a batch of
 * renders of one scene).  Each view keeps its own projected splats, instance
 * list, images and 2D gradients; darb_bin_sort runs per view between
 * darb_preprocess_multi and the raster calls.
 *
 * darb_preprocess_multi -- darb_preprocess for every view; the splat
 * parameters are read once.  Writes views[v].proj.
 */
DARB_API darb_status darb_preprocess_multi(const darb_view *views, int32_t nv, const darb_kernel *kernel, int64_t n,
                                           const darb_splats *in, void *stream);

/*
 * darb_preprocess_multi_cam_dev -- darb_preprocess_multi with the cameras read
 * from DEVICE memory: view v uses cams_dev[v] (an array of nv darb_camera), so
 * a captured graph of a batch of renders can be replayed for new poses after
 * the caller rewrites that array (the serving path).  views[v].cam still sizes
 * view v's tile grid (width, height) and must pass the host checks; the device
 * cameras are not validated (non-positive fx, fy or near_z cull every splat).
 */
DARB_API darb_status darb_preprocess_multi_cam_dev(const darb_view *views, int32_t nv, const darb_camera *cams_dev,
                                                   const darb_kernel *kernel, int64_t n, const darb_splats *in,
                                                   void *stream);

/*
 * darb_raster_fwd_multi -- darb_raster_fwd of every view in one launch over
 * all views' tiles.  Reads proj, vals, ranges, overflow_dev; writes image,
 * final_T, last (and n_contrib when non-NULL).
 */
DARB_API darb_status darb_raster_fwd_multi(const darb_view *views, int32_t nv, int64_t n, const darb_kernel *kernel,
                                           const darb_raster_opts *opts, void *stream);

/*
 * darb_raster_bwd_multi -- darb_raster_bwd (without the chain) of every view
 * in one launch over all views' tiles.  Reads the forward's inputs, final_T,
 * last and dL_dimage; zeroes and writes grads2d of every view.
 * deterministic as in darb_raster_bwd, with ws of
 * darb_raster_bwd_multi_workspace() bytes; it needs nv * n < 2^32.
 */
DARB_API darb_status darb_raster_bwd_multi(const darb_view *views, int32_t nv, int64_t n, const darb_kernel *kernel,
                                           const darb_raster_opts *opts, int32_t deterministic, void *ws,
                                           size_t ws_bytes, void *stream);
DARB_API size_t darb_raster_bwd_multi_workspace(const darb_view *views, int32_t nv, int64_t n);

/*
 * darb_raster_fwdbwd_multi -- forward, per-pixel loss gradient and backward
 * of every view in ONE launch: each tile composites its pixels, takes
 * dL/dI of `loss_kind` against views[v].target in registers and walks its
 * list backwards right away, with no checkpoint round trip through memory.
 * Writes image (and final_T, last, n_contrib when non-NULL) and zeroes and
 * accumulates grads2d with atomics.  Equal, up to the atomic summation order,
 * to darb_raster_fwd + darb_image_loss + darb_raster_bwd per view.
 */
DARB_API darb_status darb_raster_fwdbwd_multi(const darb_view *views, int32_t nv, int64_t n, const darb_kernel *kernel,
                                              const darb_raster_opts *opts, int32_t loss_kind, void *stream);

/*
 * darb_preprocess_bwd_multi -- darb_preprocess_bwd summed over the views:
 * g3d = sum_v chain(views[v].cam, views[v].grads2d), views in order, with the
 * splat parameters read once and g3d written once (overwritten).  When every
 * view's proj has dcolor and clamped set, the colour part uses them.
 */
DARB_API darb_status darb_preprocess_bwd_multi(const darb_view *views, int32_t nv, const darb_kernel *kernel, int64_t n,
                                               const darb_splats *in, const darb_grads3d *g3d, void *stream);

/*
 * Calibration probes: kernels that compute nothing of the method and measure
 * the ceilings the benchmark reports beside the published peaks.
 *   darb_probe_copy  dst[i] = src[i] for n floats (n a multiple of 4; both
 *                    16-byte aligned, not overlapping): 8 n bytes moved.
 *   darb_probe_fill  dst[i] = 0 for n floats (same conditions): 4 n bytes written.
 *   darb_probe_fma   `threads` lanes each run *chains (written back, currently 8)
 *                    independent chains of `iters` fused multiply-adds in FP32
 *                    (fp64 = 0, out holds threads floats) or FP64 (fp64 = 1, out
 *                    holds threads doubles), built like every kernel here
 *                    without packed FP32: 2 * chains * iters * threads flops.
 * Sizes beyond the buffers are the caller's error; n, threads, iters >= 0.
 */
DARB_API darb_status darb_probe_copy(const float *src, float *dst, int64_t n, void *stream);
DARB_API darb_status darb_probe_fill(float *dst, int64_t n, void *stream);
DARB_API darb_status darb_probe_fma(void *out, int64_t threads, int32_t iters, int32_t fp64, int32_t *chains,
                                    void *stream);

#ifdef __cplusplus
}
#endif

#endif /* DARB_H */
