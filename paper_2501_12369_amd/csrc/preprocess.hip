// preprocess.hip -- per-splat projection of 3D DARBFs to 2D footprints and its
// chain-rule backward (DARB Projection; Eq. of the 2x2 covariance projection
// with the correction factor psi; bounding radius of the DARBF boundaries
// section; SH colour of the 3DGS parameterisation kept by the paper).
//
// One thread per splat.  Parameters are structure-of-arrays, so each field
// load of a wavefront is one coalesced 256-byte transaction; culled splats
// stop after the 12-byte mean load.  HBM-bound.
#include "common.h"

namespace darb {

namespace {

// Real SH basis up to degree 3 (Condon-Shortley phase; index l^2 + l + m).
struct SH {
    float Y[16];
};

template <int NB>
__device__ __forceinline__ void sh_eval(float x, float y, float z, float *Y) {
    const float c0 = 0.28209479177387814f;   // 1/(2 sqrt(pi))
    const float c1 = 0.4886025119029199f;    // sqrt(3/(4 pi))
    const float c2a = 1.0925484305920792f;   // sqrt(15/pi)/2
    const float c2b = 0.31539156525252005f;  // sqrt(5/pi)/4
    const float c2c = 0.5462742152960396f;   // sqrt(15/pi)/4
    const float c3a = 0.5900435899266435f;   // sqrt(35/(2 pi))/4
    const float c3b = 2.890611442640554f;    // sqrt(105/pi)/2
    const float c3c = 0.4570457994644658f;   // sqrt(21/(2 pi))/4
    const float c3d = 0.3731763325901154f;   // sqrt(7/pi)/4
    const float c3e = 1.445305721320277f;    // sqrt(105/pi)/4
    Y[0] = c0;
    if constexpr (NB > 1) {
        Y[1] = -c1 * y;
        Y[2] = c1 * z;
        Y[3] = -c1 * x;
    }
    if constexpr (NB > 4) {
        float xx = x * x, yy = y * y, zz = z * z;
        Y[4] = c2a * (x * y);
        Y[5] = -c2a * (y * z);
        Y[6] = c2b * (2.0f * zz - xx - yy);
        Y[7] = -c2a * (x * z);
        Y[8] = c2c * (xx - yy);
        if constexpr (NB > 9) {
            Y[9] = -c3a * y * (3.0f * xx - yy);
            Y[10] = c3b * (x * y) * z;
            Y[11] = -c3c * y * (4.0f * zz - xx - yy);
            Y[12] = c3d * z * (2.0f * zz - 3.0f * xx - 3.0f * yy);
            Y[13] = -c3c * x * (4.0f * zz - xx - yy);
            Y[14] = c3e * z * (xx - yy);
            Y[15] = -c3a * x * (xx - 3.0f * yy);
        }
    }
}

// Gradient of sum_b g_b Y_b(d) with respect to d (unnormalised direction).
template <int NB>
__device__ __forceinline__ void sh_grad(float x, float y, float z, const float *g, float *out) {
    const float c1 = 0.4886025119029199f;
    const float c2a = 1.0925484305920792f;
    const float c2b = 0.31539156525252005f;
    const float c2c = 0.5462742152960396f;
    const float c3a = 0.5900435899266435f;
    const float c3b = 2.890611442640554f;
    const float c3c = 0.4570457994644658f;
    const float c3d = 0.3731763325901154f;
    const float c3e = 1.445305721320277f;
    float gx = 0.f, gy = 0.f, gz = 0.f;
    if constexpr (NB > 1) {
        gy += -c1 * g[1];
        gz += c1 * g[2];
        gx += -c1 * g[3];
    }
    if constexpr (NB > 4) {
        float xx = x * x, yy = y * y, zz = z * z;
        gx += c2a * y * g[4];
        gy += c2a * x * g[4];
        gy += -c2a * z * g[5];
        gz += -c2a * y * g[5];
        gx += -2.0f * c2b * x * g[6];
        gy += -2.0f * c2b * y * g[6];
        gz += 4.0f * c2b * z * g[6];
        gx += -c2a * z * g[7];
        gz += -c2a * x * g[7];
        gx += 2.0f * c2c * x * g[8];
        gy += -2.0f * c2c * y * g[8];
        if constexpr (NB > 9) {
            gx += -c3a * 6.0f * x * y * g[9];
            gy += -c3a * (3.0f * xx - 3.0f * yy) * g[9];
            gx += c3b * y * z * g[10];
            gy += c3b * x * z * g[10];
            gz += c3b * x * y * g[10];
            gx += c3c * 2.0f * x * y * g[11];
            gy += -c3c * (4.0f * zz - xx - 3.0f * yy) * g[11];
            gz += -c3c * 8.0f * y * z * g[11];
            gx += -c3d * 6.0f * x * z * g[12];
            gy += -c3d * 6.0f * y * z * g[12];
            gz += c3d * (6.0f * zz - 3.0f * xx - 3.0f * yy) * g[12];
            gx += -c3c * (4.0f * zz - 3.0f * xx - yy) * g[13];
            gy += c3c * 2.0f * x * y * g[13];
            gz += -c3c * 8.0f * x * z * g[13];
            gx += c3e * 2.0f * x * z * g[14];
            gy += -c3e * 2.0f * y * z * g[14];
            gz += c3e * (xx - yy) * g[14];
            gx += -c3a * (3.0f * xx - 3.0f * yy) * g[15];
            gy += c3a * 6.0f * x * y * g[15];
        }
    }
    out[0] = gx;
    out[1] = gy;
    out[2] = gz;
}

// A splat's rotation and scale parameters as loaded: quaternion (w, x, y, z), scales.
struct QS {
    float q[4], s[3];
};

__device__ __forceinline__ QS load_qs(const darb_splats &in, int n, int i) {
    QS v;
    v.q[0] = in.quats[i]; v.q[1] = in.quats[n + i]; v.q[2] = in.quats[2 * n + i]; v.q[3] = in.quats[3 * n + i];
    v.s[0] = in.scales[i]; v.s[1] = in.scales[n + i]; v.s[2] = in.scales[2 * n + i];
    return v;
}

__device__ __forceinline__ void load_mean(const darb_splats &in, int n, int i, float (&m)[3]) {
    m[0] = in.means[i];
    m[1] = in.means[n + i];
    m[2] = in.means[2 * n + i];
}

// View-independent geometry of a splat in FP64 from its FP32 parameters: unit
// quaternion, rotation, scales, 3D covariance Sigma = R diag(s^2) R^T (all nine
// entries, each summed in the order of the definition).
struct Geom64 {
    double Rq[9], qn[4], qinv, s[3], S[9];
};

// false for a zero (or non-finite) quaternion
__device__ __forceinline__ bool splat_geom64(const QS &v, Geom64 &G) {
    const double q0 = v.q[0], q1 = v.q[1], q2 = v.q[2], q3 = v.q[3];
    const double qnorm = sqrt(q0 * q0 + q1 * q1 + q2 * q2 + q3 * q3);
    G.s[0] = v.s[0];
    G.s[1] = v.s[1];
    G.s[2] = v.s[2];
    if (!(qnorm > 0.0)) return false;
    G.qinv = 1.0 / qnorm;
    const double w = q0 * G.qinv, x = q1 * G.qinv, y = q2 * G.qinv, z = q3 * G.qinv;
    G.qn[0] = w; G.qn[1] = x; G.qn[2] = y; G.qn[3] = z;
    double *Rq = G.Rq;
    Rq[0] = 1.0 - 2.0 * (y * y + z * z);
    Rq[1] = 2.0 * (x * y - w * z);
    Rq[2] = 2.0 * (x * z + w * y);
    Rq[3] = 2.0 * (x * y + w * z);
    Rq[4] = 1.0 - 2.0 * (x * x + z * z);
    Rq[5] = 2.0 * (y * z - w * x);
    Rq[6] = 2.0 * (x * z - w * y);
    Rq[7] = 2.0 * (y * z + w * x);
    Rq[8] = 1.0 - 2.0 * (x * x + y * y);
    for (int r = 0; r < 3; r++)
        for (int c = 0; c < 3; c++) {
            double acc = 0.0;
            for (int l = 0; l < 3; l++) acc += Rq[r * 3 + l] * G.s[l] * G.s[l] * Rq[c * 3 + l];
            G.S[r * 3 + c] = acc;
        }
    return true;
}

// Projection of one splat in one view.  Computed in FP64 from the FP32 inputs
// and rounded once to the FP32 records (mean2D, depth, conic factor): the
// records are the correctly rounded values of the projection's definition,
// so the rasterizer sees the same inputs whatever order a faster FP32 chain
// would have taken.  The kernel is HBM-bound; the FP64 arithmetic (vector FP64
// runs at the non-packed FP32 rate on this GPU) is hidden behind the loads.
struct Proj {
    double t[3];
    double xt, yt;        // t_x / t_z, t_y / t_z, clamped for the Jacobian
    bool cx_, cy_;        // Jacobian clamp active in x / y
    float u, v;           // mean2D (rounded)
    float l00, l01, l11;  // Q = L^T L, L = [[l00, l01], [0, l11]] (rounded)
    int radius;
    int ex, ey;           // half-extents of the tile box
};

constexpr double kMaxBoxPx = 1073741824.0;  // 2^30: the largest radius or tile-box half-extent

// t = R_cw mu + t_cw; false when the splat is not in front of the near plane.
__device__ __forceinline__ bool view_depth(const Cam &cam, const float (&m)[3], Proj &P) {
    for (int r = 0; r < 3; r++)
        P.t[r] = (double)cam.R[r * 3] * m[0] + (double)cam.R[r * 3 + 1] * m[1] + (double)cam.R[r * 3 + 2] * m[2] +
                 (double)cam.t[r];
    return P.t[2] > (double)cam.near_z;
}

// The rest of the projection of a splat in front of the camera (P.t set);
// false when culled (singular 2D covariance, or a tile box off the tile grid).
__device__ __forceinline__ bool project_rest(const Cam &cam, const KParams &kp, const Geom64 &G, Proj &P) {
    // one FP64 division (1/t_z) and reciprocals elsewhere: each product errs by an
    // FP64 rounding or two, far below the FP32 rounding of the records
    const double tz = P.t[2], itz = 1.0 / tz, fx = cam.fx, fy = cam.fy;
    P.xt = P.t[0] * itz;
    P.yt = P.t[1] * itz;
    P.cx_ = P.cy_ = false;
    if (cam.lim_x > 0.0) {
        if (P.xt > cam.lim_x) { P.xt = cam.lim_x; P.cx_ = true; }
        if (P.xt < -cam.lim_x) { P.xt = -cam.lim_x; P.cx_ = true; }
        if (P.yt > cam.lim_y) { P.yt = cam.lim_y; P.cy_ = true; }
        if (P.yt < -cam.lim_y) { P.yt = -cam.lim_y; P.cy_ = true; }
    }
    const double J00 = fx * itz, J02 = -fx * P.xt * itz, J11 = fy * itz, J12 = -fy * P.yt * itz;
    // A = J R_cw (2x3), M = A Sigma A^T
    double A[6];
    for (int c = 0; c < 3; c++) {
        A[c] = J00 * (double)cam.R[c] + J02 * (double)cam.R[6 + c];
        A[3 + c] = J11 * (double)cam.R[3 + c] + J12 * (double)cam.R[6 + c];
    }
    double AS[6];
    for (int r = 0; r < 2; r++)
        for (int c = 0; c < 3; c++)
            AS[r * 3 + c] = A[r * 3] * G.S[c] + A[r * 3 + 1] * G.S[3 + c] + A[r * 3 + 2] * G.S[6 + c];
    const double M00 = AS[0] * A[0] + AS[1] * A[1] + AS[2] * A[2];
    const double M01 = AS[0] * A[3] + AS[1] * A[4] + AS[2] * A[5];
    const double M11 = AS[3] * A[3] + AS[4] * A[4] + AS[5] * A[5];
    // Sigma'_2x2 = psi M + eps I, conic Q = Sigma'^-1
    const double psi = kp.psi, eps = cam.dilation;
    const double c00 = psi * M00 + eps, c01 = psi * M01, c11 = psi * M11 + eps;
    const double det = c00 * c11 - c01 * c01;
    if (!(det > 0.0)) return false;
    const double rs = 1.0 / sqrt(c11 * det);  // 1 / sqrt(c11 det)
    P.l11 = (float)(1.0 / sqrt(c11));
    P.l00 = (float)(c11 * rs);                             // sqrt(c11 / det)
    P.l01 = (float)(-c01 * rs);
    P.u = (float)(fx * P.t[0] * itz + (double)cam.cx);
    P.v = (float)(fy * P.t[1] * itz + (double)cam.cy);
    // radius rf sqrt(lambda_max), rf = 3 (or sqrt(e_max) beyond E = 9)
    const double mid = 0.5 * (c00 + c11);
    const double disc = mid * mid - det;
    const double lam = mid + sqrt(disc > 0.0 ? disc : 0.0);
    const double rf = kp.e_max > 9.0f ? sqrt((double)kp.e_max) : 3.0;
    // (sizes are capped at 2^30 px, beyond any image, so the conversion to int
    // is defined for every finite covariance)
    P.radius = (int)ceil(fmin(rf * sqrt(lam), kMaxBoxPx));
    // Tile box: the bounding box of the ellipse {d : d^T Sigma'^-1 d <= rf^2},
    // half-extents rf sqrt(Sigma'_xx), rf sqrt(Sigma'_yy) rounded up to whole
    // pixels.  It holds the support E <= e_max and lies inside the square of
    // half-side R; the image does not depend on it (every pixel tests E).
    P.ex = (int)ceil(fmin(rf * sqrt(c00), kMaxBoxPx));
    P.ey = (int)ceil(fmin(rf * sqrt(c11), kMaxBoxPx));
    // its rectangle on the tile grid (the binning's FP32 expression on the stored mean)
    int gx = (cam.width + kTile - 1) / kTile, gy = (cam.height + kTile - 1) / kTile;
    const float rx = (float)P.ex, ry = (float)P.ey;
    float x0 = fminf(fmaxf(floorf((P.u - rx) * 0.0625f), 0.0f), (float)gx);
    float x1 = fminf(fmaxf(floorf((P.u + rx) * 0.0625f) + 1.0f, 0.0f), (float)gx);
    float y0 = fminf(fmaxf(floorf((P.v - ry) * 0.0625f), 0.0f), (float)gy);
    float y1 = fminf(fmaxf(floorf((P.v + ry) * 0.0625f) + 1.0f, 0.0f), (float)gy);
    if (!((x1 > x0) & (y1 > y0))) return false;
    return true;
}

// The forward's Jacobian-clamp decisions, as the backward needs them.
struct Clamp {
    double xt, yt;  // the clamped t_x / t_z, t_y / t_z (used where the clamp is active)
    bool cx_, cy_;
};

// The clamp decisions alone (the splat known to be in front of the camera).
__device__ __forceinline__ void clamp_of(const Cam &cam, const float (&m)[3], Clamp &cj) {
    Proj P;
    view_depth(cam, m, P);
    const double itz = 1.0 / P.t[2];  // the forward's expression, so that the decisions agree
    cj.xt = P.t[0] * itz;
    cj.yt = P.t[1] * itz;
    cj.cx_ = cj.cy_ = false;
    if (cam.lim_x > 0.0) {
        if (cj.xt > cam.lim_x) { cj.xt = cam.lim_x; cj.cx_ = true; }
        if (cj.xt < -cam.lim_x) { cj.xt = -cam.lim_x; cj.cx_ = true; }
        if (cj.yt > cam.lim_y) { cj.yt = cam.lim_y; cj.cy_ = true; }
        if (cj.yt < -cam.lim_y) { cj.yt = -cam.lim_y; cj.cy_ = true; }
    }
}

// Whether the forward kept the splat, and its clamp decisions.
__device__ __forceinline__ bool forward_visible(const Cam &cam, const KParams &kp, const float (&m)[3], const QS &qs,
                                                Clamp &cj) {
    Proj P;
    Geom64 G;
    const bool vis = view_depth(cam, m, P) && splat_geom64(qs, G) && project_rest(cam, kp, G, P);
    cj = Clamp{P.xt, P.yt, P.cx_, P.cy_};
    return vis;
}

// Marks a loaded value as used here.  Loads whose values are used only under a
// later branch would otherwise be moved into that branch, each group behind
// the previous branch's memory round trip; pinned right after they are issued,
// a group of loads costs one round trip.
__device__ __forceinline__ void pin(float v) { asm volatile("" ::"v"(v)); }

__device__ __forceinline__ void pin_geometry(const float (&m)[3], const QS &qs) {
#pragma unroll
    for (int k = 0; k < 3; k++) pin(m[k]);
#pragma unroll
    for (int k = 0; k < 4; k++) pin(qs.q[k]);
#pragma unroll
    for (int k = 0; k < 3; k++) pin(qs.s[k]);
}

// SH coefficients of splat i, all loads issued before any use: c[b][ch]
template <int NB>
__device__ __forceinline__ void load_sh(const float *sh, int n, int i, float (&c)[NB][3]) {
#pragma unroll
    for (int b = 0; b < NB; b++)
#pragma unroll
        for (int ch = 0; ch < 3; ch++) c[b][ch] = sh[(size_t)(b * 3 + ch) * n + i];
}

// The same loads marked non-temporal: the colour part beside the binning streams
// its 576 MB of coefficients (3M splats, degree 3) without displacing the
// binning kernels' working set from the caches.
template <int NB>
__device__ __forceinline__ void load_sh_nt(const float *sh, int n, int i, float (&c)[NB][3]) {
#pragma unroll
    for (int b = 0; b < NB; b++)
#pragma unroll
        for (int ch = 0; ch < 3; ch++) c[b][ch] = __builtin_nontemporal_load(sh + (size_t)(b * 3 + ch) * n + i);
}

// Camera constants from a darb_camera in device memory (same derivation as the
// host path); the tile grid keeps the caller's width/height.  A camera with
// non-positive focal lengths or near plane culls every splat.
__device__ __forceinline__ Cam cam_from_device(const darb_camera *c, int width, int height) {
    Cam m;
    for (int r = 0; r < 3; r++) {
        for (int k = 0; k < 3; k++) m.R[r * 3 + k] = c->viewmat[r * 4 + k];
        m.t[r] = c->viewmat[r * 4 + 3];
        m.campos[r] = c->campos[r];
    }
    m.fx = c->fx;
    m.fy = c->fy;
    m.cx = c->cx;
    m.cy = c->cy;
    m.width = width;
    m.height = height;
    m.near_z = c->near_z;
    if (!(m.fx > 0.0f) || !(m.fy > 0.0f) || !(m.near_z > 0.0f)) m.near_z = INFINITY;
    if (c->jac_clamp > 0.0f && m.near_z < INFINITY) {
        m.lim_x = (double)c->jac_clamp * (0.5 * (double)width) / (double)m.fx;
        m.lim_y = (double)c->jac_clamp * (0.5 * (double)height) / (double)m.fy;
    } else {
        m.lim_x = m.lim_y = 0.0;
    }
    m.dilation = fmaxf(c->dilation, 0.0f);
    return m;
}

// Colour of a visible splat from its loaded SH coefficients; sets the clamp
// bits, and with JAC the derivative of each channel (before the clamp) with
// respect to the unit view direction u: jac[3 c + k] = d colour_c / d u_k.
template <int NB, bool JAC>
__device__ __forceinline__ void sh_colour(const Cam &cam, const float (&m)[3], const float (&c)[NB][3], float (&col)[3],
                                          uint8_t &cl, float (&jac)[9]) {
    float dx = m[0] - cam.campos[0], dy = m[1] - cam.campos[1], dz = m[2] - cam.campos[2];
    float il = rsqrtf(fmaf(dx, dx, fmaf(dy, dy, dz * dz)));
    const float ux = dx * il, uy = dy * il, uz = dz * il;
    float Y[NB];
    sh_eval<NB>(ux, uy, uz, Y);
    cl = 0;
#pragma unroll
    for (int ch = 0; ch < 3; ch++) {
        float acc = 0.0f;
#pragma unroll
        for (int b = 0; b < NB; b++) acc = fmaf(Y[b], c[b][ch], acc);
        acc += 0.5f;
        if (acc < 0.0f) cl |= (uint8_t)(1u << ch);
        col[ch] = fmaxf(acc, 0.0f);
        if constexpr (JAC) {
            float g[NB], d[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int b = 0; b < NB; b++) g[b] = c[b][ch];
            if constexpr (NB > 1) sh_grad<NB>(ux, uy, uz, g, d);
            jac[3 * ch] = d[0];
            jac[3 * ch + 1] = d[1];
            jac[3 * ch + 2] = d[2];
        }
    }
}

// Every lane stores (zeros for culled splats): whole-line writes.  The
// geometry part of the record (what the binning reads) ...
__device__ __forceinline__ void store_geom(const darb_projected &out, int i, bool vis, const Proj &P, float op) {
    reinterpret_cast<float2 *>(out.xy)[i] = vis ? make_float2(P.u, P.v) : make_float2(0.0f, 0.0f);
    out.depth[i] = vis ? (float)P.t[2] : 0.0f;
    out.radius[i] = vis ? P.radius : 0;
    reinterpret_cast<int2 *>(out.extent)[i] = vis ? make_int2(P.ex, P.ey) : make_int2(0, 0);
    reinterpret_cast<float4 *>(out.conic_o)[i] = vis ? make_float4(P.l00, P.l01, P.l11, op) : make_float4(0, 0, 0, 0);
}

// ... and its colour part (NT: the checkpoint, read only by the backward, is
// stored non-temporal).
template <bool NT = false>
__device__ __forceinline__ void store_colour(const darb_projected &out, int n, int i, bool vis, const float (&col)[3],
                                             uint8_t cl, const float (&jac)[9]) {
    if (out.dcolor) {
#pragma unroll
        for (int k = 0; k < 9; k++) {
            float *p = out.dcolor + (size_t)k * n + i;
            if constexpr (NT)
                __builtin_nontemporal_store(vis ? jac[k] : 0.0f, p);
            else
                *p = vis ? jac[k] : 0.0f;
        }
    }
    out.rgb[3 * i] = col[0];
    out.rgb[3 * i + 1] = col[1];
    out.rgb[3 * i + 2] = col[2];
    out.clamped[i] = cl;
}

__device__ __forceinline__ void store_proj(const darb_projected &out, int n, int i, bool vis, const Proj &P, float op,
                                           const float (&col)[3], uint8_t cl, const float (&jac)[9]) {
    store_colour(out, n, i, vis, col, cl, jac);
    store_geom(out, i, vis, P, op);
}

template <int DEG>
__global__ __launch_bounds__(256) void k_preprocess(Cam cam_arg, const darb_camera *cam_dev, KParams kp, int n,
                                                    darb_splats in, darb_projected out) {
    constexpr int NB = (DEG + 1) * (DEG + 1);
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const Cam cam = cam_dev ? cam_from_device(cam_dev, cam_arg.width, cam_arg.height) : cam_arg;
    // the geometry's loads are issued together (one memory round trip before the
    // projection), the SH coefficients only for the splats that survive it
    float m[3];
    load_mean(in, n, i, m);
    const QS qs = load_qs(in, n, i);
    const float op_in = in.opacity[i];
    pin_geometry(m, qs);
    Geom64 G;
    Proj P;
    const bool vis = view_depth(cam, m, P) && splat_geom64(qs, G) && project_rest(cam, kp, G, P);
    float col[3] = {0.0f, 0.0f, 0.0f};
    float jac[9] = {};
    float op = 0.0f;
    uint8_t cl = 0;
    if (vis) {
        float c[NB][3];
        load_sh<NB>(in.sh, n, i, c);
        op = op_in;
        if (out.dcolor)
            sh_colour<NB, true>(cam, m, c, col, cl, jac);
        else
            sh_colour<NB, false>(cam, m, c, col, cl, jac);
    }
    store_proj(out, n, i, vis, P, op, col, cl, jac);
}

// The two parts of k_preprocess as separate launches, each with the same
// arithmetic (so together they give its bits).  Geometry: the record the
// binning reads (xy, depth, radius, tile box, conic and opacity).
__global__ __launch_bounds__(256) void k_preprocess_geom(Cam cam, KParams kp, int n, darb_splats in,
                                                         darb_projected out) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float m[3];
    load_mean(in, n, i, m);
    const QS qs = load_qs(in, n, i);
    const float op_in = in.opacity[i];
    pin_geometry(m, qs);
    Geom64 G;
    Proj P;
    const bool vis = view_depth(cam, m, P) && splat_geom64(qs, G) && project_rest(cam, kp, G, P);
    store_geom(out, i, vis, P, vis ? op_in : 0.0f);
}

// Colour: the SH colour, clamp bits and colour checkpoint of the splats the
// geometry part kept (radius > 0; a kept splat's radius is at least 1).  It is
// meant to run beside the binning on a second stream, so it is launched with
// three one-wavefront workgroups per compute unit looping over the splats: a
// full grid of memory-bound waves would take the compute units from the
// latency-bound binning kernels and slow them by about its own duration.
#ifndef DARB_COLOUR_THREADS
#define DARB_COLOUR_THREADS 64
#endif
constexpr int kColourThreads = DARB_COLOUR_THREADS;  // threads per workgroup (a tuning constant)
#ifndef DARB_COLOUR_WGS_PER_CU
#define DARB_COLOUR_WGS_PER_CU 3
#endif
constexpr int kColourWgsPerCu = DARB_COLOUR_WGS_PER_CU;  // workgroups per compute unit (a tuning constant)

template <int DEG>
__global__ __launch_bounds__(kColourThreads) void k_preprocess_colour(Cam cam, int n, darb_splats in, darb_projected out) {
    constexpr int NB = (DEG + 1) * (DEG + 1);
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const bool vis = out.radius[i] > 0;
        float col[3] = {0.0f, 0.0f, 0.0f};
        float jac[9] = {};
        uint8_t cl = 0;
        if (vis) {
            float m[3];
            load_mean(in, n, i, m);
            float c[NB][3];
            load_sh_nt<NB>(in.sh, n, i, c);
            if (out.dcolor)
                sh_colour<NB, true>(cam, m, c, col, cl, jac);
            else
                sh_colour<NB, false>(cam, m, c, col, cl, jac);
        }
        store_colour<true>(out, n, i, vis, col, cl, jac);
    }
}

// Several views: the parameters are read once, the geometry computed once.
template <int DEG>
__global__ __launch_bounds__(256) void k_preprocess_multi(Cams cams, KParams kp, int n, darb_splats in, Projs outs) {
    constexpr int NB = (DEG + 1) * (DEG + 1);
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float m[3];
    load_mean(in, n, i, m);
    Geom64 G;
    const bool geom = splat_geom64(load_qs(in, n, i), G);
    float c[NB][3];
    float op = 0.0f;
    if (geom) {
        load_sh<NB>(in.sh, n, i, c);
        op = in.opacity[i];
    }
    auto one_view = [&](const Cam &cam, const darb_projected &out) {
        Proj P;
        const bool vis = geom && view_depth(cam, m, P) && project_rest(cam, kp, G, P);
        float col[3] = {0.0f, 0.0f, 0.0f};
        float jac[9] = {};
        uint8_t cl = 0;
        if (vis) {
            if (out.dcolor)
                sh_colour<NB, true>(cam, m, c, col, cl, jac);
            else
                sh_colour<NB, false>(cam, m, c, col, cl, jac);
        }
        store_proj(out, n, i, vis, P, vis ? op : 0.0f, col, cl, jac);
    };
    for (int v = 0; v < cams.nv; v++) {
        if (cams.dev)
            one_view(cam_from_device(cams.dev + v, cams.c[v].width, cams.c[v].height), outs.p[v]);
        else
            one_view(cams.c[v], outs.p[v]);
    }
}

// Per-view part of the gradient of one visible splat: the mean (through mu',
// J and, given as dmu_sh, the SH direction), the scales and the quaternion.
// The colour part (colour_bwd_*: Y, gv with d/d sh[b][ch] = Y[b] * gv[ch])
// runs in FP32.  The chain from the 2D conic gradient to the
// covariance, J and the splat's scales and rotation runs in FP64, on a
// projection recomputed in FP64 from the FP32 inputs with the forward's FP32
// decisions (Jacobian clamp): for a needle-like footprint the conic's small
// eigen-direction is a residual of its entries, and the FP32 chain loses it
// (about eps_32 kappa relative error in the scale and rotation gradients).
// The kernel is HBM-bound, so the FP64 arithmetic costs little.
// View direction terms of the colour of a visible splat: the unit direction
// (dx, dy, dz) and 1/|v| from the camera centre, the SH basis Y, and gv[ch] =
// dL/dcolour[ch] where the colour is not clamped (else 0).
template <int NB>
__device__ __forceinline__ void sh_view(const Cam &cam, const float (&m)[3], const float (&csh)[NB][3],
                                        const float (&grgb)[3], float (&d)[3], float &il, float (&Y)[NB],
                                        float (&gvo)[3]) {
    float vx = m[0] - cam.campos[0], vy = m[1] - cam.campos[1], vz = m[2] - cam.campos[2];
    il = rsqrtf(fmaf(vx, vx, fmaf(vy, vy, vz * vz)));
    d[0] = vx * il;
    d[1] = vy * il;
    d[2] = vz * il;
    sh_eval<NB>(d[0], d[1], d[2], Y);
#pragma unroll
    for (int ch = 0; ch < 3; ch++) {
        float acc = 0.0f;
#pragma unroll
        for (int b = 0; b < NB; b++) acc = fmaf(Y[b], csh[b][ch], acc);
        acc += 0.5f;
        gvo[ch] = (acc < 0.0f) ? 0.0f : grgb[ch];
    }
}

// The mean's gradient through the view direction, from gdir = d L / d u (u the
// unit direction): the tangential part divided by |v|.
__device__ __forceinline__ void dir_to_mean(const float (&d)[3], float il, const float (&gdir)[3], float (&out)[3]) {
    const float dd = fmaf(gdir[0], d[0], fmaf(gdir[1], d[1], gdir[2] * d[2]));
    out[0] = (gdir[0] - d[0] * dd) * il;
    out[1] = (gdir[1] - d[1] * dd) * il;
    out[2] = (gdir[2] - d[2] * dd) * il;
}

// Colour part of the chain from the SH coefficients: Y, gv (see sh_view) and
// the mean's gradient through the view direction.
template <int NB>
__device__ __forceinline__ void colour_bwd_sh(const Cam &cam, const float (&m)[3], const float (&csh)[NB][3],
                                              const float (&grgb)[3], float (&Y)[NB], float (&gvo)[3],
                                              float (&dmu_sh)[3]) {
    float d[3], il;
    sh_view<NB>(cam, m, csh, grgb, d, il, Y, gvo);
    float gdir[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int ch = 0; ch < 3; ch++) {
        const float gv = gvo[ch];
        float gsh[NB];
#pragma unroll
        for (int b = 0; b < NB; b++) gsh[b] = gv * csh[b][ch];
        if constexpr (NB > 1) {
            float gd[3];
            sh_grad<NB>(d[0], d[1], d[2], gsh, gd);
            gdir[0] += gd[0];
            gdir[1] += gd[1];
            gdir[2] += gd[2];
        }
    }
    dir_to_mean(d, il, gdir, dmu_sh);
}

// The same from the forward's checkpoint: clamp bits and d colour / d u; the SH
// coefficients are not read.
template <int NB>
__device__ __forceinline__ void colour_bwd_ckpt(const Cam &cam, const float (&m)[3], uint8_t cl, const float (&jac)[9],
                                                const float (&grgb)[3], float (&Y)[NB], float (&gvo)[3],
                                                float (&dmu_sh)[3]) {
    float vx = m[0] - cam.campos[0], vy = m[1] - cam.campos[1], vz = m[2] - cam.campos[2];
    const float il = rsqrtf(fmaf(vx, vx, fmaf(vy, vy, vz * vz)));
    const float d[3] = {vx * il, vy * il, vz * il};
    sh_eval<NB>(d[0], d[1], d[2], Y);
    float gdir[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int ch = 0; ch < 3; ch++) {
        gvo[ch] = ((cl >> ch) & 1u) ? 0.0f : grgb[ch];
#pragma unroll
        for (int k = 0; k < 3; k++) gdir[k] = fmaf(gvo[ch], jac[3 * ch + k], gdir[k]);
    }
    dir_to_mean(d, il, gdir, dmu_sh);
}

// Incoming gradients of one splat with respect to its projected quantities.
struct G2v {
    float xy[2], conic[3], op, rgb[3];
};

__device__ __forceinline__ G2v load_g2(const darb_grads2d &g2, int i) {
    G2v v;
    v.xy[0] = g2.xy[2 * i];
    v.xy[1] = g2.xy[2 * i + 1];
    v.conic[0] = g2.conic[3 * i];
    v.conic[1] = g2.conic[3 * i + 1];
    v.conic[2] = g2.conic[3 * i + 2];
    v.op = g2.opacity[i];
    v.rgb[0] = g2.rgb[3 * i];
    v.rgb[1] = g2.rgb[3 * i + 1];
    v.rgb[2] = g2.rgb[3 * i + 2];
    return v;
}

// dmu_sh: the mean's gradient through the view direction (colour part, FP32).
__device__ __forceinline__ void splat_bwd_view(const Cam &cam, const KParams &kp, const float (&m)[3],
                                               const G2v &g2, const Geom64 &G, const Clamp &P,
                                               const float (&dmu_sh)[3], float (&dmu)[3], float (&dsc)[3],
                                               float (&dqo)[4]) {

    // ---- projection in FP64: t, J (clamped as the forward decided), A = J R_cw,
    //      2D covariance and conic
    const float *Rf = cam.R;
    double R[9];
    for (int k = 0; k < 9; k++) R[k] = Rf[k];
    const double t0 = R[0] * m[0] + R[1] * m[1] + R[2] * m[2] + (double)cam.t[0];
    const double t1 = R[3] * m[0] + R[4] * m[1] + R[5] * m[2] + (double)cam.t[1];
    const double tz = R[6] * m[0] + R[7] * m[1] + R[8] * m[2] + (double)cam.t[2];
    const double itz = 1.0 / tz, itz2 = itz * itz;
    const double fx = cam.fx, fy = cam.fy;
    const double xt = P.cx_ ? (double)P.xt : t0 * itz;
    const double yt = P.cy_ ? (double)P.yt : t1 * itz;
    const double J00 = fx * itz, J02 = -fx * xt * itz, J11 = fy * itz, J12 = -fy * yt * itz;
    double A[6];
    for (int cc = 0; cc < 3; cc++) {
        A[cc] = J00 * R[cc] + J02 * R[6 + cc];
        A[3 + cc] = J11 * R[3 + cc] + J12 * R[6 + cc];
    }
    const double *Sf = G.S;
    double AS0[3], AS1[3];  // A Sigma (2x3)
    for (int cc = 0; cc < 3; cc++) {
        AS0[cc] = A[0] * Sf[cc] + A[1] * Sf[3 + cc] + A[2] * Sf[6 + cc];
        AS1[cc] = A[3] * Sf[cc] + A[4] * Sf[3 + cc] + A[5] * Sf[6 + cc];
    }
    const double psi = kp.psi, eps = cam.dilation;
    const double c00 = psi * (AS0[0] * A[0] + AS0[1] * A[1] + AS0[2] * A[2]) + eps;
    const double c01 = psi * (AS0[0] * A[3] + AS0[1] * A[4] + AS0[2] * A[5]);
    const double c11 = psi * (AS1[0] * A[3] + AS1[1] * A[4] + AS1[2] * A[5]) + eps;
    const double idet = 1.0 / (c00 * c11 - c01 * c01);
    const double a = c11 * idet, b = -c01 * idet, c = c00 * idet;

    // ---- conic -> 2D covariance: dL/dcov = -Q Ghat Q, Ghat = [[ga, gb/2], [gb/2, gc]];
    //      psi: M -> psi M + eps I
    const double ga = g2.conic[0], gb = 0.5 * (double)g2.conic[1], gc = g2.conic[2];
    const double q00 = a * ga + b * gb, q01 = a * gb + b * gc;
    const double q10 = b * ga + c * gb, q11 = b * gb + c * gc;
    const double m00 = -psi * (q00 * a + q01 * b);
    const double m01 = -psi * (q00 * b + q01 * c);
    const double m11 = -psi * (q10 * b + q11 * c);
    // M = A Sigma A^T: dA = 2 dM A Sigma
    double dA[6];
    for (int cc = 0; cc < 3; cc++) {
        dA[cc] = 2.0 * (m00 * AS0[cc] + m01 * AS1[cc]);
        dA[3 + cc] = 2.0 * (m01 * AS0[cc] + m11 * AS1[cc]);
    }
    // A = J R_cw: dJ = dA R_cw^T
    const double dJ00 = dA[0] * R[0] + dA[1] * R[1] + dA[2] * R[2];
    const double dJ02 = dA[0] * R[6] + dA[1] * R[7] + dA[2] * R[8];
    const double dJ11 = dA[3] * R[3] + dA[4] * R[4] + dA[5] * R[5];
    const double dJ12 = dA[3] * R[6] + dA[4] * R[7] + dA[5] * R[8];
    const double dxt_dtx = P.cx_ ? 0.0 : itz, dxt_dtz = P.cx_ ? 0.0 : -t0 * itz2;
    const double dyt_dty = P.cy_ ? 0.0 : itz, dyt_dtz = P.cy_ ? 0.0 : -t1 * itz2;
    double dtx = dJ02 * (-fx * dxt_dtx * itz);
    double dty = dJ12 * (-fy * dyt_dty * itz);
    double dtz = dJ00 * (-fx * itz2) + dJ11 * (-fy * itz2);
    dtz += dJ02 * (-fx * (dxt_dtz * tz - xt) * itz2);
    dtz += dJ12 * (-fy * (dyt_dtz * tz - yt) * itz2);
    // mean2D
    const double gu = g2.xy[0], gvv = g2.xy[1];
    dtx += gu * fx * itz;
    dty += gvv * fy * itz;
    dtz -= (gu * fx * t0 + gvv * fy * t1) * itz2;
    // t = R_cw mu + t_cw
    dmu[0] = dmu_sh[0] + (float)(R[0] * dtx + R[3] * dty + R[6] * dtz);
    dmu[1] = dmu_sh[1] + (float)(R[1] * dtx + R[4] * dty + R[7] * dtz);
    dmu[2] = dmu_sh[2] + (float)(R[2] * dtx + R[5] * dty + R[8] * dtz);

    // ---- scales and rotation from dM (M = B B^T, B = C diag(s), C = A Rq):
    //   ds_j = 2 s_j c_j^T dM c_j,  dRq_rj = 2 s_j^2 (A^T dM C)_rj
    const double *Rq = G.Rq;
    double C0[3], C1[3];
    for (int cc = 0; cc < 3; cc++) {
        C0[cc] = A[0] * Rq[cc] + A[1] * Rq[3 + cc] + A[2] * Rq[6 + cc];
        C1[cc] = A[3] * Rq[cc] + A[4] * Rq[3 + cc] + A[5] * Rq[6 + cc];
    }
    double dR[9];
    for (int cc = 0; cc < 3; cc++) {
        const double e0 = m00 * C0[cc] + m01 * C1[cc];
        const double e1 = m01 * C0[cc] + m11 * C1[cc];
        dsc[cc] = (float)(2.0 * G.s[cc] * (C0[cc] * e0 + C1[cc] * e1));
        const double k = 2.0 * G.s[cc] * G.s[cc];
        for (int r = 0; r < 3; r++) dR[r * 3 + cc] = k * (A[r] * e0 + A[3 + r] * e1);
    }
    // rotation gradient through the rotation vector of dR Rq^T (its antisymmetric
    // part), then to the quaternion through the normalisation
    double Mk[3][3];
    for (int r = 0; r < 3; r++)
        for (int cc = 0; cc < 3; cc++)
            Mk[r][cc] = dR[r * 3] * Rq[cc * 3] + dR[r * 3 + 1] * Rq[cc * 3 + 1] + dR[r * 3 + 2] * Rq[cc * 3 + 2];
    const double h0 = Mk[2][1] - Mk[1][2], h1 = Mk[0][2] - Mk[2][0], h2 = Mk[1][0] - Mk[0][1];
    const double w = G.qn[0], x = G.qn[1], y = G.qn[2], z = G.qn[3];
    const double s2q = 2.0 * G.qinv;
    dqo[0] = (float)(-s2q * (h0 * x + h1 * y + h2 * z));
    dqo[1] = (float)(s2q * (w * h0 + h1 * z - h2 * y));
    dqo[2] = (float)(s2q * (w * h1 + h2 * x - h0 * z));
    dqo[3] = (float)(s2q * (w * h2 + h0 * y - h1 * x));
}

// Gradients of one splat, accumulated over views by the callers.
struct Grad3 {
    float dmu[3], dsc[3], dq[4], dop;
};

template <int NB>
__device__ __forceinline__ void store_grads(const darb_grads3d &g3, int n, int i, const Grad3 &g,
                                            const float (&gsh)[NB][3], bool accumulate) {
    // every lane stores (zeros for culled splats): whole-line writes
    auto put = [&](float *p, size_t idx, float v) { p[idx] = accumulate ? p[idx] + v : v; };
#pragma unroll
    for (int c = 0; c < 3; c++) {
        put(g3.means, (size_t)c * n + i, g.dmu[c]);
        put(g3.scales, (size_t)c * n + i, g.dsc[c]);
    }
#pragma unroll
    for (int c = 0; c < 4; c++) put(g3.quats, (size_t)c * n + i, g.dq[c]);
    put(g3.opacity, i, g.dop);
#pragma unroll
    for (int b = 0; b < NB; b++)
#pragma unroll
        for (int ch = 0; ch < 3; ch++) put(g3.sh, (size_t)(b * 3 + ch) * n + i, gsh[b][ch]);
}

// CKPT: the colour part from the forward's checkpoint (ck: dcolor [9][n] and
// clamped of the view) instead of the SH coefficients.
struct Ckpt {
    const float *dcolor;
    const uint8_t *clamped;
    const int32_t *radius;  // kept iff radius > 0
};

#ifndef DARB_PBWD_THREADS
#define DARB_PBWD_THREADS 256
#endif
constexpr int kPbwdThreads = DARB_PBWD_THREADS;  // threads per workgroup (a tuning constant)

template <int DEG, bool CKPT>
__global__ __launch_bounds__(kPbwdThreads) void k_preprocess_bwd(Cam cam, KParams kp, int n, darb_splats in, Ckpt ck,
                                                        darb_grads2d g2, darb_grads3d g3, int accumulate) {
    constexpr int NB = (DEG + 1) * (DEG + 1);
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    Grad3 g = {};
    float gsh[NB][3];
#pragma unroll
    for (int b = 0; b < NB; b++) gsh[b][0] = gsh[b][1] = gsh[b][2] = 0.0f;
    // with the checkpoint the forward's radius tells the culled splats (zero
    // gradient), which then load nothing else
    bool kept = true;
    if constexpr (CKPT) kept = ck.radius[i] > 0;
    if (kept) {
        // parameters, incoming gradients and the colour checkpoint are loaded
        // together, one memory round trip before the projection
        float m[3];
        load_mean(in, n, i, m);
        const QS qs = load_qs(in, n, i);
        const G2v gin = load_g2(g2, i);
        float jac[9];
        uint8_t cl = 0;
        if constexpr (CKPT) {
#pragma unroll
            for (int k = 0; k < 9; k++) jac[k] = ck.dcolor[(size_t)k * n + i];
            cl = ck.clamped[i];
        }
        pin_geometry(m, qs);
        pin(gin.xy[0]); pin(gin.xy[1]); pin(gin.conic[0]); pin(gin.conic[1]); pin(gin.conic[2]); pin(gin.op);
        pin(gin.rgb[0]); pin(gin.rgb[1]); pin(gin.rgb[2]);
        if constexpr (CKPT) {
#pragma unroll
            for (int k = 0; k < 9; k++) pin(jac[k]);
            pin(__uint_as_float((uint32_t)cl));
        }
        // the forward's decisions (recomputed: the same expressions on the same
        // inputs); of the projection only the Jacobian clamp is kept, and the
        // FP64 geometry is rebuilt for the chain (fewer registers live across
        // the colour part)
        Clamp cj;
        bool vis;
        if constexpr (CKPT) {
            vis = true;  // the forward's radius kept it
            clamp_of(cam, m, cj);
        } else {
            vis = forward_visible(cam, kp, m, qs, cj);
        }
        if (vis) {
            float Y[NB], gv[3], dmu_sh[3];
            if constexpr (CKPT) {
                colour_bwd_ckpt<NB>(cam, m, cl, jac, gin.rgb, Y, gv, dmu_sh);
            } else {
                float csh[NB][3];
                load_sh<NB>(in.sh, n, i, csh);
                colour_bwd_sh<NB>(cam, m, csh, gin.rgb, Y, gv, dmu_sh);
            }
            Geom64 G64;
            splat_geom64(qs, G64);
            splat_bwd_view(cam, kp, m, gin, G64, cj, dmu_sh, g.dmu, g.dsc, g.dq);
            g.dop = gin.op;
#pragma unroll
            for (int b = 0; b < NB; b++)
#pragma unroll
                for (int ch = 0; ch < 3; ch++) gsh[b][ch] = Y[b] * gv[ch];
        }
    }
    store_grads<NB>(g3, n, i, g, gsh, accumulate != 0);
}

// Sum over views, in view order, of the single-view gradients (each view's
// contribution computed exactly as the single-view kernel computes it, then
// added), with the parameters read once and the result written once.
template <int DEG, bool CKPT>
__global__ __launch_bounds__(256) void k_preprocess_bwd_multi(Cams cams, KParams kp, int n, darb_splats in, G2s g2,
                                                              darb_grads3d g3) {
    constexpr int NB = (DEG + 1) * (DEG + 1);
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float m[3];
    load_mean(in, n, i, m);
    // the geometry is rebuilt per view from the loaded parameters instead of
    // kept across the loop: fewer registers live beside the colour accumulators
    const QS qs = load_qs(in, n, i);
    const bool geom = (qs.q[0] != 0.0f) | (qs.q[1] != 0.0f) | (qs.q[2] != 0.0f) | (qs.q[3] != 0.0f);
    Grad3 tot = {};
    float gsh[NB][3];
#pragma unroll
    for (int b = 0; b < NB; b++) gsh[b][0] = gsh[b][1] = gsh[b][2] = 0.0f;
    uint32_t vmask = 0;  // views where the splat is visible
    if (geom) {
        float csh[NB][3];
        if constexpr (!CKPT) load_sh<NB>(in.sh, n, i, csh);
        for (int v = 0; v < cams.nv; v++) {
            const Cam &cam = cams.c[v];
            Clamp cj;
            if (!forward_visible(cam, kp, m, qs, cj)) continue;
            vmask |= 1u << v;
            const G2v gin = load_g2(g2.g[v], i);
            float Y[NB], gv[3], dmu_sh[3];
            if constexpr (CKPT) {
                float jac[9];
#pragma unroll
                for (int k = 0; k < 9; k++) jac[k] = g2.dcolor[v][(size_t)k * n + i];
                colour_bwd_ckpt<NB>(cam, m, g2.clamped[v][i], jac, gin.rgb, Y, gv, dmu_sh);
            } else {
                colour_bwd_sh<NB>(cam, m, csh, gin.rgb, Y, gv, dmu_sh);
            }
            Geom64 G64;
            splat_geom64(qs, G64);
            Grad3 g;
            splat_bwd_view(cam, kp, m, gin, G64, cj, dmu_sh, g.dmu, g.dsc, g.dq);
            g.dop = gin.op;
#pragma unroll
            for (int c = 0; c < 3; c++) {
                tot.dmu[c] += g.dmu[c];
                tot.dsc[c] += g.dsc[c];
            }
#pragma unroll
            for (int c = 0; c < 4; c++) tot.dq[c] += g.dq[c];
            tot.dop += g.dop;
        }
        // SH coefficient gradients in a second pass over the visible views (same
        // terms and order as the single-view kernel; the 48 accumulators are not
        // live beside the FP64 chain)
        for (int v = 0; v < cams.nv; v++) {
            if (!((vmask >> v) & 1u)) continue;
            const darb_grads2d &gg = g2.g[v];
            const float grgb[3] = {gg.rgb[3 * i], gg.rgb[3 * i + 1], gg.rgb[3 * i + 2]};
            float Y[NB], gv[3];
            if constexpr (CKPT) {
                const Cam &cam = cams.c[v];
                float vx = m[0] - cam.campos[0], vy = m[1] - cam.campos[1], vz = m[2] - cam.campos[2];
                const float il = rsqrtf(fmaf(vx, vx, fmaf(vy, vy, vz * vz)));
                sh_eval<NB>(vx * il, vy * il, vz * il, Y);
                const uint8_t cl = g2.clamped[v][i];
#pragma unroll
                for (int ch = 0; ch < 3; ch++) gv[ch] = ((cl >> ch) & 1u) ? 0.0f : grgb[ch];
            } else {
                float d[3], il;
                sh_view<NB>(cams.c[v], m, csh, grgb, d, il, Y, gv);
            }
#pragma unroll
            for (int b = 0; b < NB; b++)
#pragma unroll
                for (int ch = 0; ch < 3; ch++) gsh[b][ch] += Y[b] * gv[ch];
        }
    }
    store_grads<NB>(g3, n, i, tot, gsh, false);
}

}  // namespace

#define DARB_DEG_SWITCH(deg, K, grid, s, ...)                                          \
    switch (deg) {                                                                    \
    case 0: hipLaunchKernelGGL(K<0>, grid, dim3(256), 0, s, __VA_ARGS__); break;      \
    case 1: hipLaunchKernelGGL(K<1>, grid, dim3(256), 0, s, __VA_ARGS__); break;      \
    case 2: hipLaunchKernelGGL(K<2>, grid, dim3(256), 0, s, __VA_ARGS__); break;      \
    default: hipLaunchKernelGGL(K<3>, grid, dim3(256), 0, s, __VA_ARGS__); break;     \
    }

hipError_t launch_preprocess(const Cam &cam, const darb_camera *cam_dev, const KParams &kp, int n,
                             const darb_splats &in, const darb_projected &out, hipStream_t s) {
    if (n == 0) return hipSuccess;
    dim3 grid((n + 255) / 256);
    DARB_DEG_SWITCH(in.sh_degree, k_preprocess, grid, s, cam, cam_dev, kp, n, in, out)
    return hipGetLastError();
}

hipError_t launch_preprocess_parts(const Cam &cam, const KParams &kp, int n, const darb_splats &in,
                                   const darb_projected &out, int parts, hipStream_t s) {
    if (n == 0) return hipSuccess;
    if (parts == 3) return launch_preprocess(cam, nullptr, kp, n, in, out, s);
    dim3 grid((n + 255) / 256);
    if (parts & 1) hipLaunchKernelGGL(k_preprocess_geom, grid, dim3(256), 0, s, cam, kp, n, in, out);
    if (parts & 2) {
        static int cus = 0;  // compute units of the device (queried once)
        if (cus == 0) {
            int dev = 0;
            if (hipGetDevice(&dev) != hipSuccess ||
                hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
                cus = 256;
        }
        const dim3 gc(std::min<unsigned>((unsigned)((n + kColourThreads - 1) / kColourThreads),
                                         (unsigned)(cus * kColourWgsPerCu)));
        const dim3 bc(kColourThreads);
        switch (in.sh_degree) {
        case 0: hipLaunchKernelGGL(k_preprocess_colour<0>, gc, bc, 0, s, cam, n, in, out); break;
        case 1: hipLaunchKernelGGL(k_preprocess_colour<1>, gc, bc, 0, s, cam, n, in, out); break;
        case 2: hipLaunchKernelGGL(k_preprocess_colour<2>, gc, bc, 0, s, cam, n, in, out); break;
        default: hipLaunchKernelGGL(k_preprocess_colour<3>, gc, bc, 0, s, cam, n, in, out); break;
        }
    }
    return hipGetLastError();
}

hipError_t launch_preprocess_multi(const Cams &cams, const KParams &kp, int n, const darb_splats &in,
                                   const Projs &outs, hipStream_t s) {
    if (n == 0) return hipSuccess;
    dim3 grid((n + 255) / 256);
    DARB_DEG_SWITCH(in.sh_degree, k_preprocess_multi, grid, s, cams, kp, n, in, outs)
    return hipGetLastError();
}

#define DARB_DEG_SWITCH_B(deg, K, B, grid, T, s, ...)                                       \
    switch (deg) {                                                                          \
    case 0: hipLaunchKernelGGL((K<0, B>), grid, dim3(T), 0, s, __VA_ARGS__); break;         \
    case 1: hipLaunchKernelGGL((K<1, B>), grid, dim3(T), 0, s, __VA_ARGS__); break;         \
    case 2: hipLaunchKernelGGL((K<2, B>), grid, dim3(T), 0, s, __VA_ARGS__); break;         \
    default: hipLaunchKernelGGL((K<3, B>), grid, dim3(T), 0, s, __VA_ARGS__); break;        \
    }

hipError_t launch_preprocess_bwd(const Cam &cam, const KParams &kp, int n, const darb_splats &in,
                                 const darb_projected *ckpt, const darb_grads2d &g2d, const darb_grads3d &g3d,
                                 bool accumulate, hipStream_t s) {
    if (n == 0) return hipSuccess;
    dim3 grid((n + kPbwdThreads - 1) / kPbwdThreads);
    const int acc = accumulate ? 1 : 0;
    const Ckpt ck{ckpt ? ckpt->dcolor : nullptr, ckpt ? ckpt->clamped : nullptr, ckpt ? ckpt->radius : nullptr};
    if (ck.dcolor && ck.clamped && ck.radius) {
        DARB_DEG_SWITCH_B(in.sh_degree, k_preprocess_bwd, true, grid, kPbwdThreads, s, cam, kp, n, in, ck, g2d, g3d,
                          acc)
    } else {
        DARB_DEG_SWITCH_B(in.sh_degree, k_preprocess_bwd, false, grid, kPbwdThreads, s, cam, kp, n, in, ck, g2d, g3d,
                          acc)
    }
    return hipGetLastError();
}

hipError_t launch_preprocess_bwd_multi(const Cams &cams, const KParams &kp, int n, const darb_splats &in,
                                       const G2s &g2, const darb_grads3d &g3d, hipStream_t s) {
    if (n == 0) return hipSuccess;
    dim3 grid((n + 255) / 256);
    bool ckpt = true;
    for (int v = 0; v < cams.nv; v++) ckpt = ckpt && g2.dcolor[v] && g2.clamped[v];
    if (ckpt) {
        DARB_DEG_SWITCH_B(in.sh_degree, k_preprocess_bwd_multi, true, grid, 256, s, cams, kp, n, in, g2, g3d)
    } else {
        DARB_DEG_SWITCH_B(in.sh_degree, k_preprocess_bwd_multi, false, grid, 256, s, cams, kp, n, in, g2, g3d)
    }
    return hipGetLastError();
}

}  // namespace darb
