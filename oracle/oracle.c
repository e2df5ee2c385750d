/*
 * oracle.c -- plain, slow FP64 reference for the DARB-Splatting rasterizer.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link, load or
 * call this file: only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code, header, table or constant
 * with the HIP implementation; both sides only consume the same seeded inputs.
 *
 * Every floating-point step is carried out in double precision from the FP32
 * inputs the GPU also receives (converted exactly).  The one exception is the
 * binning reference (orc_bin), which is integer / FP32 work by definition.
 *
 * Paper: "DARB-Splatting: Generalizing Splatting with Decaying Anisotropic
 * Radial Basis Functions" (arXiv 2501.12369).  Citations name the section,
 * equation or table each step follows.
 *
 * Conventions (readings of the paper where it is silent are listed in the
 * design notes and repeated at the point of use):
 *   camera frame: x right, y down, z forward; t = R_cw * mu + t_cw
 *   pixel (i, j) is evaluated at image coordinates (i, j)
 *   d = mu' - p  (projected mean minus pixel), E = d^T Q d, Q = inverse 2D cov
 *   conic stored as (a, b, c) with Q = [[a, b], [b, c]]
 *   SH coefficients, layout [(deg+1)^2][3][n]
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_GAUSS 0
#define ORC_HALF_COS 1
#define ORC_RAISED_COS 2
#define ORC_SINC 3
#define ORC_IMQ 4      /* 1 / (E/xi + 1)        (supplementary IMQ section)   */
#define ORC_IMQ_SQRT 5 /* 1 / sqrt(E/xi + 1)    (Table 1, inverse multiquadric) */
#define ORC_PARABOLA 6
/* Table 1's "modified" forms with a generic roll-off beta, u = d_M^beta / xi = E^(beta/2) / xi */
#define ORC_GAUSS_BETA 7      /* exp(-u)                                                */
#define ORC_HALF_COS_BETA 8   /* cos(u),            main lobe u <= pi/2                 */
#define ORC_RAISED_COS_BETA 9 /* 0.5 + 0.5 cos(u),  n pulses: u <= n pi                 */
#define ORC_SINC_BETA 10      /* |sin(u)| / u,      n pulses: u <= (n + 1) pi / 2       */

typedef struct {
    double viewmat[16]; /* world -> camera, row-major 4x4 */
    double campos[3];   /* camera centre, world coordinates */
    double fx, fy, cx, cy;
    int32_t width, height;
    double near_z;    /* splats with t_z <= near_z are culled */
    double jac_clamp; /* limit of |t_x/t_z| as a multiple of the half field of view; <= 0 disables */
    double dilation;  /* epsilon added to the diagonal of the 2D covariance */
} orc_camera;

typedef struct {
    int32_t kind;
    double xi;    /* scaling factor xi of Table 1 / Table 2 */
    double psi;   /* correction factor psi of Eq. (2x2 covariance projection) */
    double e_max; /* support limit on E = d_M^2 (boundaries of DARBFs) */
    double beta;  /* roll-off of the modified forms (kinds 7..10); unused otherwise */
} orc_kernel;

typedef struct {
    double alpha_min, alpha_max, t_min;
    double bg[3];
} orc_opts;

/* ------------------------------------------------------------------------ */
/* Kernel profiles F(E) with E = d_M^2, and dF/dE.                          */
/* Table 1 (tab:functions) gives the generic forms; the supplementary       */
/* sections per kernel fix beta and the support; Table 2 gives xi.          */
/* ------------------------------------------------------------------------ */

/* sin(u)/u with its limit 1 at u = 0 */
static double sinc_u(double u) {
    if (fabs(u) < 1e-4) return 1.0 - u * u / 6.0 + u * u * u * u / 120.0;
    return sin(u) / u;
}

double orc_kernel_value(int32_t kind, double xi, double E) {
    switch (kind) {
    case ORC_GAUSS: /* modified Gaussian, beta = 2: exp(-d_M^2 / xi) */
        return exp(-E / xi);
    case ORC_HALF_COS: /* half-cosine squared: cos(d_M^2 / xi) */
        return cos(E / xi);
    case ORC_RAISED_COS: { /* raised cosine, beta = 1: 0.5 + 0.5 cos(d_M / xi) */
        double u = sqrt(E) / xi;
        return 0.5 + 0.5 * cos(u);
    }
    case ORC_SINC: { /* modular sinc, beta = 1: |sin(u)| / u, u = d_M / xi; value 1 at u = 0 */
        double u = sqrt(E) / xi;
        return fabs(sinc_u(u));
    }
    case ORC_IMQ: /* inverse quadric of the supplementary section */
        return 1.0 / (E / xi + 1.0);
    case ORC_IMQ_SQRT: /* inverse multiquadric of Table 1 */
        return 1.0 / sqrt(E / xi + 1.0);
    case ORC_PARABOLA: /* 1 - d_M^2 / xi */
        return 1.0 - E / xi;
    default:
        return NAN;
    }
}

double orc_kernel_deriv(int32_t kind, double xi, double E) {
    switch (kind) {
    case ORC_GAUSS:
        return -exp(-E / xi) / xi;
    case ORC_HALF_COS:
        return -sin(E / xi) / xi;
    case ORC_RAISED_COS: {
        /* d/dE [0.5 cos(sqrt(E)/xi)] = -0.5 sin(u) / (2 xi sqrt(E)) = -sinc(u) / (4 xi^2) */
        double u = sqrt(E) / xi;
        return -sinc_u(u) / (4.0 * xi * xi);
    }
    case ORC_SINC: {
        /* F = |sin u| / u; dF/du = sgn(sin u) (u cos u - sin u) / u^2; du/dE = 1 / (2 xi^2 u) */
        double u = sqrt(E) / xi;
        double g; /* (u cos u - sin u) / u^3 */
        if (u < 1e-3)
            g = -1.0 / 3.0 + u * u / 30.0;
        else
            g = (u * cos(u) - sin(u)) / (u * u * u);
        double sgn = (u < 1e-3 || sin(u) >= 0.0) ? 1.0 : -1.0;
        return sgn * g / (2.0 * xi * xi);
    }
    case ORC_IMQ: {
        double q = E / xi + 1.0;
        return -1.0 / (xi * q * q);
    }
    case ORC_IMQ_SQRT: {
        double q = E / xi + 1.0;
        return -0.5 / (xi * q * sqrt(q));
    }
    case ORC_PARABOLA:
        return -1.0 / xi;
    default:
        return NAN;
    }
}

/* Modified forms of Table 1 with a generic roll-off beta: with d_M = sqrt(E),
 * u = d_M^beta / xi.  dF/dE = dF/du * du/dE, du/dE = (beta/2) u / E for E > 0.
 * At E = 0 the limit of du/dE is 1/xi for beta = 2 and 0 for beta > 2; for
 * beta < 2 it diverges while every gradient it feeds (dE/d mu' = 2 Q d,
 * dE/dQ = d d^T) vanishes at least as fast, so the derivative is taken as 0
 * there. */
static double modified_u(double xi, double beta, double E) { return pow(E, 0.5 * beta) / xi; }

double orc_kernel_value_beta(int32_t kind, double xi, double beta, double E) {
    if (kind < ORC_GAUSS_BETA) return orc_kernel_value(kind, xi, E);
    double u = modified_u(xi, beta, E);
    switch (kind) {
    case ORC_GAUSS_BETA:
        return exp(-u);
    case ORC_HALF_COS_BETA:
        return cos(u);
    case ORC_RAISED_COS_BETA:
        return 0.5 + 0.5 * cos(u);
    case ORC_SINC_BETA:
        return fabs(sinc_u(u));
    default:
        return NAN;
    }
}

double orc_kernel_deriv_beta(int32_t kind, double xi, double beta, double E) {
    if (kind < ORC_GAUSS_BETA) return orc_kernel_deriv(kind, xi, E);
    double u = modified_u(xi, beta, E);
    double du = E > 0.0 ? 0.5 * beta * u / E : (beta == 2.0 ? 1.0 / xi : 0.0);
    double dF; /* dF/du */
    switch (kind) {
    case ORC_GAUSS_BETA:
        dF = -exp(-u);
        break;
    case ORC_HALF_COS_BETA:
        dF = -sin(u);
        break;
    case ORC_RAISED_COS_BETA:
        dF = -0.5 * sin(u);
        break;
    case ORC_SINC_BETA: {
        /* F = |sin u| / u: dF/du = sgn(sin u) (u cos u - sin u) / u^2 */
        double g = u < 1e-3 ? -u / 3.0 + u * u * u / 30.0 : (u * cos(u) - sin(u)) / (u * u);
        dF = (u < 1e-3 || sin(u) >= 0.0) ? g : -g;
        break;
    }
    default:
        return NAN;
    }
    return dF * du;
}

/* F and dF/dE at n values of E (vectorised for the correction-factor and 1D experiments) */
void orc_kernel_values(int32_t kind, double xi, double beta, long n, const double *E, double *out) {
#pragma omp parallel for schedule(static)
    for (long i = 0; i < n; i++) out[i] = orc_kernel_value_beta(kind, xi, beta, E[i]);
}

void orc_kernel_derivs(int32_t kind, double xi, double beta, long n, const double *E, double *out) {
#pragma omp parallel for schedule(static)
    for (long i = 0; i < n; i++) out[i] = orc_kernel_deriv_beta(kind, xi, beta, E[i]);
}

/* ------------------------------------------------------------------------ */
/* Real spherical harmonics up to degree 3 (the 3DGS parameterisation that  */
/* the paper keeps, DARB Representation).  Y_{l,m} for m>0 is sqrt(2) Re and */
/* for m<0 sqrt(2) Im of the complex harmonic Y_l^{|m|} with the             */
/* Condon-Shortley phase; index k = l^2 + l + m.                             */
/* ------------------------------------------------------------------------ */

static void sh_basis(const double d[3], double Y[16], double dY[16][3]) {
    const double PI = 3.14159265358979323846;
    double x = d[0], y = d[1], z = d[2];
    double c0 = 0.5 * sqrt(1.0 / PI);
    double c1 = sqrt(3.0 / (4.0 * PI));
    double c2a = 0.5 * sqrt(15.0 / PI);
    double c2b = 0.25 * sqrt(5.0 / PI);
    double c2c = 0.25 * sqrt(15.0 / PI);
    double c3a = 0.25 * sqrt(35.0 / (2.0 * PI));
    double c3b = 0.5 * sqrt(105.0 / PI);
    double c3c = 0.25 * sqrt(21.0 / (2.0 * PI));
    double c3d = 0.25 * sqrt(7.0 / PI);
    double c3e = 0.25 * sqrt(105.0 / PI);
    memset(dY, 0, sizeof(double) * 16 * 3);

    Y[0] = c0;

    Y[1] = -c1 * y;  dY[1][1] = -c1;
    Y[2] = c1 * z;   dY[2][2] = c1;
    Y[3] = -c1 * x;  dY[3][0] = -c1;

    Y[4] = c2a * x * y;
    dY[4][0] = c2a * y; dY[4][1] = c2a * x;
    Y[5] = -c2a * y * z;
    dY[5][1] = -c2a * z; dY[5][2] = -c2a * y;
    Y[6] = c2b * (2.0 * z * z - x * x - y * y);
    dY[6][0] = -2.0 * c2b * x; dY[6][1] = -2.0 * c2b * y; dY[6][2] = 4.0 * c2b * z;
    Y[7] = -c2a * x * z;
    dY[7][0] = -c2a * z; dY[7][2] = -c2a * x;
    Y[8] = c2c * (x * x - y * y);
    dY[8][0] = 2.0 * c2c * x; dY[8][1] = -2.0 * c2c * y;

    Y[9] = -c3a * y * (3.0 * x * x - y * y);
    dY[9][0] = -c3a * 6.0 * x * y; dY[9][1] = -c3a * (3.0 * x * x - 3.0 * y * y);
    Y[10] = c3b * x * y * z;
    dY[10][0] = c3b * y * z; dY[10][1] = c3b * x * z; dY[10][2] = c3b * x * y;
    Y[11] = -c3c * y * (4.0 * z * z - x * x - y * y);
    dY[11][0] = -c3c * (-2.0 * x * y);
    dY[11][1] = -c3c * (4.0 * z * z - x * x - 3.0 * y * y);
    dY[11][2] = -c3c * (8.0 * y * z);
    Y[12] = c3d * z * (2.0 * z * z - 3.0 * x * x - 3.0 * y * y);
    dY[12][0] = c3d * (-6.0 * x * z);
    dY[12][1] = c3d * (-6.0 * y * z);
    dY[12][2] = c3d * (6.0 * z * z - 3.0 * x * x - 3.0 * y * y);
    Y[13] = -c3c * x * (4.0 * z * z - x * x - y * y);
    dY[13][0] = -c3c * (4.0 * z * z - 3.0 * x * x - y * y);
    dY[13][1] = -c3c * (-2.0 * x * y);
    dY[13][2] = -c3c * (8.0 * x * z);
    Y[14] = c3e * z * (x * x - y * y);
    dY[14][0] = c3e * 2.0 * x * z; dY[14][1] = -c3e * 2.0 * y * z; dY[14][2] = c3e * (x * x - y * y);
    Y[15] = -c3a * x * (x * x - 3.0 * y * y);
    dY[15][0] = -c3a * (3.0 * x * x - 3.0 * y * y); dY[15][1] = -c3a * (-6.0 * x * y);
}

/* exported for the basis pins in the tests: Y[16] and dY[16*3] at direction d */
void orc_sh_basis(const double *d, double *Y, double *dY) {
    double dd[16][3];
    sh_basis(d, Y, dd);
    memcpy(dY, dd, sizeof(dd));
}

/* ------------------------------------------------------------------------ */
/* Small dense-matrix helpers (row-major).                                   */
/* ------------------------------------------------------------------------ */

/* rotation matrix of a unit quaternion (w, x, y, z) */
static void quat_to_rot(const double q[4], double R[9]) {
    double w = q[0], x = q[1], y = q[2], z = q[3];
    R[0] = 1.0 - 2.0 * (y * y + z * z);
    R[1] = 2.0 * (x * y - w * z);
    R[2] = 2.0 * (x * z + w * y);
    R[3] = 2.0 * (x * y + w * z);
    R[4] = 1.0 - 2.0 * (x * x + z * z);
    R[5] = 2.0 * (y * z - w * x);
    R[6] = 2.0 * (x * z - w * y);
    R[7] = 2.0 * (y * z + w * x);
    R[8] = 1.0 - 2.0 * (x * x + y * y);
}

void orc_quat_to_rot(const double *q, double *R) {
    double n = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    double qn[4] = {q[0] / n, q[1] / n, q[2] / n, q[3] / n};
    quat_to_rot(qn, R);
}

/* C (r x c) = A (r x k) * B (k x c) */
static void matmul(const double *A, const double *B, double *C, int r, int k, int c) {
    for (int i = 0; i < r; i++)
        for (int j = 0; j < c; j++) {
            double s = 0.0;
            for (int l = 0; l < k; l++) s += A[i * k + l] * B[l * c + j];
            C[i * c + j] = s;
        }
}

static void transpose(const double *A, double *At, int r, int c) {
    for (int i = 0; i < r; i++)
        for (int j = 0; j < c; j++) At[j * r + i] = A[i * c + j];
}

/* ------------------------------------------------------------------------ */
/* Forward projection of one splat (DARB Projection, Eq. 2x2 covariance     */
/* projection; bounding radius of the DARBF boundaries section).            */
/* ------------------------------------------------------------------------ */

#define ORC_MAX_BOX_PX 1073741824.0 /* 2^30: the largest radius or tile-box half-extent */

typedef struct {
    int visible;
    double t[3];   /* camera-space mean */
    double W[9];   /* R_cw */
    double J[6];   /* affine Jacobian, 2x3 */
    int clamp_x, clamp_y;
    double xt, yt; /* (clamped) t_x / t_z and t_y / t_z */
    double A[6];   /* J W */
    double Rq[9];  /* rotation of the splat */
    double qn[4];
    double qnorm;
    double Sigma[9]; /* 3D covariance */
    double cov[4];   /* psi * A Sigma A^T + eps I */
    double det;
    double conic[3];
    double xy[2];
    double depth;
    int radius;
    int ext[2];    /* half-extents of the tile box: ceil(rf sqrt(cov_xx)), ceil(rf sqrt(cov_yy)) */
    double dir[3], vlen;
    double rgb[3];
    int clamped[3];
} orc_splat_state;

static void project_one(const orc_camera *cam, const orc_kernel *k, long n, long i,
                        const double *means, const double *scales, const double *quats,
                        const double *sh, int deg, orc_splat_state *s) {
    memset(s, 0, sizeof(*s));
    double mu[3] = {means[i], means[n + i], means[2 * n + i]};
    for (int r = 0; r < 3; r++)
        for (int c = 0; c < 3; c++) s->W[r * 3 + c] = cam->viewmat[r * 4 + c];
    for (int r = 0; r < 3; r++)
        s->t[r] = s->W[r * 3 + 0] * mu[0] + s->W[r * 3 + 1] * mu[1] + s->W[r * 3 + 2] * mu[2] +
                  cam->viewmat[r * 4 + 3];
    if (!(s->t[2] > cam->near_z)) return; /* near-plane cull */

    double q[4] = {quats[i], quats[n + i], quats[2 * n + i], quats[3 * n + i]};
    s->qnorm = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    if (!(s->qnorm > 0.0)) return;
    for (int c = 0; c < 4; c++) s->qn[c] = q[c] / s->qnorm;
    quat_to_rot(s->qn, s->Rq);

    /* Sigma = R diag(s^2) R^T  (scale + rotation parameterisation) */
    double sc[3] = {scales[i], scales[n + i], scales[2 * n + i]};
    for (int r = 0; r < 3; r++)
        for (int c = 0; c < 3; c++) {
            double v = 0.0;
            for (int l = 0; l < 3; l++) v += s->Rq[r * 3 + l] * sc[l] * sc[l] * s->Rq[c * 3 + l];
            s->Sigma[r * 3 + c] = v;
        }

    /* affine Jacobian of the perspective projection at t */
    double tz = s->t[2];
    s->xt = s->t[0] / tz;
    s->yt = s->t[1] / tz;
    if (cam->jac_clamp > 0.0) {
        double lx = cam->jac_clamp * (0.5 * cam->width) / cam->fx;
        double ly = cam->jac_clamp * (0.5 * cam->height) / cam->fy;
        if (s->xt > lx) { s->xt = lx; s->clamp_x = 1; }
        if (s->xt < -lx) { s->xt = -lx; s->clamp_x = 1; }
        if (s->yt > ly) { s->yt = ly; s->clamp_y = 1; }
        if (s->yt < -ly) { s->yt = -ly; s->clamp_y = 1; }
    }
    s->J[0] = cam->fx / tz; s->J[1] = 0.0; s->J[2] = -cam->fx * s->xt / tz;
    s->J[3] = 0.0; s->J[4] = cam->fy / tz; s->J[5] = -cam->fy * s->yt / tz;

    /* Sigma'_{2x2} = psi * [J W Sigma W^T J^T]_{2x2} + eps I */
    matmul(s->J, s->W, s->A, 2, 3, 3);
    double AS[6], At[6], M[4];
    matmul(s->A, s->Sigma, AS, 2, 3, 3);
    transpose(s->A, At, 2, 3);
    matmul(AS, At, M, 2, 3, 2);
    s->cov[0] = k->psi * M[0] + cam->dilation;
    s->cov[1] = k->psi * M[1];
    s->cov[2] = k->psi * M[2];
    s->cov[3] = k->psi * M[3] + cam->dilation;
    s->det = s->cov[0] * s->cov[3] - s->cov[1] * s->cov[1];
    if (!(s->det > 0.0)) return;
    s->conic[0] = s->cov[3] / s->det;
    s->conic[1] = -s->cov[1] / s->det;
    s->conic[2] = s->cov[0] / s->det;

    s->xy[0] = cam->fx * s->t[0] / tz + cam->cx;
    s->xy[1] = cam->fy * s->t[1] / tz + cam->cy;
    s->depth = tz;

    /* R = ceil(3 sqrt(lambda_max)) of the 2D covariance; a support beyond
     * E = 9 (several pulses) widens it to ceil(sqrt(e_max lambda_max)) */
    double mid = 0.5 * (s->cov[0] + s->cov[3]);
    double disc = mid * mid - s->det;
    double lam = mid + sqrt(disc > 0.0 ? disc : 0.0);
    double rf = k->e_max > 9.0 ? sqrt(k->e_max) : 3.0;
    /* sizes capped at 2^30 px (beyond any image): the int conversion stays defined */
    s->radius = (int)ceil(fmin(rf * sqrt(lam), ORC_MAX_BOX_PX));

    /* Tile box: the bounding box of the ellipse {d : d^T Sigma'^-1 d <= rf^2},
     * whose half-extents are rf sqrt(Sigma'_xx) and rf sqrt(Sigma'_yy) (the
     * largest |d_x| on that ellipse), rounded up to whole pixels.  It holds the
     * support E <= e_max and lies inside the paper's square of half-side R;
     * the image does not depend on the box (every pixel tests E itself). */
    s->ext[0] = (int)ceil(fmin(rf * sqrt(s->cov[0]), ORC_MAX_BOX_PX));
    s->ext[1] = (int)ceil(fmin(rf * sqrt(s->cov[3]), ORC_MAX_BOX_PX));

    /* tile rectangle of that box on the 16x16 grid; empty => not visible */
    int gx = (cam->width + 15) / 16, gy = (cam->height + 15) / 16;
    double x0 = floor((s->xy[0] - s->ext[0]) / 16.0), x1 = floor((s->xy[0] + s->ext[0]) / 16.0) + 1.0;
    double y0 = floor((s->xy[1] - s->ext[1]) / 16.0), y1 = floor((s->xy[1] + s->ext[1]) / 16.0) + 1.0;
    x0 = x0 < 0 ? 0 : (x0 > gx ? gx : x0);
    x1 = x1 < 0 ? 0 : (x1 > gx ? gx : x1);
    y0 = y0 < 0 ? 0 : (y0 > gy ? gy : y0);
    y1 = y1 < 0 ? 0 : (y1 > gy ? gy : y1);
    if ((x1 - x0) * (y1 - y0) <= 0.0) return;

    /* view-dependent colour from SH, +0.5 offset, clamped at 0 */
    double v[3] = {mu[0] - cam->campos[0], mu[1] - cam->campos[1], mu[2] - cam->campos[2]};
    s->vlen = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    for (int c = 0; c < 3; c++) s->dir[c] = s->vlen > 0.0 ? v[c] / s->vlen : 0.0;
    double Y[16], dY[16][3];
    sh_basis(s->dir, Y, dY);
    int nb = (deg + 1) * (deg + 1);
    for (int ch = 0; ch < 3; ch++) {
        double acc = 0.0;
        for (int b = 0; b < nb; b++) acc += Y[b] * sh[((long)b * 3 + ch) * n + i];
        acc += 0.5;
        s->clamped[ch] = acc < 0.0;
        s->rgb[ch] = acc < 0.0 ? 0.0 : acc;
    }
    s->visible = 1;
}

/*
 * orc_preprocess: per-splat projection.  Inputs SoA ([3][n], [4][n], [n],
 * [(deg+1)^2][3][n]).  Outputs: xy[n][2], depth[n], radius[n] (0 = culled),
 * extent[n][2] (half-extents of the tile box in pixels, 0 = culled),
 * conic[n][3], rgb[n][3], clamped[n] (bit c set when channel c is clamped),
 * visible[n], cov2d[n][3] (nullable; a, b, c of Sigma'_{2x2}).
 */
void orc_preprocess(const orc_camera *cam, const orc_kernel *k, long n, const double *means,
                    const double *scales, const double *quats, const double *sh, int deg,
                    double *xy, double *depth, int32_t *radius, int32_t *extent, double *conic, double *rgb,
                    uint8_t *clamped, int32_t *visible, double *cov2d) {
#pragma omp parallel for schedule(static)
    for (long i = 0; i < n; i++) {
        orc_splat_state s;
        project_one(cam, k, n, i, means, scales, quats, sh, deg, &s);
        visible[i] = s.visible;
        xy[2 * i] = s.visible ? s.xy[0] : 0.0;
        xy[2 * i + 1] = s.visible ? s.xy[1] : 0.0;
        depth[i] = s.visible ? s.depth : 0.0;
        radius[i] = s.visible ? s.radius : 0;
        extent[2 * i] = s.visible ? s.ext[0] : 0;
        extent[2 * i + 1] = s.visible ? s.ext[1] : 0;
        for (int c = 0; c < 3; c++) {
            conic[3 * i + c] = s.visible ? s.conic[c] : 0.0;
            rgb[3 * i + c] = s.visible ? s.rgb[c] : 0.0;
        }
        clamped[i] = s.visible ? (uint8_t)(s.clamped[0] | (s.clamped[1] << 1) | (s.clamped[2] << 2)) : 0;
        if (cov2d) {
            cov2d[3 * i] = s.cov[0];
            cov2d[3 * i + 1] = s.cov[1];
            cov2d[3 * i + 2] = s.cov[3];
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Per-pixel composite: the plain definition (front-to-back alpha blending  */
/* of the DARB footprint; Eq. half-cosine splat and the listings' alpha).   */
/* Every valid splat with 0 <= E <= e_max at the pixel is a candidate; the  */
/* candidates are blended in (depth, index) order.                          */
/* ------------------------------------------------------------------------ */

typedef struct {
    double depth;
    long id;
    double E;
} cand_t;

static int cand_cmp(const void *a, const void *b) {
    const cand_t *x = (const cand_t *)a, *y = (const cand_t *)b;
    if (x->depth < y->depth) return -1;
    if (x->depth > y->depth) return 1;
    return (x->id < y->id) ? -1 : (x->id > y->id);
}

/* conservative radius of the support {d : d^T Q d <= e_max}: sqrt(e_max / lambda_min(Q)) */
static double support_radius(const double *cq, double e_max) {
    double a = cq[0], b = cq[1], c = cq[2];
    double m = 0.5 * (a + c), det = a * c - b * b;
    double disc = m * m - det;
    double lmin = m - sqrt(disc > 0.0 ? disc : 0.0);
    if (!(lmin > 0.0) || !(det > 0.0)) return INFINITY;
    return sqrt(e_max / lmin) * (1.0 + 1e-9) + 1e-9;
}

/* Candidate prefilter: a grid of 16-pixel cells, each listing every valid
 * splat whose support bounding box overlaps it.  The prefilter only narrows
 * the loop; the exact support test below decides membership, so the result is
 * identical to scanning every splat (checked against the brute-force path). */
typedef struct {
    int gx, gy;
    long *start; /* gx*gy+1 */
    long *ids;
} cell_grid;

static void grid_build(cell_grid *g, long n, const double *xy, const double *conic, const int32_t *valid,
                       double e_max, int width, int height) {
    g->gx = (width + 15) / 16;
    g->gy = (height + 15) / 16;
    long ncell = (long)g->gx * g->gy;
    long *cnt = (long *)calloc(ncell + 1, sizeof(long));
    int *rect = (int *)malloc(sizeof(int) * 4 * (n > 0 ? n : 1));
    for (long j = 0; j < n; j++) {
        rect[4 * j] = rect[4 * j + 1] = rect[4 * j + 2] = rect[4 * j + 3] = 0;
        if (!valid[j]) continue;
        double r = support_radius(conic + 3 * j, e_max);
        double x0, x1, y0, y1;
        if (isinf(r)) {
            x0 = 0; y0 = 0; x1 = g->gx; y1 = g->gy;
        } else {
            x0 = floor((xy[2 * j] - r) / 16.0); x1 = floor((xy[2 * j] + r) / 16.0) + 1.0;
            y0 = floor((xy[2 * j + 1] - r) / 16.0); y1 = floor((xy[2 * j + 1] + r) / 16.0) + 1.0;
        }
        x0 = x0 < 0 ? 0 : (x0 > g->gx ? g->gx : x0);
        x1 = x1 < 0 ? 0 : (x1 > g->gx ? g->gx : x1);
        y0 = y0 < 0 ? 0 : (y0 > g->gy ? g->gy : y0);
        y1 = y1 < 0 ? 0 : (y1 > g->gy ? g->gy : y1);
        rect[4 * j] = (int)x0; rect[4 * j + 1] = (int)x1; rect[4 * j + 2] = (int)y0; rect[4 * j + 3] = (int)y1;
        for (int cy = (int)y0; cy < (int)y1; cy++)
            for (int cx = (int)x0; cx < (int)x1; cx++) cnt[(long)cy * g->gx + cx + 1]++;
    }
    for (long c = 0; c < ncell; c++) cnt[c + 1] += cnt[c];
    g->start = cnt;
    g->ids = (long *)malloc(sizeof(long) * (cnt[ncell] > 0 ? cnt[ncell] : 1));
    long *fill = (long *)malloc(sizeof(long) * (ncell > 0 ? ncell : 1));
    for (long c = 0; c < ncell; c++) fill[c] = cnt[c];
    for (long j = 0; j < n; j++) {
        if (!valid[j]) continue;
        for (int cy = rect[4 * j + 2]; cy < rect[4 * j + 3]; cy++)
            for (int cx = rect[4 * j]; cx < rect[4 * j + 1]; cx++) g->ids[fill[(long)cy * g->gx + cx]++] = j;
    }
    free(fill);
    free(rect);
}

static void grid_free(cell_grid *g) {
    free(g->start);
    free(g->ids);
}

typedef struct {
    long n;
    const double *xy, *conic, *opac, *rgb, *depth;
    const int32_t *valid;
    const orc_kernel *k;
    const orc_opts *o;
    const cell_grid *grid; /* NULL => scan every splat */
} comp_ctx;

/* candidates of pixel (px, py), sorted by (depth, id); returns count, *out malloc'ed */
static long gather(const comp_ctx *c, int px, int py, cand_t **out) {
    long cap = 64, m = 0;
    cand_t *v = (cand_t *)malloc(sizeof(cand_t) * cap);
    long lo = 0, hi = c->n;
    const long *ids = NULL;
    if (c->grid) {
        int cx = px / 16, cy = py / 16;
        long cell = (long)cy * c->grid->gx + cx;
        lo = c->grid->start[cell];
        hi = c->grid->start[cell + 1];
        ids = c->grid->ids;
    }
    for (long t = lo; t < hi; t++) {
        long j = ids ? ids[t] : t;
        if (!c->valid[j]) continue;
        double dx = c->xy[2 * j] - px, dy = c->xy[2 * j + 1] - py;
        const double *q = c->conic + 3 * j;
        double E = q[0] * dx * dx + 2.0 * q[1] * dx * dy + q[2] * dy * dy;
        if (E < 0.0 || E > c->k->e_max) continue;
        if (m == cap) {
            cap *= 2;
            v = (cand_t *)realloc(v, sizeof(cand_t) * cap);
        }
        v[m].depth = c->depth[j];
        v[m].id = j;
        v[m].E = E;
        m++;
    }
    qsort(v, m, sizeof(cand_t), cand_cmp);
    *out = v;
    return m;
}

static double rel_margin(double v, double thr) { return fabs(v - thr) / fabs(thr); }

/* composite one pixel; fills colour, T, last id, count, smallest decision margin.
 * If rec != NULL, records each contributor: id, E, w, alpha, T before it. */
typedef struct {
    long id;
    double E, w, alpha, T;
} contrib_t;

static long composite_pixel(const comp_ctx *c, int px, int py, double out[3], double *T_out, long *last,
                            int *ncontrib, double *margin, contrib_t **rec) {
    cand_t *v;
    long m = gather(c, px, py, &v);
    const orc_kernel *k = c->k;
    const orc_opts *o = c->o;
    double T = 1.0, C[3] = {0, 0, 0}, mg = INFINITY;
    long lastid = -1, nrec = 0;
    int cnt = 0;
    contrib_t *r = rec ? (contrib_t *)malloc(sizeof(contrib_t) * (m > 0 ? m : 1)) : NULL;
    for (long t = 0; t < m; t++) {
        long j = v[t].id;
        double E = v[t].E;
        double w = orc_kernel_value_beta(k->kind, k->xi, k->beta, E);
        double a = c->opac[j] * w;
        if (a > o->alpha_max) a = o->alpha_max;
        /* decision margins: support cut (only if it changes the outcome), alpha cut */
        if (a >= o->alpha_min * (1.0 - 1e-3)) {
            double me = rel_margin(E, k->e_max);
            if (me < mg) mg = me;
        }
        double ma = rel_margin(a, o->alpha_min);
        if (ma < mg) mg = ma;
        if (a < o->alpha_min) continue;
        double Tn = T * (1.0 - a);
        double mt = rel_margin(Tn, o->t_min);
        if (mt < mg) mg = mt;
        if (Tn < o->t_min) break;
        for (int ch = 0; ch < 3; ch++) C[ch] += a * T * c->rgb[3 * j + ch];
        if (r) {
            r[nrec].id = j; r[nrec].E = E; r[nrec].w = w; r[nrec].alpha = a; r[nrec].T = T;
            nrec++;
        }
        T = Tn;
        lastid = j;
        cnt++;
    }
    /* splats just outside the support whose inclusion would matter */
    free(v);
    for (int ch = 0; ch < 3; ch++) out[ch] = C[ch] + T * o->bg[ch];
    *T_out = T;
    *last = lastid;
    *ncontrib = cnt;
    *margin = mg;
    if (rec) *rec = r;
    return nrec;
}

/* Margin contribution of splats whose E lies just above e_max (outside the
 * candidate set): their inclusion under a slightly different rounding could
 * change the pixel.  Scans the same candidate source with a widened cut. */
static double outside_margin(const comp_ctx *c, int px, int py) {
    double mg = INFINITY;
    long lo = 0, hi = c->n;
    const long *ids = NULL;
    if (c->grid) {
        long cell = (long)(py / 16) * c->grid->gx + px / 16;
        lo = c->grid->start[cell];
        hi = c->grid->start[cell + 1];
        ids = c->grid->ids;
    }
    for (long t = lo; t < hi; t++) {
        long j = ids ? ids[t] : t;
        if (!c->valid[j]) continue;
        double dx = c->xy[2 * j] - px, dy = c->xy[2 * j + 1] - py;
        const double *q = c->conic + 3 * j;
        double E = q[0] * dx * dx + 2.0 * q[1] * dx * dy + q[2] * dy * dy;
        if (!(E > c->k->e_max)) continue;
        double me = rel_margin(E, c->k->e_max);
        if (me > 1e-2) continue;
        double w = orc_kernel_value_beta(c->k->kind, c->k->xi, c->k->beta, c->k->e_max);
        double a = c->opac[j] * w;
        if (a >= c->o->alpha_min * (1.0 - 1e-3) && me < mg) mg = me;
    }
    return mg;
}

/*
 * orc_composite: render the listed pixels (pix[p] = (x, y)).
 * xy[n][2], conic[n][3], opac[n], rgb[n][3], depth[n], valid[n].
 * Outputs per pixel: out_rgb[npix][3], out_T[npix], out_last[npix] (splat id
 * of the last contributor, -1 if none), out_ncontrib[npix], out_margin[npix]
 * (smallest relative distance of any deciding quantity to its threshold).
 * use_grid = 0 scans every splat per pixel; 1 uses the cell prefilter.
 */
void orc_composite(long n, const double *xy, const double *conic, const double *opac, const double *rgb,
                   const double *depth, const int32_t *valid, const orc_kernel *k, const orc_opts *o, int width,
                   int height, long npix, const int32_t *pix, int use_grid, double *out_rgb, double *out_T,
                   int64_t *out_last, int32_t *out_ncontrib, double *out_margin) {
    cell_grid g;
    comp_ctx c = {n, xy, conic, opac, rgb, depth, valid, k, o, NULL};
    if (use_grid) {
        grid_build(&g, n, xy, conic, valid, k->e_max * 1.01, width, height);
        c.grid = &g;
    }
#pragma omp parallel for schedule(dynamic, 64)
    for (long p = 0; p < npix; p++) {
        long last;
        int cnt;
        double mg;
        composite_pixel(&c, pix[2 * p], pix[2 * p + 1], out_rgb + 3 * p, out_T + p, &last, &cnt, &mg, NULL);
        double mo = outside_margin(&c, pix[2 * p], pix[2 * p + 1]);
        out_last[p] = last;
        out_ncontrib[p] = cnt;
        out_margin[p] = mg < mo ? mg : mo;
    }
    if (use_grid) grid_free(&g);
}

/*
 * orc_composite_bwd: gradients of L = sum_p G_p . I_p with respect to the
 * projected quantities, given the upstream gradient G[npix][3] (Backpropagation
 * and Error Calculation; derivative equations of each kernel's supplementary
 * section).  Accumulates into d_xy[n][2], d_conic[n][3] (a, scalar b, c),
 * d_opac[n], d_rgb[n][3], which the caller zero-fills.  The transmittance in
 * front of each contributor is the FP64 prefix product.
 */
void orc_composite_bwd(long n, const double *xy, const double *conic, const double *opac, const double *rgb,
                       const double *depth, const int32_t *valid, const orc_kernel *k, const orc_opts *o, int width,
                       int height, long npix, const int32_t *pix, const double *G, int use_grid, double *d_xy,
                       double *d_conic, double *d_opac, double *d_rgb) {
    cell_grid g;
    comp_ctx c = {n, xy, conic, opac, rgb, depth, valid, k, o, NULL};
    if (use_grid) {
        grid_build(&g, n, xy, conic, valid, k->e_max * 1.01, width, height);
        c.grid = &g;
    }
    /* per-pixel partials, computed in parallel, summed serially in pixel order */
    typedef struct {
        long m;
        contrib_t *r;
        double *part; /* m x 9: dxy(2) dconic(3) dopac drgb(3) */
    } pix_part;
    pix_part *pp = (pix_part *)calloc(npix > 0 ? npix : 1, sizeof(pix_part));
#pragma omp parallel for schedule(dynamic, 64)
    for (long p = 0; p < npix; p++) {
        const double *Gp = G + 3 * p;
        if (Gp[0] == 0.0 && Gp[1] == 0.0 && Gp[2] == 0.0) continue;
        int px = pix[2 * p], py = pix[2 * p + 1];
        double col[3], T, mg;
        long last;
        int cnt;
        contrib_t *r;
        long m = composite_pixel(&c, px, py, col, &T, &last, &cnt, &mg, &r);
        double *part = (double *)malloc(sizeof(double) * 9 * (m > 0 ? m : 1));
        /* S = colour contributed behind the current splat, plus the background term */
        double S[3] = {T * o->bg[0], T * o->bg[1], T * o->bg[2]};
        for (long t = m - 1; t >= 0; t--) {
            long j = r[t].id;
            double a = r[t].alpha, Tk = r[t].T;
            double dalpha = 0.0;
            for (int ch = 0; ch < 3; ch++) dalpha += Gp[ch] * (rgb[3 * j + ch] * Tk - S[ch] / (1.0 - a));
            double dx = xy[2 * j] - px, dy = xy[2 * j + 1] - py;
            const double *q = conic + 3 * j;
            /* alpha = min(alpha_max, o w): gradient passed straight through the clamp */
            double dE = opac[j] * orc_kernel_deriv_beta(k->kind, k->xi, k->beta, r[t].E) * dalpha;
            double *pt = part + 9 * t;
            pt[0] = dE * 2.0 * (q[0] * dx + q[1] * dy);
            pt[1] = dE * 2.0 * (q[1] * dx + q[2] * dy);
            pt[2] = dE * dx * dx;
            pt[3] = dE * 2.0 * dx * dy;
            pt[4] = dE * dy * dy;
            pt[5] = r[t].w * dalpha;
            for (int ch = 0; ch < 3; ch++) pt[6 + ch] = a * Tk * Gp[ch];
            for (int ch = 0; ch < 3; ch++) S[ch] += a * Tk * rgb[3 * j + ch];
        }
        pp[p].m = m;
        pp[p].r = r;
        pp[p].part = part;
    }
    for (long p = 0; p < npix; p++) {
        for (long t = 0; t < pp[p].m; t++) {
            long j = pp[p].r[t].id;
            const double *pt = pp[p].part + 9 * t;
            d_xy[2 * j] += pt[0];
            d_xy[2 * j + 1] += pt[1];
            d_conic[3 * j] += pt[2];
            d_conic[3 * j + 1] += pt[3];
            d_conic[3 * j + 2] += pt[4];
            d_opac[j] += pt[5];
            for (int ch = 0; ch < 3; ch++) d_rgb[3 * j + ch] += pt[6 + ch];
        }
        free(pp[p].r);
        free(pp[p].part);
    }
    free(pp);
    if (use_grid) grid_free(&g);
}

/*
 * orc_preprocess_bwd: chain the projected-space gradients back to the splat
 * parameters (conic -> 2D covariance -> psi -> EWA projection -> 3D
 * covariance -> scale/rotation; mean through the projection, the Jacobian and
 * the SH view direction; SH coefficients).  Overwrites d_means[3][n],
 * d_scales[3][n], d_quats[4][n], d_opac_out[n], d_sh[(deg+1)^2][3][n]; culled
 * splats get zeros.
 */
void orc_preprocess_bwd(const orc_camera *cam, const orc_kernel *k, long n, const double *means,
                        const double *scales, const double *quats, const double *sh, int deg, const double *g_xy,
                        const double *g_conic, const double *g_opac, const double *g_rgb, double *d_means,
                        double *d_scales, double *d_quats, double *d_opac_out, double *d_sh) {
    int nb = (deg + 1) * (deg + 1);
#pragma omp parallel for schedule(static)
    for (long i = 0; i < n; i++) {
        orc_splat_state s;
        project_one(cam, k, n, i, means, scales, quats, sh, deg, &s);
        for (int c = 0; c < 3; c++) { d_means[c * n + i] = 0.0; d_scales[c * n + i] = 0.0; }
        for (int c = 0; c < 4; c++) d_quats[c * n + i] = 0.0;
        d_opac_out[i] = 0.0;
        for (int b = 0; b < nb; b++)
            for (int ch = 0; ch < 3; ch++) d_sh[((long)b * 3 + ch) * n + i] = 0.0;
        if (!s.visible) continue;

        double dmu[3] = {0, 0, 0};
        d_opac_out[i] = g_opac[i];

        /* colour: rgb_ch = max(0, sum_b Y_b(dir) sh_b,ch + 0.5) */
        double Y[16], dY[16][3];
        sh_basis(s.dir, Y, dY);
        double gdir[3] = {0, 0, 0};
        for (int ch = 0; ch < 3; ch++) {
            double gv = s.clamped[ch] ? 0.0 : g_rgb[3 * i + ch];
            for (int b = 0; b < nb; b++) {
                double shv = sh[((long)b * 3 + ch) * n + i];
                d_sh[((long)b * 3 + ch) * n + i] = Y[b] * gv;
                for (int c = 0; c < 3; c++) gdir[c] += gv * shv * dY[b][c];
            }
        }
        /* dir = v / |v| */
        double dd = gdir[0] * s.dir[0] + gdir[1] * s.dir[1] + gdir[2] * s.dir[2];
        for (int c = 0; c < 3; c++) dmu[c] += (gdir[c] - s.dir[c] * dd) / s.vlen;

        /* conic Q = cov^{-1}: dL/dcov = -Q Ghat Q, Ghat = [[ga, gb/2], [gb/2, gc]] */
        double Q[4] = {s.conic[0], s.conic[1], s.conic[1], s.conic[2]};
        double Gh[4] = {g_conic[3 * i], 0.5 * g_conic[3 * i + 1], 0.5 * g_conic[3 * i + 1], g_conic[3 * i + 2]};
        double QG[4], dcov[4];
        matmul(Q, Gh, QG, 2, 2, 2);
        matmul(QG, Q, dcov, 2, 2, 2);
        for (int c = 0; c < 4; c++) dcov[c] = -dcov[c];
        /* cov = psi M + eps I */
        double dM[4];
        for (int c = 0; c < 4; c++) dM[c] = k->psi * dcov[c];
        /* M = A Sigma A^T: dSigma = A^T dM A, dA = 2 dM A Sigma */
        double At[6], AtdM[6], dSigma[9], dMA[6], dA[6];
        transpose(s.A, At, 2, 3);
        matmul(At, dM, AtdM, 3, 2, 2);
        matmul(AtdM, s.A, dSigma, 3, 2, 3);
        matmul(dM, s.A, dMA, 2, 2, 3);
        matmul(dMA, s.Sigma, dA, 2, 3, 3);
        for (int c = 0; c < 6; c++) dA[c] *= 2.0;
        /* A = J W: dJ = dA W^T */
        double Wt[9], dJ[6];
        transpose(s.W, Wt, 3, 3);
        matmul(dA, Wt, dJ, 2, 3, 3);
        /* J(t) entries: J00 = fx/tz, J02 = -fx xt/tz, J11 = fy/tz, J12 = -fy yt/tz */
        double tx = s.t[0], ty = s.t[1], tz = s.t[2];
        double fx = cam->fx, fy = cam->fy;
        double dt[3] = {0, 0, 0};
        double dxt_dtx = s.clamp_x ? 0.0 : 1.0 / tz, dxt_dtz = s.clamp_x ? 0.0 : -tx / (tz * tz);
        double dyt_dty = s.clamp_y ? 0.0 : 1.0 / tz, dyt_dtz = s.clamp_y ? 0.0 : -ty / (tz * tz);
        dt[2] += dJ[0] * (-fx / (tz * tz)) + dJ[4] * (-fy / (tz * tz));
        dt[0] += dJ[2] * (-fx * dxt_dtx / tz);
        dt[2] += dJ[2] * (-fx * (dxt_dtz * tz - s.xt) / (tz * tz));
        dt[1] += dJ[5] * (-fy * dyt_dty / tz);
        dt[2] += dJ[5] * (-fy * (dyt_dtz * tz - s.yt) / (tz * tz));
        /* mean2D: (fx tx/tz + cx, fy ty/tz + cy) */
        double gx = g_xy[2 * i], gy = g_xy[2 * i + 1];
        dt[0] += gx * fx / tz;
        dt[1] += gy * fy / tz;
        dt[2] += -gx * fx * tx / (tz * tz) - gy * fy * ty / (tz * tz);
        /* t = W mu + t_cw */
        for (int c = 0; c < 3; c++) dmu[c] += s.W[0 * 3 + c] * dt[0] + s.W[1 * 3 + c] * dt[1] + s.W[2 * 3 + c] * dt[2];
        for (int c = 0; c < 3; c++) d_means[c * n + i] = dmu[c];

        /* Sigma = Mq Mq^T with Mq = Rq diag(s): dMq = 2 dSigma Mq */
        double sc[3] = {scales[i], scales[n + i], scales[2 * n + i]};
        double Mq[9], dMq[9];
        for (int r = 0; r < 3; r++)
            for (int c = 0; c < 3; c++) Mq[r * 3 + c] = s.Rq[r * 3 + c] * sc[c];
        matmul(dSigma, Mq, dMq, 3, 3, 3);
        for (int c = 0; c < 9; c++) dMq[c] *= 2.0;
        double dR[9];
        for (int c = 0; c < 3; c++) {
            double acc = 0.0;
            for (int r = 0; r < 3; r++) {
                acc += dMq[r * 3 + c] * s.Rq[r * 3 + c];
                dR[r * 3 + c] = dMq[r * 3 + c] * sc[c];
            }
            d_scales[c * n + i] = acc;
        }
        /* rotation entries as functions of the unit quaternion (w, x, y, z) */
        double w = s.qn[0], x = s.qn[1], y = s.qn[2], z = s.qn[3];
        double dq[4];
        dq[0] = dR[1] * (-2 * z) + dR[2] * (2 * y) + dR[3] * (2 * z) + dR[5] * (-2 * x) + dR[6] * (-2 * y) +
                dR[7] * (2 * x);
        dq[1] = dR[1] * (2 * y) + dR[2] * (2 * z) + dR[3] * (2 * y) + dR[4] * (-4 * x) + dR[5] * (-2 * w) +
                dR[6] * (2 * z) + dR[7] * (2 * w) + dR[8] * (-4 * x);
        dq[2] = dR[0] * (-4 * y) + dR[1] * (2 * x) + dR[2] * (2 * w) + dR[3] * (2 * x) + dR[5] * (2 * z) +
                dR[6] * (-2 * w) + dR[7] * (2 * z) + dR[8] * (-4 * y);
        dq[3] = dR[0] * (-4 * z) + dR[1] * (-2 * w) + dR[2] * (2 * x) + dR[3] * (2 * w) + dR[4] * (-4 * z) +
                dR[5] * (2 * y) + dR[6] * (2 * x) + dR[7] * (2 * y);
        /* qn = q / |q| */
        double qd = dq[0] * w + dq[1] * x + dq[2] * y + dq[3] * z;
        double qn4[4] = {w, x, y, z};
        for (int c = 0; c < 4; c++) d_quats[c * n + i] = (dq[c] - qn4[c] * qd) / s.qnorm;
    }
}

/* ------------------------------------------------------------------------ */
/* Binning reference: integer / FP32 by definition (tile-based               */
/* rasterization with a bounding box, DARBF boundaries section).             */
/* ------------------------------------------------------------------------ */

typedef struct {
    uint64_t key;
    uint32_t id;
} bin_entry;

static int bin_cmp(const void *a, const void *b) {
    const bin_entry *x = (const bin_entry *)a, *y = (const bin_entry *)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    return (x->id < y->id) ? -1 : (x->id > y->id);
}

static int clamp_tile(float v, int hi) {
    float c = fminf(fmaxf(v, 0.0f), (float)hi);
    return (int)c;
}

/*
 * orc_bin: every splat with half-extents (rx, ry) > 0 covers the tiles
 *   x in [clamp(floor((u - rx) / 16)), clamp(floor((u + rx) / 16) + 1)), same for y with ry,
 * evaluated in FP32; one entry per covered tile with key (tile << 32) | bits(depth)
 * and value = splat index.  Entries are ordered by (key, index).  ranges[t] =
 * (#entries with tile < t, #entries with tile <= t).  Returns K; keys/vals are
 * written only when vals is given and K <= cap (ranges need no sort).
 *
 * The order is produced by a sort on (key, index); the entries are first
 * grouped by tile (the high half of the key) and each tile's group is then
 * sorted on its own, which is the same total order.
 */
long orc_bin(long n, const float *xy, const int32_t *extent, const float *depth, int width, int height, long cap,
             uint64_t *keys, uint32_t *vals, uint32_t *ranges) {
    int gx = (width + 15) / 16, gy = (height + 15) / 16;
    long ntile = (long)gx * gy;
    long K = 0;
    int *rect = (int *)malloc(sizeof(int) * 4 * (n > 0 ? n : 1));
    long *cnt = (long *)calloc(ntile + 1, sizeof(long));
    for (long i = 0; i < n; i++) {
        rect[4 * i] = rect[4 * i + 1] = rect[4 * i + 2] = rect[4 * i + 3] = 0;
        if (extent[2 * i] <= 0 || extent[2 * i + 1] <= 0) continue;
        float u = xy[2 * i], v = xy[2 * i + 1], rx = (float)extent[2 * i], ry = (float)extent[2 * i + 1];
        rect[4 * i] = clamp_tile(floorf((u - rx) * 0.0625f), gx);
        rect[4 * i + 1] = clamp_tile(floorf((u + rx) * 0.0625f) + 1.0f, gx);
        rect[4 * i + 2] = clamp_tile(floorf((v - ry) * 0.0625f), gy);
        rect[4 * i + 3] = clamp_tile(floorf((v + ry) * 0.0625f) + 1.0f, gy);
        long w = rect[4 * i + 1] - rect[4 * i], h = rect[4 * i + 3] - rect[4 * i + 2];
        if (w <= 0 || h <= 0) continue;
        K += w * h;
        for (int ty = rect[4 * i + 2]; ty < rect[4 * i + 3]; ty++)
            for (int tx = rect[4 * i]; tx < rect[4 * i + 1]; tx++) cnt[(long)ty * gx + tx + 1]++;
    }
    /* ranges from the per-tile counts */
    for (long t = 0; t < ntile; t++) cnt[t + 1] += cnt[t];
    for (long t = 0; t < ntile; t++) { ranges[2 * t] = (uint32_t)cnt[t]; ranges[2 * t + 1] = (uint32_t)cnt[t + 1]; }
    if (vals && K <= cap && K > 0) {
        bin_entry *e = (bin_entry *)malloc(sizeof(bin_entry) * K);
        long *pos = (long *)malloc(sizeof(long) * (ntile > 0 ? ntile : 1));
        for (long t = 0; t < ntile; t++) pos[t] = cnt[t];
        for (long i = 0; i < n; i++) {
            uint32_t db;
            memcpy(&db, &depth[i], 4);
            for (int ty = rect[4 * i + 2]; ty < rect[4 * i + 3]; ty++)
                for (int tx = rect[4 * i]; tx < rect[4 * i + 1]; tx++) {
                    long t = (long)ty * gx + tx;
                    e[pos[t]].key = ((uint64_t)t << 32) | db;
                    e[pos[t]].id = (uint32_t)i;
                    pos[t]++;
                }
        }
#pragma omp parallel for schedule(dynamic, 16)
        for (long t = 0; t < ntile; t++) qsort(e + cnt[t], cnt[t + 1] - cnt[t], sizeof(bin_entry), bin_cmp);
        for (long t = 0; t < K; t++) {
            if (keys) keys[t] = e[t].key;
            vals[t] = e[t].id;
        }
        free(pos);
        free(e);
    }
    free(cnt);
    free(rect);
    return K;
}

/* number of OpenMP threads the oracle's parallel loops use */
#ifdef _OPENMP
#include <omp.h>
#endif
int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* thread count of the following parallel loops (timing runs on fewer cores) */
void orc_set_num_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
