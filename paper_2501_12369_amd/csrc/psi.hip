// psi.hip -- the correction-factor experiment of the paper on the GPU
// (Mathematical Expressions of Monte Carlo Experiments; the psi regression of
// the extended results): a 3D DARBF with covariance Sigma is sampled on an
// N x N x N grid, summed along z with Simpson's rule into a 2D density, and the
// density's weighted covariance (a', b', d') is compared with the upper-left
// 2x2 block (a, b, d) of Sigma.  Over m covariances the linear map
// (a, b, c, d, e, f) -> (a', b', d') is fitted by least squares, and the scalar
// psi by the least-squares ratio of the two 2x2 blocks.
//
// One workgroup per (sample, x row): each lane walks the z column of one or
// more y positions (the Simpson sum in FP64), the row's three moments are
// reduced across the workgroup; a second kernel combines the rows of a sample,
// a third solves the 6 x 6 normal equations in FP64.  ALU-bound (one profile
// evaluation per grid point); nothing is read from memory but the covariance.
#include "common.h"

namespace darb {

namespace {

constexpr int kPsiThreads = 256;

// The grid of a sample: n points per axis (n odd) spanning [-L_a, L_a] on axis
// a, L_a = margin * sqrt(e_max * Sigma_aa), the half-extent of the support
// {p : p^T Sigma^-1 p <= e_max} along that axis (the box that holds it).
struct PsiGrid {
    int n;
    float margin;
};

__device__ __forceinline__ void sample_extent(const double *sig, const PsiGrid &g, float e_max, double (&L)[3]) {
    L[0] = g.margin * sqrt((double)e_max * sig[0]);
    L[1] = g.margin * sqrt((double)e_max * sig[3]);
    L[2] = g.margin * sqrt((double)e_max * sig[5]);
}

__device__ __forceinline__ double coord(double L, int k, int n) { return L * (2.0 * k / (double)(n - 1) - 1.0); }

// Inverse covariance (xx, xy, xz, yy, yz, zz) of a sample.
__device__ __forceinline__ void sample_inverse(const double *sig, double (&inv)[6]) {
    const double a = sig[0], b = sig[1], c = sig[2], d = sig[3], e = sig[4], f = sig[5];
    const double A = d * f - e * e, B = -(b * f - c * e), C = b * e - c * d;
    const double det = a * A + b * B + c * C;
    const double id = 1.0 / det;
    inv[0] = A * id;
    inv[1] = B * id;
    inv[2] = C * id;
    inv[3] = (a * f - c * c) * id;
    inv[4] = -(a * e - b * c) * id;
    inv[5] = (a * d - b * b) * id;
}

__device__ __forceinline__ double simpson_weight(int k, int n) {
    return (k == 0 || k == n - 1) ? 1.0 : ((k & 1) ? 4.0 : 2.0);
}

__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// row moments of sample s, x row i: (sum w, sum w y, sum w y^2) with the 2D
// density w(x_i, y_j) = Simpson sum over z of F(E(x_i, y_j, z_k))
template <int KIND>
__global__ __launch_bounds__(kPsiThreads) void k_psi_rows(const double *sigma, PsiGrid g, KParams kp, double *rows) {
    const int i = blockIdx.x, s = blockIdx.y;
    double inv[6], L[3];
    sample_inverse(sigma + 6 * (size_t)s, inv);
    sample_extent(sigma + 6 * (size_t)s, g, kp.e_max, L);
    const double x = coord(L[0], i, g.n);
    // E = p^T inv p in FP32 from FP64 coefficients
    const float qxx = (float)inv[0], qxy = (float)inv[1], qxz = (float)inv[2], qyy = (float)inv[3],
                qyz = (float)inv[4], qzz = (float)inv[5];
    const float xf = (float)x;
    double m0 = 0.0, m1 = 0.0, m2 = 0.0;
    for (int j = threadIdx.x; j < g.n; j += kPsiThreads) {
        const double y = coord(L[1], j, g.n);
        const float yf = (float)y;
        // the (x, y) part of E and of its z-linear term
        const float exy = fmaf(qxx * xf, xf, fmaf(2.0f * qxy * xf, yf, qyy * yf * yf));
        const float lin = 2.0f * fmaf(qxz, xf, qyz * yf);
        double col = 0.0;
        for (int k = 0; k < g.n; k++) {
            const float z = (float)coord(L[2], k, g.n);
            // E >= 0 up to rounding near the centre: clamped there, not cut
            const float E = fmaxf(fmaf(fmaf(qzz, z, lin), z, exy), 0.0f);
            const float w = E <= kp.e_max ? profile<KIND>(E, kp) : 0.0f;
            col += simpson_weight(k, g.n) * (double)w;
        }
        m0 += col;
        m1 += col * y;
        m2 += col * y * y;
    }
    __shared__ double red[3][kPsiThreads / 64];
    m0 = wave_sum_d(m0);
    m1 = wave_sum_d(m1);
    m2 = wave_sum_d(m2);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) {
        red[0][w] = m0;
        red[1][w] = m1;
        red[2][w] = m2;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double t0 = 0.0, t1 = 0.0, t2 = 0.0;
        for (int k = 0; k < kPsiThreads / 64; k++) {
            t0 += red[0][k];
            t1 += red[1][k];
            t2 += red[2][k];
        }
        double *r = rows + 3 * ((size_t)s * g.n + i);
        r[0] = t0;
        r[1] = t1;
        r[2] = t2;
    }
}

// weighted 2x2 covariance of sample s from its row moments (one wavefront per sample)
__global__ __launch_bounds__(64) void k_psi_cov(const double *sigma, const double *rows, PsiGrid g, float e_max,
                                                double *cov2) {
    const int s = blockIdx.x, lane = threadIdx.x;
    double L[3];
    sample_extent(sigma + 6 * (size_t)s, g, e_max, L);
    double S0 = 0, Sx = 0, Sy = 0, Sxx = 0, Sxy = 0, Syy = 0;
    for (int i = lane; i < g.n; i += 64) {
        const double x = coord(L[0], i, g.n);
        const double *r = rows + 3 * ((size_t)s * g.n + i);
        S0 += r[0];
        Sx += x * r[0];
        Sxx += x * x * r[0];
        Sy += r[1];
        Sxy += x * r[1];
        Syy += r[2];
    }
    S0 = wave_sum_d(S0);
    Sx = wave_sum_d(Sx);
    Sy = wave_sum_d(Sy);
    Sxx = wave_sum_d(Sxx);
    Sxy = wave_sum_d(Sxy);
    Syy = wave_sum_d(Syy);
    if (lane == 0) {
        const double mx = Sx / S0, my = Sy / S0;
        cov2[3 * (size_t)s] = Sxx / S0 - mx * mx;
        cov2[3 * (size_t)s + 1] = Sxy / S0 - mx * my;
        cov2[3 * (size_t)s + 2] = Syy / S0 - my * my;
    }
}

// Least squares over the m samples, one wavefront: the sums of the normal
// equations are reduced across lanes, lane 0 solves them (Gaussian elimination
// with partial pivoting, FP64).  Row r of the fit (a', b', d' for r = 0, 1, 2)
// holds the weights of (a, b, c, d, e, f) at fit[6 r .. 6 r + 5]; fit[18] is
// the scalar psi.
__global__ __launch_bounds__(64) void k_psi_fit(const double *sigma, const double *cov2, int m, double *fit) {
    const int lane = threadIdx.x;
    double XtX[21], XtY[18], num = 0.0, den = 0.0;  // XtX upper triangle, row-major
    for (int k = 0; k < 21; k++) XtX[k] = 0.0;
    for (int k = 0; k < 18; k++) XtY[k] = 0.0;
    for (int s = lane; s < m; s += 64) {
        const double *x = sigma + 6 * (size_t)s;  // a = xx, b = xy, c = xz, d = yy, e = yz, f = zz
        const double *y = cov2 + 3 * (size_t)s;   // a', b', d'
        int t = 0;
        for (int r = 0; r < 6; r++)
            for (int c = r; c < 6; c++) XtX[t++] += x[r] * x[c];
        for (int r = 0; r < 6; r++)
            for (int o = 0; o < 3; o++) XtY[3 * r + o] += x[r] * y[o];
        num += y[0] * x[0] + 2.0 * y[1] * x[1] + y[2] * x[3];
        den += x[0] * x[0] + 2.0 * x[1] * x[1] + x[3] * x[3];
    }
    for (int k = 0; k < 21; k++) XtX[k] = wave_sum_d(XtX[k]);
    for (int k = 0; k < 18; k++) XtY[k] = wave_sum_d(XtY[k]);
    num = wave_sum_d(num);
    den = wave_sum_d(den);
    if (lane != 0) return;
    double A[6][9];
    int t = 0;
    for (int r = 0; r < 6; r++)
        for (int c = r; c < 6; c++) {
            A[r][c] = XtX[t];
            A[c][r] = XtX[t];
            t++;
        }
    for (int r = 0; r < 6; r++)
        for (int o = 0; o < 3; o++) A[r][6 + o] = XtY[3 * r + o];
    for (int col = 0; col < 6; col++) {
        int piv = col;
        for (int r = col + 1; r < 6; r++)
            if (fabs(A[r][col]) > fabs(A[piv][col])) piv = r;
        if (piv != col)
            for (int c = 0; c < 9; c++) {
                const double tmp = A[col][c];
                A[col][c] = A[piv][c];
                A[piv][c] = tmp;
            }
        const double p = A[col][col];
        for (int r = 0; r < 6; r++) {
            if (r == col) continue;
            const double f = A[r][col] / p;
            for (int c = col; c < 9; c++) A[r][c] -= f * A[col][c];
        }
    }
    for (int o = 0; o < 3; o++)
        for (int r = 0; r < 6; r++) fit[6 * o + r] = A[r][6 + o] / A[r][r];
    fit[18] = num / den;
}

template <int KIND>
void rows_launch(const double *sigma, const PsiGrid &g, const KParams &kp, int m, double *rows, hipStream_t s) {
    hipLaunchKernelGGL((k_psi_rows<KIND>), dim3(g.n, m), dim3(kPsiThreads), 0, s, sigma, g, kp, rows);
}

}  // namespace

size_t psi_workspace(int m, int n) { return (size_t)3 * m * n * sizeof(double); }

hipError_t launch_psi_calibrate(int kind, const KParams &kp, int m, const double *sigma, int n, float margin, void *ws,
                                double *cov2, double *fit, hipStream_t s) {
    if (m <= 0) return hipSuccess;
    const PsiGrid g{n, margin};
    double *rows = static_cast<double *>(ws);
    switch (kind) {
    case DARB_GAUSS: rows_launch<DARB_GAUSS>(sigma, g, kp, m, rows, s); break;
    case DARB_HALF_COS: rows_launch<DARB_HALF_COS>(sigma, g, kp, m, rows, s); break;
    case DARB_RAISED_COS: rows_launch<DARB_RAISED_COS>(sigma, g, kp, m, rows, s); break;
    case DARB_SINC: rows_launch<DARB_SINC>(sigma, g, kp, m, rows, s); break;
    case DARB_IMQ: rows_launch<DARB_IMQ>(sigma, g, kp, m, rows, s); break;
    case DARB_IMQ_SQRT: rows_launch<DARB_IMQ_SQRT>(sigma, g, kp, m, rows, s); break;
    case DARB_PARABOLA: rows_launch<DARB_PARABOLA>(sigma, g, kp, m, rows, s); break;
    default: rows_launch<DARB_GAUSS_BETA>(sigma, g, kp, m, rows, s); break;
    }
    hipLaunchKernelGGL(k_psi_cov, dim3(m), dim3(64), 0, s, sigma, rows, g, kp.e_max, cov2);
    if (fit) hipLaunchKernelGGL(k_psi_fit, dim3(1), dim3(64), 0, s, sigma, cov2, m, fit);
    return hipGetLastError();
}

}  // namespace darb
