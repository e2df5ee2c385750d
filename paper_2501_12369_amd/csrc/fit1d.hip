// fit1d.hip -- the paper's 1D signal-reconstruction experiment (Assessing
// DARBFs through 1D Simulations; the extended 1D results): a target signal
// sampled at m points is approximated by a mixture of n_comp DARBF components
// f(x) = sum_k a_k F(E_k(x)),  E_k(x) = ((x - mu_k) / sigma_k)^2 = d_M^2 in 1D,
// each component restricted to E <= e_max, and the mean squared error
//   L = (1/m) sum_x (f(x) - t(x))^2
// is minimised by Adam over (mu_k, log sigma_k, a_k).
//
// Many independent problems (signals x kernels x component counts, the
// paper's parameter sweep) run in one persistent launch: one workgroup per
// problem keeps its components in LDS and runs every optimisation step --
// forward over its samples, residual, gradient sums, Adam -- with workgroup
// barriers between the phases; nothing leaves the chip between steps but the
// optional per-step loss.  ALU-bound.
#include "common.h"

namespace darb {

namespace {

constexpr int kFitThreads = 256;
constexpr int kFitMaxComp = 64;
constexpr int kFitMaxSamples = 4096;
constexpr int kFitWaves = kFitThreads / 64;

struct FitArgs {
    int batch, n, m, steps, step0;
    float lr_mu, lr_ls, lr_a, beta1, beta2, eps;
};

__device__ __forceinline__ float wave_sum_f(float v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Adam on one parameter held in LDS (bias corrections bc1 = 1 - beta1^t, bc2 = 1 - beta2^t)
__device__ __forceinline__ void adam(float &p, float g, float *m1, float *m2, int idx, float lr, const FitArgs &A,
                                     float bc1, float bc2) {
    const float a = fmaf(A.beta1, m1[idx], (1.0f - A.beta1) * g);
    const float v = fmaf(A.beta2, m2[idx], (1.0f - A.beta2) * (g * g));
    m1[idx] = a;
    m2[idx] = v;
    p = p - (lr / bc1) * (a / (sqrtf(v) / sqrtf(bc2) + A.eps));
}

// Step: (1) every lane evaluates f at its samples and stores the residual in
// LDS; (2) wavefront w owns the components k = w, w + 4, ...: its lanes sum the
// three gradients over all samples, a wavefront reduction gives the totals,
// and lane 0 applies Adam to that component's three parameters.
template <int KIND>
__global__ __launch_bounds__(kFitThreads) void k_fit1d(KParams kp, FitArgs A, const float *x, const float *target,
                                                       float *params, float *adam_m, float *adam_v, float *loss) {
    const int b = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int n = A.n, m = A.m;
    __shared__ float mu[kFitMaxComp], ls[kFitMaxComp], amp[kFitMaxComp];
    __shared__ float xs[kFitMaxSamples], res[kFitMaxSamples];
    __shared__ float lred[kFitWaves];
    float *P = params + (size_t)b * 3 * n;
    float *M1 = adam_m + (size_t)b * 3 * n;
    float *M2 = adam_v + (size_t)b * 3 * n;
    const float *t = target + (size_t)b * m;
    for (int k = tid; k < n; k += kFitThreads) {
        mu[k] = P[k];
        ls[k] = P[n + k];
        amp[k] = P[2 * n + k];
    }
    for (int j = tid; j < m; j += kFitThreads) xs[j] = x[j];
    __syncthreads();
    const float inv_m2 = 2.0f / (float)m;
    float p1 = powf(A.beta1, (float)A.step0), p2 = powf(A.beta2, (float)A.step0);
    for (int step = 0; step < A.steps; step++) {
        p1 *= A.beta1;
        p2 *= A.beta2;
        float lsum = 0.0f;
        for (int j = tid; j < m; j += kFitThreads) {
            const float xj = xs[j];
            float f = 0.0f;
            for (int k = 0; k < n; k++) {
                const float u = (xj - mu[k]) * expf(-ls[k]);
                const float E = u * u;
                f = (E <= kp.e_max) ? fmaf(amp[k], profile<KIND>(E, kp), f) : f;
            }
            const float r = f - t[j];
            res[j] = r;
            lsum = fmaf(r, r, lsum);
        }
        lsum = wave_sum_f(lsum);
        if (lane == 0) lred[wv] = lsum;
        __syncthreads();
        for (int k = wv; k < n; k += kFitWaves) {
            const float is = expf(-ls[k]), mk = mu[k], ak = amp[k];
            float g_mu = 0.0f, g_ls = 0.0f, g_a = 0.0f;
            for (int j = lane; j < m; j += 64) {
                const float d = xs[j] - mk;
                const float u = d * is;
                const float E = u * u;
                if (E <= kp.e_max) {
                    const float r = res[j];
                    const float w = profile<KIND>(E, kp);
                    const float ra = r * ak * profile_deriv<KIND>(E, w, kp);
                    g_a = fmaf(r, w, g_a);
                    g_mu = fmaf(ra, -2.0f * d * is * is, g_mu);  // dE/dmu = -2 (x - mu) / sigma^2
                    g_ls = fmaf(ra, -2.0f * E, g_ls);           // dE/dlog sigma = -2 E
                }
            }
            g_mu = wave_sum_f(g_mu) * inv_m2;
            g_ls = wave_sum_f(g_ls) * inv_m2;
            g_a = wave_sum_f(g_a) * inv_m2;
            if (lane == 0) {
                adam(mu[k], g_mu, M1, M2, k, A.lr_mu, A, 1.0f - p1, 1.0f - p2);
                adam(ls[k], g_ls, M1, M2, n + k, A.lr_ls, A, 1.0f - p1, 1.0f - p2);
                adam(amp[k], g_a, M1, M2, 2 * n + k, A.lr_a, A, 1.0f - p1, 1.0f - p2);
            }
        }
        if (tid == 0 && loss) {
            float s = 0.0f;
            for (int w = 0; w < kFitWaves; w++) s += lred[w];
            loss[(size_t)b * A.steps + step] = s / (float)m;
        }
        __syncthreads();
    }
    for (int k = tid; k < n; k += kFitThreads) {
        P[k] = mu[k];
        P[n + k] = ls[k];
        P[2 * n + k] = amp[k];
    }
}

template <int KIND>
void fit_launch(const KParams &kp, const FitArgs &A, const float *x, const float *t, float *p, float *m1, float *m2,
                float *loss, hipStream_t s) {
    hipLaunchKernelGGL((k_fit1d<KIND>), dim3(A.batch), dim3(kFitThreads), 0, s, kp, A, x, t, p, m1, m2, loss);
}

}  // namespace

int fit1d_max_components() { return kFitMaxComp; }
int fit1d_max_samples() { return kFitMaxSamples; }

hipError_t launch_fit1d(int kind, const KParams &kp, int batch, int n, int m, const float *x, const float *target,
                        float *params, float *adam_m, float *adam_v, int steps, int step0, const float lr[3],
                        float beta1, float beta2, float eps, float *loss, hipStream_t s) {
    if (batch == 0 || steps == 0) return hipSuccess;
    const FitArgs A{batch, n, m, steps, step0, lr[0], lr[1], lr[2], beta1, beta2, eps};
    switch (kind) {
    case DARB_GAUSS: fit_launch<DARB_GAUSS>(kp, A, x, target, params, adam_m, adam_v, loss, s); break;
    case DARB_HALF_COS: fit_launch<DARB_HALF_COS>(kp, A, x, target, params, adam_m, adam_v, loss, s); break;
    case DARB_RAISED_COS: fit_launch<DARB_RAISED_COS>(kp, A, x, target, params, adam_m, adam_v, loss, s); break;
    case DARB_SINC: fit_launch<DARB_SINC>(kp, A, x, target, params, adam_m, adam_v, loss, s); break;
    case DARB_IMQ: fit_launch<DARB_IMQ>(kp, A, x, target, params, adam_m, adam_v, loss, s); break;
    case DARB_IMQ_SQRT: fit_launch<DARB_IMQ_SQRT>(kp, A, x, target, params, adam_m, adam_v, loss, s); break;
    case DARB_PARABOLA: fit_launch<DARB_PARABOLA>(kp, A, x, target, params, adam_m, adam_v, loss, s); break;
    default: fit_launch<DARB_GAUSS_BETA>(kp, A, x, target, params, adam_m, adam_v, loss, s); break;
    }
    return hipGetLastError();
}

}  // namespace darb
