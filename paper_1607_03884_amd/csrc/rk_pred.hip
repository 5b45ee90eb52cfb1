// Learned predictor in the integration call: input features of every state,
// batched network inference (rk_mlp.hip), decoding into the starting values
// of the first Radau step, and cost bins from the predicted step counts.
#include <hip/hip_runtime.h>
#include <cmath>

#include "rk_internal.h"

namespace rk {

namespace {

constexpr double kPatmF = 101325.0;
constexpr double kLog2_10 = 3.321928094887362;    // log2(10)

// X[s] = standardised [T / 1000, ln(P / 1 atm), Y_1..Y_K]
__global__ void feature_kernel(int64_t n, int K, const double *__restrict__ yin, const float *__restrict__ shift,
                               const float *__restrict__ scale, float *__restrict__ X) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int D = K + 2;
    if (i >= n * D) return;
    const int64_t s = i / D;
    const int j = (int)(i % D);
    double f;
    if (j == 0) f = yin[s] / 1000.0;
    else if (j == 1) f = log(fmax(yin[(size_t)(K + 1) * n + s], 1e-300) / kPatmF);
    else f = yin[(size_t)(j - 1) * n + s];
    X[i] = (float)((f - (double)shift[j]) / (double)scale[j]);
}

// pred[s][0..3N) = first-step stage values z_ic, pred[s][3N] = first step size
// (0: the default rule), pred[s][3N+1] = predicted step attempts.
// Stage values: t = symlog(z / sc) with sc = atol + rtol |y0|, |t| <= 40.
// First step: t = log10(h / dt) in [-15, 0], rounded to the nearest power of
// two times dt, h = dt 2^-q (exact), so that nearby predictions give the same
// step.  A non-finite network output decodes to 0.
__global__ void decode_kernel(int64_t n, int N, const float *__restrict__ Y, const float *__restrict__ shift,
                              const float *__restrict__ scale, const double *__restrict__ yin, double dt, double atol,
                              double rtol, double *__restrict__ pred) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int D = 3 * N + 2;
    if (i >= n * D) return;
    const int64_t s = i / D;
    const int j = (int)(i % D);
    double t = (double)Y[i] * (double)scale[j] + (double)shift[j];
    double v = 0.0;
    if (!isfinite(t)) {
        v = 0.0;
    } else if (j < 3 * N) {
        const int c = j % N;
        t = fmin(fmax(t, -40.0), 40.0);
        const double mag = expm1(fabs(t));
        const double sc = atol + rtol * fabs(yin[(size_t)c * n + s]);
        v = (t < 0.0 ? -mag : mag) * sc;
    } else if (j == 3 * N) {
        const int q = (int)rint(-fmin(fmax(t, -15.0), 0.0) * kLog2_10);
        v = ldexp(dt, -q);
    } else {
        v = exp10(fmin(fmax(t, 0.0), 7.0));
    }
    pred[i] = isfinite(v) ? v : 0.0;
}

__global__ void steps_bin_kernel(int64_t n, int D, const double *__restrict__ pred, int nbins, int *__restrict__ bins) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const double steps = pred[s * D + D - 1];
    // log2 of 1..4096 predicted attempts over the bins
    bins[s] = min(nbins - 1, max(0, (int)(log2(fmax(steps, 1.0)) * nbins / 12.0)));
}

unsigned nblk(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

hipError_t launch_predictor(Predictor &pr, int64_t n, const double *yin, double dt, double atol, double rtol,
                            int nbins, int *bins, hipStream_t st) {
    if (n == 0) return hipSuccess;
    const int K = pr.K, N = K + 1, Din = K + 2, Dout = 3 * N + 2;
    hipLaunchKernelGGL(feature_kernel, dim3(nblk(n * Din)), dim3(256), 0, st, n, K, yin, pr.in_shift, pr.in_scale, pr.X);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = pr.net->forward(n, pr.X, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(decode_kernel, dim3(nblk(n * Dout)), dim3(256), 0, st, n, N, pr.net->pre.back(), pr.out_shift,
                       pr.out_scale, yin, dt, atol, rtol, pr.pred);
    if (nbins > 0 && bins)
        hipLaunchKernelGGL(steps_bin_kernel, dim3(nblk(n)), dim3(256), 0, st, n, Dout, pr.pred, nbins, bins);
    return hipGetLastError();
}

}  // namespace rk
