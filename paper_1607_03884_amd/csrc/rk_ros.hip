// Rodas3 Rosenbrock integration with a group of lanes cooperating on one
// state: the non-exponential Rosenbrock direction the paper's conclusions
// recommend for GPU chemical kinetics (Sec. 4), on the same source terms,
// analytical Jacobian, register-row LU and substitutions as the wavefront
// Radau IIA kernels (16 lanes per state for N <= 16, a wavefront for N <= 56).
//
// Rodas3 (Sandu et al.; four stages, order 3, embedded order 2, L-stable,
// gamma = 1/2) in the transformed form:
//   (1/(h gamma) I - J) u_i = f(y + sum_{j<i} a_ij u_j) + sum_{j<i} (c_ij / h) u_j,
//   y_new = y + sum_i m_i u_i, error estimate u_4,
// a21 = 0, a31 = 2, a32 = 0, a41 = 2, a42 = 0, a43 = 1;
// c21 = 4, c31 = 1, c32 = -1, c41 = 1, c42 = -1, c43 = -8/3; m = (2, 0, 1, 1).
// Stages 1 and 2 evaluate f at y (f(y) of the step), so a step costs one
// Jacobian (at every new y), one real FP64 factorisation, two source-term
// evaluations inside the step and one at its end, and four substitutions.
// Step control: err = RMS of u_4 / (atol + rtol max(|y|, |y_new|)) (a
// non-finite err rejects), accept when err <= 1,
// h_new = h min(6, max(0.2, 0.9 err^(-1/3))), no growth right after a
// rejection, the Jacobian kept after a rejection; initial step, last-step
// rule and failure statuses as the Radau IIA kernels.
#include <hip/hip_runtime.h>
#include <algorithm>

#include "rk_group_impl.h"

namespace rk {

namespace {

constexpr double kRosGamma = 0.5;

template <int G, int NC>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(G == 16 ? 2 : 1))) void rodas3_group_kernel(
    DevMech m, RadauParams rp, int64_t n, const double *__restrict__ yin, double *__restrict__ yout,
    int32_t *__restrict__ cnt, int *__restrict__ queue, const int *__restrict__ order) {
    extern __shared__ double smem[];
    const int r = threadIdx.x & (G - 1);
    const int grp = threadIdx.x / G;
    const int N = m.N, K = m.K;
    GL L = group_lds<NC>(smem + (size_t)grp * group_lds_doubles(NC, m.R), m.R);
    stage_tables<G, NC>(m, smem, L);
    const bool comp = r < N;
    const double dt = rp.dt, atol = rp.atol, rtol = rp.rtol;
    LUR<double, NC> E;
    bool have = false, drained = false, last = false, reject = false, need_j = true;
    int qnext = 0, qend = 0;
    int64_t s = 0;
    double y = 0.0, h = 0.0;
    int status = 0, nstep = 0, nacc = 0;
    auto bump = [&](int k, int v) {
        if (r == 0) L.ctr[k] += v;
    };
    for (;;) {
        if (!have && !drained) {
            if (qnext >= qend) {
                int q0 = 0;
                if (r == 0) q0 = atomicAdd(queue, rp.tile);
                qnext = gbi<G>(q0, 0);
                qend = qnext + rp.tile;
            }
            const int qi = qnext++;
            if (qi >= n) {
                drained = true;
            } else {
                s = order ? (int64_t)order[qi] : (int64_t)qi;
                const double P = yin[(size_t)(K + 1) * n + s];
                L.hist[3] = P;
                y = comp ? yin[(size_t)r * n + s] : 0.0;
                const bool bad_l = (comp && !isfinite(y)) || (r == 0 && !(y > 0.0)) ||
                                   (r == 0 && !(P > 0.0 && isfinite(P)));
                nstep = nacc = 0;
                if (r < K_NCTR) L.ctr[r] = 0;
                if (gsum<G>(bad_l ? 1.0 : 0.0) > 0.0) {
                    if (comp) yout[(size_t)r * n + s] = y;
                    if (r == 0) {
                        yout[(size_t)(K + 1) * n + s] = P;
                        cnt[(size_t)C_STATUS * n + s] = RK_ST_NONFINITE;
                        for (int c = 1; c < kNumCounters; ++c) cnt[(size_t)c * n + s] = 0;
                    }
                } else {
                    have = true;
                    status = RK_ST_OK;
                    L.hist[4] = 0.0;
                    h = rp.h0;
                    last = false;
                    if (1.0001 * h >= dt) { h = dt; last = true; }
                    const double f0 = rhs_g<G>(m, L, r, y, P);
                    if (r < NC) L.f0s[r] = f0;
                    bump(K_NFEV, 1);
                    reject = false;
                    need_j = true;
                }
            }
        }
        if (__ballot(have) == 0ull && __ballot(!drained) == 0ull) break;
        if (!have) continue;

        bool done = false;
        const double P = L.hist[3];
        if (nstep >= rp.nmax) {
            status = RK_ST_STEP_LIMIT;
            done = true;
        } else if (0.1 * h <= kU * L.hist[4] || h < 1e-300) {
            status = RK_ST_H_UNDERFLOW;
            done = true;
        } else {
            if (need_j) {
                jac_g<G, NC>(m, L, r, y, P);
                bump(K_NJEV, 1);
                need_j = false;
            }
            ++nstep;
            // E = 1/(h gamma) I - J, factored with FP64 partial pivoting
            const double *row = L.J + (r < NC ? r : 0) * (NC + 1);
#pragma unroll
            for (int c = 0; c < NC; ++c) E.a[c] = -(comp ? row[c] : 0.0);
            const double gh = 1.0 / (h * kRosGamma);
#pragma unroll
            for (int c = 0; c < NC; ++c)
                if (c == r) E.a[c] += gh;
            sync_wave();
            factor_real<double, G>(E, L, r, N);
            bump(K_NLU, 1);
            const double f0 = comp ? L.f0s[r] : 0.0;
            // c_ij / h
            const double c21 = 4.0 / h, c31 = 1.0 / h, c32 = -1.0 / h, c43 = (-8.0 / 3.0) / h;
            // stages 1 and 2 at y
            const double u1 = solve_real<double, G>(E, r, N, f0);
            const double u2 = solve_real<double, G>(E, r, N, comp ? f0 + c21 * u1 : 0.0);
            // stages 3 and 4: one source-term body for both
            double u3 = 0.0, u4 = 0.0;
#pragma nounroll
            for (int st = 2; st < 4; ++st) {
                const double arg = st == 2 ? (y + 2.0 * u1) + 0.0 * u2 : ((y + 2.0 * u1) + 0.0 * u2) + 1.0 * u3;
                const double fs = rhs_g<G>(m, L, r, arg, P);
                // c41 = c31, c42 = c32
                const double rhs = st == 2 ? (fs + c31 * u1) + c32 * u2 : ((fs + c31 * u1) + c32 * u2) + c43 * u3;
                const double us = solve_real<double, G>(E, r, N, comp ? rhs : 0.0);
                u3 = st == 2 ? us : u3;
                u4 = st == 3 ? us : u4;
            }
            bump(K_NFEV, 2);
            const double yn = comp ? (((y + 2.0 * u1) + 0.0 * u2) + 1.0 * u3) + 1.0 * u4 : 0.0;
            const double sc = comp ? atol + rtol * fmax(fabs(y), fabs(yn)) : 1.0;
            const double en = sqrt(gsum<G>(comp ? (u4 / sc) * (u4 / sc) : 0.0) / N);
            const double err = isfinite(en) ? fmax(en, 1e-10) : 1e300;
            const double fac = fmin(6.0, fmax(0.2, 0.9 * pow(err, -1.0 / 3.0)));
            if (err <= 1.0) {
                ++nacc;
                y = yn;
                const double t = last ? dt : L.hist[4] + h;
                L.hist[4] = t;
                if (last) {
                    done = true;
                } else {
                    const double fn = rhs_g<G>(m, L, r, y, P);
                    if (r < NC) L.f0s[r] = fn;
                    bump(K_NFEV, 1);
                    need_j = true;
                    double hn = h * fac;
                    if (reject) hn = fmin(hn, h);
                    reject = false;
                    if (t + 1.0001 * hn >= dt) {
                        h = dt - t;
                        last = true;
                    } else {
                        h = hn;
                    }
                }
            } else {
                bump(K_NREJ, 1);
                reject = true;
                last = false;
                h = h * fac;
            }
        }
        if (done) {
            if (comp) yout[(size_t)r * n + s] = y;
            if (r == 0) {
                yout[(size_t)(K + 1) * n + s] = L.hist[3];
                cnt[(size_t)C_STATUS * n + s] = status;
                cnt[(size_t)C_NSTEP * n + s] = nstep;
                cnt[(size_t)C_NACC * n + s] = nacc;
                cnt[(size_t)C_NREJ * n + s] = L.ctr[K_NREJ];
                cnt[(size_t)C_NNEWT * n + s] = 0;
                cnt[(size_t)C_NNFAIL * n + s] = 0;
                cnt[(size_t)C_NFEV * n + s] = L.ctr[K_NFEV];
                cnt[(size_t)C_NJEV * n + s] = L.ctr[K_NJEV];
                cnt[(size_t)C_NLU * n + s] = L.ctr[K_NLU];
                cnt[(size_t)C_FLAGS * n + s] = 0;
            }
            have = false;
        }
    }
}

__global__ void reset_ros_queue_kernel(int *q) {
    if (threadIdx.x < 4) q[threadIdx.x] = 0;
}

template <int G, int NC>
void launch_ros(const DevMech &m, const RadauParams &p, int64_t n, const double *yin, double *yout, int32_t *cnt,
                int *queue, const int *order, int grid, hipStream_t st) {
    const size_t lds = block_lds_bytes<G, NC>(m.K, m.R, m.nsp, m.n3b);
    hipLaunchKernelGGL((rodas3_group_kernel<G, NC>), dim3(grid), dim3(kWave), lds, st, m, p, n, yin, yout, cnt, queue,
                       order);
}

}  // namespace

hipError_t launch_rodas3_group(const DevMech &m, const RadauParams &p, int64_t n, const double *yin, double *yout,
                               int32_t *counters, int *queue, const int *order, int grid, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(reset_ros_queue_kernel, dim3(1), dim3(64), 0, st, queue);
    const int N = m.N;
    if (N <= 14) launch_ros<16, 14>(m, p, n, yin, yout, counters, queue, order, grid, st);
    else if (N <= 16) launch_ros<16, 16>(m, p, n, yin, yout, counters, queue, order, grid, st);
    else if (N <= 54) launch_ros<64, 54>(m, p, n, yin, yout, counters, queue, order, grid, st);
    else if (N <= 56) launch_ros<64, 56>(m, p, n, yin, yout, counters, queue, order, grid, st);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace rk
