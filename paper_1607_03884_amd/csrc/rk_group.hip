// Host side of the group-cooperative integrator: launch shape per mechanism
// size, the queue reset, the mixed-precision hand-back pass and occupancy.
// The kernels themselves are in rk_group_impl.h, instantiated by
// rk_group16.hip (16 lanes per state) and rk_group64.hip (a wavefront per
// state), which compile in parallel.
#include <hip/hip_runtime.h>
#include <algorithm>
#include <cstdint>

#include "rk_group_impl.h"

namespace rk {

namespace {

__global__ void reset_queue_kernel(int *q) {
    if (threadIdx.x < 4) q[threadIdx.x] = 0;
}

// indices of the states the mixed-precision pass handed back (status FALLBACK)
__global__ void collect_fallback_kernel(const int32_t *__restrict__ cnt, int64_t n, int *__restrict__ list,
                                        int *__restrict__ count) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && cnt[(size_t)C_STATUS * n + i] == kStatusFallback) list[atomicAdd(count, 1)] = (int)i;
}

__global__ void zero_i32_kernel(int32_t *__restrict__ p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

// launch shape per mechanism size: lanes per state and register columns
struct GroupShape {
    int G, NC;
};

GroupShape group_shape(int N) {
    if (N <= 14) return {16, 14};
    if (N <= 16) return {16, 16};
    if (N <= 54) return {64, 54};
    if (N <= 56) return {64, 56};
    return {0, 0};
}

hipError_t launch_shape(const GroupShape &g, bool fp32, const DevMech &m, const RadauParams &p, int64_t n,
                        const double *yin, double *yout, int32_t *cnt, int *queue, const int *order,
                        const int *work_n, const double *pred, int grid, hipStream_t st) {
    if (g.G == 16)
        return launch_group16(g.NC, fp32, m, p, n, yin, yout, cnt, queue, order, work_n, pred, grid, st);
    return launch_group64(g.NC, fp32, m, p, n, yin, yout, cnt, queue, order, work_n, pred, grid, st);
}

}  // namespace

hipError_t launch_zero_i32(int32_t *p, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(zero_i32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n);
    return hipGetLastError();
}

bool group_supported(int N) { return group_shape(N).G != 0; }

int group_states_per_block(int N) {
    const GroupShape g = group_shape(N);
    return g.G ? kWave / g.G : 0;
}

size_t group_lds_bytes(const DevMech &m) {
    const GroupShape g = group_shape(m.N);
    if (!g.G) return 0;
    const size_t slices = (size_t)(kWave / g.G) * group_lds_doubles(g.NC, m.R) * sizeof(double);
    return slices + shared_tables(g.G, m.K, m.nsp, m.n3b).bytes;
}

hipError_t launch_radau_group(const DevMech &m, const RadauParams &p, int64_t n, const double *yin, double *yout,
                              int32_t *counters, int *queue, int *fb_list, const int *order, const double *pred,
                              bool mixed, int grid, hipStream_t st) {
    if (n == 0) return hipSuccess;
    const GroupShape g = group_shape(m.N);
    if (!g.G) return hipErrorInvalidValue;
    hipLaunchKernelGGL(reset_queue_kernel, dim3(1), dim3(64), 0, st, queue);
    if (!mixed) return launch_shape(g, false, m, p, n, yin, yout, counters, queue, order, nullptr, pred, grid, st);
    // mixed pass over every state, then an FP64 pass over the states it handed back
    hipError_t e = launch_shape(g, true, m, p, n, yin, yout, counters, queue, order, nullptr, pred, grid, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(collect_fallback_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, counters, n,
                       fb_list, queue + 1);
    // the FP64 pass starts the handed-back states cold
    return launch_shape(g, false, m, p, n, yin, yout, counters, queue + 2, fb_list, queue + 1, nullptr, grid, st);
}

hipError_t launch_lu_solve(int N, bool fp32, int64_t n, double gh, double ah, double bh, const double *J,
                           const double *sc, const double *b, double *x, hipStream_t st) {
    const GroupShape g = group_shape(N);
    if (!g.G) return hipErrorInvalidValue;
    if (n == 0) return hipSuccess;
    if (g.G == 16) return lu_solve_group16(g.NC, fp32, N, n, gh, ah, bh, J, sc, b, x, st);
    return lu_solve_group64(g.NC, fp32, N, n, gh, ah, bh, J, sc, b, x, st);
}

int group_max_blocks(const DevMech &m) {
    const GroupShape g = group_shape(m.N);
    if (!g.G) return 1;
    const size_t lds = group_lds_bytes(m);
    const int per_cu = g.G == 16 ? occupancy_group16(g.NC, lds) : occupancy_group64(g.NC, lds);
    int dev = 0, cus = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    return std::max(1, per_cu) * std::max(1, cus);
}

}  // namespace rk
