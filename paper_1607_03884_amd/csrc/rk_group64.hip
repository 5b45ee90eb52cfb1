// Instantiations of the group kernel with one wavefront per state:
// register columns NC = 54 and 56 (N <= NC), FP64 and FP32 factors.
#include <algorithm>

#include "rk_group_impl.h"

namespace rk {

hipError_t launch_group64(int NC, bool fp32, const DevMech &m, const RadauParams &p, int64_t n, const double *yin,
                          double *yout, int32_t *cnt, int *queue, const int *order, const int *work_n,
                          const double *pred, int grid, hipStream_t st) {
    if (NC == 54) {
        if (fp32) launch_one<float, 64, 54>(m, p, n, yin, yout, cnt, queue, order, work_n, pred, grid, st);
        else launch_one<double, 64, 54>(m, p, n, yin, yout, cnt, queue, order, work_n, pred, grid, st);
        return hipGetLastError();
    }
    if (NC == 56) {
        if (fp32) launch_one<float, 64, 56>(m, p, n, yin, yout, cnt, queue, order, work_n, pred, grid, st);
        else launch_one<double, 64, 56>(m, p, n, yin, yout, cnt, queue, order, work_n, pred, grid, st);
        return hipGetLastError();
    }
    return hipErrorInvalidValue;
}

hipError_t lu_solve_group64(int NC, bool fp32, int N, int64_t n, double gh, double ah, double bh, const double *J,
                            const double *sc, const double *b, double *x, hipStream_t st) {
    if (NC == 54) {
        if (fp32) launch_lu_solve_one<float, 64, 54>(N, n, gh, ah, bh, J, sc, b, x, st);
        else launch_lu_solve_one<double, 64, 54>(N, n, gh, ah, bh, J, sc, b, x, st);
        return hipGetLastError();
    }
    if (NC == 56) {
        if (fp32) launch_lu_solve_one<float, 64, 56>(N, n, gh, ah, bh, J, sc, b, x, st);
        else launch_lu_solve_one<double, 64, 56>(N, n, gh, ah, bh, J, sc, b, x, st);
        return hipGetLastError();
    }
    return hipErrorInvalidValue;
}

int occupancy_group64(int NC, size_t lds) {
    if (NC == 54) return std::min(occupancy_one<double, 64, 54>(lds), occupancy_one<float, 64, 54>(lds));
    if (NC == 56) return std::min(occupancy_one<double, 64, 56>(lds), occupancy_one<float, 64, 56>(lds));
    return 1;
}

}  // namespace rk
