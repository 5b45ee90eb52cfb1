// Instantiations of the group kernel with 16 lanes per state (four states per wavefront):
// register columns NC = 14 and 16 (N <= NC), FP64 and FP32 factors.
#include <algorithm>

#include "rk_group_impl.h"

namespace rk {

hipError_t launch_group16(int NC, bool fp32, const DevMech &m, const RadauParams &p, int64_t n, const double *yin,
                          double *yout, int32_t *cnt, int *queue, const int *order, const int *work_n,
                          const double *pred, int grid, hipStream_t st) {
    if (NC == 14) {
        if (fp32) launch_one<float, 16, 14>(m, p, n, yin, yout, cnt, queue, order, work_n, pred, grid, st);
        else launch_one<double, 16, 14>(m, p, n, yin, yout, cnt, queue, order, work_n, pred, grid, st);
        return hipGetLastError();
    }
    if (NC == 16) {
        if (fp32) launch_one<float, 16, 16>(m, p, n, yin, yout, cnt, queue, order, work_n, pred, grid, st);
        else launch_one<double, 16, 16>(m, p, n, yin, yout, cnt, queue, order, work_n, pred, grid, st);
        return hipGetLastError();
    }
    return hipErrorInvalidValue;
}

hipError_t lu_solve_group16(int NC, bool fp32, int N, int64_t n, double gh, double ah, double bh, const double *J,
                            const double *sc, const double *b, double *x, hipStream_t st) {
    if (NC == 14) {
        if (fp32) launch_lu_solve_one<float, 16, 14>(N, n, gh, ah, bh, J, sc, b, x, st);
        else launch_lu_solve_one<double, 16, 14>(N, n, gh, ah, bh, J, sc, b, x, st);
        return hipGetLastError();
    }
    if (NC == 16) {
        if (fp32) launch_lu_solve_one<float, 16, 16>(N, n, gh, ah, bh, J, sc, b, x, st);
        else launch_lu_solve_one<double, 16, 16>(N, n, gh, ah, bh, J, sc, b, x, st);
        return hipGetLastError();
    }
    return hipErrorInvalidValue;
}

int occupancy_group16(int NC, size_t lds) {
    if (NC == 14) return std::min(occupancy_one<double, 16, 14>(lds), occupancy_one<float, 16, 14>(lds));
    if (NC == 16) return std::min(occupancy_one<double, 16, 16>(lds), occupancy_one<float, 16, 16>(lds));
    return 1;
}

}  // namespace rk
