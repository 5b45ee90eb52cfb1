// Internal types of the rkchem library (host and device).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>
#include <string>
#include <utility>
#include <vector>

#include "../../include/rkchem.h"

namespace rk {

constexpr double kRu = 8.314462618;     // J/(mol K)
constexpr double kPatm = 101325.0;      // Pa
constexpr int kWave = 64;

// Reaction parameter record (doubles per reaction).
enum RPar { P_A = 0, P_B, P_EAR, P_A0, P_B0, P_EA0R, P_TA, P_T3, P_T1, P_T2, P_DNU, P_NPAR = 12 };

// Jacobian-column list entry of species m: e = reaction << 5 | slots holding
// m (bits 0-3: r0, r1, p0, p1) | 16 if m's efficiency there is not 1;
// em1 = that efficiency - 1 (0 unless bit 4).  16 bytes: one load per entry.
struct JlEnt {
    double em1;
    int e, pad;
};

// Third-body list entry: efficiency - 1 of species k.
struct TbEnt {
    double em1;
    int k, pad;
};

// Device view of a mechanism.  Reaction/species tables are read with
// wavefront-uniform indices, so the loads are scalar (constant cache).
struct DevMech {
    int K, R, N, n3b;
    int nsp;               // entries of sp_rx
    const double *W;       // [K]  kg/mol
    const double *invW;    // [K]
    const double *Tmid;    // [K]
    const double *thermo;  // [K][2][7]: low range then high range
    const int4 *rsp;       // [R]  reactant slots r0, r1, product slots p0, p1 (-1 = empty)
    const int *rinfo;      // [R]  kind | nr << 4 | np << 8 | (third-body row + 1) << 12
    const double *rpar;    // [R][P_NPAR]
    const double4 *rhead;  // [R]: A, b, E_a/R, sum of nu (the parameters every reaction reads)
    const double *eff;     // [n3b][K] collision efficiencies
    const int *sp_off;     // [K+1] species -> reaction list offsets
    const int2 *sp_rx;     // [sp_off[K]] (reaction, net stoichiometric coefficient)
    // species m -> the reactions whose rate depends on C_m other than through
    // the mixture total of a third body: m fills a reactant or product slot,
    // or m has a non-default collision efficiency (reaction order)
    const int *jl_off;     // [K+1]
    const JlEnt *jl;       // [jl_off[K]]
    // third-body row b -> the species with a non-default efficiency:
    // [M]_b = sum_k C_k + sum over the list of (efficiency - 1) C_k
    const int *tb_off;     // [n3b+1]
    const TbEnt *tb;       // (efficiency - 1, species), 16 bytes: one load per entry
    const int2 *tbr;       // [R]: a reaction's range in tb (empty for elementary reactions)
};

// Radau IIA constants and integrator parameters (computed on the host).
struct RadauParams {
    double dt, atol, rtol, kappa, h0;
    int kmax, nmax;
    int pred_use;            // bit 1: predicted first step size, bit 2: predicted stage values
    int tile;                // queue entries a group (block) takes per atomic grab
    int fd_jac;              // first-order forward-difference Jacobian instead of the analytical one
    int method;              // 0: Radau IIA, 1: Rodas3 (Rosenbrock; wave variant)
    int force_fb;            // FP32 variants: take the fallback at the first accepted step (tests)
    int fp64_solves;         // block variant: FP64-accurate solves (three refinement sweeps) from the start
    double g, a, b;          // eigenvalues of A^-1: g, a +- i b
    double T[9], Ti[9];      // T^-1 A^-1 T = [[g,0,0],[0,a,-b],[0,b,a]] (row-major)
    double c1, c2;           // collocation nodes (c3 = 1)
    double d[3];             // error-estimate weights
};

// Per-lane scratch layout (element offsets; element e of a lane lives at
// base[e * 64], consecutive lanes in consecutive doubles).
struct LaneLayout {
    int y, f0, sc, Z, W, F, dW, Zs, ev, vv, tmp, sc2;
    int J, E1, E2r, E2i, p1, p2;
    int C, cp, h, s, dcp, wdot, dwdT, sS;
    int total;
};

// Per-state counters written by the integrators: [kNumCounters][n].
enum Counter { C_STATUS = 0, C_NSTEP, C_NACC, C_NREJ, C_NNEWT, C_NNFAIL, C_NFEV, C_NJEV, C_NLU, C_FLAGS, kNumCounters };
// status a mixed-precision pass gives a state it hands to the FP64 pass
constexpr int kStatusFallback = 4;
// C_FLAGS bits
constexpr int kFlagFp32Fallback = 1, kFlagPredKept = 2, kFlagPredFallback = 4;

LaneLayout lane_layout(int K);

// Launchers (rk_kernels.hip).
hipError_t launch_rhs(const DevMech &m, int64_t n, const double *y, double *f, double *scratch, hipStream_t st);
hipError_t launch_jac(const DevMech &m, int64_t n, const double *y, double *J, double *scratch, hipStream_t st);
hipError_t launch_radau_lane(const DevMech &m, const RadauParams &p, int64_t n, const double *yin, double *yout,
                             double *scratch, int32_t *counters, const int *order, hipStream_t st);
hipError_t launch_gather_head(const double *src, int64_t n, int64_t m, int rows, double *dst, hipStream_t st);
// cost binning: proxy key per state, counting sort into a queue order (costliest bins first)
constexpr int kProxyLanes = 65536;
size_t proxy_scratch_doubles(int K);
hipError_t launch_binning(const DevMech &m, int64_t n, const double *yin, double dt, double atol, double rtol,
                          int nbins, int *bins, int *order, int *hist, double *scratch, hipStream_t st);
size_t lane_scratch_doubles(int K, int64_t n);
// group-cooperative variant (16 lanes per state for N <= 16, a wavefront per
// state for N <= 56), persistent work queue
bool group_supported(int N);
int group_states_per_block(int N);
hipError_t launch_radau_group(const DevMech &m, const RadauParams &p, int64_t n, const double *yin, double *yout,
                              int32_t *counters, int *queue, int *fb_list, const int *order, const double *pred,
                              bool mixed, int grid, hipStream_t st);
int group_max_blocks(const DevMech &m);
// per-family entry points (rk_group16.hip, rk_group64.hip): NC = register columns
hipError_t launch_group16(int NC, bool fp32, const DevMech &m, const RadauParams &p, int64_t n, const double *yin,
                          double *yout, int32_t *cnt, int *queue, const int *order, const int *work_n,
                          const double *pred, int grid, hipStream_t st);
hipError_t launch_group64(int NC, bool fp32, const DevMech &m, const RadauParams &p, int64_t n, const double *yin,
                          double *yout, int32_t *cnt, int *queue, const int *order, const int *work_n,
                          const double *pred, int grid, hipStream_t st);
hipError_t lu_solve_group16(int NC, bool fp32, int N, int64_t n, double gh, double ah, double bh, const double *J,
                            const double *sc, const double *b, double *x, hipStream_t st);
hipError_t lu_solve_group64(int NC, bool fp32, int N, int64_t n, double gh, double ah, double bh, const double *J,
                            const double *sc, const double *b, double *x, hipStream_t st);
// factor and solve E1 = gh I - J, E2 = (ah + i bh) I - J with the group
// kernels' routines (kernel-level test entry; N <= 56)
hipError_t launch_lu_solve(int N, bool fp32, int64_t n, double gh, double ah, double bh, const double *J,
                           const double *sc, const double *b, double *x, hipStream_t st);
int occupancy_group16(int NC, size_t lds);
int occupancy_group64(int NC, size_t lds);
hipError_t launch_zero_i32(int32_t *p, int64_t n, hipStream_t st);
// Rodas3 (Rosenbrock) with the wavefront kernels' building blocks (rk_ros.hip)
hipError_t launch_rodas3_group(const DevMech &m, const RadauParams &p, int64_t n, const double *yin, double *yout,
                               int32_t *counters, int *queue, const int *order, int grid, hipStream_t st);
// block-cooperative variant (rk_block.hip): one 512-lane block per state,
// FP32 factors in registers, J in a per-block slab of global memory
bool block_supported(int N);
size_t block_lds_bytes(const DevMech &m);
size_t block_slab_doubles(int N, int grid);
int block_max_blocks(const DevMech &m);
hipError_t launch_radau_block(const DevMech &m, const RadauParams &p, int64_t n, const double *yin, double *yout,
                              int32_t *counters, int *queue, const int *order, double *slab, const double *pred,
                              int grid, hipStream_t st);
size_t group_lds_bytes(const DevMech &m);   // per block

// Device buffers of one integration call (rk_api.cpp): the handle's
// workspaces, or the static array of the no-allocation entry (rk_noalloc.hip).
struct Work {
    int32_t *counters = nullptr;   // [kNumCounters][n]
    int *queue = nullptr;          // four queue heads / counts
    int *fb_list = nullptr;        // [n] states handed from the FP32 to the FP64 pass
    int *bins = nullptr, *order = nullptr, *hist = nullptr;
    double *proxy = nullptr;       // proxy-key evaluation scratch
    double *lane = nullptr;        // lane-kernel working set
    double *slab = nullptr;        // block-kernel Jacobian slabs
    bool allow_predictor = false;
};

// Predictor network (rk_mlp.hip): FP32 masters, BF16 copy used in products.
struct Mlp {
    std::vector<int> dims;
    float *params = nullptr, *grads = nullptr, *adam_m = nullptr, *adam_v = nullptr, *part = nullptr;
    uint16_t *wbf = nullptr;
    std::vector<float *> acts, pre, dacts;   // per layer: post-activation, pre-activation, gradient
    int64_t cap_b = 0;
    int steps = 0;
    ~Mlp();
    int64_t count() const;
    hipError_t init(const std::vector<int> &d);
    hipError_t ensure_batch(int64_t B);
    hipError_t refresh_bf16(hipStream_t st);
    hipError_t forward(int64_t B, const float *x, hipStream_t st);
    hipError_t backward(int64_t B, const float *x, const float *t, const float *mask, const float *wout,
                        float inv_count, float *loss, hipStream_t st);
    hipError_t adam(float lr, hipStream_t st);
};

// Loaded predictor for one global step size (device copies of the
// standardisation and the network) and its per-call buffers.
struct Predictor {
    double dt = 0.0;
    int K = 0;
    std::vector<int> dims;
    float *in_shift = nullptr, *in_scale = nullptr, *out_shift = nullptr, *out_scale = nullptr;
    Mlp *net = nullptr;
    float *X = nullptr;       // [n][K+2] features
    double *pred = nullptr;   // [n][3N+2] stage values, first step, step attempts
    int64_t cap = 0;
    ~Predictor();
    hipError_t ensure(int64_t n);
};

hipError_t launch_predictor(Predictor &pr, int64_t n, const double *yin, double dt, double atol, double rtol,
                            int nbins, int *bins, hipStream_t st);
hipError_t launch_sort_bins(const int *bins, int64_t n, int nbins, int *order, int *hist, hipStream_t st);

}  // namespace rk

// Handle (host side).
struct rk_mech {
    int K = 0, R = 0, E = 0, n3b = 0;
    std::string name;
    // host copies
    std::vector<double> W, Tmid, thermo, rpar, eff;
    std::vector<double4> rhead;
    std::vector<int> rinfo, comp;
    std::vector<int4> rsp;
    std::vector<int> sp_off;
    std::vector<int2> sp_rx;
    std::vector<int> jl_off, tb_off;
    std::vector<rk::JlEnt> jl;
    std::vector<rk::TbEnt> tb;
    std::vector<int2> tbr;
    // device
    rk::DevMech dev{};
    void *dev_block = nullptr;
    int device = 0;
    // options
    int variant = -1;          // -1 auto, 0 lane, 1 wave, 2 mixed (FP32 factors), 3 block (N > 56)
    int kmax = 7, nmax = 100000;
    int force_fb = 0, fp64_solves = 0;
    int fd_jac = 0;            // Jacobian by forward differences (lane and wave variants)
    int method = 0;            // 0 Radau IIA, 1 Rodas3
    double kappa = 0.0, h0 = 0.0;
    // workspace of the last call
    double *scratch = nullptr;
    size_t scratch_cap = 0;    // doubles
    int32_t *counters = nullptr;
    int64_t counters_cap = 0;  // states
    int *queue = nullptr;      // work-queue heads and fallback count (device)
    int *fb_list = nullptr;    // states handed from the mixed to the FP64 pass (device)
    int64_t fb_cap = 0;
    // cost binning
    int nbins = 0;             // 0: queue in input order
    int *bins = nullptr, *order = nullptr, *hist = nullptr;
    int64_t bin_cap = 0;
    double *proxy_scratch = nullptr;
    // autotuner: chosen (bins, grid percent) per dt, trial buffers
    bool autotune = false;
    int pred_use = 3;
    struct Tuned {
        double dt;
        int bins, grid_pct, tile;
        float ms;
    };
    std::vector<Tuned> tuned;
    int grid_pct = 100;
    int tile = 1;              // queue entries per grab
    int last_tile = 1;
    double *tune_buf = nullptr;
    size_t tune_cap = 0;
    int last_nbins = 0, last_grid = 0;
    std::vector<rk::Predictor *> predictors;   // one per global step size
    int group_blocks = 0;      // resident blocks of the group kernel (cached)
    int block_blocks = 0;      // resident blocks of the block kernel (cached)
    double *block_slab = nullptr;   // per-block Jacobian slabs of the block kernel
    size_t block_slab_cap = 0;      // doubles
    int64_t last_n = 0;
    int32_t *last_counters = nullptr;   // counters of the last call (handle or static array)
    int *last_order = nullptr;          // its queue order (nullptr: input order)
    hipStream_t last_stream = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    bool have_run = false;
};

// integration call shared by radau_integrate (w == nullptr) and the
// no-allocation entry (w = its static buffers)
int rk_integrate_common(rk_mech *m, int64_t n, double dt, const double *yin, double *yout, double atol, double rtol,
                        void *stream, const rk::Work *w);
// record an error message for rk_last_error (thread-local) and return code
int rk_fail(int code, const char *msg);
