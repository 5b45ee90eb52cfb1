/*
 * rkchem — batched constant-pressure Radau IIA chemical-kinetics integration
 * on AMD Instinct MI355X (gfx950).
 *
 * The library integrates many independent thermochemical states over one
 * global time step, as in the paper's GPU study of stiff kinetics integrators
 * (Curtis, Niemeyer & Sung, Sec. 2.1-2.2): each state is a constant-pressure,
 * adiabatic, homogeneous reactor in (T, Y_1..Y_K); the integrator is the
 * three-stage, fifth-order Radau IIA method with simplified Newton iterations
 * on an analytical Jacobian, an embedded error estimate and adaptive step
 * control under absolute/relative tolerances (Sec. 2.1).  One call integrates
 * every state from t = 0 to t = dt.
 *
 * All compute runs in the library's HIP kernels on the current HIP device.
 * Pointers named `d_*` are device pointers the caller owns (e.g. from torch);
 * the library owns mechanism handles and its internal workspaces.
 *
 * Error handling: functions return 0 on success or a negative RK_E* code; the
 * message of the last failing call on the calling thread is returned by
 * rk_last_error().  Per-state integration failures are not errors: they are
 * reported as status codes through stats_get().
 */
#ifndef RKCHEM_H
#define RKCHEM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* return codes */
#define RK_OK 0
#define RK_EIO (-1)      /* mechanism file cannot be opened */
#define RK_EPARSE (-2)   /* mechanism file malformed */
#define RK_EINVAL (-3)   /* invalid argument or mechanism that fails validation */
#define RK_EHIP (-4)     /* HIP runtime error */
#define RK_ENOMEM (-5)   /* device allocation failed */

/* per-state status codes */
#define RK_ST_OK 0           /* reached t = dt */
#define RK_ST_STEP_LIMIT 1   /* more step attempts than the limit (option nmax) */
#define RK_ST_H_UNDERFLOW 2  /* step size too small to advance t (0.1 h <= u t) */
#define RK_ST_NONFINITE 3    /* input state not finite, T <= 0 or P <= 0; y_out = y_in */

typedef struct rk_mech rk_mech;

/* Statistics of the last radau_integrate call on a handle. */
typedef struct rk_stats {
    int64_t n_states;
    int64_t steps;            /* step attempts (Newton started), summed over states */
    int64_t accepted, rejected;
    int64_t newton_iters, newton_fail;
    int64_t f_evals, jac_evals, lu_factor;
    int64_t n_failed;         /* states whose status is not RK_ST_OK */
    int32_t max_steps, min_steps;
    /* divergence D = 1 - sum_i d_i / (w max_i d_i) over groups of w consecutive
     * states (d_i = step attempts of state i), the paper's Eq. (3); histogram
     * of D in 20 bins of width 0.05, for w = 64 (one wavefront) and w = 32 */
    int64_t d_hist64[20];
    int64_t d_hist32[20];
    double d_mean64, d_mean32;
    double kernel_ms;         /* device time of the last call (HIP events) */
    int64_t fp32_fallback;    /* states the mixed variant re-ran with FP64 factors
                                 (block variant: switched to FP64-accurate solves) */
    int32_t nbins_used;       /* cost bins of the work queue (0: input order) */
    int32_t grid_used;        /* blocks launched for the integrator */
    int64_t predictor_kept;     /* states whose predicted first step converged */
    int64_t predictor_fallback; /* states restarted cold after the prediction failed */
    /* D (Eq. 3) over groups of 64 consecutive entries of the work-queue order
     * the integrator drew states in (equal to d_hist64 when no bins are used) */
    int64_t d_hist64_queue[20];
    double d_mean64_queue;
    int32_t tile_used;        /* queue entries a group (block) took per atomic grab */
    int32_t reserved;
} rk_stats;

/* mech_load — read a mechanism file and upload it to the current device.
 * Defines the source terms the integrator works on: the paper integrates
 * constant-pressure, mass-fraction-based reactor equations whose rates and
 * analytical Jacobian come from a chemical kinetic model of species
 * thermodynamics and reversible reactions (Sec. 2.1; test models Sec. 2.2).
 *   path: text mechanism (species with element counts and molar masses,
 *         two-range NASA-7 thermodynamics, reversible reactions with 1-2
 *         species per side: elementary, third-body, Troe falloff; SI units).
 *   out:  receives a handle owned by the library; release with mech_free.
 * Validates element balance of every reaction, NASA-7 continuity of cp, h, s
 * at T_mid (relative 1e-6) and positive molar masses.
 * Returns RK_OK, RK_EIO, RK_EPARSE, RK_EINVAL or RK_EHIP/RK_ENOMEM. */
int mech_load(const char *path, rk_mech **out);

/* mech_free — release a handle and its device memory (NULL is a no-op).
 * Synchronises the handle's last stream first. */
void mech_free(rk_mech *mech);

/* mech_dims — number of species K and reactions R of a handle. */
int mech_dims(const rk_mech *mech, int32_t *K, int32_t *R);

/* radau_integrate — integrate n_states independent states over [0, dt]:
 * the paper's batched problem (Sec. 2.1, Sec. 2.2): every state is an
 * independent constant-pressure adiabatic reactor advanced over one global
 * time step by the three-stage fifth-order Radau IIA method with adaptive
 * steps under the absolute and relative tolerances of Sec. 2.1 (paper:
 * atol 1e-10, rtol 1e-6); global steps of 1e-6 s and 1e-4 s in Sec. 3.
 *   d_y_in, d_y_out: device arrays of (K+2)*n_states doubles, component-major
 *       (struct of arrays): element (c, i) at c*n_states + i, c = 0 temperature
 *       [K], c = 1..K mass fractions Y_k, c = K+1 pressure [Pa].  Pressure is
 *       copied through unchanged.  d_y_out may equal d_y_in.
 *   atol, rtol: tolerances of the error and Newton norms (paper: 1e-10, 1e-6).
 *   stream: hipStream_t to enqueue on (NULL = default stream).  The call
 *       returns after enqueueing; results are ready when the stream is.
 * One call in flight per handle: a second call on the same handle must not
 * start before the first one's stream work has been ordered before it.
 * Returns RK_EINVAL for dt <= 0 or not finite, atol < 0, rtol <= 0,
 * n_states < 0, a NULL or host-memory state array with n_states > 0, or a
 * variant, method or Jacobian option (radau_set_option) that does not fit the
 * mechanism or each other; RK_ENOMEM / RK_EHIP on runtime failures.
 * Failures of individual states go to their status (stats_get); a failed
 * state keeps its last accepted solution in d_y_out. */
int radau_integrate(rk_mech *mech, int64_t n_states, double dt, const double *d_y_in, double *d_y_out,
                    double atol, double rtol, void *stream);

/* radau_integrate_noalloc — radau_integrate for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the same kernels and results as
 * radau_integrate with the handle's "wave" or "mixed" variant in input order
 * ("auto" runs "wave"), but every scratch buffer of the call (queue heads,
 * FP32-to-FP64 hand-back list, per-state counters) lives in one static device
 * array of 11.5 MB that each device holds for the life of the process;
 * nothing is allocated, by the library or anything it calls.  The caller
 * still passes the state arrays (as radau_integrate).  The predictor, cost
 * bins and autotuner of the handle are not used.
 * Limits: n_states <= 262144 (RK_EINVAL beyond); K + 1 <= 56 and variant
 * "auto", "wave" or "mixed" (RK_EINVAL otherwise).
 * Sharing: every call on a device uses that device's one array, so calls
 * that overlap on a device (any handles, any streams) race and must be
 * ordered by the caller; stats_get after this call reads the array, which
 * the next no-allocation call on the device overwrites. */
int radau_integrate_noalloc(rk_mech *mech, int64_t n_states, double dt, const double *d_y_in, double *d_y_out,
                            double atol, double rtol, void *stream);

/* stats_get — statistics of the last radau_integrate on this handle,
 * including the thread-divergence measure D of Eq. (3) (Sec. 3.3) over
 * groups of 64 and 32 consecutive states of the input order and over the
 * groups of 64 consecutive states of the executed work-queue order.
 * Synchronises that call's stream.  per_state_steps and per_state_status are
 * optional HOST arrays of n_states int32 (step attempts, status code). */
int stats_get(rk_mech *mech, rk_stats *out, int32_t *per_state_steps, int32_t *per_state_status);

/* radau_set_option — integrator options of a handle (strings):
 *   "variant"  "auto" (default: "wave" when K + 1 <= 56, "block" when
 *              K + 1 <= 153, else "lane") |
 *              "lane" (one lane per state, the paper's per-thread pattern;
 *              any K; the matrices live in global memory, so large
 *              mechanisms are slow) |
 *              "wave" (a group of lanes cooperates on one state, the paper's
 *              per-block pattern: 16 lanes for K + 1 <= 16, a whole wavefront
 *              for K + 1 <= 56; LU factors in registers; persistent work
 *              queue) |
 *              "mixed" (as "wave" with the iteration matrices equilibrated and
 *              factored in FP32; every solve takes one refinement step
 *              against the FP64 matrices; source terms, residuals, error
 *              estimate and control in FP64; a state whose Newton iteration
 *              diverges twice in a row after its first accepted step is
 *              re-integrated from its initial value with FP64 factors).
 *              "wave" and "mixed" return RK_EINVAL for K + 1 > 56.
 *              "block" (57 <= K + 1 <= 153, R + third-body rows up to about
 *              2000: a block of 512 lanes
 *              cooperates on one state, the per-block pattern for large
 *              mechanisms (Sec. 1.2, Sec. 4); iteration matrices equilibrated
 *              and factored in FP32 (the complex one in registers, three
 *              lanes per row; the real one in LDS), J in FP64 in device
 *              memory; every solve refined against the FP64
 *              matrices until the last correction is below 1e-8 in the error
 *              weights (one to four sweeps; a correction larger than the
 *              one before it ends the sweeps unapplied); a state whose
 *              Newton iteration
 *              diverges twice in a row after its first accepted step continues
 *              with three to six sweeps per solve and
 *              counts in fp32_fallback; predictor as for "wave";
 *              persistent work queue).
 *              RK_EINVAL outside those sizes.
 *   "binning"  number of cost bins (0..64, default 0): one source-term
 *              evaluation per state gives the key ||dt f(y0)|| (RMS in the
 *              error weights); states are queued costliest bin first
 *   "grid_pct" share of the resident capacity launched for the persistent
 *              kernels (10..100, default 100)
 *   "tile"     queue entries a group (block) takes per atomic grab (1..64,
 *              default 1); results do not depend on it
 *   "autotune" "1": on the first call per dt with at least 4096 states (1024
 *              for "block"), time the integrator on the first min(n, S)
 *              states (S = 32768 for K + 1 <= 16, 8192 for K + 1 <= 56, 1024
 *              for "block") and keep the fastest schedule: bins
 *              {0, 8, 16, 32} x grid {100, 75, 50} % ("block": bins {0, 16},
 *              grid 100 %; "lane": bins only) at tile 1, then tile {2, 4} at
 *              the best of those; the choice is reported by stats_get
 *              (nbins_used, grid_used, tile_used); this call blocks the host;
 *              "0": forget the choices
 *   "predictor" path of a predictor file (network widths K+2 -> ... -> 3(K+1)+2,
 *              standardisation, parameters) trained for one global step size;
 *              calls with that dt and the "wave", "mixed" or "block" variant
 *              start each state's first step from the predicted step size
 *              (rounded to dt times a power of two) and stage values and keep
 *              them only if Newton converges on that attempt, else restart the
 *              state exactly as a cold start; with "binning" (or "autotune")
 *              the bin key becomes the predicted step count.  A file for
 *              another K is refused (RK_EINVAL).  "none" removes all
 *              predictors.
 *   "predictor_use" "both" (default) | "h0" (predicted first step size only,
 *              stage values start at zero) | "z0" (predicted stage values with
 *              the default first step size) | "bins" (no warm start: the
 *              network only keys the cost bins by its predicted step counts,
 *              so every state's result is bitwise that of a cold start)
 *   "method"   "radau" (default) | "rodas3": Rosenbrock integration instead
 *              of Radau IIA, the semi-implicit direction the paper's
 *              conclusions recommend (Sec. 4): Rodas3 (Sandu et al.; four
 *              stages, order 3, embedded order 2, L-stable), one real FP64
 *              factorisation of 1/(h gamma) I - J per step size, Jacobian at
 *              every new y; variant "wave" (or "auto" for K + 1 <= 56) with
 *              the analytical Jacobian, RK_EINVAL otherwise
 *   "jacobian" "analytical" (default) | "fd": first-order forward-difference
 *              Jacobian (the alternative Sec. 3.4 compares with the analytical
 *              one): column j from (f(y + inc_j e_j) - f(y)) / inc_j with
 *              CVODE's dense difference-quotient increments
 *              inc_j = max(sqrt(u) |y_j|, 1000 |h| u N ||f(y)||_w w_j),
 *              w_j = atol + rtol |y_j|: N more source-term evaluations per
 *              Jacobian; variants "lane" and "wave" (RK_EINVAL otherwise)
 *   "force_fallback" "0" (default) | "1": test switch of the FP32 variants'
 *              fallbacks: "mixed" hands every state to the FP64 pass at its
 *              first accepted step; "block" switches every state to
 *              FP64-accurate solves after its first accepted step
 *   "block_solves" "fp32_refined" (default) | "fp64_accurate": the block
 *              variant refines every solve at least three times from the first step
 *              (FP64-accurate solves from FP32 factors and FP64 residuals
 *              wherever cond(E) * 2^-24 is well below 1; counted in
 *              fp32_fallback)
 *   "kmax"     max Newton iterations per step (default 7)
 *   "kappa"    Newton stopping constant (0 = default: max(10u/rtol, min(0.03, rtol^0.5)))
 *   "nmax"     step-attempt limit per state (default 100000)
 *   "h0"       initial step size in seconds (default min(dt, 1e-6))
 * Returns RK_EINVAL for an unknown key or a malformed value. */
int radau_set_option(rk_mech *mech, const char *key, const char *value);

/* rk_last_error — message of the last failing call on this thread ("" if none). */
const char *rk_last_error(void);

/* ---- kernel-level entry points used by the parity tests ------------------ */

/* rk_dbg_rhs — source terms f(y) for n states: d_y as in radau_integrate,
 * d_f receives (K+1)*n doubles, component-major (dT/dt, dY_k/dt). */
int rk_dbg_rhs(rk_mech *mech, int64_t n, const double *d_y, double *d_f, void *stream);

/* rk_dbg_jacobian — analytical Jacobian for n states: d_J receives
 * (K+1)^2 * n doubles, element (r, c) of state i at (r*(K+1) + c)*n + i. */
int rk_dbg_jacobian(rk_mech *mech, int64_t n, const double *d_y, double *d_J, void *stream);

/* rk_dbg_lu_solve — the integrator's own formation, LU factorisation with
 * partial pivoting and substitutions of the two Radau IIA iteration matrices
 * (the real and complex systems of the transformed simplified Newton
 * iteration that the paper's Radau IIA solves, Sec. 2.1), applied to given
 * Jacobians: x1 = E1^-1 b1 and x2 + i x3 = E2^-1 (b2 + i b3), with
 * E1 = g/h I - J and E2 = (a + i b)/h I - J (g, a +- i b the eigenvalues of
 * the inverse Radau IIA coefficient matrix).  K + 1 <= 56 (wavefront kernels).
 *   fp32: 0 = FP64 factors; 1 = FP32 factors of the matrices equilibrated with
 *         the error weights d_sc, solved without refinement (the factors' own
 *         accuracy).
 *   d_J: (K+1)^2 * n doubles as rk_dbg_jacobian; d_sc: (K+1) * n error
 *   weights (component-major, used by fp32 = 1); d_b, d_x: 3 (K+1) n doubles,
 *   element (v, r) of system i at (v (K+1) + r) n + i, v = 0 real right-hand
 *   side / solution, v = 1, 2 real and imaginary parts of the complex one.
 * RK_EINVAL for n < 0, h <= 0, K + 1 > 56 or non-device arrays. */
int rk_dbg_lu_solve(rk_mech *mech, int64_t n, int fp32, double h, const double *d_J, const double *d_sc,
                    const double *d_b, double *d_x, void *stream);

/* ---- learned stage/step predictor network --------------------------------
 * A multilayer perceptron with widths dims[0] -> ... -> dims[n-1], GELU
 * (x Phi(x), erf form) on hidden layers, linear output.  Parameters are FP32
 * masters used as BF16 (round-to-nearest-even) in every product, with FP32
 * accumulation.  Flat parameter order: per layer W [d_out][d_in] row-major,
 * then b [d_out].  Device arrays (d_*) are row-major [B][width] float32.
 * Loss: sum_b mask_b sum_o w_o (y_bo - t_bo)^2 * inv_count.  The forward
 * pass runs on the matrix cores (FP32 MFMA with the BF16-valued weights). */
typedef struct rk_mlp rk_mlp;

/* rk_mlp_create — allocate a network on the current device (2..8 widths,
 * each 1..4096); parameters start at zero.  RK_EINVAL / RK_ENOMEM. */
int rk_mlp_create(int32_t n_dims, const int32_t *dims, rk_mlp **out);
void rk_mlp_free(rk_mlp *mlp);
int64_t rk_mlp_param_count(const rk_mlp *mlp);
/* host float32 arrays of rk_mlp_param_count entries; set also resets Adam */
int rk_mlp_set_params(rk_mlp *mlp, const float *host_params, int64_t count);
int rk_mlp_get_params(const rk_mlp *mlp, float *host_params, int64_t count);
/* d_y[B][dims[n-1]] = network(d_x[B][dims[0]]) */
int rk_mlp_forward(rk_mlp *mlp, int64_t batch, const float *d_x, float *d_y, void *stream);
/* loss (d_loss, one float) and its gradient (d_grad, param_count floats, may
 * be NULL) at the current parameters; inv_count = 1 / sum(mask); no update.
 * Synchronises the stream (reads the mask). */
int rk_mlp_grads(rk_mlp *mlp, int64_t batch, const float *d_x, const float *d_t, const float *d_mask,
                 const float *d_wout, float *d_grad, float *d_loss, void *stream);
/* one Adam step (beta 0.9, 0.999, eps 1e-8, learning rate lr) on the loss */
int rk_mlp_train_step(rk_mlp *mlp, int64_t batch, const float *d_x, const float *d_t, const float *d_mask,
                      const float *d_wout, float inv_count, float lr, float *d_loss, void *stream);
const char *rk_mlp_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
