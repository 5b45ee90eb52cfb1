/*
 * CPU FP64 oracle for batched constant-pressure Radau IIA chemical kinetics.
 *
 * TEST INFRASTRUCTURE ONLY.  This code is the independent reference that the
 * HIP library is checked against; it shares no code, header, table or constant
 * generator with that library.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load it.
 *
 * What it computes (the paper delegates the equations to pyJac and Radau IIA
 * to Hairer & Wanner; Sec. 2.1):
 *   - the adiabatic constant-pressure reactor in (T, Y_1..Y_K): species source
 *     terms from mass-action kinetics with Arrhenius forward rates, reverse
 *     rates from NASA-7 equilibrium constants, third-body and Troe falloff
 *     modifiers (Sec. 2.1, "constant-pressure, mass-fraction-based");
 *   - the exact analytical Jacobian of that right-hand side;
 *   - the 3-stage, order-5 Radau IIA method with simplified Newton, embedded
 *     error estimate and adaptive step control, tolerances atol/rtol
 *     (Sec. 2.1), one independent IVP per state, OpenMP over states
 *     (Sec. 3, CPU runs).
 * Everything is double precision; built with -ffp-contract=off.
 */
#ifndef RK_ORACLE_H
#define RK_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define OR_RU 8.314462618     /* J/(mol K) */
#define OR_PATM 101325.0      /* Pa */

typedef struct {
    int kind;                 /* 0 elementary, 1 third body, 2 Troe falloff */
    int nr, np;
    int reac[2], prod[2];
    double A, b, Ea;          /* forward (high-pressure limit for kind 2) */
    double A0, b0, Ea0;       /* kind 2 low-pressure limit */
    double troe[4];           /* a, T***, T*, T** */
    double *eff;              /* [K] collision efficiencies (kind 1, 2), else NULL */
} or_reaction;

typedef struct {
    int K, R, E;
    double *W;                /* [K] kg/mol */
    int *comp;                /* [K*E] */
    double *Tlow, *Tmid, *Thigh;
    double *alow, *ahigh;     /* [K*7] */
    or_reaction *rx;          /* [R] */
} or_mech;

/* integrator status per state */
enum { OR_OK = 0, OR_STEP_LIMIT = 1, OR_H_UNDERFLOW = 2, OR_NONFINITE = 3 };

typedef struct {
    int kmax;                 /* max Newton iterations per step (default 7) */
    double kappa;             /* Newton stopping constant; <= 0 -> default rule */
    double h0;                /* initial step; <= 0 -> min(dt, 1e-6 s) */
    int nmax;                 /* step attempts limit (default 100000) */
    int untransformed;        /* 1: solve the 3N x 3N Newton system directly */
    int isothermal;           /* 1: dT/dt = 0 (used only to relax burnt templates) */
    int fd_jac;               /* 1: first-order forward-difference Jacobian (Sec. 3.4) */
} or_opts;

typedef struct {
    int32_t status;
    int32_t nstep;            /* step attempts (Newton started) */
    int32_t naccept, nreject, nnewton, nnewtfail, nfev, njev, nlu;
    int32_t warm;             /* warm start: 0 none, 1 kept, 2 Newton failed -> cold restart */
    double h_first;           /* size of the first accepted step */
} or_result;

int  or_mech_load(const char *path, or_mech **out);
void or_mech_free(or_mech *m);
int  or_mech_dims(const or_mech *m, int *K, int *R, int *E);

/* First-order forward-difference Jacobian of the chemistry right-hand side
 * (the alternative to the analytical Jacobian compared in Sec. 3.4), with
 * CVODE's dense difference-quotient increments: column j uses
 * inc_j = max(sqrt(u) |y_j|, m w_j), w_j = atol + rtol |y_j|,
 * m = 1000 |h| u N ||f(y)||_w (||.||_w the weighted RMS norm; m = 1 when
 * f(y) = 0).  J is row-major N x N; f0 = f(y). */
void or_jac_fd(const or_mech *m, const double *y, double P, const double *f0, double h, double atol, double rtol,
               double *J);
/* the same rule applied to f_i(y) = sum_j A_ij y_j^2 (tests of the increments) */
void or_jac_fd_quadratic(int N, const double *A, const double *y, double h, double atol, double rtol, double *J);

/* Rodas3 (Sandu et al.; four-stage L-stable Rosenbrock method of order 3 with
 * an embedded order-2 estimate), the semi-implicit method the paper's
 * conclusions recommend (Sec. 4): adaptive integration of n states over
 * [0, dt] (same layout, options and result records as or_integrate_batch;
 * nnewton = nnewtfail = 0), fixed steps, one step of a linear system, and
 * its coefficient table (gamma, a and c 4x4 strictly lower, m, e). */
int or_integrate_rodas3(const or_mech *m, int64_t n, double dt, const double *y_in, double *y_out, double atol,
                        double rtol, const or_opts *o, or_result *res, int nthreads);
int or_rodas3_fixed_steps(const or_mech *m, const double *y_row, double dt, int nsteps, double *y_out);
int or_rodas3_linear_step(int N, const double *M, const double *y0, double h, double *y1);
void or_rodas3_table(double *gamma, double *a, double *c, double *m, double *e);

/* default options */
void or_default_opts(or_opts *o);

/* thermo of every species at T: cp/R, h/(RT), s/R  (each [K]) */
void or_thermo(const or_mech *m, double T, double *cp, double *h, double *s);

/* rates of progress q[R] and production rates wdot[K] (mol/m^3/s) at (T, Y, P) */
void or_rates(const or_mech *m, const double *TY, double P, double *q, double *wdot);
/* as or_rates, also returning the forward and reverse parts qf, qr (q = qf - qr) */
void or_rates2(const or_mech *m, const double *TY, double P, double *q, double *wdot, double *qf, double *qr);

/* right-hand side f[N] of y = (T, Y_1..Y_K) at pressure P */
void or_rhs(const or_mech *m, const double *y, double P, double *f);

/* analytical Jacobian, row-major N x N: J[i*N+j] = d f_i / d y_j */
void or_jac(const or_mech *m, const double *y, double P, double *J);

/* complex-step Jacobian (step 1e-30 i on each column) */
void or_jac_cs(const or_mech *m, const double *y, double P, double *J);

/* Radau IIA constants: A[9] (row-major), c[3], b[3], gamma, alpha, beta of
 * eig(A^-1), T[9], Tinv[9] (T^-1 A^-1 T = [[g,0,0],[0,a,-b],[0,b,a]]), d[3] */
void or_radau_constants(double *A, double *c, double *b, double *ev, double *T, double *Tinv, double *d);

/* batch integration over [0, dt]; rows are (T, Y_1..Y_K, P), row-major
 * [n][K+2].  h0 may be NULL (per-state initial steps otherwise). */
int or_integrate_batch(const or_mech *m, int64_t n, double dt, const double *y_in, double *y_out,
                       double atol, double rtol, const or_opts *o, const double *h0,
                       or_result *res, int nthreads);

/* as or_integrate_batch, also returning the stage increments Z = (z1, z2, z3)
 * of each state's first accepted step in zfirst[n][3N] (may be NULL) */
int or_integrate_batch2(const or_mech *m, int64_t n, double dt, const double *y_in, double *y_out,
                        double atol, double rtol, const or_opts *o, const double *h0,
                        or_result *res, int nthreads, double *zfirst);

/* as or_integrate_batch2, with an optional warm start per state: the first
 * step attempt uses step size hw[i] (<= 0: the default rule) and Newton
 * starting values zw[i][3N] (NULL: zero).  If Newton does not converge on
 * that attempt the state restarts exactly as a cold start (default initial
 * step, zero starting values, controller memory reset).  hw or zw may be NULL;
 * a state is warm if hw[i] > 0 or zw is given. */
int or_integrate_batch3(const or_mech *m, int64_t n, double dt, const double *y_in, double *y_out,
                        double atol, double rtol, const or_opts *o, const double *hw, const double *zw,
                        or_result *res, int nthreads, double *zfirst);

/* Radau IIA on the linear system y' = M y (row-major N x N), for the
 * closed-form checks.  Accepted step sizes are written to hrec (capacity cap). */
int or_integrate_linear(int N, const double *M, const double *y0, double dt, double atol, double rtol,
                        const or_opts *o, double *y_out, or_result *res, double *hrec, int cap);

/* One Radau step of fixed size h on the chemistry RHS with Newton iterated to
 * convergence (no error control); used for fixed-step refinement studies. */
int or_fixed_steps(const or_mech *m, const double *y_row, double dt, int nsteps, double *y_out);

#ifdef __cplusplus
}
#endif
#endif
