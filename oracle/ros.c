/* Oracle Rosenbrock integrator (test infrastructure only; see oracle.h).
 *
 * The paper's conclusions (Sec. 4) recommend non-exponential Rosenbrock
 * solvers as the next semi-implicit method for GPU chemical kinetics.  This
 * file restates one published L-stable Rosenbrock method, Rodas3 of Sandu et
 * al. (four stages, order 3, embedded order 2, gamma = 1/2), in the
 * transformed form of Hairer & Wanner (Solving ODEs II, Sec. IV.7):
 *   (1/(h gamma) I - J) u_i = f(y + sum_{j<i} a_ij u_j) + sum_{j<i} (c_ij / h) u_j,
 *   y_new = y + sum_i m_i u_i,   error estimate sum_i e_i u_i = u_4,
 * with J the Jacobian at y (one real factorisation per step size, no Newton
 * iteration).  Step control (the usual Rosenbrock controller; readings noted
 * in the design notes): err = RMS of u_4 / (atol + rtol max(|y|, |y_new|)),
 * accept when err <= 1 (a non-finite err rejects), h_new = h min(6, max(0.2,
 * 0.9 err^(-1/3))), no growth
 * right after a rejection, J kept after a rejection (same y); the initial
 * step, the last-step rule and the failure rules are the Radau oracle's. */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include "oracle.h"

#define UROUND 2.220446049250313e-16

/* Rodas3: strictly lower-triangular a and c, stage weights m, error weights e */
static const double RG = 0.5;
static const double RA[4][4] = {{0, 0, 0, 0}, {0, 0, 0, 0}, {2, 0, 0, 0}, {2, 0, 1, 0}};
static const double RC[4][4] = {{0, 0, 0, 0}, {4, 0, 0, 0}, {1, -1, 0, 0}, {1, -1, -8.0 / 3.0, 0}};
static const double RM[4] = {2, 0, 1, 1};
static const double RE[4] = {0, 0, 0, 1};

void or_rodas3_table(double *gamma, double *a, double *c, double *m, double *e) {
    *gamma = RG;
    for (int i = 0; i < 4; ++i) {
        for (int j = 0; j < 4; ++j) { a[i * 4 + j] = RA[i][j]; c[i * 4 + j] = RC[i][j]; }
        m[i] = RM[i];
        e[i] = RE[i];
    }
}

/* dense LU with partial pivoting, row-major, and its solve */
static void lu(int n, double *a, int *piv) {
    for (int k = 0; k < n; ++k) {
        int p = k;
        for (int i = k + 1; i < n; ++i) if (fabs(a[i * n + k]) > fabs(a[p * n + k])) p = i;
        piv[k] = p;
        if (p != k) for (int j = 0; j < n; ++j) { double t = a[k * n + j]; a[k * n + j] = a[p * n + j]; a[p * n + j] = t; }
        for (int i = k + 1; i < n; ++i) {
            double l = a[i * n + k] / a[k * n + k];
            a[i * n + k] = l;
            for (int j = k + 1; j < n; ++j) a[i * n + j] -= l * a[k * n + j];
        }
    }
}

static void lus(int n, const double *a, const int *piv, double *b) {
    for (int k = 0; k < n; ++k) { int p = piv[k]; if (p != k) { double t = b[k]; b[k] = b[p]; b[p] = t; } }
    for (int i = 0; i < n; ++i) for (int j = 0; j < i; ++j) b[i] -= a[i * n + j] * b[j];
    for (int i = n - 1; i >= 0; --i) {
        for (int j = i + 1; j < n; ++j) b[i] -= a[i * n + j] * b[j];
        b[i] /= a[i * n + i];
    }
}

typedef struct {
    int N;
    void (*f)(void *ctx, const double *y, double *out);
    void (*jac)(void *ctx, const double *y, double *J);
    void *ctx;
} rproblem;

/* One Rodas3 step of size h from y (J = Jacobian at y, f0 = f(y)): the new
 * value into yn, the error-estimate vector into err_v.  Work: 5 N + N*N. */
static void rodas3_step(const rproblem *pb, const double *y, const double *f0, const double *J, double h,
                        double *yn, double *err_v, double *E, int *piv, double *u, double *w, int *nfev) {
    const int N = pb->N;
    for (int i = 0; i < N * N; ++i) E[i] = -J[i];
    for (int i = 0; i < N; ++i) E[i * N + i] += 1.0 / (h * RG);
    lu(N, E, piv);
    double *yi = w, *fi = w + N;
    for (int s = 0; s < 4; ++s) {
        /* stage argument y + sum a_sj u_j; f at y for the stages with no a terms */
        int at_y = 1;
        for (int j = 0; j < s; ++j) if (RA[s][j] != 0.0) at_y = 0;
        if (at_y) {
            memcpy(fi, f0, sizeof(double) * N);
        } else {
            for (int c = 0; c < N; ++c) {
                double v = y[c];
                for (int j = 0; j < s; ++j) v += RA[s][j] * u[j * N + c];
                yi[c] = v;
            }
            pb->f(pb->ctx, yi, fi);
            ++*nfev;
        }
        double *us = u + s * N;
        for (int c = 0; c < N; ++c) {
            double v = fi[c];
            for (int j = 0; j < s; ++j) v += RC[s][j] / h * u[j * N + c];
            us[c] = v;
        }
        lus(N, E, piv, us);
    }
    for (int c = 0; c < N; ++c) {
        double v = y[c], e = 0.0;
        for (int s = 0; s < 4; ++s) { v += RM[s] * u[s * N + c]; e += RE[s] * u[s * N + c]; }
        yn[c] = v;
        err_v[c] = e;
    }
}

/* Adaptive Rodas3 over [0, dt] in place; counters as the Radau oracle's
 * (nnewton and nnewtfail stay 0: no Newton iteration). */
static int ros_core(const rproblem *pb, double dt, double *y, double atol, double rtol, const or_opts *o,
                    or_result *res) {
    const int N = pb->N;
    memset(res, 0, sizeof *res);
    const int nmax = o->nmax > 0 ? o->nmax : 100000;
    double *J = malloc(sizeof(double) * N * N * 2);
    double *E = J + N * N;
    int *piv = malloc(sizeof(int) * N);
    double *buf = malloc(sizeof(double) * 10 * N);
    double *f0 = buf, *yn = f0 + N, *ev = yn + N, *u = ev + N, *w = u + 4 * N;
    for (int i = 0; i < N; ++i) if (!isfinite(y[i])) { res->status = OR_NONFINITE; goto done; }
    double t = 0.0;
    double h = o->h0 > 0 ? o->h0 : fmin(dt, 1e-6);
    int last = 0, reject = 0, need_j = 1, first = 1;
    if (t + 1.0001 * h >= dt) { h = dt - t; last = 1; }
    pb->f(pb->ctx, y, f0);
    res->nfev++;
    for (;;) {
        if (res->nstep >= nmax) { res->status = OR_STEP_LIMIT; break; }
        if (0.1 * h <= UROUND * t || h < 1e-300) { res->status = OR_H_UNDERFLOW; break; }
        if (need_j) { pb->jac(pb->ctx, y, J); res->njev++; need_j = 0; }
        res->nstep++;
        rodas3_step(pb, y, f0, J, h, yn, ev, E, piv, u, w, &res->nfev);
        res->nlu++;
        double s2 = 0.0;
        for (int i = 0; i < N; ++i) {
            const double sc = atol + rtol * fmax(fabs(y[i]), fabs(yn[i]));
            s2 += (ev[i] / sc) * (ev[i] / sc);
        }
        /* a stage that left the domain of f (e.g. T <= 0) gives a non-finite
         * estimate: the step is rejected (no Newton iteration catches it) */
        const double en = sqrt(s2 / N);
        double err = isfinite(en) ? fmax(en, 1e-10) : 1e300;
        double fac = fmin(6.0, fmax(0.2, 0.9 * pow(err, -1.0 / 3.0)));
        if (err <= 1.0) {
            res->naccept++;
            if (first) { res->h_first = h; first = 0; }
            memcpy(y, yn, sizeof(double) * N);
            t = last ? dt : t + h;
            if (last) break;
            pb->f(pb->ctx, y, f0);
            res->nfev++;
            need_j = 1;
            double hn = h * fac;
            if (reject) hn = fmin(hn, h);
            reject = 0;
            if (t + 1.0001 * hn >= dt) { h = dt - t; last = 1; } else { h = hn; }
        } else {
            res->nreject++;
            reject = 1;
            last = 0;
            h = h * fac;
        }
    }
done:
    free(J); free(piv); free(buf);
    return res->status;
}

typedef struct { const or_mech *m; double P; } rchem;
static void rchem_f(void *c, const double *y, double *f) { rchem *x = c; or_rhs(x->m, y, x->P, f); }
static void rchem_j(void *c, const double *y, double *J) { rchem *x = c; or_jac(x->m, y, x->P, J); }

int or_integrate_rodas3(const or_mech *m, int64_t n, double dt, const double *y_in, double *y_out, double atol,
                        double rtol, const or_opts *o, or_result *res, int nthreads) {
    const int K = m->K, N = K + 1, S = K + 2;
    or_opts dflt;
    if (!o) { or_default_opts(&dflt); o = &dflt; }
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    #pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < n; ++i) {
        const double *row = y_in + i * S;
        double *out = y_out + i * S;
        int bad = !(row[0] > 0.0) || !(row[K + 1] > 0.0);
        for (int c = 0; c < S; ++c) bad = bad || !isfinite(row[c]);
        if (bad) {
            memset(&res[i], 0, sizeof res[i]);
            res[i].status = OR_NONFINITE;
            memcpy(out, row, sizeof(double) * S);
            continue;
        }
        double *y = malloc(sizeof(double) * N);
        memcpy(y, row, sizeof(double) * N);
        rchem cx = { m, row[K + 1] };
        rproblem pb = { N, rchem_f, rchem_j, &cx };
        ros_core(&pb, dt, y, atol, rtol, o, &res[i]);
        memcpy(out, y, sizeof(double) * N);
        out[K + 1] = row[K + 1];
        free(y);
    }
    return 0;
}

/* nsteps fixed Rodas3 steps of size dt / nsteps (convergence studies) */
int or_rodas3_fixed_steps(const or_mech *m, const double *y_row, double dt, int nsteps, double *y_out) {
    const int N = m->K + 1;
    rchem cx = { m, y_row[m->K + 1] };
    rproblem pb = { N, rchem_f, rchem_j, &cx };
    double *J = malloc(sizeof(double) * N * N * 2), *E = J + N * N;
    int *piv = malloc(sizeof(int) * N);
    double *buf = malloc(sizeof(double) * 10 * N);
    double *y = buf, *f0 = y + N, *yn = f0 + N, *ev = yn + N, *u = ev + N, *w = u + 4 * N;
    memcpy(y, y_row, sizeof(double) * N);
    int nfev = 0;
    const double h = dt / nsteps;
    for (int k = 0; k < nsteps; ++k) {
        pb.f(pb.ctx, y, f0);
        pb.jac(pb.ctx, y, J);
        /* w needs 2 N; u 4 N; the stage buffers share buf's tail */
        rodas3_step(&pb, y, f0, J, h, yn, ev, E, piv, u, w, &nfev);
        memcpy(y, yn, sizeof(double) * N);
    }
    memcpy(y_out, y, sizeof(double) * N);
    free(J); free(piv); free(buf);
    return 0;
}

/* one Rodas3 step of y' = M y (N x N row-major) from y0 with step h */
typedef struct { int N; const double *M; } rlin;
static void rlin_f(void *c, const double *y, double *f) {
    const rlin *x = c;
    for (int i = 0; i < x->N; ++i) {
        double s = 0.0;
        for (int j = 0; j < x->N; ++j) s += x->M[i * x->N + j] * y[j];
        f[i] = s;
    }
}

int or_rodas3_linear_step(int N, const double *M, const double *y0, double h, double *y1) {
    double *J = malloc(sizeof(double) * N * N * 2), *E = J + N * N;
    int *piv = malloc(sizeof(int) * N);
    double *buf = malloc(sizeof(double) * 8 * N);
    double *f0 = buf, *ev = f0 + N, *u = ev + N, *w = u + 4 * N;
    rlin lx = { N, M };
    rproblem pb = { N, rlin_f, NULL, &lx };
    memcpy(J, M, sizeof(double) * N * N);
    rlin_f(&lx, y0, f0);
    int nfev = 0;
    rodas3_step(&pb, y0, f0, J, h, y1, ev, E, piv, u, w, &nfev);
    free(J); free(piv); free(buf);
    return 0;
}
