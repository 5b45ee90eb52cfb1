/* Oracle Radau IIA integrator (test infrastructure only; see oracle.h).
 *
 * The paper uses the three-stage, fifth-order Radau IIA method with its
 * built-in adaptive stepping and Jacobian reuse (Sec. 2.1) and cites Hairer &
 * Wanner, Solving ODEs II, for the algorithm.  This file restates that
 * published algorithm:
 *   stage equations  z_i = h sum_j a_ij f(y0 + z_j), y1 = y0 + z_3;
 *   simplified Newton with the Jacobian J frozen at y0, either on the full
 *   3N x 3N system (I - h A (x) J) dZ = -Z + h (A (x) I) F(Z), or, after the
 *   change of basis W = (T^-1 (x) I) Z with T^-1 A^-1 T = [[g,0,0],[0,a,-b],[0,b,a]],
 *   as one real N x N system with E1 = (g/h) I - J and one complex one with
 *   E2 = ((a + i b)/h) I - J;
 *   embedded error estimate err = E1^-1 [f(y0) + (d1 z1 + d2 z2 + d3 z3)/h];
 *   step-size control with the predictive (Gustafsson) controller, and the
 *   Jacobian / factorisation reuse rules.
 * Every quantity the paper leaves open is given a reading in the design notes;
 * the numbered readings are repeated at the point of use below. */
#define _GNU_SOURCE
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include "oracle.h"

void or_rhs_iso(const or_mech *m, const double *y, double P, double *f);
void or_jac_iso(const or_mech *m, const double *y, double P, double *J);

#define UROUND 2.220446049250313e-16

/* ------------------------------------------------------------------------- */
/* dense LU with partial pivoting (row-major), real and complex               */
/* ------------------------------------------------------------------------- */
static void lu_r(int n, double *a, int *piv) {
    for (int k = 0; k < n; ++k) {
        int p = k;
        for (int i = k + 1; i < n; ++i) if (fabs(a[i * n + k]) > fabs(a[p * n + k])) p = i;
        piv[k] = p;
        if (p != k) for (int j = 0; j < n; ++j) { double t = a[k * n + j]; a[k * n + j] = a[p * n + j]; a[p * n + j] = t; }
        double d = a[k * n + k];
        for (int i = k + 1; i < n; ++i) {
            double l = a[i * n + k] / d;
            a[i * n + k] = l;
            for (int j = k + 1; j < n; ++j) a[i * n + j] -= l * a[k * n + j];
        }
    }
}

static void lus_r(int n, const double *a, const int *piv, double *b) {
    for (int k = 0; k < n; ++k) { int p = piv[k]; if (p != k) { double t = b[k]; b[k] = b[p]; b[p] = t; } }
    for (int i = 0; i < n; ++i) for (int j = 0; j < i; ++j) b[i] -= a[i * n + j] * b[j];
    for (int i = n - 1; i >= 0; --i) {
        for (int j = i + 1; j < n; ++j) b[i] -= a[i * n + j] * b[j];
        b[i] /= a[i * n + i];
    }
}

static void lu_c(int n, double complex *a, int *piv) {
    for (int k = 0; k < n; ++k) {
        int p = k;
        for (int i = k + 1; i < n; ++i) if (cabs(a[i * n + k]) > cabs(a[p * n + k])) p = i;
        piv[k] = p;
        if (p != k) for (int j = 0; j < n; ++j) { double complex t = a[k * n + j]; a[k * n + j] = a[p * n + j]; a[p * n + j] = t; }
        double complex d = a[k * n + k];
        for (int i = k + 1; i < n; ++i) {
            double complex l = a[i * n + k] / d;
            a[i * n + k] = l;
            for (int j = k + 1; j < n; ++j) a[i * n + j] -= l * a[k * n + j];
        }
    }
}

static void lus_c(int n, const double complex *a, const int *piv, double complex *b) {
    for (int k = 0; k < n; ++k) { int p = piv[k]; if (p != k) { double complex t = b[k]; b[k] = b[p]; b[p] = t; } }
    for (int i = 0; i < n; ++i) for (int j = 0; j < i; ++j) b[i] -= a[i * n + j] * b[j];
    for (int i = n - 1; i >= 0; --i) {
        for (int j = i + 1; j < n; ++j) b[i] -= a[i * n + j] * b[j];
        b[i] /= a[i * n + i];
    }
}

/* ------------------------------------------------------------------------- */
/* Radau IIA (s = 3) coefficients                                             */
/* ------------------------------------------------------------------------- */
typedef struct {
    double A[9], c[3], b[3], g, a, bt, T[9], Ti[9], d[3];
} rconst;

static void inv3(const double *m, double *r) {
    double det = m[0] * (m[4] * m[8] - m[5] * m[7]) - m[1] * (m[3] * m[8] - m[5] * m[6])
               + m[2] * (m[3] * m[7] - m[4] * m[6]);
    r[0] = (m[4] * m[8] - m[5] * m[7]) / det; r[1] = (m[2] * m[7] - m[1] * m[8]) / det;
    r[2] = (m[1] * m[5] - m[2] * m[4]) / det; r[3] = (m[5] * m[6] - m[3] * m[8]) / det;
    r[4] = (m[0] * m[8] - m[2] * m[6]) / det; r[5] = (m[2] * m[3] - m[0] * m[5]) / det;
    r[6] = (m[3] * m[7] - m[4] * m[6]) / det; r[7] = (m[1] * m[6] - m[0] * m[7]) / det;
    r[8] = (m[0] * m[4] - m[1] * m[3]) / det;
}

/* null vector of a rank-2 complex 3x3 matrix: cross product of the pair of rows
 * with the largest cross product */
static void null3(const double complex *B, double complex *v) {
    double best = -1.0;
    for (int p = 0; p < 3; ++p) for (int q = p + 1; q < 3; ++q) {
        const double complex *r = &B[p * 3], *s = &B[q * 3];
        double complex w[3] = { r[1] * s[2] - r[2] * s[1], r[2] * s[0] - r[0] * s[2], r[0] * s[1] - r[1] * s[0] };
        double nw = cabs(w[0]) + cabs(w[1]) + cabs(w[2]);
        if (nw > best) { best = nw; v[0] = w[0]; v[1] = w[1]; v[2] = w[2]; }
    }
}

static void radau_consts(rconst *k) {
    double s6 = sqrt(6.0);
    double A[9] = { (88.0 - 7.0 * s6) / 360.0, (296.0 - 169.0 * s6) / 1800.0, (-2.0 + 3.0 * s6) / 225.0,
                    (296.0 + 169.0 * s6) / 1800.0, (88.0 + 7.0 * s6) / 360.0, (-2.0 - 3.0 * s6) / 225.0,
                    (16.0 - s6) / 36.0, (16.0 + s6) / 36.0, 1.0 / 9.0 };
    memcpy(k->A, A, sizeof A);
    k->c[0] = (4.0 - s6) / 10.0; k->c[1] = (4.0 + s6) / 10.0; k->c[2] = 1.0;
    k->b[0] = A[6]; k->b[1] = A[7]; k->b[2] = A[8];
    /* eigenvalues of A: one real 1/g, a complex pair; those of A^-1: g, a +- i b */
    double c81 = cbrt(81.0), c9 = cbrt(9.0);
    k->g = 30.0 / (6.0 + c81 - c9);
    double al = (12.0 - c81 + c9) / 60.0, be = sqrt(3.0) * (c81 + c9) / 60.0, nr = al * al + be * be;
    k->a = al / nr;
    k->bt = be / nr;
    double Ai[9];
    inv3(A, Ai);
    /* T = [v1, Re v, Im v] with A^-1 v1 = g v1 and A^-1 v = (a - i b) v */
    double complex B[9], v[3];
    for (int i = 0; i < 9; ++i) B[i] = Ai[i];
    for (int i = 0; i < 3; ++i) B[i * 4] -= k->g;
    null3(B, v);
    double v1[3] = { creal(v[0]), creal(v[1]), creal(v[2]) };
    for (int i = 0; i < 9; ++i) B[i] = Ai[i];
    for (int i = 0; i < 3; ++i) B[i * 4] -= (k->a - k->bt * I);
    null3(B, v);
    for (int i = 0; i < 3; ++i) {
        k->T[i * 3 + 0] = v1[i];
        k->T[i * 3 + 1] = creal(v[i]);
        k->T[i * 3 + 2] = cimag(v[i]);
    }
    inv3(k->T, k->Ti);
    /* error-estimate weights */
    k->d[0] = -(13.0 + 7.0 * s6) / 3.0;
    k->d[1] = (-13.0 + 7.0 * s6) / 3.0;
    k->d[2] = -1.0 / 3.0;
}

void or_radau_constants(double *A, double *c, double *b, double *ev, double *T, double *Tinv, double *d) {
    rconst k;
    radau_consts(&k);
    memcpy(A, k.A, sizeof k.A); memcpy(c, k.c, sizeof k.c); memcpy(b, k.b, sizeof k.b);
    ev[0] = k.g; ev[1] = k.a; ev[2] = k.bt;
    memcpy(T, k.T, sizeof k.T); memcpy(Tinv, k.Ti, sizeof k.Ti); memcpy(d, k.d, sizeof k.d);
}

void or_default_opts(or_opts *o) {
    o->kmax = 7; o->kappa = 0.0; o->h0 = 0.0; o->nmax = 100000; o->untransformed = 0; o->isothermal = 0;
    o->fd_jac = 0;
}

/* ------------------------------------------------------------------------- */
/* generic problem interface                                                  */
/* ------------------------------------------------------------------------- */
typedef struct {
    int N;
    void (*f)(void *ctx, const double *y, double *out);
    void (*jac)(void *ctx, const double *y, double *J);
    void *ctx;
} problem;

/* First-order forward differences of f around y (Sec. 3.4's finite-difference
 * Jacobian), increments by CVODE's dense difference-quotient rule: the larger
 * of sqrt(u) |y_j| and a floor proportional to the step size, the weighted
 * norm of f(y) and the error weight of component j.  f0 = f(y); work: 2 N. */
static void fd_jacobian(const problem *pb, const double *y, const double *f0, double h, double atol, double rtol,
                        double *J, double *work) {
    const int N = pb->N;
    double *yp = work, *fp = work + N;
    double fn = 0.0;
    for (int i = 0; i < N; ++i) {
        const double w = atol + rtol * fabs(y[i]);
        fn += (f0[i] / w) * (f0[i] / w);
    }
    fn = sqrt(fn / N);
    const double minc = fn != 0.0 ? 1000.0 * fabs(h) * UROUND * N * fn : 1.0;
    memcpy(yp, y, sizeof(double) * N);
    for (int j = 0; j < N; ++j) {
        const double w = atol + rtol * fabs(y[j]);
        const double inc = fmax(sqrt(UROUND) * fabs(y[j]), minc * w);
        yp[j] = y[j] + inc;
        pb->f(pb->ctx, yp, fp);
        yp[j] = y[j];
        for (int i = 0; i < N; ++i) J[i * N + j] = (fp[i] - f0[i]) / inc;
    }
}

/* scaled RMS norm over n entries with weights sc (period N) */
static double rms(const double *v, const double *sc, int n, int N) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) { double t = v[i] / sc[i % N]; s += t * t; }
    return sqrt(s / n);
}

static int finite_vec(const double *v, int n) {
    for (int i = 0; i < n; ++i) if (!isfinite(v[i])) return 0;
    return 1;
}

/* Integrate y over [0, dt] in place. */
static int radau_core(const problem *pb, double dt, double *y, double atol, double rtol, const or_opts *o,
                      double h0, int warm, const double *zw, or_result *res, double *hrec, int cap,
                      double *zfirst) {
    const int N = pb->N, N3 = 3 * N;
    rconst k;
    radau_consts(&k);
    memset(res, 0, sizeof *res);
    const int kmax = o->kmax > 0 ? o->kmax : 7;
    const int nmax = o->nmax > 0 ? o->nmax : 100000;
    /* (reading) Newton stopping constant: max(10 u / rtol, min(0.03, sqrt(rtol))) */
    const double kappa = o->kappa > 0 ? o->kappa : fmax(10.0 * UROUND / rtol, fmin(0.03, sqrt(rtol)));
    const double safe = 0.9, facl = 5.0, facr = 0.125, thet = 1e-3;

    size_t nd = (size_t)N * N;
    double *J = malloc(sizeof(double) * nd);
    double *E1 = malloc(sizeof(double) * (o->untransformed ? 9 * nd : nd) + sizeof(double) * nd);
    double *Ebig = E1 + nd;                                   /* 3N x 3N when untransformed */
    double complex *E2 = malloc(sizeof(double complex) * nd);
    int *p1 = malloc(sizeof(int) * (N3 + 2 * N));
    int *p2 = p1 + N, *pb3 = p2 + N;
    double *w = malloc(sizeof(double) * (20 * N + 2 * N3));
    double *f0 = w, *sc = f0 + N, *Z = sc + N, *W = Z + N3, *F = W + N3, *dZ = F + N3, *dW = dZ + N3;
    double *Zs = dW + N3, *e = Zs + N3, *v = e + N, *ytmp = v + N, *rhs = ytmp + N;
    double complex *cz = malloc(sizeof(double complex) * N);
    double *fdw = malloc(sizeof(double) * 2 * N);

    if (!finite_vec(y, N)) { res->status = OR_NONFINITE; goto done; }

    double t = 0.0;
    const double hcold = o->h0 > 0 ? o->h0 : fmin(dt, 1e-6);
    double h = h0 > 0 ? h0 : hcold;
    int last = 0;
    if (t + 1.0001 * h >= dt) { h = dt - t; last = 1; }
    pb->f(pb->ctx, y, f0); res->nfev++;
    for (int i = 0; i < N; ++i) sc[i] = atol + rtol * fabs(y[i]);
    int first = 1, reject = 0, jac_fresh = 0, nacc = 0;
    double eta = 1.0, theta = 1.0, hacc = h, erracc = 1e-2, hlast = h;
    enum { NEW_JAC, NEW_LU, SAME } action = NEW_JAC;

    for (;;) {
        if (action == NEW_JAC) {
            if (o->fd_jac) {
                fd_jacobian(pb, y, f0, h, atol, rtol, J, fdw);
                res->nfev += N;
            } else {
                pb->jac(pb->ctx, y, J);
            }
            res->njev++;
            jac_fresh = 1;
            action = NEW_LU;
        }
        if (action == NEW_LU) {
            for (size_t i = 0; i < nd; ++i) { E1[i] = -J[i]; E2[i] = -J[i]; }
            for (int i = 0; i < N; ++i) { E1[i * N + i] += k.g / h; E2[i * N + i] += (k.a + k.bt * I) / h; }
            lu_r(N, E1, p1);
            lu_c(N, E2, p2);
            if (o->untransformed) {
                /* I - h A (x) J */
                for (int bi = 0; bi < 3; ++bi) for (int bj = 0; bj < 3; ++bj)
                    for (int i = 0; i < N; ++i) for (int j = 0; j < N; ++j)
                        Ebig[(size_t)(bi * N + i) * N3 + bj * N + j] =
                            (bi == bj && i == j ? 1.0 : 0.0) - h * k.A[bi * 3 + bj] * J[i * N + j];
                lu_r(N3, Ebig, pb3);
            }
            res->nlu++;
        }
        action = SAME;
        if (res->nstep >= nmax) { res->status = OR_STEP_LIMIT; break; }
        /* (reading) step too small: it no longer advances t (Hairer-Wanner code criterion) */
        if (0.1 * h <= UROUND * t || h < 1e-300) { res->status = OR_H_UNDERFLOW; break; }
        res->nstep++;

        /* starting values: zero on the first step, otherwise the previous
         * step's collocation cubic q (q(0)=0, q(c_i)=z_i) evaluated at the new
         * stage abscissae, tau = 1 + c_i h/h_old, minus q(1) = z_3 */
        if (first) {
            if (warm && zw) memcpy(Z, zw, sizeof(double) * N3);
            else memset(Z, 0, sizeof(double) * N3);
        } else {
            double tn[4] = { 0.0, k.c[0], k.c[1], 1.0 };
            for (int i = 0; i < 3; ++i) {
                double tau = 1.0 + k.c[i] * h / hlast;
                double L[4];
                for (int mm = 1; mm < 4; ++mm) {
                    L[mm] = 1.0;
                    for (int nn = 0; nn < 4; ++nn) if (nn != mm) L[mm] *= (tau - tn[nn]) / (tn[mm] - tn[nn]);
                }
                for (int c = 0; c < N; ++c)
                    Z[i * N + c] = L[1] * Zs[c] + L[2] * Zs[N + c] + L[3] * Zs[2 * N + c] - Zs[2 * N + c];
            }
        }
        for (int i = 0; i < 3; ++i) for (int c = 0; c < N; ++c)
            W[i * N + c] = k.Ti[i * 3] * Z[c] + k.Ti[i * 3 + 1] * Z[N + c] + k.Ti[i * 3 + 2] * Z[2 * N + c];

        /* simplified Newton */
        eta = pow(fmax(eta, UROUND), 0.8);
        int converged = 0, newt = 0, diverged = 0;
        double dn_old = 1.0;
        for (int it = 1; it <= kmax; ++it) {
            for (int i = 0; i < 3; ++i) {
                for (int c = 0; c < N; ++c) ytmp[c] = y[c] + Z[i * N + c];
                pb->f(pb->ctx, ytmp, F + i * N);
            }
            res->nfev += 3;
            if (o->untransformed) {
                for (int i = 0; i < 3; ++i) for (int c = 0; c < N; ++c) {
                    double acc = -Z[i * N + c];
                    for (int j = 0; j < 3; ++j) acc += h * k.A[i * 3 + j] * F[j * N + c];
                    dZ[i * N + c] = acc;
                }
                lus_r(N3, Ebig, pb3, dZ);
            } else {
                for (int c = 0; c < N; ++c) {
                    double G[3];
                    for (int i = 0; i < 3; ++i)
                        G[i] = k.Ti[i * 3] * F[c] + k.Ti[i * 3 + 1] * F[N + c] + k.Ti[i * 3 + 2] * F[2 * N + c];
                    dW[c] = G[0] - k.g / h * W[c];
                    double r2 = G[1] - (k.a * W[N + c] - k.bt * W[2 * N + c]) / h;
                    double r3 = G[2] - (k.bt * W[N + c] + k.a * W[2 * N + c]) / h;
                    cz[c] = r2 + r3 * I;
                }
                lus_r(N, E1, p1, dW);
                lus_c(N, E2, p2, cz);
                for (int c = 0; c < N; ++c) { dW[N + c] = creal(cz[c]); dW[2 * N + c] = cimag(cz[c]); }
                for (int i = 0; i < 3; ++i) for (int c = 0; c < N; ++c)
                    dZ[i * N + c] = k.T[i * 3] * dW[c] + k.T[i * 3 + 1] * dW[N + c] + k.T[i * 3 + 2] * dW[2 * N + c];
            }
            res->nnewton++;
            newt = it;
            double dn = rms(dZ, sc, N3, N);
            if (!isfinite(dn)) { diverged = 1; break; }
            if (it >= 2) {
                double th = dn / dn_old;
                theta = th;
                if (th >= 0.99) { diverged = 1; break; }
                eta = th / (1.0 - th);
                /* predicted error after the remaining iterations */
                if (pow(th, kmax - it) / (1.0 - th) * dn > kappa) { diverged = 1; break; }
            }
            dn_old = fmax(dn, UROUND);
            for (int i = 0; i < N3; ++i) Z[i] += dZ[i];
            if (!o->untransformed) for (int i = 0; i < N3; ++i) W[i] += dW[i];
            else for (int i = 0; i < 3; ++i) for (int c = 0; c < N; ++c)
                W[i * N + c] = k.Ti[i * 3] * Z[c] + k.Ti[i * 3 + 1] * Z[N + c] + k.Ti[i * 3 + 2] * Z[2 * N + c];
            if (eta * dn <= kappa) { converged = 1; break; }
        }
        if (!converged && warm) {
            /* the warm start did not converge: restart as a cold start */
            res->nnewtfail++;
            res->warm = 2;
            warm = 0;
            h = hcold;
            last = 0;
            if (t + 1.0001 * h >= dt) { h = dt - t; last = 1; }
            eta = 1.0;
            theta = 1.0;
            hacc = h;
            erracc = 1e-2;
            hlast = h;
            action = NEW_LU;
            continue;
        }
        if (warm) { res->warm = 1; warm = 0; }
        if (!converged) {
            /* (reading) Newton failure: halve h and redo; fresh J if stale */
            res->nnewtfail++;
            h *= 0.5;
            reject = 1;
            last = 0;
            action = jac_fresh ? NEW_LU : NEW_JAC;
            (void)diverged;
            continue;
        }

        /* embedded error estimate */
        for (int c = 0; c < N; ++c) {
            double dz = (k.d[0] * Z[c] + k.d[1] * Z[N + c] + k.d[2] * Z[2 * N + c]) / h;
            v[c] = dz;
            e[c] = f0[c] + dz;
            double y1 = y[c] + Z[2 * N + c];
            rhs[c] = atol + rtol * fmax(fabs(y[c]), fabs(y1));
        }
        lus_r(N, E1, p1, e);
        double err = fmax(rms(e, rhs, N, N), 1e-10);
        if (err >= 1.0 && (first || reject)) {
            for (int c = 0; c < N; ++c) ytmp[c] = y[c] + e[c];
            pb->f(pb->ctx, ytmp, e);
            res->nfev++;
            for (int c = 0; c < N; ++c) e[c] += v[c];
            lus_r(N, E1, p1, e);
            err = fmax(rms(e, rhs, N, N), 1e-10);
        }
        if (!isfinite(err)) err = 1e300;

        /* new step size */
        double fac = fmin(safe, safe * (2 * kmax + 1) / (double)(2 * kmax + newt));
        double quot = fmax(facr, fmin(facl, pow(err, 0.25) / fac));
        double hnew = h / quot;
        if (err < 1.0) {
            /* accepted */
            first = 0;
            nacc++;
            res->naccept++;
            if (nacc > 1) {
                double facgus = (hacc / h) * pow(err * err / erracc, 0.25) / safe;
                facgus = fmax(facr, fmin(facl, facgus));
                quot = fmax(quot, facgus);
                hnew = h / quot;
            }
            hacc = h;
            erracc = fmax(1e-2, err);
            if (res->naccept == 1) {
                res->h_first = h;
                if (zfirst) memcpy(zfirst, Z, sizeof(double) * N3);
            }
            if (hrec && res->naccept <= cap) hrec[res->naccept - 1] = h;
            memcpy(Zs, Z, sizeof(double) * N3);
            hlast = h;
            for (int c = 0; c < N; ++c) y[c] += Z[2 * N + c];
            t = last ? dt : t + h;
            for (int c = 0; c < N; ++c) sc[c] = atol + rtol * fabs(y[c]);
            jac_fresh = 0;
            if (last) { res->status = OR_OK; break; }
            pb->f(pb->ctx, y, f0);
            res->nfev++;
            if (reject) hnew = fmin(hnew, h);
            reject = 0;
            if (t + 1.0001 * hnew >= dt) {   /* last step: no tail shorter than 1e-4 h */
                h = dt - t;
                last = 1;
            } else {
                double qt = hnew / h;
                if (theta <= thet && qt >= 1.0 && qt <= 1.2) { action = SAME; continue; }
                h = hnew;
            }
            action = theta <= thet ? NEW_LU : NEW_JAC;
        } else {
            /* rejected */
            res->nreject++;
            reject = 1;
            last = 0;
            h = first ? 0.1 * h : hnew;
            action = jac_fresh ? NEW_LU : NEW_JAC;
        }
    }
done:
    free(J); free(E1); free(E2); free(p1); free(w); free(cz); free(fdw);
    return res->status;
}

/* ------------------------------------------------------------------------- */
/* chemistry and linear problems                                              */
/* ------------------------------------------------------------------------- */
typedef struct { const or_mech *m; double P; int iso; } chem_ctx;

static void chem_f(void *c, const double *y, double *f) {
    chem_ctx *x = c;
    if (x->iso) or_rhs_iso(x->m, y, x->P, f); else or_rhs(x->m, y, x->P, f);
}
static void chem_j(void *c, const double *y, double *J) {
    chem_ctx *x = c;
    if (x->iso) or_jac_iso(x->m, y, x->P, J); else or_jac(x->m, y, x->P, J);
}

void or_jac_fd(const or_mech *m, const double *y, double P, const double *f0, double h, double atol, double rtol,
               double *J) {
    const int N = m->K + 1;
    chem_ctx cx = { m, P, 0 };
    problem pb = { N, chem_f, chem_j, &cx };
    double *work = malloc(sizeof(double) * 2 * N);
    fd_jacobian(&pb, y, f0, h, atol, rtol, J, work);
    free(work);
}

typedef struct { int N; const double *A; } quad_ctx;
static void quad_f(void *c, const double *y, double *f) {
    quad_ctx *x = c;
    for (int i = 0; i < x->N; ++i) {
        double s = 0.0;
        for (int j = 0; j < x->N; ++j) s += x->A[i * x->N + j] * y[j] * y[j];
        f[i] = s;
    }
}

void or_jac_fd_quadratic(int N, const double *A, const double *y, double h, double atol, double rtol, double *J) {
    quad_ctx cx = { N, A };
    problem pb = { N, quad_f, NULL, &cx };
    double *work = malloc(sizeof(double) * 3 * N);
    quad_f(&cx, y, work + 2 * N);
    fd_jacobian(&pb, y, work + 2 * N, h, atol, rtol, J, work);
    free(work);
}

static int integrate_rows(const or_mech *m, int64_t n, double dt, const double *y_in, double *y_out,
                          double atol, double rtol, const or_opts *o, const double *h0, int warm_h,
                          const double *zw, or_result *res, int nthreads, double *zfirst) {
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
        double *y = malloc(sizeof(double) * N);
        memcpy(y, row, sizeof(double) * N);
        chem_ctx cx = { m, row[K + 1], o->isothermal };
        problem pb = { N, chem_f, chem_j, &cx };
        int bad = !(row[0] > 0.0) || !(row[K + 1] > 0.0) || !finite_vec(row, S);
        if (bad) {
            memset(&res[i], 0, sizeof res[i]);
            res[i].status = OR_NONFINITE;
            memcpy(out, row, sizeof(double) * S);
        } else {
            const double hi = h0 ? h0[i] : 0.0;
            const int warm = warm_h ? (hi > 0.0 || zw != NULL) : 0;
            radau_core(&pb, dt, y, atol, rtol, o, hi, warm, zw ? zw + i * 3 * N : NULL, &res[i], NULL, 0,
                       zfirst ? zfirst + i * 3 * N : NULL);
            memcpy(out, y, sizeof(double) * N);
            out[K + 1] = row[K + 1];
        }
        free(y);
    }
    return 0;
}

int or_integrate_batch2(const or_mech *m, int64_t n, double dt, const double *y_in, double *y_out,
                        double atol, double rtol, const or_opts *o, const double *h0,
                        or_result *res, int nthreads, double *zfirst) {
    return integrate_rows(m, n, dt, y_in, y_out, atol, rtol, o, h0, 0, NULL, res, nthreads, zfirst);
}

int or_integrate_batch3(const or_mech *m, int64_t n, double dt, const double *y_in, double *y_out,
                        double atol, double rtol, const or_opts *o, const double *hw, const double *zw,
                        or_result *res, int nthreads, double *zfirst) {
    return integrate_rows(m, n, dt, y_in, y_out, atol, rtol, o, hw, 1, zw, res, nthreads, zfirst);
}

typedef struct { int N; const double *M; } lin_ctx;
static void lin_f(void *c, const double *y, double *f) {
    lin_ctx *x = c;
    for (int i = 0; i < x->N; ++i) { double s = 0.0; for (int j = 0; j < x->N; ++j) s += x->M[i * x->N + j] * y[j]; f[i] = s; }
}
static void lin_j(void *c, const double *y, double *J) {
    lin_ctx *x = c;
    (void)y;
    memcpy(J, x->M, sizeof(double) * x->N * x->N);
}

int or_integrate_linear(int N, const double *M, const double *y0, double dt, double atol, double rtol,
                        const or_opts *o, double *y_out, or_result *res, double *hrec, int cap) {
    or_opts dflt;
    if (!o) { or_default_opts(&dflt); o = &dflt; }
    lin_ctx cx = { N, M };
    problem pb = { N, lin_f, lin_j, &cx };
    memcpy(y_out, y0, sizeof(double) * N);
    return radau_core(&pb, dt, y_out, atol, rtol, o, 0.0, 0, NULL, res, hrec, cap, NULL);
}

int or_integrate_batch(const or_mech *m, int64_t n, double dt, const double *y_in, double *y_out,
                       double atol, double rtol, const or_opts *o, const double *h0,
                       or_result *res, int nthreads) {
    return or_integrate_batch2(m, n, dt, y_in, y_out, atol, rtol, o, h0, res, nthreads, NULL);
}

/* Fixed-step Radau IIA: nsteps equal steps of size dt/nsteps, the collocation
 * equations solved by full Newton (J refreshed each iteration) to 1e-14
 * relative change; no error control.  Used for refinement studies. */
int or_fixed_steps(const or_mech *m, const double *y_row, double dt, int nsteps, double *y_out) {
    const int K = m->K, N = K + 1, N3 = 3 * N;
    rconst k;
    radau_consts(&k);
    double P = y_row[K + 1];
    double *y = malloc(sizeof(double) * (N + N3 * 3 + N + (size_t)N * N * 3 + (size_t)N3 * N3));
    double *Z = y + N, *F = Z + N3, *R = F + N3, *yt = R + N3, *Js = yt + N, *Mb = Js + (size_t)N * N * 3;
    int *piv = malloc(sizeof(int) * N3);
    memcpy(y, y_row, sizeof(double) * N);
    double h = dt / nsteps;
    int ok = 0;
    for (int st = 0; st < nsteps; ++st) {
        memset(Z, 0, sizeof(double) * N3);
        for (int it = 0; it < 50; ++it) {
            for (int i = 0; i < 3; ++i) {
                for (int c = 0; c < N; ++c) yt[c] = y[c] + Z[i * N + c];
                or_rhs(m, yt, P, F + i * N);
                or_jac(m, yt, P, Js + (size_t)i * N * N);
            }
            /* residual G(Z) = Z - h (A (x) I) F(Z); Newton matrix I - h a_ij J(y0+z_j) */
            for (int i = 0; i < 3; ++i) for (int c = 0; c < N; ++c) {
                double acc = Z[i * N + c];
                for (int j = 0; j < 3; ++j) acc -= h * k.A[i * 3 + j] * F[j * N + c];
                R[i * N + c] = -acc;
            }
            for (int bi = 0; bi < 3; ++bi) for (int bj = 0; bj < 3; ++bj)
                for (int i = 0; i < N; ++i) for (int j = 0; j < N; ++j)
                    Mb[(size_t)(bi * N + i) * N3 + bj * N + j] =
                        (bi == bj && i == j ? 1.0 : 0.0) - h * k.A[bi * 3 + bj] * Js[(size_t)bj * N * N + i * N + j];
            lu_r(N3, Mb, piv);
            lus_r(N3, Mb, piv, R);
            double ch = 0.0;
            for (int i = 0; i < N3; ++i) {
                Z[i] += R[i];
                double sc = 1e-300 + fabs(y[i % N]) + fabs(Z[i]);
                ch = fmax(ch, fabs(R[i]) / sc);
            }
            if (ch < 1e-14) break;
        }
        for (int c = 0; c < N; ++c) y[c] += Z[2 * N + c];
        if (!finite_vec(y, N)) { ok = -1; break; }
    }
    memcpy(y_out, y, sizeof(double) * N);
    y_out[K + 1] = P;
    free(y); free(piv);
    return ok;
}
