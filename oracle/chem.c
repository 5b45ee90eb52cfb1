/* Oracle thermochemistry: source terms and the analytical Jacobian
 * (test infrastructure only; see oracle.h).
 *
 * State y = (T, Y_1..Y_K) at constant pressure P.  Mixture relations:
 *   1/Wbar = sum_k Y_k / W_k,  rho = P Wbar / (R T),  C_k = rho Y_k / W_k,
 *   dY_k/dt = W_k wdot_k / rho,
 *   dT/dt  = -(sum_k h_k wdot_k) / (rho cp),  cp = sum_k Y_k cp_k / W_k,
 * with molar h_k, cp_k from NASA-7 polynomials and wdot from mass-action
 * kinetics (Arrhenius forward constants, reverse constants through the
 * equilibrium constant, third-body and Troe falloff modifiers).  The paper
 * takes these from pyJac's constant-pressure, mass-fraction formulation
 * (Sec. 2.1); here they are written out from the textbook definitions. */
#define _GNU_SOURCE
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "oracle.h"

/* real instantiation */
#define SC double
#define FN(x) x##_r
#define EXPF exp
#define LOGF log
#define RE(x) (x)
#include "chem_generic.inc"
#undef SC
#undef FN
#undef EXPF
#undef LOGF
#undef RE

/* complex instantiation (complex-step derivative check) */
#define SC double complex
#define FN(x) x##_c
#define EXPF cexp
#define LOGF clog
#define RE(x) creal(x)
#include "chem_generic.inc"
#undef SC
#undef FN
#undef EXPF
#undef LOGF
#undef RE

void or_thermo(const or_mech *m, double T, double *cp, double *h, double *s) { thermo_r(m, T, cp, h, s); }

/* forward and reverse parts of each rate of progress (q = qf - qr), optional */
void or_rates2(const or_mech *m, const double *TY, double P, double *q, double *wdot, double *qf, double *qr) {
    const int K = m->K;
    double *C = malloc(sizeof(double) * 4 * K);
    double *cp = C + K, *h = cp + K, *s = h + K;
    double T = TY[0], sumYW = 0.0;
    for (int k = 0; k < K; ++k) sumYW += TY[1 + k] / m->W[k];
    double rho = P / sumYW / (OR_RU * T);
    for (int k = 0; k < K; ++k) C[k] = rho * TY[1 + k] / m->W[k];
    kinetics_r(m, T, C, q, wdot, cp, h, s, qf, qr);
    free(C);
}

void or_rates(const or_mech *m, const double *TY, double P, double *q, double *wdot) {
    or_rates2(m, TY, P, q, wdot, NULL, NULL);
}

void or_rhs(const or_mech *m, const double *y, double P, double *f) { rhs_r(m, y, P, f, 0); }

void or_rhs_iso(const or_mech *m, const double *y, double P, double *f) { rhs_r(m, y, P, f, 1); }

void or_jac_cs(const or_mech *m, const double *y, double P, double *J) {
    const int N = m->K + 1;
    const double hcs = 1e-30;
    double complex *yc = malloc(sizeof(double complex) * 2 * N);
    double complex *fc = yc + N;
    for (int col = 0; col < N; ++col) {
        for (int i = 0; i < N; ++i) yc[i] = y[i];
        yc[col] += hcs * I;
        rhs_c(m, yc, P, fc, 0);
        for (int i = 0; i < N; ++i) J[i * N + col] = cimag(fc[i]) / hcs;
    }
    free(yc);
}

/* Analytical Jacobian by the chain rule through C_k(T, Y), k_f(T), K_c(T),
 * [M](C), P_r, the Troe factor F(T, P_r), cp(T, Y) and h_k(T).
 *   dq_j/dC_m, dq_j/dT|_C          per reaction
 *   S_j = sum_m dq_j/dC_m C_m       (density coupling through rho(T, Y))
 *   dC_m/dT = -C_m/T,  dC_l/dY_m = delta_lm rho/W_m - C_l Wbar/W_m            */
static void jac_impl(const or_mech *m, const double *y, double P, double *J, int isothermal) {
    const int K = m->K, N = K + 1;
    double *buf = calloc((size_t)K * K + 12 * (size_t)K, sizeof(double));
    double *Mkm = buf;                        /* d wdot_k / d C_m  (T fixed) */
    double *C = Mkm + (size_t)K * K, *cp = C + K, *h = cp + K, *s = h + K, *dcp = s + K;
    double *wdot = dcp + K, *dwdT = wdot + K, *sS = dwdT + K, *dqdC = sS + K, *dPf = dqdC + K, *dPr = dPf + K;
    double T = y[0];
    double sumYW = 0.0;
    for (int k = 0; k < K; ++k) sumYW += y[1 + k] / m->W[k];
    double Wbar = 1.0 / sumYW;
    double rho = P * Wbar / (OR_RU * T);
    for (int k = 0; k < K; ++k) C[k] = rho * y[1 + k] / m->W[k];
    thermo_r(m, T, cp, h, s);
    for (int k = 0; k < K; ++k) {
        const double *a = (T < m->Tmid[k]) ? &m->alow[k * 7] : &m->ahigh[k * 7];
        dcp[k] = a[1] + 2.0 * a[2] * T + 3.0 * a[3] * T * T + 4.0 * a[4] * T * T * T;  /* d(cp/R)/dT */
    }
    double lnT = log(T), RT = OR_RU * T;
    for (int j = 0; j < m->R; ++j) {
        const or_reaction *x = &m->rx[j];
        double kf = x->A * exp(x->b * lnT - x->Ea / RT);
        double dlnkf_dT = x->b / T + x->Ea / (RT * T);
        double Mc = 0.0, dlnkf_dM = 0.0;
        if (x->kind != 0)
            for (int k = 0; k < K; ++k) Mc += x->eff[k] * C[k];
        if (x->kind == 2) {
            double k0 = x->A0 * exp(x->b0 * lnT - x->Ea0 / RT);
            double dlnk0_dT = x->b0 / T + x->Ea0 / (RT * T);
            double Pr = k0 * Mc / kf;
            double dlnPr_dT = dlnk0_dT - dlnkf_dT;
            double a = x->troe[0], T3 = x->troe[1], T1 = x->troe[2], T2 = x->troe[3];
            double Fc = (1.0 - a) * exp(-T / T3) + a * exp(-T / T1) + exp(-T2 / T);
            double dFc = -(1.0 - a) / T3 * exp(-T / T3) - a / T1 * exp(-T / T1) + T2 / (T * T) * exp(-T2 / T);
            double L = log10(Fc);
            double dL = dFc / (Fc * M_LN10);
            double c = -0.4 - 0.67 * L, nn = 0.75 - 1.27 * L;
            double xx = log10(Pr) + c;
            double den = nn - 0.14 * xx;
            double f1 = xx / den;
            double g1 = 1.0 + f1 * f1;
            double log10F = L / g1;
            /* temperature derivative of log10 F at fixed [M] */
            double dx_T = dlnPr_dT / M_LN10 - 0.67 * dL;
            double dn_T = -1.27 * dL;
            double df1_T = (nn * dx_T - xx * dn_T) / (den * den);
            double dlog10F_T = dL / g1 - 2.0 * L * f1 * df1_T / (g1 * g1);
            /* [M] derivative of log10 F at fixed T */
            double dx_M = 1.0 / (Mc * M_LN10);
            double df1_M = nn * dx_M / (den * den);
            double dlog10F_M = -2.0 * L * f1 * df1_M / (g1 * g1);
            double F = pow(10.0, log10F);
            kf = kf * (Pr / (1.0 + Pr)) * F;
            dlnkf_dT = dlnkf_dT + dlnPr_dT / (1.0 + Pr) + M_LN10 * dlog10F_T;
            dlnkf_dM = 1.0 / (Mc * (1.0 + Pr)) + M_LN10 * dlog10F_M;
        }
        double dS = 0.0, dH = 0.0;
        for (int t = 0; t < x->np; ++t) { dS += s[x->prod[t]]; dH += h[x->prod[t]]; }
        for (int t = 0; t < x->nr; ++t) { dS -= s[x->reac[t]]; dH -= h[x->reac[t]]; }
        int dnu = x->np - x->nr;
        double Kc = exp(dS - dH + dnu * log(OR_PATM / RT));
        double dlnKc_dT = dH / T - dnu / T;    /* van 't Hoff: dH here is Delta H/(R T) */
        double kr = kf / Kc;
        /* concentration products and their partial derivatives (slot rule) */
        double Pf = 1.0, Pp = 1.0;
        for (int t = 0; t < x->nr; ++t) Pf *= C[x->reac[t]];
        for (int t = 0; t < x->np; ++t) Pp *= C[x->prod[t]];
        for (int k = 0; k < K; ++k) { dPf[k] = 0.0; dPr[k] = 0.0; }
        for (int t = 0; t < x->nr; ++t) {
            double o = 1.0;
            for (int u = 0; u < x->nr; ++u) if (u != t) o *= C[x->reac[u]];
            dPf[x->reac[t]] += o;
        }
        for (int t = 0; t < x->np; ++t) {
            double o = 1.0;
            for (int u = 0; u < x->np; ++u) if (u != t) o *= C[x->prod[u]];
            dPr[x->prod[t]] += o;
        }
        double Rj = kf * Pf - kr * Pp;
        double dRdT = Rj * dlnkf_dT + kr * Pp * dlnKc_dT;
        double qj, dqdT;
        for (int mm = 0; mm < K; ++mm) dqdC[mm] = kf * dPf[mm] - kr * dPr[mm];
        if (x->kind == 1) {
            qj = Mc * Rj;
            dqdT = Mc * dRdT;
            for (int mm = 0; mm < K; ++mm) dqdC[mm] = Mc * dqdC[mm] + x->eff[mm] * Rj;
        } else if (x->kind == 2) {
            qj = Rj;
            dqdT = dRdT;
            for (int mm = 0; mm < K; ++mm) dqdC[mm] += Rj * dlnkf_dM * x->eff[mm];
        } else {
            qj = Rj;
            dqdT = dRdT;
        }
        double Sj = 0.0;
        for (int mm = 0; mm < K; ++mm) Sj += dqdC[mm] * C[mm];
        /* scatter nu_kj times the reaction derivatives */
        int sp[4], nu[4], ns = 0;
        for (int t = 0; t < x->nr + x->np; ++t) {
            int k = t < x->nr ? x->reac[t] : x->prod[t - x->nr];
            int v = t < x->nr ? -1 : 1;
            int found = 0;
            for (int u = 0; u < ns; ++u) if (sp[u] == k) { nu[u] += v; found = 1; }
            if (!found) { sp[ns] = k; nu[ns] = v; ++ns; }
        }
        for (int u = 0; u < ns; ++u) {
            if (nu[u] == 0) continue;
            int k = sp[u];
            wdot[k] += nu[u] * qj;
            dwdT[k] += nu[u] * dqdT;
            sS[k] += nu[u] * Sj;
            for (int mm = 0; mm < K; ++mm) Mkm[(size_t)k * K + mm] += nu[u] * dqdC[mm];
        }
    }
    /* assemble */
    double cpmix = 0.0, dcpmix = 0.0, H = 0.0, dHdT = 0.0;
    for (int k = 0; k < K; ++k) {
        cpmix += y[1 + k] * cp[k] * OR_RU / m->W[k];
        dcpmix += y[1 + k] * dcp[k] * OR_RU / m->W[k];
        H += h[k] * RT * wdot[k];
    }
    double fT = -H / (rho * cpmix);
    for (int k = 0; k < K; ++k) {
        double fk = m->W[k] * wdot[k] / rho;
        double dwdT_Y = dwdT[k] - sS[k] / T;           /* d wdot_k/dT at fixed Y */
        J[(1 + k) * N + 0] = m->W[k] / rho * dwdT_Y + fk / T;
        dHdT += cp[k] * OR_RU * wdot[k] + h[k] * RT * dwdT_Y;
        for (int mm = 0; mm < K; ++mm) {
            double dwdY = rho / m->W[mm] * Mkm[(size_t)k * K + mm] - Wbar / m->W[mm] * sS[k];
            J[(1 + k) * N + 1 + mm] = m->W[k] / rho * dwdY + fk * Wbar / m->W[mm];
        }
    }
    if (isothermal) {
        for (int c = 0; c < N; ++c) J[c] = 0.0;
    } else {
        J[0] = -dHdT / (rho * cpmix) - fT * (-1.0 / T + dcpmix / cpmix);
        for (int mm = 0; mm < K; ++mm) {
            double dHdY = 0.0;
            for (int k = 0; k < K; ++k) {
                double dwdY = rho / m->W[mm] * Mkm[(size_t)k * K + mm] - Wbar / m->W[mm] * sS[k];
                dHdY += h[k] * RT * dwdY;
            }
            J[1 + mm] = -dHdY / (rho * cpmix) - fT * (cp[mm] * OR_RU / (m->W[mm] * cpmix) - Wbar / m->W[mm]);
        }
    }
    free(buf);
}

void or_jac(const or_mech *m, const double *y, double P, double *J) { jac_impl(m, y, P, J, 0); }

void or_jac_iso(const or_mech *m, const double *y, double P, double *J) { jac_impl(m, y, P, J, 1); }
