// Device code of the rkchem library for gfx950: source terms, analytical
// Jacobian, batched dense LU (real and complex) and the Radau IIA integrator
// with one state per lane (the paper's per-thread pattern, Sec. 1.2).
//
// Every per-state array lives in a global scratch block laid out
// [wave][element][64 lanes]: element e of lane l is at base[e * 64] with
// base = scratch + wave * total * 64 + l, so the 64 lanes of a wavefront touch
// 64 consecutive doubles for every element (one 512-byte coalesced access).
// Mechanism tables are indexed by wavefront-uniform loop counters and are read
// through scalar loads.
#include <hip/hip_runtime.h>
#include <cmath>

#include "rk_internal.h"

namespace rk {

namespace {

constexpr double kU = 2.220446049250313e-16;   // unit roundoff of binary64

struct Lane {
    double *b;
    __device__ __forceinline__ double &operator[](int e) const { return b[(size_t)e * kWave]; }
};

enum { ACT_JAC = 0, ACT_LU = 1, ACT_SAME = 2 };

// ---------------------------------------------------------------------------
// thermodynamics: cp/R, h/(RT), s/R (and d(cp/R)/dT) of every species
// thermo table per species and range: [0..4] cp coefficients a1..a5,
// [5..9] a1, a2/2, a3/3, a4/4, a5/5, [10] a6, [11..14] a2, a3/2, a4/3, a5/4, [15] a7
// ---------------------------------------------------------------------------
__device__ __forceinline__ void thermo(const DevMech &m, const LaneLayout &L, Lane M, double T, bool want_dcp) {
    const double lnT = log(T), invT = 1.0 / T;
    for (int k = 0; k < m.K; ++k) {
        const double *lo = m.thermo + (size_t)k * 32;
        const double *hi = lo + 16;
        const bool low = T < m.Tmid[k];
        double a[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) a[i] = low ? lo[i] : hi[i];
        M[L.cp + k] = a[0] + T * (a[1] + T * (a[2] + T * (a[3] + T * a[4])));
        M[L.h + k] = a[5] + T * (a[6] + T * (a[7] + T * (a[8] + T * a[9]))) + a[10] * invT;
        M[L.s + k] = a[0] * lnT + T * (a[11] + T * (a[12] + T * (a[13] + T * a[14]))) + a[15];
        if (want_dcp) M[L.dcp + k] = a[1] + T * (2.0 * a[2] + T * (3.0 * a[3] + T * 4.0 * a[4]));
    }
}

struct MixState {
    double T, P, Wbar, rho;
};

// concentrations C_k = rho Y_k / W_k from y at offset yo
__device__ __forceinline__ MixState mixture(const DevMech &m, const LaneLayout &L, Lane M, int yo, double P) {
    MixState x;
    x.T = M[yo];
    x.P = P;
    double s = 0.0;
    for (int k = 0; k < m.K; ++k) s += M[yo + 1 + k] * m.invW[k];
    x.Wbar = 1.0 / s;
    x.rho = P * x.Wbar / (kRu * x.T);
    for (int k = 0; k < m.K; ++k) M[L.C + k] = x.rho * M[yo + 1 + k] * m.invW[k];
    return x;
}

// ---------------------------------------------------------------------------
// source terms f(y): y at offset yo, f to offset fo
// ---------------------------------------------------------------------------
__device__ void rhs(const DevMech &m, const LaneLayout &L, Lane M, int yo, int fo, double P) {
    const int K = m.K;
    const MixState x = mixture(m, L, M, yo, P);
    const double T = x.T;
    thermo(m, L, M, T, false);
    for (int k = 0; k < K; ++k) M[L.wdot + k] = 0.0;
    const double lnT = log(T), invT = 1.0 / T, lnPRT = log(kPatm / (kRu * T));
    for (int j = 0; j < m.R; ++j) {
        const int4 sp = m.rsp[j];
        const int info = m.rinfo[j];
        const double *p = m.rpar + (size_t)j * P_NPAR;
        const int kind = info & 15;
        double kf = p[P_A] * exp(p[P_B] * lnT - p[P_EAR] * invT);
        double Mc = 0.0;
        if (kind != 0) {
            const double *e = m.eff + (size_t)((info >> 12) - 1) * K;
            for (int k = 0; k < K; ++k) Mc += e[k] * M[L.C + k];
        }
        if (kind == 2) {
            const double k0 = p[P_A0] * exp(p[P_B0] * lnT - p[P_EA0R] * invT);
            const double Pr = k0 * Mc / kf;
            const double Fc = (1.0 - p[P_TA]) * exp(-T / p[P_T3]) + p[P_TA] * exp(-T / p[P_T1]) + exp(-p[P_T2] * invT);
            const double lF = log10(Fc);
            const double c = -0.4 - 0.67 * lF, nn = 0.75 - 1.27 * lF;
            const double xx = log10(Pr) + c;
            const double f1 = xx / (nn - 0.14 * xx);
            kf = kf * (Pr / (1.0 + Pr)) * exp10(lF / (1.0 + f1 * f1));
        }
        double dS = M[L.s + sp.z] - M[L.s + sp.x];
        double dH = M[L.h + sp.z] - M[L.h + sp.x];
        double cf = kf * M[L.C + sp.x];
        if (sp.y >= 0) { dS -= M[L.s + sp.y]; dH -= M[L.h + sp.y]; cf *= M[L.C + sp.y]; }
        if (sp.w >= 0) { dS += M[L.s + sp.w]; dH += M[L.h + sp.w]; }
        const double Kc = exp(dS - dH + p[P_DNU] * lnPRT);
        double cr = kf / Kc * M[L.C + sp.z];
        if (sp.w >= 0) cr *= M[L.C + sp.w];
        double q = cf - cr;
        if (kind == 1) q *= Mc;
        M[L.wdot + sp.x] -= q;
        if (sp.y >= 0) M[L.wdot + sp.y] -= q;
        M[L.wdot + sp.z] += q;
        if (sp.w >= 0) M[L.wdot + sp.w] += q;
    }
    double cpmix = 0.0, hw = 0.0;
    for (int k = 0; k < K; ++k) {
        cpmix += M[yo + 1 + k] * M[L.cp + k] * m.invW[k];
        hw += M[L.h + k] * M[L.wdot + k];
    }
    // cp and h carry a factor R (and h a factor T); they cancel in dT/dt up to T
    M[fo] = -hw * T / (x.rho * cpmix);
    const double invrho = 1.0 / x.rho;
    for (int k = 0; k < K; ++k) M[fo + 1 + k] = m.W[k] * M[L.wdot + k] * invrho;
}

// ---------------------------------------------------------------------------
// analytical Jacobian J = df/dy (row-major N x N at offset jo) at y (offset yo)
//
// Per reaction j: rate of progress q_j, dq_j/dT at fixed C, dq_j/dC_m, and
// S_j = sum_m C_m dq_j/dC_m.  Accumulated per species:
//   Mkm = sum_j nu_kj dq_j/dC_m  (kept in the Y block of J until assembly),
//   dwdT_k = sum_j nu_kj dq_j/dT|_C,  sS_k = sum_j nu_kj S_j.
// With dC_m/dT = -C_m/T and dC_l/dY_m = delta_lm rho/W_m - C_l Wbar/W_m:
//   d wdot_k/dT|_Y = dwdT_k - sS_k / T
//   d wdot_k/dY_m  = (rho/W_m) Mkm - (Wbar/W_m) sS_k
// and f_k = W_k wdot_k / rho, f_T = -sum h_k wdot_k / (rho cp) are
// differentiated through rho(T, Y) and cp(T, Y).
// ---------------------------------------------------------------------------
__device__ void jacobian(const DevMech &m, const LaneLayout &L, Lane M, int yo, int jo, double P) {
    const int K = m.K, N = m.N;
    const MixState x = mixture(m, L, M, yo, P);
    const double T = x.T, rho = x.rho, Wbar = x.Wbar;
    thermo(m, L, M, T, true);
    for (int i = 0; i < N * N; ++i) M[jo + i] = 0.0;
    for (int k = 0; k < K; ++k) { M[L.wdot + k] = 0.0; M[L.dwdT + k] = 0.0; M[L.sS + k] = 0.0; }
    const double lnT = log(T), invT = 1.0 / T, lnPRT = log(kPatm / (kRu * T));
    for (int j = 0; j < m.R; ++j) {
        const int4 sp = m.rsp[j];
        const int info = m.rinfo[j];
        const double *p = m.rpar + (size_t)j * P_NPAR;
        const int kind = info & 15;
        const double *eff = kind ? m.eff + (size_t)((info >> 12) - 1) * K : nullptr;
        double kf = p[P_A] * exp(p[P_B] * lnT - p[P_EAR] * invT);
        double dlnkf = (p[P_B] + p[P_EAR] * invT) * invT;
        double Mc = 0.0, dlnkf_dM = 0.0;
        if (kind != 0)
            for (int k = 0; k < K; ++k) Mc += eff[k] * M[L.C + k];
        if (kind == 2) {
            const double k0 = p[P_A0] * exp(p[P_B0] * lnT - p[P_EA0R] * invT);
            const double dlnk0 = (p[P_B0] + p[P_EA0R] * invT) * invT;
            const double Pr = k0 * Mc / kf;
            const double dlnPr = dlnk0 - dlnkf;
            const double ta = p[P_TA], t3 = p[P_T3], t1 = p[P_T1], t2 = p[P_T2];
            const double e3 = exp(-T / t3), e1 = exp(-T / t1), e2 = exp(-t2 * invT);
            const double Fc = (1.0 - ta) * e3 + ta * e1 + e2;
            const double dFc = -(1.0 - ta) / t3 * e3 - ta / t1 * e1 + t2 * invT * invT * e2;
            const double lF = log10(Fc);
            const double dlF = dFc / (Fc * M_LN10);
            const double c = -0.4 - 0.67 * lF, nn = 0.75 - 1.27 * lF;
            const double xx = log10(Pr) + c;
            const double den = nn - 0.14 * xx;
            const double f1 = xx / den, g1 = 1.0 + f1 * f1;
            const double l10F = lF / g1;
            // d log10F along T (fixed [M]) and along [M] (fixed T)
            const double dxT = dlnPr / M_LN10 - 0.67 * dlF, dnT = -1.27 * dlF;
            const double df1T = (nn * dxT - xx * dnT) / (den * den);
            const double dl10F_T = dlF / g1 - 2.0 * lF * f1 * df1T / (g1 * g1);
            const double df1M = nn / (Mc * M_LN10) / (den * den);
            const double dl10F_M = -2.0 * lF * f1 * df1M / (g1 * g1);
            kf = kf * (Pr / (1.0 + Pr)) * exp10(l10F);
            dlnkf = dlnkf + dlnPr / (1.0 + Pr) + M_LN10 * dl10F_T;
            dlnkf_dM = 1.0 / (Mc * (1.0 + Pr)) + M_LN10 * dl10F_M;
        }
        double dS = M[L.s + sp.z] - M[L.s + sp.x];
        double dH = M[L.h + sp.z] - M[L.h + sp.x];
        const double Cr0 = M[L.C + sp.x], Cp0 = M[L.C + sp.z];
        double Cr1 = 1.0, Cp1 = 1.0;
        if (sp.y >= 0) { dS -= M[L.s + sp.y]; dH -= M[L.h + sp.y]; Cr1 = M[L.C + sp.y]; }
        if (sp.w >= 0) { dS += M[L.s + sp.w]; dH += M[L.h + sp.w]; Cp1 = M[L.C + sp.w]; }
        const double dnu = p[P_DNU];
        const double Kc = exp(dS - dH + dnu * lnPRT);
        const double dlnKc = (dH - dnu) * invT;      // van 't Hoff, dH = Delta h / (R T)
        const double kr = kf / Kc;
        const double Pf = Cr0 * Cr1, Pp = Cp0 * Cp1;
        const double Rj = kf * Pf - kr * Pp;
        const double dRdT = Rj * dlnkf + kr * Pp * dlnKc;
        const int nr = (info >> 4) & 15, np = (info >> 8) & 15;
        const double sMA = (kind == 1) ? Mc : 1.0;               // factor of the mass-action part
        const double q = sMA * Rj;
        const double dqdT = sMA * dRdT;
        const double ctb = (kind == 1) ? Rj : (kind == 2 ? Rj * dlnkf_dM : 0.0);  // dense part: ctb * eff_m
        // Euler: sum_m C_m d(prod C)/dC_m = order * prod C
        const double Sj = sMA * (nr * kf * Pf - np * kr * Pp) + ctb * Mc;
        // mass-action partials (slot rule): (species, value) pairs
        const int em[4] = {sp.x, sp.y, sp.z, sp.w};
        const double ev[4] = {sMA * kf * Cr1, sMA * kf * Cr0, -sMA * kr * Cp1, -sMA * kr * Cp0};
        const double nu[4] = {-1.0, -1.0, 1.0, 1.0};
        for (int a = 0; a < 4; ++a) {
            const int k = em[a];
            if (k < 0) continue;
            const double v = nu[a];
            M[L.wdot + k] += v * q;
            M[L.dwdT + k] += v * dqdT;
            M[L.sS + k] += v * Sj;
            const int row = jo + (1 + k) * N + 1;
            for (int b = 0; b < 4; ++b) {
                if (em[b] < 0) continue;
                M[row + em[b]] += v * ev[b];
            }
            if (ctb != 0.0) {
                const double vc = v * ctb;
                for (int mm = 0; mm < K; ++mm) M[row + mm] += vc * eff[mm];
            }
        }
    }
    // assembly
    double cpmix = 0.0, dcpmix = 0.0, hw = 0.0, dHdT = 0.0, hsS = 0.0;
    for (int k = 0; k < K; ++k) {
        const double Yk = M[yo + 1 + k];
        cpmix += Yk * M[L.cp + k] * m.invW[k];
        dcpmix += Yk * M[L.dcp + k] * m.invW[k];
        const double hk = M[L.h + k] * T;   // molar enthalpy / R
        hw += hk * M[L.wdot + k];
        dHdT += M[L.cp + k] * M[L.wdot + k] + hk * (M[L.dwdT + k] - M[L.sS + k] * invT);
        hsS += hk * M[L.sS + k];
    }
    // quantities below carry a factor 1/R relative to SI; they cancel in f_T
    const double rcp = rho * cpmix;
    const double fT = -hw / rcp;
    M[jo] = -dHdT / rcp - fT * (-invT + dcpmix / cpmix);
    for (int mm = 0; mm < K; ++mm) {
        double hM = 0.0;
        for (int k = 0; k < K; ++k) hM += M[L.h + k] * T * M[jo + (1 + k) * N + 1 + mm];
        const double dHdY = (rho * hM - Wbar * hsS) * m.invW[mm];
        M[jo + 1 + mm] = -dHdY / rcp - fT * (M[L.cp + mm] * m.invW[mm] / cpmix - Wbar * m.invW[mm]);
    }
    const double invrho = 1.0 / rho;
    for (int k = 0; k < K; ++k) {
        const double Wk = m.W[k];
        const double fk = Wk * M[L.wdot + k] * invrho;
        const double a = Wbar * (fk - Wk * M[L.sS + k] * invrho);
        const int row = jo + (1 + k) * N;
        M[row] = Wk * invrho * (M[L.dwdT + k] - M[L.sS + k] * invT) + fk * invT;
        for (int mm = 0; mm < K; ++mm) M[row + 1 + mm] = (Wk * M[row + 1 + mm] + a) * m.invW[mm];
    }
}

// ---------------------------------------------------------------------------
// dense LU with partial pivoting, in place (row-major), pivots stored as doubles
// ---------------------------------------------------------------------------
__device__ void lu_real(Lane M, int N, int ao, int po) {
    for (int k = 0; k < N; ++k) {
        int p = k;
        double amax = fabs(M[ao + k * N + k]);
        for (int i = k + 1; i < N; ++i) {
            const double v = fabs(M[ao + i * N + k]);
            if (v > amax) { amax = v; p = i; }
        }
        M[po + k] = (double)p;
        if (p != k)
            for (int j = 0; j < N; ++j) {
                const double t = M[ao + k * N + j];
                M[ao + k * N + j] = M[ao + p * N + j];
                M[ao + p * N + j] = t;
            }
        const double inv = 1.0 / M[ao + k * N + k];
        for (int i = k + 1; i < N; ++i) {
            const double l = M[ao + i * N + k] * inv;
            M[ao + i * N + k] = l;
            for (int j = k + 1; j < N; ++j) M[ao + i * N + j] -= l * M[ao + k * N + j];
        }
    }
}

__device__ void lu_solve_real(Lane M, int N, int ao, int po, int bo) {
    for (int k = 0; k < N; ++k) {
        const int p = (int)M[po + k];
        if (p != k) { const double t = M[bo + k]; M[bo + k] = M[bo + p]; M[bo + p] = t; }
    }
    for (int i = 1; i < N; ++i) {
        double acc = M[bo + i];
        for (int j = 0; j < i; ++j) acc -= M[ao + i * N + j] * M[bo + j];
        M[bo + i] = acc;
    }
    for (int i = N - 1; i >= 0; --i) {
        double acc = M[bo + i];
        for (int j = i + 1; j < N; ++j) acc -= M[ao + i * N + j] * M[bo + j];
        M[bo + i] = acc / M[ao + i * N + i];
    }
}

__device__ void lu_cplx(Lane M, int N, int ar, int ai, int po) {
    for (int k = 0; k < N; ++k) {
        int p = k;
        double amax = M[ar + k * N + k] * M[ar + k * N + k] + M[ai + k * N + k] * M[ai + k * N + k];
        for (int i = k + 1; i < N; ++i) {
            const double re = M[ar + i * N + k], im = M[ai + i * N + k];
            const double v = re * re + im * im;
            if (v > amax) { amax = v; p = i; }
        }
        M[po + k] = (double)p;
        if (p != k)
            for (int j = 0; j < N; ++j) {
                double t = M[ar + k * N + j]; M[ar + k * N + j] = M[ar + p * N + j]; M[ar + p * N + j] = t;
                t = M[ai + k * N + j]; M[ai + k * N + j] = M[ai + p * N + j]; M[ai + p * N + j] = t;
            }
        const double dr = M[ar + k * N + k], di = M[ai + k * N + k];
        const double dd = 1.0 / (dr * dr + di * di);
        const double ir = dr * dd, ii = -di * dd;       // 1 / pivot
        for (int i = k + 1; i < N; ++i) {
            const double xr = M[ar + i * N + k], xi = M[ai + i * N + k];
            const double lr = xr * ir - xi * ii, li = xr * ii + xi * ir;
            M[ar + i * N + k] = lr;
            M[ai + i * N + k] = li;
            for (int j = k + 1; j < N; ++j) {
                const double ur = M[ar + k * N + j], ui = M[ai + k * N + j];
                M[ar + i * N + j] -= lr * ur - li * ui;
                M[ai + i * N + j] -= lr * ui + li * ur;
            }
        }
    }
}

__device__ void lu_solve_cplx(Lane M, int N, int ar, int ai, int po, int br, int bi) {
    for (int k = 0; k < N; ++k) {
        const int p = (int)M[po + k];
        if (p != k) {
            double t = M[br + k]; M[br + k] = M[br + p]; M[br + p] = t;
            t = M[bi + k]; M[bi + k] = M[bi + p]; M[bi + p] = t;
        }
    }
    for (int i = 1; i < N; ++i) {
        double xr = M[br + i], xi = M[bi + i];
        for (int j = 0; j < i; ++j) {
            const double lr = M[ar + i * N + j], li = M[ai + i * N + j];
            const double yr = M[br + j], yi = M[bi + j];
            xr -= lr * yr - li * yi;
            xi -= lr * yi + li * yr;
        }
        M[br + i] = xr;
        M[bi + i] = xi;
    }
    for (int i = N - 1; i >= 0; --i) {
        double xr = M[br + i], xi = M[bi + i];
        for (int j = i + 1; j < N; ++j) {
            const double ur = M[ar + i * N + j], ui = M[ai + i * N + j];
            const double yr = M[br + j], yi = M[bi + j];
            xr -= ur * yr - ui * yi;
            xi -= ur * yi + ui * yr;
        }
        const double dr = M[ar + i * N + i], di = M[ai + i * N + i];
        const double dd = 1.0 / (dr * dr + di * di);
        M[br + i] = (xr * dr + xi * di) * dd;
        M[bi + i] = (xi * dr - xr * di) * dd;
    }
}

// scaled RMS norm of n entries at offset vo with weights at so (period N)
__device__ __forceinline__ double wrms(Lane M, int vo, int so, int n, int N) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) {
        const double t = M[vo + i] / M[so + (i % N)];
        s += t * t;
    }
    return sqrt(s / n);
}

// First-order forward-difference Jacobian into J at jo (the alternative to
// the analytical Jacobian that Sec. 3.4 compares): column j from
// (f(y + inc_j e_j) - f(y)) / inc_j with CVODE's dense difference-quotient
// increments inc_j = max(sqrt(u) |y_j|, m w_j), w_j = atol + rtol |y_j|,
// m = 1000 |h| u N ||f(y)||_w (1 when f(y) = 0).  f(y) is at fo; the
// perturbed state goes to tmp, its source terms to ev: N evaluations.
__device__ void jacobian_fd(const DevMech &m, const LaneLayout &L, Lane M, int yo, int fo, int jo, double P,
                            double h, double atol, double rtol) {
    const int N = m.N;
    double fn = 0.0;
    for (int i = 0; i < N; ++i) {
        const double q = M[fo + i] / (atol + rtol * fabs(M[yo + i]));
        fn += q * q;
    }
    fn = sqrt(fn / N);
    const double minc = fn != 0.0 ? 1000.0 * fabs(h) * kU * N * fn : 1.0;
    for (int i = 0; i < N; ++i) M[L.tmp + i] = M[yo + i];
    for (int j = 0; j < N; ++j) {
        const double yj = M[yo + j];
        const double inc = fmax(sqrt(kU) * fabs(yj), minc * (atol + rtol * fabs(yj)));
        M[L.tmp + j] = yj + inc;
        rhs(m, L, M, L.tmp, L.ev, P);
        M[L.tmp + j] = yj;
        for (int i = 0; i < N; ++i) M[jo + i * N + j] = (M[L.ev + i] - M[fo + i]) / inc;
    }
}

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void rhs_kernel(DevMech m, LaneLayout L, int64_t n, const double *__restrict__ y,
                                                 double *__restrict__ f, double *__restrict__ scratch) {
    const int64_t s = (int64_t)blockIdx.x * kWave + threadIdx.x;
    if (s >= n) return;
    Lane M{scratch + (size_t)blockIdx.x * L.total * kWave + threadIdx.x};
    for (int c = 0; c < m.N; ++c) M[L.y + c] = y[(size_t)c * n + s];
    rhs(m, L, M, L.y, L.f0, y[(size_t)(m.K + 1) * n + s]);
    for (int c = 0; c < m.N; ++c) f[(size_t)c * n + s] = M[L.f0 + c];
}

__global__ __launch_bounds__(64) void jac_kernel(DevMech m, LaneLayout L, int64_t n, const double *__restrict__ y,
                                                 double *__restrict__ J, double *__restrict__ scratch) {
    const int64_t s = (int64_t)blockIdx.x * kWave + threadIdx.x;
    if (s >= n) return;
    Lane M{scratch + (size_t)blockIdx.x * L.total * kWave + threadIdx.x};
    for (int c = 0; c < m.N; ++c) M[L.y + c] = y[(size_t)c * n + s];
    jacobian(m, L, M, L.y, L.J, y[(size_t)(m.K + 1) * n + s]);
    for (int i = 0; i < m.N * m.N; ++i) J[(size_t)i * n + s] = M[L.J + i];
}

// Radau IIA, one state per lane.  The step logic restates Hairer & Wanner's
// published algorithm (simplified Newton in transformed variables, embedded
// error estimate, predictive step control, Jacobian/LU reuse rules); the
// readings of the points the paper leaves open are the library's documented
// defaults (kappa, kmax, h0, the failure rules).
__global__ __launch_bounds__(64) void radau_lane_kernel(DevMech m, LaneLayout L, RadauParams rp, int64_t n,
                                                        const double *__restrict__ yin, double *__restrict__ yout,
                                                        double *__restrict__ scratch, int32_t *__restrict__ cnt,
                                                        const int *__restrict__ order) {
    const int64_t slot = (int64_t)blockIdx.x * kWave + threadIdx.x;
    if (slot >= n) return;
    const int64_t s = order ? (int64_t)order[slot] : slot;
    Lane M{scratch + (size_t)blockIdx.x * L.total * kWave + threadIdx.x};
    const int N = m.N, K = m.K, N3 = 3 * N;
    const double P = yin[(size_t)(K + 1) * n + s];
    bool bad = !(P > 0.0) || !isfinite(P);
    for (int c = 0; c < N; ++c) {
        const double v = yin[(size_t)c * n + s];
        M[L.y + c] = v;
        bad = bad || !isfinite(v);
    }
    bad = bad || !(M[L.y] > 0.0);
    int status = RK_ST_OK, nstep = 0, nacc = 0, nrej = 0, nnewt = 0, nnf = 0, nfev = 0, njev = 0, nlu = 0;
    if (bad) {
        for (int c = 0; c < K + 2; ++c) yout[(size_t)c * n + s] = yin[(size_t)c * n + s];
        status = RK_ST_NONFINITE;
    } else {
        const double dt = rp.dt, atol = rp.atol, rtol = rp.rtol, kappa = rp.kappa;
        const int kmax = rp.kmax;
        double t = 0.0, h = rp.h0;
        bool last = false;
        if (t + 1.0001 * h >= dt) { h = dt - t; last = true; }
        rhs(m, L, M, L.y, L.f0, P);
        ++nfev;
        for (int c = 0; c < N; ++c) M[L.sc + c] = atol + rtol * fabs(M[L.y + c]);
        bool first = true, reject = false, jac_fresh = false;
        double eta = 1.0, theta = 1.0, hacc = h, erracc = 1e-2, hlast = h;
        int action = ACT_JAC;
        for (;;) {
            if (action == ACT_JAC) {
                if (rp.fd_jac) {
                    jacobian_fd(m, L, M, L.y, L.f0, L.J, P, h, atol, rtol);
                    nfev += N;
                } else {
                    jacobian(m, L, M, L.y, L.J, P);
                }
                ++njev;
                jac_fresh = true;
                action = ACT_LU;
            }
            if (action == ACT_LU) {
                const double gh = rp.g / h, ah = rp.a / h, bh = rp.b / h;
                for (int i = 0; i < N * N; ++i) {
                    const double j = M[L.J + i];
                    M[L.E1 + i] = -j;
                    M[L.E2r + i] = -j;
                    M[L.E2i + i] = 0.0;
                }
                for (int i = 0; i < N; ++i) {
                    M[L.E1 + i * N + i] += gh;
                    M[L.E2r + i * N + i] += ah;
                    M[L.E2i + i * N + i] = bh;
                }
                lu_real(M, N, L.E1, L.p1);
                lu_cplx(M, N, L.E2r, L.E2i, L.p2);
                ++nlu;
            }
            action = ACT_SAME;
            if (nstep >= rp.nmax) { status = RK_ST_STEP_LIMIT; break; }
            if (0.1 * h <= kU * t || h < 1e-300) { status = RK_ST_H_UNDERFLOW; break; }   // no longer advances t
            ++nstep;

            // starting values: zero on the first step, else the previous step's
            // collocation polynomial (Newton divided differences on the nodes
            // 0, c1, c2, 1) continued to the new stage abscissae
            if (first) {
                for (int i = 0; i < N3; ++i) M[L.Z + i] = 0.0;
            } else {
                const double c1 = rp.c1, c2 = rp.c2, r = h / hlast;
                const double t1 = 1.0 + c1 * r, t2 = 1.0 + c2 * r, t3 = 1.0 + r;
                for (int c = 0; c < N; ++c) {
                    const double z1 = M[L.Zs + c], z2 = M[L.Zs + N + c], z3 = M[L.Zs + 2 * N + c];
                    const double d01 = z1 / c1, d12 = (z2 - z1) / (c2 - c1), d23 = (z3 - z2) / (1.0 - c2);
                    const double d012 = (d12 - d01) / c2, d123 = (d23 - d12) / (1.0 - c1);
                    const double d0123 = d123 - d012;
                    M[L.Z + c] = t1 * (d01 + (t1 - c1) * (d012 + (t1 - c2) * d0123)) - z3;
                    M[L.Z + N + c] = t2 * (d01 + (t2 - c1) * (d012 + (t2 - c2) * d0123)) - z3;
                    M[L.Z + 2 * N + c] = t3 * (d01 + (t3 - c1) * (d012 + (t3 - c2) * d0123)) - z3;
                }
            }
            for (int c = 0; c < N; ++c) {
                const double z1 = M[L.Z + c], z2 = M[L.Z + N + c], z3 = M[L.Z + 2 * N + c];
                M[L.W + c] = rp.Ti[0] * z1 + rp.Ti[1] * z2 + rp.Ti[2] * z3;
                M[L.W + N + c] = rp.Ti[3] * z1 + rp.Ti[4] * z2 + rp.Ti[5] * z3;
                M[L.W + 2 * N + c] = rp.Ti[6] * z1 + rp.Ti[7] * z2 + rp.Ti[8] * z3;
            }

            // simplified Newton iteration
            eta = pow(fmax(eta, kU), 0.8);
            bool converged = false;
            int newt = 0;
            double dn_old = 1.0;
            for (int it = 1; it <= kmax; ++it) {
                for (int i = 0; i < 3; ++i) {
                    for (int c = 0; c < N; ++c) M[L.tmp + c] = M[L.y + c] + M[L.Z + i * N + c];
                    rhs(m, L, M, L.tmp, L.F + i * N, P);
                }
                nfev += 3;
                const double gh = rp.g / h, ah = rp.a / h, bh = rp.b / h;
                for (int c = 0; c < N; ++c) {
                    const double F1 = M[L.F + c], F2 = M[L.F + N + c], F3 = M[L.F + 2 * N + c];
                    const double G1 = rp.Ti[0] * F1 + rp.Ti[1] * F2 + rp.Ti[2] * F3;
                    const double G2 = rp.Ti[3] * F1 + rp.Ti[4] * F2 + rp.Ti[5] * F3;
                    const double G3 = rp.Ti[6] * F1 + rp.Ti[7] * F2 + rp.Ti[8] * F3;
                    const double W1 = M[L.W + c], W2 = M[L.W + N + c], W3 = M[L.W + 2 * N + c];
                    M[L.dW + c] = G1 - gh * W1;
                    M[L.dW + N + c] = G2 - (ah * W2 - bh * W3);
                    M[L.dW + 2 * N + c] = G3 - (bh * W2 + ah * W3);
                }
                lu_solve_real(M, N, L.E1, L.p1, L.dW);
                lu_solve_cplx(M, N, L.E2r, L.E2i, L.p2, L.dW + N, L.dW + 2 * N);
                // back to stage increments dZ = (T (x) I) dW, kept in F
                for (int c = 0; c < N; ++c) {
                    const double w1 = M[L.dW + c], w2 = M[L.dW + N + c], w3 = M[L.dW + 2 * N + c];
                    M[L.F + c] = rp.T[0] * w1 + rp.T[1] * w2 + rp.T[2] * w3;
                    M[L.F + N + c] = rp.T[3] * w1 + rp.T[4] * w2 + rp.T[5] * w3;
                    M[L.F + 2 * N + c] = rp.T[6] * w1 + rp.T[7] * w2 + rp.T[8] * w3;
                }
                ++nnewt;
                newt = it;
                const double dn = wrms(M, L.F, L.sc, N3, N);
                if (!isfinite(dn)) break;
                if (it >= 2) {
                    const double th = dn / dn_old;
                    theta = th;
                    if (th >= 0.99) break;
                    eta = th / (1.0 - th);
                    if (pow(th, (double)(kmax - it)) / (1.0 - th) * dn > kappa) break;
                }
                dn_old = fmax(dn, kU);
                for (int i = 0; i < N3; ++i) {
                    M[L.Z + i] += M[L.F + i];
                    M[L.W + i] += M[L.dW + i];
                }
                if (eta * dn <= kappa) { converged = true; break; }
            }
            if (!converged) {
                ++nnf;
                h *= 0.5;
                reject = true;
                last = false;
                action = jac_fresh ? ACT_LU : ACT_JAC;
                continue;
            }

            // embedded error estimate
            const double invh = 1.0 / h;
            for (int c = 0; c < N; ++c) {
                const double z3 = M[L.Z + 2 * N + c];
                const double dz = (rp.d[0] * M[L.Z + c] + rp.d[1] * M[L.Z + N + c] + rp.d[2] * z3) * invh;
                M[L.vv + c] = dz;
                M[L.ev + c] = M[L.f0 + c] + dz;
                const double yc = M[L.y + c];
                M[L.sc2 + c] = atol + rtol * fmax(fabs(yc), fabs(yc + z3));
            }
            lu_solve_real(M, N, L.E1, L.p1, L.ev);
            double err = fmax(wrms(M, L.ev, L.sc2, N, N), 1e-10);
            if (err >= 1.0 && (first || reject)) {
                for (int c = 0; c < N; ++c) M[L.tmp + c] = M[L.y + c] + M[L.ev + c];
                rhs(m, L, M, L.tmp, L.ev, P);
                ++nfev;
                for (int c = 0; c < N; ++c) M[L.ev + c] += M[L.vv + c];
                lu_solve_real(M, N, L.E1, L.p1, L.ev);
                err = fmax(wrms(M, L.ev, L.sc2, N, N), 1e-10);
            }
            if (!isfinite(err)) err = 1e300;

            // step-size selection
            const double fac = fmin(0.9, 0.9 * (2 * kmax + 1) / (double)(2 * kmax + newt));
            double quot = fmax(0.125, fmin(5.0, pow(err, 0.25) / fac));
            double hnew = h / quot;
            if (err < 1.0) {
                first = false;
                ++nacc;
                if (nacc > 1) {
                    double fg = (hacc / h) * pow(err * err / erracc, 0.25) / 0.9;
                    fg = fmax(0.125, fmin(5.0, fg));
                    quot = fmax(quot, fg);
                    hnew = h / quot;
                }
                hacc = h;
                erracc = fmax(1e-2, err);
                for (int i = 0; i < N3; ++i) M[L.Zs + i] = M[L.Z + i];
                hlast = h;
                for (int c = 0; c < N; ++c) {
                    const double yc = M[L.y + c] + M[L.Z + 2 * N + c];
                    M[L.y + c] = yc;
                    M[L.sc + c] = atol + rtol * fabs(yc);
                }
                t = last ? dt : t + h;
                jac_fresh = false;
                if (last) break;
                rhs(m, L, M, L.y, L.f0, P);
                ++nfev;
                if (reject) hnew = fmin(hnew, h);
                reject = false;
                if (t + 1.0001 * hnew >= dt) {   // last step: no tail shorter than 1e-4 h
                    h = dt - t;
                    last = true;
                } else {
                    const double qt = hnew / h;
                    if (theta <= 1e-3 && qt >= 1.0 && qt <= 1.2) { action = ACT_SAME; continue; }
                    h = hnew;
                }
                action = theta <= 1e-3 ? ACT_LU : ACT_JAC;
            } else {
                ++nrej;
                reject = true;
                last = false;
                h = first ? 0.1 * h : hnew;
                action = jac_fresh ? ACT_LU : ACT_JAC;
            }
        }
        for (int c = 0; c < N; ++c) yout[(size_t)c * n + s] = M[L.y + c];
        yout[(size_t)(K + 1) * n + s] = P;
    }
    cnt[(size_t)C_STATUS * n + s] = status;
    cnt[(size_t)C_NSTEP * n + s] = nstep;
    cnt[(size_t)C_NACC * n + s] = nacc;
    cnt[(size_t)C_NREJ * n + s] = nrej;
    cnt[(size_t)C_NNEWT * n + s] = nnewt;
    cnt[(size_t)C_NNFAIL * n + s] = nnf;
    cnt[(size_t)C_NFEV * n + s] = nfev;
    cnt[(size_t)C_NJEV * n + s] = njev;
    cnt[(size_t)C_NLU * n + s] = nlu;
}

// ---------------------------------------------------------------------------
// cost binning: key = ||dt f(y0)||, RMS in the error weights, one source-term
// evaluation per state; bin = floor(log2(1 + key) * nbins / 64) clamped.
// States are then ordered by descending bin (costliest first) with a
// counting sort whose atomics are aggregated per block.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void proxy_bin_kernel(DevMech m, LaneLayout L, int64_t n, const double *__restrict__ yin,
                                                       double dt, double atol, double rtol, int nbins,
                                                       int *__restrict__ bins, double *__restrict__ scratch,
                                                       int64_t nlanes) {
    Lane M{scratch + (size_t)blockIdx.x * L.total * kWave + threadIdx.x};
    const int N = m.N, K = m.K;
    for (int64_t s = (int64_t)blockIdx.x * kWave + threadIdx.x; s < n; s += nlanes) {
        const double P = yin[(size_t)(K + 1) * n + s];
        bool ok = P > 0.0 && isfinite(P);
        for (int c = 0; c < N; ++c) {
            const double v = yin[(size_t)c * n + s];
            M[L.y + c] = v;
            ok = ok && isfinite(v);
        }
        ok = ok && M[L.y] > 0.0;
        int b = nbins - 1;
        if (ok) {
            rhs(m, L, M, L.y, L.f0, P);
            double acc = 0.0;
            for (int c = 0; c < N; ++c) {
                const double t = dt * M[L.f0 + c] / (atol + rtol * fabs(M[L.y + c]));
                acc += t * t;
            }
            const double key = sqrt(acc / N);
            if (isfinite(key)) b = min(nbins - 1, max(0, (int)(log2(1.0 + key) * nbins / 64.0)));
        }
        bins[s] = b;
    }
}

__global__ __launch_bounds__(256) void bin_hist_kernel(const int *__restrict__ bins, int64_t n, int nbins,
                                                       int *__restrict__ hist) {
    __shared__ int h[64];
    if (threadIdx.x < 64) h[threadIdx.x] = 0;
    __syncthreads();
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < n; s += (int64_t)gridDim.x * blockDim.x)
        atomicAdd(&h[bins[s]], 1);
    __syncthreads();
    if (threadIdx.x < nbins && h[threadIdx.x]) atomicAdd(&hist[threadIdx.x], h[threadIdx.x]);
}

// cursor[b] = first queue position of bin b, bins in descending order
__global__ void bin_scan_kernel(const int *__restrict__ hist, int nbins, int *__restrict__ cursor) {
    if (threadIdx.x == 0) {
        int acc = 0;
        for (int b = nbins - 1; b >= 0; --b) {
            cursor[b] = acc;
            acc += hist[b];
        }
    }
}

// each block scatters a contiguous chunk: one global atomic per bin per block
__global__ __launch_bounds__(256) void bin_scatter_kernel(const int *__restrict__ bins, int64_t n, int64_t chunk,
                                                          int *__restrict__ cursor, int *__restrict__ order) {
    __shared__ int cnt[64], base[64];
    if (threadIdx.x < 64) cnt[threadIdx.x] = 0;
    __syncthreads();
    const int64_t s0 = (int64_t)blockIdx.x * chunk, s1 = min(n, s0 + chunk);
    for (int64_t s = s0 + threadIdx.x; s < s1; s += blockDim.x) atomicAdd(&cnt[bins[s]], 1);
    __syncthreads();
    if (threadIdx.x < 64) {
        base[threadIdx.x] = cnt[threadIdx.x] ? atomicAdd(&cursor[threadIdx.x], cnt[threadIdx.x]) : 0;
        cnt[threadIdx.x] = 0;
    }
    __syncthreads();
    for (int64_t s = s0 + threadIdx.x; s < s1; s += blockDim.x) {
        const int b = bins[s];
        order[base[b] + atomicAdd(&cnt[b], 1)] = (int)s;
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
LaneLayout lane_layout(int K) {
    const int N = K + 1, N2 = N * N;
    LaneLayout L{};
    int o = 0;
    auto take = [&o](int n) { const int r = o; o += n; return r; };
    L.y = take(N); L.f0 = take(N); L.sc = take(N);
    L.Z = take(3 * N); L.W = take(3 * N); L.F = take(3 * N); L.dW = take(3 * N); L.Zs = take(3 * N);
    L.ev = take(N); L.vv = take(N); L.tmp = take(N); L.sc2 = take(N);
    L.J = take(N2); L.E1 = take(N2); L.E2r = take(N2); L.E2i = take(N2); L.p1 = take(N); L.p2 = take(N);
    L.C = take(K); L.cp = take(K); L.h = take(K); L.s = take(K); L.dcp = take(K);
    L.wdot = take(K); L.dwdT = take(K); L.sS = take(K);
    L.total = o;
    return L;
}

size_t lane_scratch_doubles(int K, int64_t n) {
    const int64_t waves = (n + kWave - 1) / kWave;
    return (size_t)waves * kWave * (size_t)lane_layout(K).total;
}

static unsigned grid_of(int64_t n) { return (unsigned)((n + kWave - 1) / kWave); }

namespace {
__global__ void zero_ints_kernel(int *p, int n) {
    if ((int)threadIdx.x < n) p[threadIdx.x] = 0;
}
// first m states of a component-major [rows][n] array into a [rows][m] one
__global__ void gather_head_kernel(const double *__restrict__ src, int64_t n, int64_t m, int rows,
                                   double *__restrict__ dst) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m * rows) {
        const int64_t r = i / m, c = i % m;
        dst[i] = src[r * n + c];
    }
}
}  // namespace

hipError_t launch_gather_head(const double *src, int64_t n, int64_t m, int rows, double *dst, hipStream_t st) {
    if (m <= 0) return hipSuccess;
    hipLaunchKernelGGL(gather_head_kernel, dim3((unsigned)((m * rows + 255) / 256)), dim3(256), 0, st, src, n, m, rows,
                       dst);
    return hipGetLastError();
}

hipError_t launch_rhs(const DevMech &m, int64_t n, const double *y, double *f, double *scratch, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(rhs_kernel, dim3(grid_of(n)), dim3(kWave), 0, st, m, lane_layout(m.K), n, y, f, scratch);
    return hipGetLastError();
}

hipError_t launch_jac(const DevMech &m, int64_t n, const double *y, double *J, double *scratch, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(jac_kernel, dim3(grid_of(n)), dim3(kWave), 0, st, m, lane_layout(m.K), n, y, J, scratch);
    return hipGetLastError();
}

hipError_t launch_radau_lane(const DevMech &m, const RadauParams &p, int64_t n, const double *yin, double *yout,
                             double *scratch, int32_t *counters, const int *order, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(radau_lane_kernel, dim3(grid_of(n)), dim3(kWave), 0, st, m, lane_layout(m.K), p, n, yin, yout,
                       scratch, counters, order);
    return hipGetLastError();
}

LaneLayout proxy_layout(int K) {
    // only what one source-term evaluation touches
    const int N = K + 1;
    LaneLayout L{};
    int o = 0;
    auto take = [&o](int n) { const int r = o; o += n; return r; };
    L.y = take(N); L.f0 = take(N);
    L.C = take(K); L.cp = take(K); L.h = take(K); L.s = take(K); L.wdot = take(K);
    L.total = o;
    return L;
}

size_t proxy_scratch_doubles(int K) { return (size_t)kProxyLanes * proxy_layout(K).total; }

hipError_t launch_binning(const DevMech &m, int64_t n, const double *yin, double dt, double atol, double rtol,
                          int nbins, int *bins, int *order, int *hist, double *scratch, hipStream_t st) {
    if (n == 0) return hipSuccess;
    if (nbins < 1 || nbins > 64) return hipErrorInvalidValue;
    hipLaunchKernelGGL(proxy_bin_kernel, dim3(kProxyLanes / kWave), dim3(kWave), 0, st, m, proxy_layout(m.K), n, yin, dt,
                       atol, rtol, nbins, bins, scratch, (int64_t)kProxyLanes);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_sort_bins(bins, n, nbins, order, hist, st);
}

hipError_t launch_sort_bins(const int *bins, int64_t n, int nbins, int *order, int *hist, hipStream_t st) {
    if (n == 0) return hipSuccess;
    if (nbins < 1 || nbins > 64) return hipErrorInvalidValue;
    hipLaunchKernelGGL(zero_ints_kernel, dim3(1), dim3(128), 0, st, hist, 128);
    hipLaunchKernelGGL(bin_hist_kernel, dim3(256), dim3(256), 0, st, bins, n, nbins, hist);
    hipLaunchKernelGGL(bin_scan_kernel, dim3(1), dim3(64), 0, st, hist, nbins, hist + 64);
    const int64_t chunk = 4096;
    hipLaunchKernelGGL(bin_scatter_kernel, dim3((unsigned)((n + chunk - 1) / chunk)), dim3(256), 0, st, bins, n, chunk,
                       hist + 64, order);
    return hipGetLastError();
}

}  // namespace rk
