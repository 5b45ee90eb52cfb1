// Radau IIA with a group of G lanes cooperating on one state (the paper's
// per-block pattern, Sec. 1.2): G = 16 (a quarter wavefront, four states per
// wavefront) for mechanisms with N = K + 1 <= 16 unknowns, G = 64 (one state
// per wavefront) for N <= 56.
//
// Lane r of a group owns component r of every vector (r = 0 temperature,
// r = 1..K mass fractions) and row r of the iteration matrices.  The LU
// factors of E1 (real) and E2 (complex) stay in registers (NC columns per
// row): partial pivoting is done by row ownership (the pivot row is chosen
// among the rows not yet used, its lane records the elimination position,
// nothing moves), so every register index is a compile-time constant.
// Per-species and per-reaction intermediates of the source terms and of the
// Jacobian go through the group's slice of LDS, the reactions in chunks of at
// most 64; J itself is assembled and kept in LDS.
//
// Work distribution: a persistent grid whose groups pull states from a device
// queue (one atomic per state), so a group that finishes a cheap state starts
// the next one at once instead of idling until the costliest state of its
// wavefront is done.  The states may be visited in a caller-supplied order.
#pragma once
#include <hip/hip_runtime.h>
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <type_traits>

#include "rk_internal.h"

namespace rk {

namespace {

constexpr double kU = 2.220446049250313e-16;

__device__ __forceinline__ void sync_wave() { __syncthreads(); }   // blocks are one wavefront

// In-row (16-lane) data-parallel moves.  Every reduction below gives the same
// bits in all lanes of the group (pairwise combinations of equal operands, then
// a fixed-order combination of the four rows for G = 64), so group control
// decisions taken on reduced values are uniform within the group.
template <int CTRL>
__device__ __forceinline__ double dpp(double v) {
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const int lo = __builtin_amdgcn_mov_dpp((int)(uint32_t)u, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(uint32_t)(u >> 32), CTRL, 0xF, 0xF, false);
    return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}
template <int CTRL>
__device__ __forceinline__ uint64_t dppu(uint64_t u) {
    const int lo = __builtin_amdgcn_mov_dpp((int)(uint32_t)u, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(uint32_t)(u >> 32), CTRL, 0xF, 0xF, false);
    return ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
}
constexpr int kRowMirror = 0x140, kRowHalfMirror = 0x141, kQuadXor2 = 0x4E, kQuadXor1 = 0xB1;

// value of a lane of the wavefront (wave-uniform result)
__device__ __forceinline__ uint64_t rlaneu(uint64_t u, int lane) {
    const int lo = __builtin_amdgcn_readlane((int)(uint32_t)u, lane);
    const int hi = __builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), lane);
    return ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
}
__device__ __forceinline__ double rlane(double v, int lane) {
    return __builtin_bit_cast(double, rlaneu(__builtin_bit_cast(uint64_t, v), lane));
}
__device__ __forceinline__ float rlane(float v, int lane) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), lane));
}

template <int G>
__device__ __forceinline__ double gsum(double v) {
    v = v + dpp<kRowMirror>(v);        // lanes i, 15-i
    v = v + dpp<kRowHalfMirror>(v);    // ... and 7-i, 8+i (within each half)
    v = v + dpp<kQuadXor2>(v);
    v = v + dpp<kQuadXor1>(v);
    if constexpr (G == 64) v = (rlane(v, 0) + rlane(v, 16)) + (rlane(v, 32) + rlane(v, 48));
    return v;
}

template <int G>
__device__ __forceinline__ uint64_t gmaxu(uint64_t v) {
    uint64_t o;
    o = dppu<kRowMirror>(v); v = o > v ? o : v;
    o = dppu<kRowHalfMirror>(v); v = o > v ? o : v;
    o = dppu<kQuadXor2>(v); v = o > v ? o : v;
    o = dppu<kQuadXor1>(v); v = o > v ? o : v;
    if constexpr (G == 64) {
        const uint64_t a = rlaneu(v, 0), b = rlaneu(v, 16), c = rlaneu(v, 32), d = rlaneu(v, 48);
        const uint64_t ab = a > b ? a : b, cd = c > d ? c : d;
        v = ab > cd ? ab : cd;
    }
    return v;
}

template <int G>
__device__ __forceinline__ uint32_t gmaxu32(uint32_t v) {
    auto mx = [](uint32_t a, uint32_t b) { return a > b ? a : b; };
    v = mx(v, (uint32_t)__builtin_amdgcn_mov_dpp((int)v, kRowMirror, 0xF, 0xF, false));
    v = mx(v, (uint32_t)__builtin_amdgcn_mov_dpp((int)v, kRowHalfMirror, 0xF, 0xF, false));
    v = mx(v, (uint32_t)__builtin_amdgcn_mov_dpp((int)v, kQuadXor2, 0xF, 0xF, false));
    v = mx(v, (uint32_t)__builtin_amdgcn_mov_dpp((int)v, kQuadXor1, 0xF, 0xF, false));
    if constexpr (G == 64) {
        const uint32_t a = (uint32_t)__builtin_amdgcn_readlane((int)v, 0), b = (uint32_t)__builtin_amdgcn_readlane((int)v, 16);
        const uint32_t c = (uint32_t)__builtin_amdgcn_readlane((int)v, 32), d = (uint32_t)__builtin_amdgcn_readlane((int)v, 48);
        v = mx(mx(a, b), mx(c, d));
    }
    return v;
}

template <int G>
__device__ __forceinline__ double gb(double v, int src) { return __shfl(v, src, G); }
template <int G>
__device__ __forceinline__ float gb(float v, int src) { return __shfl(v, src, G); }
template <int G>
__device__ __forceinline__ int gbi(int v, int src) { return __shfl(v, src, G); }

// Pivot choice: lane whose non-negative magnitude is largest; key = magnitude
// bits with the log2(G) low mantissa bits replaced by (G - 1 - lane), so equal
// magnitudes go to the lowest lane; rows already used carry key 0.
template <int G>
__device__ __forceinline__ int gpivot(double mag, bool used, int lane) {
    constexpr uint64_t kMask = G - 1;
    const uint64_t key = used ? 0ull : ((__builtin_bit_cast(uint64_t, mag) & ~kMask) | (uint64_t)(kMask - lane));
    return (int)kMask - (int)(gmaxu<G>(key) & kMask);
}
// The same on FP32 magnitudes (FP32 factors): 32-bit keys, half the moves;
// magnitudes within 2^-(23 - log2 G) of each other count as equal.
template <int G>
__device__ __forceinline__ int gpivot(float mag, bool used, int lane) {
    constexpr uint32_t kMask = G - 1;
    const uint32_t key = used ? 0u : ((__builtin_bit_cast(uint32_t, mag) & ~kMask) | (kMask - (uint32_t)lane));
    return (int)kMask - (int)(gmaxu32<G>(key) & kMask);
}

// LDS slice of one group (doubles).  J is row-major with an odd leading
// dimension NC + 1, so lanes reading down a column hit distinct banks.
struct GL {
    double *C, *h, *s, *rec, *J, *prow, *vx;
    double *zs;       // previous step's stage values, [3][NC] (parked here, not in registers)
    double *hist;     // h of the last accepted step, its error, h of the last step, pressure, time
    double *f0s;      // f(y0) of the current step, [NC]
    double *q;        // net rates of all reactions (source terms): the record chunk when R <= 64
    int *ctr;         // rarely read per-state counters (lane 0 updates them)
    // mechanism tables read inside loops, staged in block-shared LDS: the
    // species -> reaction lists (entry = reaction << 4 | (nu + 8)) always,
    // the dense collision efficiencies for 16-lane groups (null otherwise:
    // the wavefront groups use the sparse rows in global memory)
    const int *spoff;
    const int *sprx;
    const double *eff;
};

// per-state counters kept in LDS
enum { K_NREJ = 0, K_NNEWT, K_NNF, K_NFEV, K_NJEV, K_NLU, K_NCTR };

__host__ __device__ constexpr int rec_chunk(int R) { return R < 64 ? R : 64; }

__host__ __device__ constexpr int group_lds_doubles(int NC, int R) {
    return 3 * NC + 8 * rec_chunk(R) + NC * (NC + 1) + 2 * NC + NC + 3 * NC + 5 + NC + (K_NCTR + 1) / 2 +
           (R > 64 ? R : 0);
}

// Block-shared LDS copies of mechanism tables (after the group slices): the
// packed species -> reaction lists, and for 16-lane groups (small
// mechanisms, four groups per block) the collision efficiencies.
struct SharedTables {
    int off_spoff, off_sprx, off_eff, bytes;
};

__host__ __device__ inline SharedTables shared_tables(int G, int K, int nsp, int n3b) {
    SharedTables t;
    t.off_spoff = 0;
    t.off_sprx = (K + 1) * 4;
    t.off_eff = ((t.off_sprx + nsp * 4) + 7) / 8 * 8;
    t.bytes = t.off_eff + (G == 16 ? n3b * K * 8 : 0);
    return t;
}

template <int G, int NC>
__host__ __device__ inline size_t block_lds_bytes(int K, int R, int nsp, int n3b) {
    return (size_t)(kWave / G) * group_lds_doubles(NC, R) * sizeof(double) + shared_tables(G, K, nsp, n3b).bytes;
}

template <int NC>
__device__ __forceinline__ GL group_lds(double *base, int R) {
    GL L;
    L.C = base;
    L.h = base + NC;
    L.s = base + 2 * NC;
    L.rec = base + 3 * NC;
    L.J = L.rec + 8 * rec_chunk(R);
    L.prow = L.J + NC * (NC + 1);
    L.vx = L.prow + 2 * NC;
    L.zs = L.vx + NC;
    L.hist = L.zs + 3 * NC;
    L.f0s = L.hist + 5;
    L.ctr = reinterpret_cast<int *>(L.f0s + NC);
    L.q = R > 64 ? L.f0s + NC + (K_NCTR + 1) / 2 : L.rec;
    return L;
}

// Stage the species lists (and, for 16-lane groups, the efficiencies) in the
// block-shared LDS after the group slices, once per block.
template <int G, int NC>
__device__ __forceinline__ void stage_tables(const DevMech &m, double *smem, GL &L) {
    const int K = m.K;
    const SharedTables tb = shared_tables(G, K, m.nsp, m.n3b);
    char *sh = reinterpret_cast<char *>(smem + (size_t)(kWave / G) * group_lds_doubles(NC, m.R));
    int *so = reinterpret_cast<int *>(sh + tb.off_spoff);
    int *sx = reinterpret_cast<int *>(sh + tb.off_sprx);
    for (int i = threadIdx.x; i <= K; i += kWave) so[i] = m.sp_off[i];
    for (int i = threadIdx.x; i < m.nsp; i += kWave) {
        const int2 e = m.sp_rx[i];
        sx[i] = (e.x << 4) | (e.y + 8);
    }
    L.spoff = so;
    L.sprx = sx;
    if constexpr (G == 16) {
        double *se = reinterpret_cast<double *>(sh + tb.off_eff);
        for (int i = threadIdx.x; i < m.n3b * K; i += kWave) se[i] = m.eff[i];
        L.eff = se;
    } else {
        L.eff = nullptr;
    }
    sync_wave();
}

struct Thermo {
    double cp, h, s, dcp;
};

__device__ __forceinline__ Thermo species_thermo(const DevMech &m, int k, double T, double lnT, double invT) {
    const double *lo = m.thermo + (size_t)k * 32;
    const double *a = T < m.Tmid[k] ? lo : lo + 16;
    Thermo t;
    t.cp = a[0] + T * (a[1] + T * (a[2] + T * (a[3] + T * a[4])));
    t.h = a[5] + T * (a[6] + T * (a[7] + T * (a[8] + T * a[9]))) + a[10] * invT;
    t.s = a[0] * lnT + T * (a[11] + T * (a[12] + T * (a[13] + T * a[14]))) + a[15];
    t.dcp = a[1] + T * (2.0 * a[2] + T * (3.0 * a[3] + T * 4.0 * a[4]));
    return t;
}

// Per-reaction quantities at (T, C): forward constant (incl. falloff) and its
// log-derivatives, equilibrium constant.
struct RxEval {
    double kf, kr, dlnkf, dlnkf_dM, dlnKc, Mc, Pf, Pp;
    int kind, nr, np;
    int4 sp;
};

// The table entries every reaction needs (slots, kind word, Arrhenius
// parameters, sum of nu).
struct RxHead {
    int4 sp;
    int info;
    int2 tbr;      // third-body row's range in the sparse efficiency entries
    double A, B, EaR, dnu;
};

__device__ __forceinline__ RxHead rx_head(const DevMech &m, int j) {
    const double4 hp = m.rhead[j];     // 32 bytes: a third of a full parameter record
    return RxHead{m.rsp[j], m.rinfo[j], m.tbr[j], hp.x, hp.y, hp.z, hp.w};
}

__device__ __forceinline__ RxEval eval_reaction(const DevMech &m, const GL &L, int j, const RxHead &hd, double T,
                                                double lnT, double invT, double lnPRT, double ctot, bool derivs) {
    RxEval e;
    e.sp = hd.sp;
    const int info = hd.info;
    const double *p = m.rpar + (size_t)j * P_NPAR;
    e.kind = info & 15;
    e.nr = (info >> 4) & 15;
    e.np = (info >> 8) & 15;
    double kf = hd.A * exp(hd.B * lnT - hd.EaR * invT);
    double dlnkf = (hd.B + hd.EaR * invT) * invT;
    double Mc = 0.0, dlnkf_dM = 0.0;
    if (e.kind != 0) {
        const int b = (info >> 12) - 1;
        if (L.eff) {
            // 16-lane groups: the dense row staged in LDS
            const double *ef = L.eff + (size_t)b * m.K;
#pragma unroll 4
            for (int k = 0; k < m.K; ++k) Mc += ef[k] * L.C[k];
        } else {
            // [M] = sum_k eff_k C_k = sum_k C_k + sum over the non-default
            // efficiencies of (eff_k - 1) C_k
            // (entries fetched eight at a time so their loads overlap)
            Mc = ctot;
            const int p1 = hd.tbr.y;
            for (int p = hd.tbr.x; p < p1; p += 8) {
                TbEnt te[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) te[u] = p + u < p1 ? m.tb[p + u] : TbEnt{0.0, 0, 0};
#pragma unroll
                for (int u = 0; u < 8; ++u)
                    if (p + u < p1) Mc += te[u].em1 * L.C[te[u].k];
            }
        }
    }
    if (e.kind == 2) {
        const double k0 = p[P_A0] * exp(p[P_B0] * lnT - p[P_EA0R] * invT);
        const double Pr = k0 * Mc / kf;
        const double ta = p[P_TA], t3 = p[P_T3], t1 = p[P_T1], t2 = p[P_T2];
        const double e3 = exp(-T / t3), e1 = exp(-T / t1), e2 = exp(-t2 * invT);
        const double Fc = (1.0 - ta) * e3 + ta * e1 + e2;
        const double lF = log10(Fc);
        const double c = -0.4 - 0.67 * lF, nn = 0.75 - 1.27 * lF;
        const double xx = log10(Pr) + c;
        const double den = nn - 0.14 * xx;
        const double f1 = xx / den, g1 = 1.0 + f1 * f1;
        if (derivs) {
            const double dlnk0 = (p[P_B0] + p[P_EA0R] * invT) * invT;
            const double dlnPr = dlnk0 - dlnkf;
            const double dFc = -(1.0 - ta) / t3 * e3 - ta / t1 * e1 + t2 * invT * invT * e2;
            const double dlF = dFc / (Fc * M_LN10);
            const double dxT = dlnPr / M_LN10 - 0.67 * dlF, dnT = -1.27 * dlF;
            const double df1T = (nn * dxT - xx * dnT) / (den * den);
            const double dl10F_T = dlF / g1 - 2.0 * lF * f1 * df1T / (g1 * g1);
            const double df1M = nn / (Mc * M_LN10) / (den * den);
            const double dl10F_M = -2.0 * lF * f1 * df1M / (g1 * g1);
            dlnkf = dlnkf + dlnPr / (1.0 + Pr) + M_LN10 * dl10F_T;
            dlnkf_dM = 1.0 / (Mc * (1.0 + Pr)) + M_LN10 * dl10F_M;
        }
        kf = kf * (Pr / (1.0 + Pr)) * exp10(lF / g1);
    }
    const int4 sp = e.sp;
    double dS = L.s[sp.z] - L.s[sp.x];
    double dH = L.h[sp.z] - L.h[sp.x];
    double Pf = L.C[sp.x], Pp = L.C[sp.z];
    if (sp.y >= 0) { dS -= L.s[sp.y]; dH -= L.h[sp.y]; Pf *= L.C[sp.y]; }
    if (sp.w >= 0) { dS += L.s[sp.w]; dH += L.h[sp.w]; Pp *= L.C[sp.w]; }
    const double dnu = hd.dnu;
    // k_r = k_f / K_c = k_f exp(-ln K_c)
    e.kf = kf;
    e.kr = kf * exp(-(dS - dH + dnu * lnPRT));
    e.dlnkf = dlnkf;
    e.dlnkf_dM = dlnkf_dM;
    e.dlnKc = (dH - dnu) * invT;
    e.Mc = Mc;
    e.Pf = Pf;
    e.Pp = Pp;
    return e;
}

struct Mix {
    double T, Wbar, rho, invW, Y, lnT, invT, lnPRT, ctot;
    bool isY;
    int k;
};

// mixture quantities and concentrations/thermo into LDS; returns lane data
template <int G>
__device__ __forceinline__ Mix mixture(const DevMech &m, const GL &L, int r, double yv, double P, Thermo &th) {
    Mix x;
    x.T = gb<G>(yv, 0);
    x.k = r - 1;
    x.isY = r >= 1 && r <= m.K;
    x.Y = x.isY ? yv : 0.0;
    x.invW = x.isY ? m.invW[x.k] : 0.0;
    const double sumYW = gsum<G>(x.Y * x.invW);
    x.Wbar = 1.0 / sumYW;
    x.rho = P * x.Wbar / (kRu * x.T);
    x.ctot = x.rho * sumYW;       // total concentration sum_k C_k
    x.lnT = log(x.T);
    x.invT = 1.0 / x.T;
    x.lnPRT = log(kPatm / (kRu * x.T));
    sync_wave();
    if (x.isY) {
        th = species_thermo(m, x.k, x.T, x.lnT, x.invT);
        L.C[x.k] = x.rho * x.Y * x.invW;
        L.h[x.k] = th.h;
        L.s[x.k] = th.s;
    } else {
        th = Thermo{0.0, 0.0, 0.0, 0.0};
    }
    sync_wave();
    return x;
}

// f(y): lane r in, lane r out.  Reaction rates of one chunk go to LDS, then
// each species lane adds its entries of that chunk in reaction order.
template <int G>
__device__ __forceinline__ double rhs_g(const DevMech &m, const GL &L, int r, double yv, double P) {
    Thermo th;
    const Mix x = mixture<G>(m, L, r, yv, P, th);
    const int R = m.R;
    // all reaction rates first (no barrier between rounds, so the loads of
    // one round overlap the arithmetic of the previous), then each species
    // lane sums its list in reaction order
    for (int j = r; j < R; j += G) {
        const RxEval e = eval_reaction(m, L, j, rx_head(m, j), x.T, x.lnT, x.invT, x.lnPRT, x.ctot, false);
        double q = e.kf * e.Pf - e.kr * e.Pp;
        if (e.kind == 1) q *= e.Mc;
        L.q[j] = q;
    }
    sync_wave();
    double wdot = 0.0;
    const int iend = x.isY ? L.spoff[x.k + 1] : 0;
    // four list entries per round: their loads (entry, then rate) overlap;
    // the sum keeps the list order
    for (int i = x.isY ? L.spoff[x.k] : 0; i < iend; i += 4) {
        int ev[4];
        double qv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) ev[u] = i + u < iend ? L.sprx[i + u] : 8;
#pragma unroll
        for (int u = 0; u < 4; ++u) qv[u] = L.q[ev[u] >> 4];
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (i + u < iend) wdot += ((ev[u] & 15) - 8) * qv[u];
    }
    sync_wave();
    const double hw = gsum<G>(x.isY ? th.h * wdot : 0.0);
    const double cpm = gsum<G>(x.isY ? x.Y * th.cp * x.invW : 0.0);
    if (r == 0) return -hw * x.T / (x.rho * cpm);
    return x.isY ? m.W[x.k] * wdot / x.rho : 0.0;
}

// Jacobian into L.J (row-major NC x (NC + 1); rows/columns beyond N are 0)
template <int G, int NC>
__device__ __forceinline__ void jac_g(const DevMech &m, const GL &L, int r, double yv, double P) {
    constexpr int LD = NC + 1;
    const int K = m.K, R = m.R, CH = rec_chunk(R);
    Thermo th;
    const Mix x = mixture<G>(m, L, r, yv, P, th);
    const double T = x.T, invT = x.invT, rho = x.rho, Wbar = x.Wbar;
    for (int i = r; i < NC * LD; i += G) L.J[i] = 0.0;
    double wdot = 0.0, dwdT = 0.0, sS = 0.0, ck = 0.0;
    int i = x.isY ? L.spoff[x.k] : 0;
    const int iend = x.isY ? L.spoff[x.k + 1] : 0;
    int jp = x.isY ? m.jl_off[x.k] : 0;
    const int jpend = x.isY ? m.jl_off[x.k + 1] : 0;
    for (int j0 = 0; j0 < R; j0 += CH) {
        const int j1 = min(R, j0 + CH);
        // per-reaction records: q, dq/dT|C, S, dense coefficient, 4 mass-action partials
        for (int j = j0 + r; j < j1; j += G) {
            const RxEval e = eval_reaction(m, L, j, rx_head(m, j), T, x.lnT, invT, x.lnPRT, x.ctot, true);
            const double Rj = e.kf * e.Pf - e.kr * e.Pp;
            const double dRdT = Rj * e.dlnkf + e.kr * e.Pp * e.dlnKc;
            const double sMA = e.kind == 1 ? e.Mc : 1.0;
            const double ctb = e.kind == 1 ? Rj : (e.kind == 2 ? Rj * e.dlnkf_dM : 0.0);
            const int4 sp = e.sp;
            const double Cr0 = L.C[sp.x], Cr1 = sp.y >= 0 ? L.C[sp.y] : 1.0;
            const double Cp0 = L.C[sp.z], Cp1 = sp.w >= 0 ? L.C[sp.w] : 1.0;
            double *rc = L.rec + 8 * (j - j0);
            rc[0] = sMA * Rj;
            rc[1] = sMA * dRdT;
            rc[2] = sMA * (e.nr * e.kf * e.Pf - e.np * e.kr * e.Pp) + ctb * e.Mc;
            rc[3] = ctb;
            rc[4] = sMA * e.kf * Cr1;
            rc[5] = sMA * e.kf * Cr0;
            rc[6] = -sMA * e.kr * Cp1;
            rc[7] = -sMA * e.kr * Cp0;
        }
        sync_wave();
        // Mkm = sum_j nu_kj dq_j/dC_m into the Y block; lane r owns column r
        // (species r-1) and walks the reactions of this chunk in its species'
        // list (mass-action slots and non-default efficiencies); the common
        // third-body part sum_j nu_kj ctb_j of row k is added with the row pass
        if (x.isY) {
            for (; jp < jpend; ++jp) {
                const JlEnt en = m.jl[jp];
                const int e = en.e, j = e >> 5;
                if (j >= j1) break;
                const int4 sp = m.rsp[j];
                const double *rc = L.rec + 8 * (j - j0);
                double dq = 0.0;
                if (e & 1) dq += rc[4];
                if (e & 2) dq += rc[5];
                if (e & 4) dq += rc[6];
                if (e & 8) dq += rc[7];
                if (e & 16) dq += rc[3] * en.em1;
                if (dq != 0.0) {
                    L.J[(1 + sp.x) * LD + r] -= dq;
                    if (sp.y >= 0) L.J[(1 + sp.y) * LD + r] -= dq;
                    L.J[(1 + sp.z) * LD + r] += dq;
                    if (sp.w >= 0) L.J[(1 + sp.w) * LD + r] += dq;
                }
            }
        }
        // species sums over this chunk, in reaction order (four list entries
        // per round so their loads overlap)
        for (bool more = true; more && i < iend;) {
            int ev[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) ev[u] = i + u < iend ? L.sprx[i + u] : (R << 4);
            double4 rv[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int jr = ev[u] >> 4;
                const double *rc = L.rec + 8 * (jr < j1 ? jr - j0 : 0);
                rv[u] = double4{rc[0], rc[1], rc[2], rc[3]};
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int jr = ev[u] >> 4, nu = (ev[u] & 15) - 8;
                more = more && jr < j1;
                if (more) {
                    wdot += nu * rv[u].x;
                    dwdT += nu * rv[u].y;
                    sS += nu * rv[u].z;
                    ck += nu * rv[u].w;     // third-body coefficient (0 for elementary reactions)
                    ++i;
                }
            }
        }
        sync_wave();
    }
    // temperature row (lane r: column r)
    const double hk = th.h * T;
    const double cpmix = gsum<G>(x.Y * th.cp * x.invW);
    const double dcpmix = gsum<G>(x.Y * th.dcp * x.invW);
    const double hw = gsum<G>(x.isY ? hk * wdot : 0.0);
    const double dHdT = gsum<G>(x.isY ? th.cp * wdot + hk * (dwdT - sS * invT) : 0.0);
    const double hsS = gsum<G>(x.isY ? hk * sS : 0.0);
    const double hck = gsum<G>(x.isY ? hk * ck : 0.0);
    const double rcp = rho * cpmix;
    const double fT = -hw / rcp;
    if (x.isY) {
        double hM = 0.0;
        for (int k = 0; k < K; ++k) hM += L.h[k] * T * L.J[(1 + k) * LD + r];
        hM += hck;      // the rows' third-body constants, summed with the enthalpies
        const double dHdY = (rho * hM - Wbar * hsS) * x.invW;
        L.J[r] = -dHdY / rcp - fT * (th.cp * x.invW / cpmix - Wbar * x.invW);
    }
    if (r == 0) L.J[0] = -dHdT / rcp - fT * (-invT + dcpmix / cpmix);
    sync_wave();
    // species rows (lane r: row r)
    if (x.isY) {
        const double Wk = m.W[x.k];
        const double fk = Wk * wdot / rho;
        const double a = Wbar * (fk - Wk * sS / rho);
        double *row = L.J + r * LD;
        row[0] = Wk / rho * (dwdT - sS * invT) + fk * invT;
        const __attribute__((address_space(4))) double *iw = (const __attribute__((address_space(4))) double *)m.invW;
        for (int c = 1; c <= K; ++c) row[c] = (Wk * (row[c] + ck) + a) * iw[c - 1];
    }
    sync_wave();
}

// First-order forward-difference Jacobian into L.J (the alternative to the
// analytical Jacobian that Sec. 3.4 compares): column c from
// (f(y + inc_c e_c) - f(y)) / inc_c, CVODE's dense difference-quotient
// increments inc_c = max(sqrt(u) |y_c|, m w_c), w_c = atol + rtol |y_c|,
// m = 1000 |h| u N ||f(y)||_w (1 when f(y) = 0).  f(y) of the step is in
// L.f0s; one group-cooperative source-term evaluation per column.
template <int G, int NC>
__device__ __forceinline__ void jac_fd_g(const DevMech &m, const GL &L, int r, double yv, double P, double h,
                                          double atol, double rtol) {
    constexpr int LD = NC + 1;
    const int N = m.N;
    const bool comp = r < N;
    const double f0 = comp ? L.f0s[r] : 0.0;
    const double w = comp ? atol + rtol * fabs(yv) : 1.0;
    const double fn = sqrt(gsum<G>(comp ? (f0 / w) * (f0 / w) : 0.0) / N);
    const double minc = fn != 0.0 ? 1000.0 * fabs(h) * kU * N * fn : 1.0;
    const double inc_l = comp ? fmax(sqrt(kU) * fabs(yv), minc * w) : 1.0;
    for (int i = r; i < NC * LD; i += G) L.J[i] = 0.0;
    sync_wave();
#pragma nounroll
    for (int c = 0; c < N; ++c) {
        const double inc = gb<G>(inc_l, c);
        const double fp = rhs_g<G>(m, L, r, yv + (r == c ? inc : 0.0), P);
        if (comp) L.J[r * LD + c] = (fp - f0) / inc;
    }
    sync_wave();
}

// ---------------------------------------------------------------------------
// LU with partial pivoting by row ownership, then rows moved to pivot order.
// Step k picks, among the rows not yet used, the one with the largest
// magnitude in column k; its lane broadcasts the row (through LDS for G = 16,
// where the four groups of a wavefront pivot on different lanes, with
// readlane for G = 64) and the remaining rows are eliminated (every register
// index is a compile-time constant).  Afterwards the rows are permuted so
// that lane k holds row k of L\U (P E = L U), which lets the substitutions
// broadcast from lane k with a constant lane index.
// ---------------------------------------------------------------------------
// S is the storage (and elimination) precision of the factors: double for
// the plain path, float for the mixed path.  Substitutions run in double.
// With float factors the matrix is equilibrated first: columns scaled by the
// error weights sc_c (a similarity with rows 1/sc_r) and rows by their
// largest entry; rs = row factor of the lane's row, cs = sc of its column.
template <typename S, int NC>
struct LUR {
    S a[NC];
    double dinv;      // 1 / U_kk of the lane's row
    int src;          // lane whose row became pivot at step r (the lane's own r beyond N)
    double rs, cs;
};

template <typename S, int NC>
struct LUC {
    S re[NC], im[NC];
    double dr, di;    // 1 / U_kk
    int src;
    double rs, cs;
};

// value of lane k of the group; k is a constant once the calling loops are
// unrolled (row_newbcast:k DPP within a 16-lane row, readlane for G = 64)
template <int G>
__device__ __forceinline__ double bcast(double v, int k) {
    if constexpr (G == 64) {
        return rlane(v, k);
    } else {
        switch (k) {
            case 0: return dpp<0x150>(v);
            case 1: return dpp<0x151>(v);
            case 2: return dpp<0x152>(v);
            case 3: return dpp<0x153>(v);
            case 4: return dpp<0x154>(v);
            case 5: return dpp<0x155>(v);
            case 6: return dpp<0x156>(v);
            case 7: return dpp<0x157>(v);
            case 8: return dpp<0x158>(v);
            case 9: return dpp<0x159>(v);
            case 10: return dpp<0x15A>(v);
            case 11: return dpp<0x15B>(v);
            case 12: return dpp<0x15C>(v);
            case 13: return dpp<0x15D>(v);
            case 14: return dpp<0x15E>(v);
            default: return dpp<0x15F>(v);
        }
    }
}

template <typename S, int G, int NC>
__device__ __forceinline__ void factor_real(LUR<S, NC> &F, const GL &L, int r, int N) {
    bool used = r >= N;
    int src = r;
    double dinv = 0.0;
#pragma unroll
    for (int k = 0; k < NC; ++k) {
        if (k < N) {
            const int p = gpivot<G>(fabs(F.a[k]), used, r);
            if (r == k) src = p;
            if constexpr (G == 64) {
                if (r == p) {
                    used = true;
                    dinv = 1.0 / (double)F.a[k];
                }
                const S pk = rlane(F.a[k], p);
                const S l = F.a[k] / pk;
                if (!used) F.a[k] = l;
#pragma unroll
                for (int c = k + 1; c < NC; ++c) {
                    const S pc = rlane(F.a[c], p);
                    if (!used) F.a[c] -= l * pc;
                }
            } else {
                if (r == p) {
                    used = true;
                    dinv = 1.0 / (double)F.a[k];
#pragma unroll
                    for (int c = k; c < NC; ++c) L.prow[c] = (double)F.a[c];
                }
                sync_wave();
                if (!used) {
                    const S l = F.a[k] / (S)L.prow[k];
                    F.a[k] = l;
#pragma unroll
                    for (int c = k + 1; c < NC; ++c) F.a[c] -= l * (S)L.prow[c];
                }
                sync_wave();
            }
        }
    }
    // lane k takes the row that became pivot at step k
#pragma unroll
    for (int c = 0; c < NC; ++c) F.a[c] = gb<G>(F.a[c], src);
    F.dinv = gb<G>(dinv, src);
    F.src = src;
}

template <typename S, int G, int NC>
__device__ __forceinline__ void factor_cplx(LUC<S, NC> &F, const GL &L, int r, int N) {
    bool used = r >= N;
    int src = r;
    double dr = 0.0, di = 0.0;
#pragma unroll
    for (int k = 0; k < NC; ++k) {
        if (k < N) {
            const double mr = F.re[k], mi = F.im[k];
            const int p = gpivot<G>((S)(mr * mr + mi * mi), used, r);
            if (r == k) src = p;
            if (r == p) {
                used = true;
                const double dd = 1.0 / (mr * mr + mi * mi);
                dr = mr * dd;
                di = -mi * dd;
                if constexpr (G != 64) {
#pragma unroll
                    for (int c = k; c < NC; ++c) { L.prow[c] = (double)F.re[c]; L.prow[NC + c] = (double)F.im[c]; }
                }
            }
            S pr, pi;
            if constexpr (G == 64) {
                pr = rlane(F.re[k], p);
                pi = rlane(F.im[k], p);
            } else {
                sync_wave();
                pr = (S)L.prow[k];
                pi = (S)L.prow[NC + k];
            }
            const S dd = (S)1 / (pr * pr + pi * pi);
            const S ir = pr * dd, ii = -pi * dd;
            const S xr = F.re[k], xi = F.im[k];
            const S lr = xr * ir - xi * ii, li = xr * ii + xi * ir;
            if (!used) {
                F.re[k] = lr;
                F.im[k] = li;
            }
#pragma unroll
            for (int c = k + 1; c < NC; ++c) {
                S ur, ui;
                if constexpr (G == 64) {
                    ur = rlane(F.re[c], p);
                    ui = rlane(F.im[c], p);
                } else {
                    ur = (S)L.prow[c];
                    ui = (S)L.prow[NC + c];
                }
                if (!used) {
                    F.re[c] -= lr * ur - li * ui;
                    F.im[c] -= lr * ui + li * ur;
                }
            }
            if constexpr (G != 64) sync_wave();
        }
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        F.re[c] = gb<G>(F.re[c], src);
        F.im[c] = gb<G>(F.im[c], src);
    }
    F.dr = gb<G>(dr, src);
    F.di = gb<G>(di, src);
    F.src = src;
}

// The two iteration matrices of a step from the lane's row of J (unit stride,
// NC entries): E1 = gh I - J (real), E2 = (ah + i bh) I - J (complex).  With
// FP32 factors they are equilibrated first: E'' = diag(1/(sc_r m_r)) E diag(sc_c),
// the column scaling applied in FP64 before rounding, the row factor m_r (the
// power of two at or below the row maximum, so exact) afterwards.
template <typename S, int G, int NC>
__device__ __forceinline__ void form_matrices(LUR<S, NC> &E1, LUC<S, NC> &E2, const double *row, bool comp, int r,
                                              double scv, double gh, double ah, double bh) {
    if constexpr (std::is_same<S, float>::value) {
        double m1 = 0.0, m2 = 0.0;
        const double isc = 1.0 / scv;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const double j = comp ? row[c] : 0.0;
            const double w = bcast<G>(scv, c) * isc;
            const double v1 = ((c == r ? gh : 0.0) - j) * w, v2 = ((c == r ? ah : 0.0) - j) * w;
            m1 = fmax(m1, fabs(v1));
            m2 = fmax(m2, fabs(v2));
            E1.a[c] = (S)v1;
            E2.re[c] = (S)v2;
        }
        const double e2i = bh;      // imaginary part: diagonal only, scale w = 1
        m2 = fmax(m2, e2i);
        const double i1 = 1.0 / exp2(floor(log2(m1))), i2 = 1.0 / exp2(floor(log2(m2)));
        const S f1 = (S)i1, f2 = (S)i2;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            E1.a[c] *= f1;
            E2.re[c] *= f2;
            E2.im[c] = (S)(c == r ? e2i * i2 : 0.0);
        }
        E1.rs = isc * i1;
        E2.rs = isc * i2;
        E1.cs = E2.cs = scv;
    } else {
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const double j = comp ? row[c] : 0.0;
            E1.a[c] = -j;
            E2.re[c] = -j;
            E2.im[c] = 0.0;
        }
#pragma unroll
        for (int c = 0; c < NC; ++c)
            if (c == r) { E1.a[c] += gh; E2.re[c] += ah; E2.im[c] = bh; }
    }
}

// factor entry widened to double at its point of use: the empty asm keeps the
// compiler from hoisting the conversions of all entries out of the Newton loop
// (which would hold a double copy of both factorisations in registers)
__device__ __forceinline__ double wide(double v) { return v; }
__device__ __forceinline__ double wide(float v) {
    asm volatile("" : "+v"(v));
    return (double)v;
}

// x = E^-1 b, component r in lane r in and out
template <typename S, int G, int NC>
__device__ __forceinline__ double solve_real(const LUR<S, NC> &F, int r, int N, double b) {
    constexpr bool eq = std::is_same<S, float>::value;     // equilibrated (FP32) factors
    double acc = gb<G>(eq ? b * F.rs : b, F.src);        // P b (equilibrated)
#pragma unroll
    for (int k = 0; k < NC; ++k)
        if (k < N) {
            const double yk = bcast<G>(acc, k);
            if (r > k) acc -= wide(F.a[k]) * yk;
        }
#pragma unroll
    for (int k = NC - 1; k >= 0; --k)
        if (k < N) {
            if (r == k) acc *= F.dinv;
            const double xk = bcast<G>(acc, k);
            if (r < k) acc -= wide(F.a[k]) * xk;
        }
    return r < N ? (eq ? acc * F.cs : acc) : 0.0;
}

template <typename S, int G, int NC>
__device__ __forceinline__ void solve_cplx(const LUC<S, NC> &F, int r, int N, double &br, double &bi) {
    constexpr bool eq = std::is_same<S, float>::value;
    double ar = gb<G>(eq ? br * F.rs : br, F.src), ai = gb<G>(eq ? bi * F.rs : bi, F.src);
#pragma unroll
    for (int k = 0; k < NC; ++k)
        if (k < N) {
            const double yr = bcast<G>(ar, k), yi = bcast<G>(ai, k);
            if (r > k) {
                const double lr = wide(F.re[k]), li = wide(F.im[k]);
                ar -= lr * yr - li * yi;
                ai -= lr * yi + li * yr;
            }
        }
#pragma unroll
    for (int k = NC - 1; k >= 0; --k)
        if (k < N) {
            if (r == k) {
                const double tr = ar * F.dr - ai * F.di;
                ai = ar * F.di + ai * F.dr;
                ar = tr;
            }
            const double xr = bcast<G>(ar, k), xi = bcast<G>(ai, k);
            if (r < k) {
                const double ur = wide(F.re[k]), ui = wide(F.im[k]);
                ar -= ur * xr - ui * xi;
                ai -= ur * xi + ui * xr;
            }
        }
    br = r < N ? (eq ? ar * F.cs : ar) : 0.0;
    bi = r < N ? (eq ? ai * F.cs : ai) : 0.0;
}

// FP64 product of the iteration matrix c I - J (J row-major in LDS) with x
// (component r in lane r), used for residuals of the mixed-precision solves
template <int NC>
__device__ __forceinline__ double ematvec(const GL &L, int r, int N, double c, double x) {
    sync_wave();
    if (r < NC) L.vx[r] = x;
    sync_wave();
    double acc = c * x;
    const double *row = L.J + (r < NC ? r : 0) * (NC + 1);
#pragma unroll
    for (int k = 0; k < NC; ++k)
        if (k < N) acc -= row[k] * L.vx[k];
    sync_wave();
    return r < N ? acc : 0.0;
}

// Substitutions with FP32 factors in FP32 arithmetic.  The factors are only
// accurate to FP32 (of the equilibrated matrices), so an FP32 substitution
// loses nothing the FP64 refinement that follows does not restore, and it
// halves the cross-lane moves (one readlane or DPP move per value, not two).
template <int CTRL>
__device__ __forceinline__ float dppf(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}
template <int G>
__device__ __forceinline__ float bcastf(float v, int k) {
    if constexpr (G == 64) {
        return rlane(v, k);
    } else {
        switch (k) {
            case 0: return dppf<0x150>(v);
            case 1: return dppf<0x151>(v);
            case 2: return dppf<0x152>(v);
            case 3: return dppf<0x153>(v);
            case 4: return dppf<0x154>(v);
            case 5: return dppf<0x155>(v);
            case 6: return dppf<0x156>(v);
            case 7: return dppf<0x157>(v);
            case 8: return dppf<0x158>(v);
            case 9: return dppf<0x159>(v);
            case 10: return dppf<0x15A>(v);
            case 11: return dppf<0x15B>(v);
            case 12: return dppf<0x15C>(v);
            case 13: return dppf<0x15D>(v);
            case 14: return dppf<0x15E>(v);
            default: return dppf<0x15F>(v);
        }
    }
}
// factor entry read at its point of use (keeps the compiler from hoisting
// copies of both factorisations out of the Newton loop)
__device__ __forceinline__ float keepf(float v) {
    asm volatile("" : "+v"(v));
    return v;
}

// x = E1^-1 b1 and (x2 + i x3) = E2^-1 (b2 + i b3) with FP32 factors, the two
// substitutions interleaved in one sweep (two independent dependency chains),
// component r in lane r in and out
template <int G, int NC>
__device__ __forceinline__ void solve_pair_f32(const LUR<float, NC> &F1, const LUC<float, NC> &F2, int r, int N,
                                               double &b1, double &br, double &bi) {
    float a1 = gb<G>((float)(b1 * F1.rs), F1.src);
    float ar = gb<G>((float)(br * F2.rs), F2.src), ai = gb<G>((float)(bi * F2.rs), F2.src);
#pragma unroll
    for (int k = 0; k < NC; ++k)
        if (k < N) {
            const float y1 = bcastf<G>(a1, k), yr = bcastf<G>(ar, k), yi = bcastf<G>(ai, k);
            if (r > k) {
                a1 -= keepf(F1.a[k]) * y1;
                const float lr = keepf(F2.re[k]), li = keepf(F2.im[k]);
                ar -= lr * yr - li * yi;
                ai -= lr * yi + li * yr;
            }
        }
    const float d1 = (float)F1.dinv, dr = (float)F2.dr, di = (float)F2.di;
#pragma unroll
    for (int k = NC - 1; k >= 0; --k)
        if (k < N) {
            if (r == k) {
                a1 *= d1;
                const float tr = ar * dr - ai * di;
                ai = ar * di + ai * dr;
                ar = tr;
            }
            const float x1 = bcastf<G>(a1, k), xr = bcastf<G>(ar, k), xi = bcastf<G>(ai, k);
            if (r < k) {
                a1 -= keepf(F1.a[k]) * x1;
                const float ur = keepf(F2.re[k]), ui = keepf(F2.im[k]);
                ar -= ur * xr - ui * xi;
                ai -= ur * xi + ui * xr;
            }
        }
    b1 = r < N ? (double)a1 * F1.cs : 0.0;
    br = r < N ? (double)ar * F2.cs : 0.0;
    bi = r < N ? (double)ai * F2.cs : 0.0;
}

// x = E1^-1 b with FP32 factors in FP32 arithmetic
template <int G, int NC>
__device__ __forceinline__ double solve_real_f32(const LUR<float, NC> &F, int r, int N, double b) {
    float acc = gb<G>((float)(b * F.rs), F.src);
#pragma unroll
    for (int k = 0; k < NC; ++k)
        if (k < N) {
            const float yk = bcastf<G>(acc, k);
            if (r > k) acc -= keepf(F.a[k]) * yk;
        }
    const float d = (float)F.dinv;
#pragma unroll
    for (int k = NC - 1; k >= 0; --k)
        if (k < N) {
            if (r == k) acc *= d;
            const float xk = bcastf<G>(acc, k);
            if (r < k) acc -= keepf(F.a[k]) * xk;
        }
    return r < N ? (double)acc * F.cs : 0.0;
}

// J x for three vectors (J row-major in LDS, FP64), one sweep over the row;
// the vectors go through the pivot-row and product buffers (contiguous, 3 NC)
template <int NC>
__device__ __forceinline__ void jv3(const GL &L, int r, int N, double x1, double x2, double x3, double &j1,
                                    double &j2, double &j3) {
    double *vb = L.prow;
    sync_wave();
    if (r < NC) {
        vb[r] = x1;
        vb[NC + r] = x2;
        vb[2 * NC + r] = x3;
    }
    sync_wave();
    double s1 = 0.0, s2 = 0.0, s3 = 0.0;
    const double *row = L.J + (r < NC ? r : 0) * (NC + 1);
#pragma unroll
    for (int k = 0; k < NC; ++k)
        if (k < N) {
            const double a = row[k];
            s1 += a * vb[k];
            s2 += a * vb[NC + k];
            s3 += a * vb[2 * NC + k];
        }
    sync_wave();
    j1 = r < N ? s1 : 0.0;
    j2 = r < N ? s2 : 0.0;
    j3 = r < N ? s3 : 0.0;
}

enum { ACT_JAC = 0, ACT_LU = 1, ACT_SAME = 2 };

// One step attempt per group per loop iteration: the groups of a wavefront run
// the same sequence of phases (refill, Jacobian, factorisation, Newton, error
// estimate, control) with per-group masks, and a group whose state is done
// takes the next state from the queue in the next iteration without waiting
// for the other groups of its wavefront.  The wavefront leaves the loop when
// no group holds a state.
// G = 16: at most 256 registers, so two wavefronts share each SIMD (the LDS
// slices of eight 4-state blocks fit a CU); the few spills cost far less than
// the latency the second wavefront hides.
template <typename S, int G, int NC, bool FDJ = false>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(G == 16 ? 2 : 1))) void radau_group_kernel(DevMech m, RadauParams rp, int64_t n,
                                                         const double *__restrict__ yin, double *__restrict__ yout,
                                                         int32_t *__restrict__ cnt, int *__restrict__ queue,
                                                         const int *__restrict__ order,
                                                         const int *__restrict__ work_n,
                                                         const double *__restrict__ pred) {
    constexpr bool kMixed = std::is_same<S, float>::value;
    extern __shared__ double smem[];
    const int r = threadIdx.x & (G - 1);
    const int grp = threadIdx.x / G;
    const int N = m.N, K = m.K;
    GL L = group_lds<NC>(smem + (size_t)grp * group_lds_doubles(NC, m.R), m.R);
    stage_tables<G, NC>(m, smem, L);
    const bool comp = r < N;                       // lane holds a state component
    const double dt = rp.dt, atol = rp.atol, rtol = rp.rtol, kappa = rp.kappa;
    const int kmax = rp.kmax;

    const int64_t nwork = work_n ? (int64_t)*work_n : n;
    LUR<S, NC> E1;
    LUC<S, NC> E2;
    int ndiv_row = 0;      // consecutive Newton divergences since the last accepted step
    bool warm = false;     // first attempt starts from the predictor
    int flags = 0;
    const int PD = 3 * N + 2;
    bool have = false, drained = false;
    int qnext = 0, qend = 0;     // queue entries taken by this group and not yet started
    int64_t s = 0;
    // per-state values that are read rarely live in LDS: pressure L.hist[3],
    // time L.hist[4], f(y0) L.f0s; the error weights are recomputed from y
    double y = 0.0, h = 0.0;
    auto scw = [&]() { return comp ? atol + rtol * fabs(y) : 1.0; };
    double eta = 1.0, theta = 1.0;
    bool last = false, first = true, reject = false, jac_fresh = false;
    int action = ACT_JAC;
    int status = 0, nstep = 0, nacc = 0;
    // counter increments go to LDS (lane 0 of the group), read once at the end
    auto bump = [&](int k, int v) {
        if (r == 0) L.ctr[k] += v;
    };

    for (;;) {
        // ---- refill: take the next state of the queue --------------------------
        if (!have && !drained) {
            // the group takes rp.tile consecutive queue entries per atomic
            if (qnext >= qend) {
                int q0 = 0;
                if (r == 0) q0 = atomicAdd(queue, rp.tile);
                qnext = gbi<G>(q0, 0);
                qend = qnext + rp.tile;
            }
            const int qi = qnext++;
            if (qi >= nwork) {
                drained = true;
            } else {
                s = order ? (int64_t)order[qi] : (int64_t)qi;
                const double P = yin[(size_t)(K + 1) * n + s];
                L.hist[3] = P;
                y = comp ? yin[(size_t)r * n + s] : 0.0;
                const bool bad_l = (comp && !isfinite(y)) || (r == 0 && !(y > 0.0)) ||
                                   (r == 0 && !(P > 0.0 && isfinite(P)));
                nstep = nacc = 0;
                if (r < K_NCTR) L.ctr[r] = 0;
                if (gsum<G>(bad_l ? 1.0 : 0.0) > 0.0) {
                    status = RK_ST_NONFINITE;
                    if (comp) yout[(size_t)r * n + s] = y;
                    if (r == 0) yout[(size_t)(K + 1) * n + s] = P;
                    if (r == 0) {
                        cnt[(size_t)C_STATUS * n + s] = status;
                        for (int c = 1; c < kNumCounters; ++c) cnt[(size_t)c * n + s] = 0;
                    }
                } else {
                    have = true;
                    status = RK_ST_OK;
                    flags = 0;
                    L.hist[4] = 0.0;
                    warm = pred != nullptr;
                    h = rp.h0;
                    if (warm) {
                        // warm start: predicted first step (0: the default rule) and stage values
                        const double *ps = pred + (size_t)s * PD;
                        if ((rp.pred_use & 1) && ps[3 * N] > 0.0) h = ps[3 * N];
                        warm = rp.pred_use != 0;
                    }
                    last = false;
                    if (1.0001 * h >= dt) { h = dt; last = true; }
                    const double f0 = rhs_g<G>(m, L, r, y, P);
                    if (r < NC) L.f0s[r] = f0;
                    bump(K_NFEV, 1);
                    first = true;
                    reject = false;
                    jac_fresh = false;
                    eta = 1.0;
                    theta = 1.0;
                    L.hist[0] = h;        // h of the last accepted step
                    L.hist[1] = 1e-2;     // its error
                    L.hist[2] = h;        // h of the last step (stage extrapolation)
                    ndiv_row = 0;
                    action = ACT_JAC;
                }
            }
        }
        if (__ballot(have) == 0ull && __ballot(!drained) == 0ull) break;
        if (!have) continue;

        // ---- one step attempt ---------------------------------------------------
        if (action == ACT_JAC) {
            if constexpr (FDJ) {
                jac_fd_g<G, NC>(m, L, r, y, L.hist[3], h, atol, rtol);
                bump(K_NFEV, N);
            } else {
                jac_g<G, NC>(m, L, r, y, L.hist[3]);
            }
            bump(K_NJEV, 1);
            jac_fresh = true;
            action = ACT_LU;
        }
        if (action == ACT_LU) {
            form_matrices<S, G, NC>(E1, E2, L.J + (r < NC ? r : 0) * (NC + 1), comp, r, scw(), rp.g / h, rp.a / h,
                                    rp.b / h);
            sync_wave();
            factor_real<S, G>(E1, L, r, N);
            factor_cplx<S, G>(E2, L, r, N);
            bump(K_NLU, 1);
        }
        action = ACT_SAME;
        bool done = false;
        if (nstep >= rp.nmax) {
            status = RK_ST_STEP_LIMIT;
            done = true;
        } else if (0.1 * h <= kU * L.hist[4] || h < 1e-300) {   // the step no longer advances t
            status = RK_ST_H_UNDERFLOW;
            done = true;
        } else {
            ++nstep;
            // starting values (collocation polynomial of the previous step)
            double Z1, Z2, Z3;
            if (first) {
                // predicted stage values (re-read here rather than held in registers)
                const bool zw = warm && comp && (rp.pred_use & 2) != 0;
                const double *ps = pred + (size_t)s * PD;
                Z1 = zw ? ps[r] : 0.0;
                Z2 = zw ? ps[N + r] : 0.0;
                Z3 = zw ? ps[2 * N + r] : 0.0;
            } else {
                const double c1 = rp.c1, c2 = rp.c2, q = h / L.hist[2];
                const double Zs1 = r < NC ? L.zs[r] : 0.0;
                const double Zs2 = r < NC ? L.zs[NC + r] : 0.0;
                const double Zs3 = r < NC ? L.zs[2 * NC + r] : 0.0;
                const double t1 = 1.0 + c1 * q, t2 = 1.0 + c2 * q, t3 = 1.0 + q;
                const double d01 = Zs1 / c1, d12 = (Zs2 - Zs1) / (c2 - c1), d23 = (Zs3 - Zs2) / (1.0 - c2);
                const double d012 = (d12 - d01) / c2, d123 = (d23 - d12) / (1.0 - c1);
                const double d0123 = d123 - d012;
                Z1 = t1 * (d01 + (t1 - c1) * (d012 + (t1 - c2) * d0123)) - Zs3;
                Z2 = t2 * (d01 + (t2 - c1) * (d012 + (t2 - c2) * d0123)) - Zs3;
                Z3 = t3 * (d01 + (t3 - c1) * (d012 + (t3 - c2) * d0123)) - Zs3;
            }
            double W1 = rp.Ti[0] * Z1 + rp.Ti[1] * Z2 + rp.Ti[2] * Z3;
            double W2 = rp.Ti[3] * Z1 + rp.Ti[4] * Z2 + rp.Ti[5] * Z3;
            double W3 = rp.Ti[6] * Z1 + rp.Ti[7] * Z2 + rp.Ti[8] * Z3;

            eta = pow(fmax(eta, kU), 0.8);
            bool converged = false, diverged = false;
            int newt = 0;
            double dn_old = 1.0;
            for (int it = 1; it <= kmax; ++it) {
                // one source-term body for the three stages (smaller code, no
                // interleaving of three evaluations competing for registers)
                double F1 = 0.0, F2 = 0.0, F3 = 0.0;
#pragma nounroll
                for (int i = 0; i < 3; ++i) {
                    const double zi = i == 0 ? Z1 : (i == 1 ? Z2 : Z3);
                    const double fi = rhs_g<G>(m, L, r, y + zi, L.hist[3]);
                    F1 = i == 0 ? fi : F1;
                    F2 = i == 1 ? fi : F2;
                    F3 = i == 2 ? fi : F3;
                }
                bump(K_NFEV, 3);
                const double gh = rp.g / h, ah = rp.a / h, bh = rp.b / h;
                const double G1 = rp.Ti[0] * F1 + rp.Ti[1] * F2 + rp.Ti[2] * F3;
                const double G2 = rp.Ti[3] * F1 + rp.Ti[4] * F2 + rp.Ti[5] * F3;
                const double G3 = rp.Ti[6] * F1 + rp.Ti[7] * F2 + rp.Ti[8] * F3;
                const double b1 = comp ? G1 - gh * W1 : 0.0;
                const double b2 = comp ? G2 - (ah * W2 - bh * W3) : 0.0;
                const double b3 = comp ? G3 - (bh * W2 + ah * W3) : 0.0;
                double dW1, dW2, dW3;
                if constexpr (kMixed) {
                    // both systems in one FP32 sweep, then one refinement step
                    // against the FP64 matrices (residuals in FP64)
                    dW1 = b1;
                    dW2 = b2;
                    dW3 = b3;
                    solve_pair_f32<G, NC>(E1, E2, r, N, dW1, dW2, dW3);
                    double j1, j2, j3;
                    jv3<NC>(L, r, N, dW1, dW2, dW3, j1, j2, j3);
                    double q1 = comp ? b1 - (gh * dW1 - j1) : 0.0;
                    double q2 = comp ? b2 - ((ah * dW2 - j2) - bh * dW3) : 0.0;
                    double q3 = comp ? b3 - ((ah * dW3 - j3) + bh * dW2) : 0.0;
                    solve_pair_f32<G, NC>(E1, E2, r, N, q1, q2, q3);
                    dW1 += q1;
                    dW2 += q2;
                    dW3 += q3;
                } else {
                    dW1 = solve_real<S, G>(E1, r, N, b1);
                    dW2 = b2;
                    dW3 = b3;
                    solve_cplx<S, G>(E2, r, N, dW2, dW3);
                }
                const double dZ1 = rp.T[0] * dW1 + rp.T[1] * dW2 + rp.T[2] * dW3;
                const double dZ2 = rp.T[3] * dW1 + rp.T[4] * dW2 + rp.T[5] * dW3;
                const double dZ3 = rp.T[6] * dW1 + rp.T[7] * dW2 + rp.T[8] * dW3;
                bump(K_NNEWT, 1);
                newt = it;
                const double sc = scw();
                const double dn = sqrt(gsum<G>(comp ? (dZ1 * dZ1 + dZ2 * dZ2 + dZ3 * dZ3) / (sc * sc) : 0.0) / (3 * N));
                if (!isfinite(dn)) { diverged = true; break; }
                if (it >= 2) {
                    const double th = dn / dn_old;
                    theta = th;
                    if (th >= 0.99) { diverged = true; break; }
                    eta = th / (1.0 - th);
                    if (pow(th, (double)(kmax - it)) / (1.0 - th) * dn > kappa) break;
                }
                dn_old = fmax(dn, kU);
                Z1 += dZ1; Z2 += dZ2; Z3 += dZ3;
                W1 += dW1; W2 += dW2; W3 += dW3;
                if (eta * dn <= kappa) { converged = true; break; }
            }
            if (!converged && warm) {
                // the prediction did not converge: restart the state exactly as a cold
                // start (default first step, zero starting values, controller memory)
                bump(K_NNF, 1);
                warm = false;
                flags |= kFlagPredFallback;
                h = rp.h0;
                last = false;
                if (1.0001 * h >= dt) { h = dt; last = true; }
                eta = 1.0;
                theta = 1.0;
                L.hist[0] = h;
                L.hist[1] = 1e-2;
                L.hist[2] = h;
                action = ACT_LU;
            } else if (!converged) {
                bump(K_NNF, 1);
                h *= 0.5;
                reject = true;
                last = false;
                action = jac_fresh ? ACT_LU : ACT_JAC;
                ndiv_row = diverged ? ndiv_row + 1 : 0;
                if (kMixed && !first && ndiv_row >= 2) {   // after start-up: hand the state to the FP64 pass
                    status = kStatusFallback;
                    done = true;
                }
            } else {
                if (warm) { flags |= kFlagPredKept; warm = false; }
                // embedded error estimate
                const double invh = 1.0 / h;
                const double dz = (rp.d[0] * Z1 + rp.d[1] * Z2 + rp.d[2] * Z3) * invh;
                const double sc2 = comp ? atol + rtol * fmax(fabs(y), fabs(y + Z3)) : 1.0;
                const double gh = rp.g / h;
                double v = comp ? L.f0s[r] + dz : 0.0;
                double ev;
                if constexpr (kMixed) {
                    ev = solve_real_f32<G, NC>(E1, r, N, v);
                    ev += solve_real_f32<G, NC>(E1, r, N, v - ematvec<NC>(L, r, N, gh, ev));   // FP64 residual
                } else {
                    ev = solve_real<S, G>(E1, r, N, v);
                }
                double err = fmax(sqrt(gsum<G>(comp ? (ev / sc2) * (ev / sc2) : 0.0) / N), 1e-10);
                if (err >= 1.0 && (first || reject)) {
                    const double fe = rhs_g<G>(m, L, r, y + ev, L.hist[3]);
                    bump(K_NFEV, 1);
                    v = comp ? fe + dz : 0.0;
                    if constexpr (kMixed) {
                        ev = solve_real_f32<G, NC>(E1, r, N, v);
                        ev += solve_real_f32<G, NC>(E1, r, N, v - ematvec<NC>(L, r, N, gh, ev));
                    } else {
                        ev = solve_real<S, G>(E1, r, N, v);
                    }
                    err = fmax(sqrt(gsum<G>(comp ? (ev / sc2) * (ev / sc2) : 0.0) / N), 1e-10);
                }
                if (!isfinite(err)) err = 1e300;

                const double fac = fmin(0.9, 0.9 * (2 * kmax + 1) / (double)(2 * kmax + newt));
                double quot = fmax(0.125, fmin(5.0, pow(err, 0.25) / fac));
                double hnew = h / quot;
                if (err < 1.0) {
                    first = false;
                    ndiv_row = 0;
                    ++nacc;
                    if (nacc > 1) {
                        double fg = (L.hist[0] / h) * pow(err * err / L.hist[1], 0.25) / 0.9;
                        fg = fmax(0.125, fmin(5.0, fg));
                        quot = fmax(quot, fg);
                        hnew = h / quot;
                    }
                    L.hist[0] = h;
                    L.hist[1] = fmax(1e-2, err);
                    L.hist[2] = h;
                    if (r < NC) {
                        L.zs[r] = Z1;
                        L.zs[NC + r] = Z2;
                        L.zs[2 * NC + r] = Z3;
                    }
                    y = comp ? y + Z3 : 0.0;
                    const double t = last ? dt : L.hist[4] + h;
                    L.hist[4] = t;
                    jac_fresh = false;
                    if (kMixed && rp.force_fb) {    // host-forced hand-back (tests of the FP64 pass)
                        status = kStatusFallback;
                        done = true;
                    } else if (last) {
                        done = true;
                    } else {
                        const double f0 = rhs_g<G>(m, L, r, y, L.hist[3]);
                        if (r < NC) L.f0s[r] = f0;
                        bump(K_NFEV, 1);
                        if (reject) hnew = fmin(hnew, h);
                        reject = false;
                        if (t + 1.0001 * hnew >= dt) {   // last step: no tail shorter than 1e-4 h
                            h = dt - t;
                            last = true;
                            action = theta <= 1e-3 ? ACT_LU : ACT_JAC;
                        } else {
                            const double qt = hnew / h;
                            if (theta <= 1e-3 && qt >= 1.0 && qt <= 1.2) {
                                action = ACT_SAME;
                            } else {
                                h = hnew;
                                action = theta <= 1e-3 ? ACT_LU : ACT_JAC;
                            }
                        }
                    }
                } else {
                    bump(K_NREJ, 1);
                    reject = true;
                    last = false;
                    h = first ? 0.1 * h : hnew;
                    action = jac_fresh ? ACT_LU : ACT_JAC;
                }
            }
        }
        if (done) {
            // a state handed to the FP64 pass leaves y_out alone: that pass
            // restarts it from y_in, which may be the same array
            const bool handed = status == kStatusFallback;
            if (comp && !handed) yout[(size_t)r * n + s] = y;
            if (r == 0) {
                if (!handed) yout[(size_t)(K + 1) * n + s] = L.hist[3];
                cnt[(size_t)C_STATUS * n + s] = status;
                cnt[(size_t)C_NSTEP * n + s] = nstep;
                cnt[(size_t)C_NACC * n + s] = nacc;
                cnt[(size_t)C_NREJ * n + s] = L.ctr[K_NREJ];
                cnt[(size_t)C_NNEWT * n + s] = L.ctr[K_NNEWT];
                cnt[(size_t)C_NNFAIL * n + s] = L.ctr[K_NNF];
                cnt[(size_t)C_NFEV * n + s] = L.ctr[K_NFEV];
                cnt[(size_t)C_NJEV * n + s] = L.ctr[K_NJEV];
                cnt[(size_t)C_NLU * n + s] = L.ctr[K_NLU];
                // the FP64 pass over handed-back states keeps the mixed pass's flags
                const int32_t prev = work_n ? cnt[(size_t)C_FLAGS * n + s] : 0;
                cnt[(size_t)C_FLAGS * n + s] = prev | flags | (status == kStatusFallback ? kFlagFp32Fallback : 0);
            }
            have = false;
        }
    }
}



// Kernel-level test entry: the integrator's own formation, factorisation and
// substitutions applied to a given J.  One group per system; the system's J
// (element (r, c) of system i at (r * N + c) * n + i) is staged in LDS in the
// integrator's row layout.  x1 = E1^-1 b1 and x2 + i x3 = E2^-1 (b2 + i b3)
// with E1 = g/h I - J, E2 = (a + i b)/h I - J; b and x are [3][N][n].  FP32
// factors are equilibrated with the error weights sc ([N][n]) and solved in
// FP32 without refinement, so x shows the FP32 path's own accuracy.
template <typename S, int G, int NC>
__global__ __launch_bounds__(64) void lu_solve_kernel(int N, int64_t n, double gh, double ah, double bh,
                                                      const double *__restrict__ J, const double *__restrict__ sc,
                                                      const double *__restrict__ b, double *__restrict__ x) {
    extern __shared__ double smem[];
    const int r = threadIdx.x & (G - 1), grp = threadIdx.x / G;
    double *Js = smem + (size_t)grp * (NC * (NC + 1) + 2 * NC);
    GL L{};
    L.prow = Js + NC * (NC + 1);
    const int64_t i = (int64_t)blockIdx.x * (kWave / G) + grp;
    const bool live = i < n;
    const bool comp = live && r < N;
    for (int e = r; e < NC * (NC + 1); e += G) {
        const int rr = e / (NC + 1), cc = e - rr * (NC + 1);
        Js[e] = (live && rr < N && cc < N) ? J[((size_t)rr * N + cc) * n + i] : 0.0;
    }
    sync_wave();
    LUR<S, NC> E1;
    LUC<S, NC> E2;
    const double scv = comp ? sc[(size_t)r * n + i] : 1.0;
    form_matrices<S, G, NC>(E1, E2, Js + (r < NC ? r : 0) * (NC + 1), comp, r, scv, gh, ah, bh);
    sync_wave();
    factor_real<S, G>(E1, L, r, N);
    factor_cplx<S, G>(E2, L, r, N);
    double b1 = comp ? b[(size_t)r * n + i] : 0.0;
    double b2 = comp ? b[((size_t)N + r) * n + i] : 0.0;
    double b3 = comp ? b[((size_t)2 * N + r) * n + i] : 0.0;
    if constexpr (std::is_same<S, float>::value) {
        solve_pair_f32<G, NC>(E1, E2, r, N, b1, b2, b3);
    } else {
        b1 = solve_real<S, G>(E1, r, N, b1);
        solve_cplx<S, G>(E2, r, N, b2, b3);
    }
    if (comp) {
        x[(size_t)r * n + i] = b1;
        x[((size_t)N + r) * n + i] = b2;
        x[((size_t)2 * N + r) * n + i] = b3;
    }
}

template <typename S, int G, int NC>
void launch_lu_solve_one(int N, int64_t n, double gh, double ah, double bh, const double *J, const double *sc,
                         const double *b, double *x, hipStream_t st) {
    const int per = kWave / G;
    const size_t lds = (size_t)per * (NC * (NC + 1) + 2 * NC) * sizeof(double);
    hipLaunchKernelGGL((lu_solve_kernel<S, G, NC>), dim3((unsigned)((n + per - 1) / per)), dim3(kWave), lds, st, N,
                       n, gh, ah, bh, J, sc, b, x);
}

// enqueue one instantiation on its persistent grid (FP64 factors with the
// forward-difference Jacobian when p.fd_jac is set)
template <typename S, int G, int NC>
void launch_one(const DevMech &m, const RadauParams &p, int64_t n, const double *yin, double *yout, int32_t *cnt,
                int *queue, const int *order, const int *work_n, const double *pred, int grid, hipStream_t st) {
    const size_t lds = block_lds_bytes<G, NC>(m.K, m.R, m.nsp, m.n3b);
    if constexpr (std::is_same<S, double>::value) {
        if (p.fd_jac) {
            hipLaunchKernelGGL((radau_group_kernel<S, G, NC, true>), dim3(grid), dim3(kWave), lds, st, m, p, n, yin,
                               yout, cnt, queue, order, work_n, pred);
            return;
        }
    }
    hipLaunchKernelGGL((radau_group_kernel<S, G, NC>), dim3(grid), dim3(kWave), lds, st, m, p, n, yin, yout, cnt, queue,
                       order, work_n, pred);
}

template <typename S, int G, int NC>
int occupancy_one(size_t lds) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, radau_group_kernel<S, G, NC>, kWave, lds) != hipSuccess)
        per_cu = 1;
    return per_cu;
}

}  // namespace
}  // namespace rk
