// Radau IIA with a whole block (eight wavefronts, 512 lanes) cooperating on
// one state, for mechanisms whose iteration matrices do not fit one wavefront
// (57 <= N <= 153 unknowns, e.g. 150 species and temperature): the paper's
// per-block pattern for large models (Sec. 1.2, Sec. 4).
//
// Lane t < N owns component t of every vector (t = 0 temperature, t = 1..K
// mass fractions).  The iteration matrices E1 (real) and E2 (complex) are
// factored in FP32 with three lanes per row: lane t = part * 170 + row holds
// columns [part * CW, part * CW + CW) of that row of both factors in registers
// (CW = 51).  Pivoting is by row ownership as in the wavefront kernels (the
// pivot row is chosen among the rows not yet used and records its elimination
// position; nothing moves), so every register index is a compile-time
// constant.  Pivot search, pivot-row broadcast and the substitutions talk
// through LDS: two barriers per elimination step and one per substitution
// step, shared by the two matrices.  The FP64 Jacobian lives in a per-block
// slab of global memory, column-major (lane r reads row r of a column with
// its neighbours: coalesced); it forms E1/E2 and gives the FP64 residuals of
// the refinement step that follows every FP32 solve.
//
// Every solve is refined against the FP64 matrices until the last
// correction is below 1e-8 in the error weights (one to four sweeps); a
// correction larger than the one before it ends the sweeps unapplied (the
// iterate is then at the FP64 rounding floor, or cond(E) * 2^-24 >= 1 and
// further sweeps would amplify the error).  A state whose Newton iteration
// diverges twice in a row after its first accepted step switches to at least
// three (at most six) sweeps per solve for the rest of the call.
//
// The FP32 factors are least accurate along the linear invariants: the
// element (and total-mass) weights w satisfy w^T J = 0, so w^T E = (g/h) w^T
// and E's smallest singular values, near g/h, lie in those directions, while
// the largest follow ||J||; cond(E) grows like h ||J|| / g.  Where
// cond(E) * 2^-24 approaches 1 the sweeps contract slowly and the sum of the
// mass fractions keeps the error of the last Newton solve, a fraction of the
// last increment (the exact solve would conserve it to rounding).
//
// Work distribution: a persistent grid whose blocks pull states from a device
// queue, optionally in a caller-supplied order.  A state's first step attempt
// may start from the predictor's step size and stage values, kept only if
// Newton converges (else the state restarts cold), as in the wavefront kernels.
#include <hip/hip_runtime.h>
#include <algorithm>
#include <cmath>
#include <cstdint>

#include "rk_group_impl.h"

namespace rk {

namespace {

constexpr int BT = 512;         // lanes per block (eight wavefronts)
constexpr int BP = 3;           // lanes per matrix row
constexpr int BRP = 170;        // rows per part: lane t = part * BRP + row
constexpr int NPB = 176;        // padded vector length in LDS
constexpr int kCW = 51;         // register columns per part (N <= 153)
constexpr int BCH = 192;        // reactions per Jacobian record chunk
constexpr int CWP = 52;         // part stride of the pivot-row buffers (16-byte segments)

// LDS of one block, offsets in doubles.  The matrix-vector product reuses the
// substitution relay for its input vector.
struct BlockLds {
    int C, h, s, Mc, q, red, key, bci, hist, ctr, svec, yb, xb, relay, scr, zs, f0s, col, prow, e1, total;
};

__host__ __device__ inline BlockLds block_layout(int R, int n3b, int N) {
    BlockLds b{};
    int o = 0;
    b.C = o; o += NPB;
    b.h = o; o += NPB;
    b.s = o; o += NPB;
    b.Mc = o; o += (n3b + 7) / 8 * 8;             // third-body concentration of every efficiency row
    b.q = o; o += ((R > 8 * BCH ? R : 8 * BCH) + 1) / 2 * 2;   // reaction rates, or Jacobian records
    b.red = o; o += 32;                            // 2 phases x 2 values x 8 wavefronts
    b.key = o; o += 32;                            // 2 buffers x 2 keys x 8 wavefronts
    b.bci = o; o += 4;
    b.hist = o; o += 8;
    b.ctr = o; o += 4;
    b.svec = o; o += NPB;
    b.yb = o; o += 3 * NPB;                        // forward results: E1, E2 real, E2 imaginary
    b.xb = o; o += 3 * NPB;                        // back-substitution results
    b.relay = o; o += 3 * NPB;                     // running sums handed to the next part
    b.scr = o; o += 9 * NPB;                       // row maxima / matrix-vector partial sums
    b.zs = o; o += 3 * NPB;
    b.f0s = o; o += NPB;
    b.col = o; o += 3 * NPB;                       // floats: 2 buffers x 3 arrays x NPB
    b.prow = o; o += 3 * NPB;                      // floats: 2 buffers x 3 arrays x NPB (16-byte aligned)
    b.e1 = o; o += (N * BP * kCW + 1) / 2;          // floats: factors of E1, column-major (ld N)
    b.total = o;
    return b;
}

struct BL {
    double *C, *h, *s, *Mc, *q, *red, *hist, *svec, *yb, *xb, *relay, *scr, *zs, *f0s;
    uint64_t *key;
    int *bci, *ctr;
    float *col, *prow;
    float *e1;        // E1 and its factors: entry (row, c) at e1[c * N + row]
};

__device__ __forceinline__ BL block_lds(double *base, int R, int n3b, int N) {
    const BlockLds o = block_layout(R, n3b, N);
    BL L;
    L.C = base + o.C;
    L.h = base + o.h;
    L.s = base + o.s;
    L.Mc = base + o.Mc;
    L.q = base + o.q;
    L.red = base + o.red;
    L.key = reinterpret_cast<uint64_t *>(base + o.key);
    L.bci = reinterpret_cast<int *>(base + o.bci);
    L.hist = base + o.hist;
    L.ctr = reinterpret_cast<int *>(base + o.ctr);
    L.svec = base + o.svec;
    L.yb = base + o.yb;
    L.xb = base + o.xb;
    L.relay = base + o.relay;
    L.scr = base + o.scr;
    L.zs = base + o.zs;
    L.f0s = base + o.f0s;
    L.col = reinterpret_cast<float *>(base + o.col);
    L.prow = reinterpret_cast<float *>(base + o.prow);
    L.e1 = reinterpret_cast<float *>(base + o.e1);
    return L;
}

__device__ __forceinline__ int wave_of(int t) { return t >> 6; }

// block sums of two values: wavefront sums, then the eight partial sums in a
// fixed order, so every lane gets the same bits; ph alternates the LDS slots
__device__ __forceinline__ void bsum2(double &a, double &b, double *red, int &ph) {
    const double wa = gsum<64>(a), wb = gsum<64>(b);
    double *sl = red + ph * 16;
    const int t = threadIdx.x;
    if ((t & 63) == 0) {
        sl[wave_of(t)] = wa;
        sl[8 + wave_of(t)] = wb;
    }
    __syncthreads();
    a = ((sl[0] + sl[1]) + (sl[2] + sl[3])) + ((sl[4] + sl[5]) + (sl[6] + sl[7]));
    b = ((sl[8] + sl[9]) + (sl[10] + sl[11])) + ((sl[12] + sl[13]) + (sl[14] + sl[15]));
    ph ^= 1;
}

struct MixB {
    double T, Wbar, rho, invW, Y, lnT, invT, lnPRT;
    bool isY;
    int k;
};

// mixture quantities (temperature reaches every lane through the block sum)
// and concentrations / thermo of the species lanes into LDS
__device__ __forceinline__ MixB mixture_b(const DevMech &m, const BL &L, int t, double yv, double P, Thermo &th,
                                          int &ph) {
    MixB x;
    x.k = t - 1;
    x.isY = t >= 1 && t <= m.K;
    x.Y = x.isY ? yv : 0.0;
    x.invW = x.isY ? m.invW[x.k] : 0.0;
    double syw = x.Y * x.invW, tt = t == 0 ? yv : 0.0;
    bsum2(syw, tt, L.red, ph);
    x.T = tt;
    x.Wbar = 1.0 / syw;
    x.rho = P * x.Wbar / (kRu * x.T);
    x.lnT = log(x.T);
    x.invT = 1.0 / x.T;
    x.lnPRT = log(kPatm / (kRu * x.T));
    if (x.isY) {
        th = species_thermo(m, x.k, x.T, x.lnT, x.invT);
        L.C[x.k] = x.rho * x.Y * x.invW;
        L.h[x.k] = th.h;
        L.s[x.k] = th.s;
    } else {
        th = Thermo{0.0, 0.0, 0.0, 0.0};
    }
    __syncthreads();
    // [M] of every efficiency row, once per evaluation: wavefront w takes rows
    // w, w + 8, ...; its lanes read the row coalesced and reduce in a fixed order
    // (four rows per pass, so the loads of the four overlap)
    const int w = wave_of(t), ln = t & 63, K = m.K;
    for (int b0 = w; b0 < m.n3b; b0 += 32) {
        double acc[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int b = b0 + 8 * u;
            acc[u] = 0.0;
            if (b < m.n3b) {
                const double *er = m.eff + (size_t)b * K;
                for (int k = ln; k < K; k += 64) acc[u] += er[k] * L.C[k];
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const double v = gsum<64>(acc[u]);
            if (ln == 0 && b0 + 8 * u < m.n3b) L.Mc[b0 + 8 * u] = v;
        }
    }
    __syncthreads();
    return x;
}

// Per-reaction quantities (as eval_reaction of the wavefront kernels, with
// the third-body concentration taken from the per-row values in LDS)
__device__ __forceinline__ RxEval eval_reaction_b(const DevMech &m, const BL &L, int j, double T, double lnT,
                                                  double invT, double lnPRT, bool derivs) {
    RxEval e;
    e.sp = m.rsp[j];
    const int info = m.rinfo[j];
    const double *p = m.rpar + (size_t)j * P_NPAR;
    e.kind = info & 15;
    e.nr = (info >> 4) & 15;
    e.np = (info >> 8) & 15;
    double kf = p[P_A] * exp(p[P_B] * lnT - p[P_EAR] * invT);
    double dlnkf = (p[P_B] + p[P_EAR] * invT) * invT;
    double Mc = 0.0, dlnkf_dM = 0.0;
    if (e.kind != 0) Mc = L.Mc[(info >> 12) - 1];
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
    const double dnu = p[P_DNU];
    const double Kc = exp(dS - dH + dnu * lnPRT);
    e.kf = kf;
    e.kr = kf / Kc;
    e.dlnkf = dlnkf;
    e.dlnkf_dM = dlnkf_dM;
    e.dlnKc = (dH - dnu) * invT;
    e.Mc = Mc;
    e.Pf = Pf;
    e.Pp = Pp;
    return e;
}

// f(y): component t in lane t (0 beyond N)
__device__ __forceinline__ double rhs_b(const DevMech &m, const BL &L, int t, double yv, double P, int &ph) {
    Thermo th;
    const MixB x = mixture_b(m, L, t, yv, P, th, ph);
    for (int j = t; j < m.R; j += BT) {
        const RxEval e = eval_reaction_b(m, L, j, x.T, x.lnT, x.invT, x.lnPRT, false);
        double q = e.kf * e.Pf - e.kr * e.Pp;
        if (e.kind == 1) q *= e.Mc;
        L.q[j] = q;
    }
    __syncthreads();
    double wdot = 0.0;
    if (x.isY) {
        // eight list entries per round: their loads (entry, then rate)
        // overlap; the sum keeps the list order
        const int i1 = m.sp_off[x.k + 1];
        for (int i = m.sp_off[x.k]; i < i1; i += 8) {
            int2 ev[8];
            double qv[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) ev[u] = i + u < i1 ? m.sp_rx[i + u] : int2{0, 0};
#pragma unroll
            for (int u = 0; u < 8; ++u) qv[u] = L.q[ev[u].x];
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (i + u < i1) wdot += ev[u].y * qv[u];
        }
    }
    double hw = x.isY ? th.h * wdot : 0.0, cpm = x.isY ? x.Y * th.cp * x.invW : 0.0;
    bsum2(hw, cpm, L.red, ph);
    if (t == 0) return -hw * x.T / (x.rho * cpm);
    return x.isY ? m.W[x.k] * wdot / x.rho : 0.0;
}

// Jacobian into the slab JS (column-major, leading dimension LDJ): lane t
// accumulates column t (species t - 1) over the reactions with non-returning
// atomic adds (the lane's own column, so the adds land in program order and
// the result is deterministic; no round trip per update), then owns row t
// for the final species-row pass.  A third-body term nu_kj ctb_j eff_j(m) is
// split as nu_kj ctb_j (1 + (eff_j(m) - 1)): the first part is the same for
// every column m of row k, so it is summed per row (c_k) and added in the
// species-row pass; only efficiencies other than 1 go through the columns.
__device__ __forceinline__ void jac_b(const DevMech &m, const BL &L, int t, double yv, double P, double *JS, int LDJ,
                                      int &ph) {
    const int K = m.K, R = m.R, N = m.N;
    Thermo th;
    const MixB x = mixture_b(m, L, t, yv, P, th, ph);
    const double T = x.T, invT = x.invT, rho = x.rho, Wbar = x.Wbar;
    for (int i = t; i < N * LDJ; i += BT) JS[i] = 0.0;
    __syncthreads();
    double *col = JS + (size_t)(t < N ? t : 0) * LDJ;
    double wdot = 0.0, dwdT = 0.0, sS = 0.0, ck = 0.0;
    int i = x.isY ? m.sp_off[x.k] : 0;
    const int iend = x.isY ? m.sp_off[x.k + 1] : 0;
    int jp = x.isY ? m.jl_off[x.k] : 0;
    const int jpend = x.isY ? m.jl_off[x.k + 1] : 0;
    double *rec = L.q;
    for (int j0 = 0; j0 < R; j0 += BCH) {
        const int j1 = min(R, j0 + BCH);
        for (int j = j0 + t; j < j1; j += BT) {
            const RxEval e = eval_reaction_b(m, L, j, T, x.lnT, invT, x.lnPRT, true);
            const double Rj = e.kf * e.Pf - e.kr * e.Pp;
            const double dRdT = Rj * e.dlnkf + e.kr * e.Pp * e.dlnKc;
            const double sMA = e.kind == 1 ? e.Mc : 1.0;
            const double ctb = e.kind == 1 ? Rj : (e.kind == 2 ? Rj * e.dlnkf_dM : 0.0);
            const int4 sp = e.sp;
            const double Cr0 = L.C[sp.x], Cr1 = sp.y >= 0 ? L.C[sp.y] : 1.0;
            const double Cp0 = L.C[sp.z], Cp1 = sp.w >= 0 ? L.C[sp.w] : 1.0;
            double *rc = rec + 8 * (j - j0);
            rc[0] = sMA * Rj;
            rc[1] = sMA * dRdT;
            rc[2] = sMA * (e.nr * e.kf * e.Pf - e.np * e.kr * e.Pp) + ctb * e.Mc;
            rc[3] = ctb;
            rc[4] = sMA * e.kf * Cr1;
            rc[5] = sMA * e.kf * Cr0;
            rc[6] = -sMA * e.kr * Cp1;
            rc[7] = -sMA * e.kr * Cp0;
        }
        __syncthreads();
        // column m (lane m + 1): the reactions of this chunk in species m's
        // list, in reaction order (reactions outside the list contribute 0)
        if (x.isY) {
            // entries fetched four at a time so their loads overlap
            bool more = true;
            while (more && jp < jpend) {
                JlEnt en[4];
                int4 spv[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) en[u] = jp + u < jpend ? m.jl[jp + u] : JlEnt{0.0, R << 5, 0};
#pragma unroll
                for (int u = 0; u < 4; ++u) spv[u] = (en[u].e >> 5) < j1 ? m.rsp[en[u].e >> 5] : int4{0, -1, 0, -1};
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int e = en[u].e, j = e >> 5;
                    more = more && j < j1;
                    if (more) {
                        const int4 sp = spv[u];
                        const double *rc = rec + 8 * (j - j0);
                        double dq = 0.0;
                        if (e & 1) dq += rc[4];
                        if (e & 2) dq += rc[5];
                        if (e & 4) dq += rc[6];
                        if (e & 8) dq += rc[7];
                        if (e & 16) dq += rc[3] * en[u].em1;
                        if (dq != 0.0) {
                            unsafeAtomicAdd(col + 1 + sp.x, -dq);
                            if (sp.y >= 0) unsafeAtomicAdd(col + 1 + sp.y, -dq);
                            unsafeAtomicAdd(col + 1 + sp.z, dq);
                            if (sp.w >= 0) unsafeAtomicAdd(col + 1 + sp.w, dq);
                        }
                        ++jp;
                    }
                }
            }
        }
        // (four list entries per round so their loads overlap; list order kept)
        for (bool more = true; more && i < iend;) {
            int2 ev[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) ev[u] = i + u < iend ? m.sp_rx[i + u] : int2{R, 0};
            double4 rv[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const double *rc = rec + 8 * (ev[u].x < j1 ? ev[u].x - j0 : 0);
                rv[u] = double4{rc[0], rc[1], rc[2], rc[3]};
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                more = more && ev[u].x < j1;
                if (more) {
                    wdot += ev[u].y * rv[u].x;
                    dwdT += ev[u].y * rv[u].y;
                    sS += ev[u].y * rv[u].z;
                    ck += ev[u].y * rv[u].w;    // third-body coefficient (0 for elementary reactions)
                    ++i;
                }
            }
        }
        __syncthreads();
    }
    // temperature row (lane t: column t)
    const double hk = th.h * T;
    double cpmix = x.Y * th.cp * x.invW, dcpmix = x.Y * th.dcp * x.invW;
    bsum2(cpmix, dcpmix, L.red, ph);
    double hw = x.isY ? hk * wdot : 0.0, dHdT = x.isY ? th.cp * wdot + hk * (dwdT - sS * invT) : 0.0;
    bsum2(hw, dHdT, L.red, ph);
    double hsS = x.isY ? hk * sS : 0.0, hck = x.isY ? hk * ck : 0.0;
    bsum2(hsS, hck, L.red, ph);
    const double rcp = rho * cpmix;
    const double fT = -hw / rcp;
    if (x.isY) {
        double hM = 0.0;
        for (int k = 0; k < K; ++k) hM += L.h[k] * T * col[1 + k];
        hM += hck;      // the rows' third-body constants, summed with the enthalpies
        const double dHdY = (rho * hM - Wbar * hsS) * x.invW;
        col[0] = -dHdY / rcp - fT * (th.cp * x.invW / cpmix - Wbar * x.invW);
    }
    if (t == 0) col[0] = -dHdT / rcp - fT * (-invT + dcpmix / cpmix);
    __syncthreads();
    // species rows (lane t: row t, coalesced over t for every column)
    if (x.isY) {
        const double Wk = m.W[x.k];
        const double fk = Wk * wdot / rho;
        const double a = Wbar * (fk - Wk * sS / rho);
        JS[t] = Wk / rho * (dwdT - sS * invT) + fk * invT;
        const __attribute__((address_space(4))) double *iw = (const __attribute__((address_space(4))) double *)m.invW;
        // batches of 16 columns: all loads of a batch issue before its stores
        for (int c0 = 1; c0 <= K; c0 += 16) {
            double v[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) v[u] = c0 + u <= K ? JS[(size_t)(c0 + u) * LDJ + t] : 0.0;
#pragma unroll
            for (int u = 0; u < 16; ++u)
                if (c0 + u <= K) JS[(size_t)(c0 + u) * LDJ + t] = (Wk * (v[u] + ck) + a) * iw[c0 + u - 1];
        }
    }
    __syncthreads();
}

// FP32 factors of one row segment of E2 (equilibrated; those of E1 are in
// LDS), the lane's elimination positions and, for the lane that holds its
// row's pivot entry, the reciprocal of that entry
template <int CW>
struct BLU {
    float re[CW], im[CW];
    int pos1, pos2;
    double d1, d2r, d2i;
    double rs1, rs2;    // row scale factors 1 / (sc_r m_r)
};

// pivot key: magnitude bits with the 8 low bits replaced by 255 - row (ties go
// to the lowest row); 0 = not a candidate
__device__ __forceinline__ uint64_t pkey(double mag, int row) {
    return (__builtin_bit_cast(uint64_t, mag) & ~255ull) | (uint64_t)(255 - row);
}

// Form E1 = g/h I - J, E2 = (a + i b)/h I - J from the slab, equilibrate them
// (columns by the error weights, rows by the power of two at or below the
// row maximum) and factor both: P E = L U, unit L stored below the diagonal.
template <int CW>
__device__ __forceinline__ void form_factor(BLU<CW> &F, const BL &L, const double *JS, int LDJ, int part, int row,
                                            bool active, int N, double gh, double ah, double bh) {
    const int t = threadIdx.x;
    double m1 = 0.0, m2 = 0.0;
    const double iscr = active ? 1.0 / L.svec[row] : 0.0;
    float *e1 = L.e1 + (active ? row : 0);      // this row of E1: entry c at e1[c * N]
#pragma unroll
    for (int j = 0; j < CW; ++j) {
        const int c = part * CW + j;
        const bool in = active && c < N;
        const double jv = in ? JS[(size_t)c * LDJ + row] : 0.0;
        const double w = in ? L.svec[c] * iscr : 0.0;
        const double v1 = ((c == row ? gh : 0.0) - jv) * w, v2 = ((c == row ? ah : 0.0) - jv) * w;
        m1 = fmax(m1, fabs(v1));
        m2 = fmax(m2, fabs(v2));
        if (active) e1[(size_t)c * N] = (float)v1;
        F.re[j] = (float)v2;
    }
    m2 = fmax(m2, bh);   // imaginary part: diagonal only (scale 1 there)
    if (active) {
        L.scr[part * NPB + row] = m1;
        L.scr[(3 + part) * NPB + row] = m2;
    }
    __syncthreads();
    if (active) {
        m1 = fmax(fmax(L.scr[row], L.scr[NPB + row]), L.scr[2 * NPB + row]);
        m2 = fmax(fmax(L.scr[3 * NPB + row], L.scr[4 * NPB + row]), L.scr[5 * NPB + row]);
    }
    if (!(m1 > 0.0) || !isfinite(m1)) m1 = 1.0;
    if (!(m2 > 0.0) || !isfinite(m2)) m2 = 1.0;
    const double i1 = 1.0 / exp2(floor(log2(m1))), i2 = 1.0 / exp2(floor(log2(m2)));
    const float f1 = (float)i1, f2 = (float)i2;
#pragma unroll
    for (int j = 0; j < CW; ++j) {
        const int c = part * CW + j;
        if (active) e1[(size_t)c * N] *= f1;
        F.re[j] *= f2;
        F.im[j] = (float)((active && c == row) ? bh * i2 : 0.0);
    }
    F.rs1 = iscr * i1;
    F.rs2 = iscr * i2;
    F.pos1 = F.pos2 = active ? N : -1;
    F.d1 = F.d2r = F.d2i = 0.0;
    bool u1 = !active, u2 = !active;
    const int w = wave_of(t), ln = t & 63;
    int buf = 0;
    for (int pk = 0; pk < BP; ++pk) {
#pragma unroll
        for (int c = 0; c < CW; ++c) {
            const int k = pk * CW + c;
            if (k < N) {
                float *cb = L.col + buf * 3 * NPB;
                float *pb = L.prow + buf * 3 * NPB;
                uint64_t *kb = L.key + buf * 16;
                const bool mine = active && part == pk;
                // pivot candidates: this column of every row, keys of the unused rows
                uint64_t k1 = 0, k2 = 0;
                if (mine) {
                    const float xr = F.re[c], xi = F.im[c], xa = e1[(size_t)k * N];
                    cb[row] = xa;
                    cb[NPB + row] = xr;
                    cb[2 * NPB + row] = xi;
                    if (!u1) k1 = pkey(fabs((double)xa), row);
                    if (!u2) k2 = pkey((double)xr * xr + (double)xi * xi, row);
                }
                k1 = gmaxu<64>(k1);
                k2 = gmaxu<64>(k2);
                if (ln == 0) {
                    kb[w] = k1;
                    kb[8 + w] = k2;
                }
                __syncthreads();
                k1 = kb[0];
                k2 = kb[8];
#pragma unroll
                for (int v = 1; v < 8; ++v) {
                    k1 = kb[v] > k1 ? kb[v] : k1;
                    k2 = kb[8 + v] > k2 ? kb[8 + v] : k2;
                }
                const int p1 = 255 - (int)(k1 & 255), p2 = 255 - (int)(k2 & 255);
                // pivot rows publish their segments; every row forms its multipliers
                if (active && row == p1) {
                    u1 = true;
                    F.pos1 = k;
#pragma unroll
                    for (int j4 = 0; j4 < (CW + 3) / 4; ++j4) {
                        const int j = 4 * j4;
                        const float *ec = e1 + (size_t)(part * CW + j) * N;
                        reinterpret_cast<float4 *>(pb + part * CWP)[j4] =
                            make_float4(ec[0], j + 1 < CW ? ec[N] : 0.0f, j + 2 < CW ? ec[2 * (size_t)N] : 0.0f,
                                        j + 3 < CW ? ec[3 * (size_t)N] : 0.0f);
                    }
                    if (part == pk) F.d1 = 1.0 / (double)cb[row];
                }
                if (active && row == p2) {
                    u2 = true;
                    F.pos2 = k;
                    float4 *wr = reinterpret_cast<float4 *>(pb + NPB + part * CWP);
                    float4 *wi = reinterpret_cast<float4 *>(pb + 2 * NPB + part * CWP);
#pragma unroll
                    for (int j4 = 0; j4 < (CW + 3) / 4; ++j4) {
                        const int j = 4 * j4;
                        wr[j4] = make_float4(F.re[j], j + 1 < CW ? F.re[j + 1] : 0.0f, j + 2 < CW ? F.re[j + 2] : 0.0f,
                                             j + 3 < CW ? F.re[j + 3] : 0.0f);
                        wi[j4] = make_float4(F.im[j], j + 1 < CW ? F.im[j + 1] : 0.0f, j + 2 < CW ? F.im[j + 2] : 0.0f,
                                             j + 3 < CW ? F.im[j + 3] : 0.0f);
                    }
                    if (part == pk) {
                        const double mr = F.re[c], mi = F.im[c];
                        const double dd = 1.0 / (mr * mr + mi * mi);
                        F.d2r = mr * dd;
                        F.d2i = -mi * dd;
                    }
                }
                float l1 = 0.0f, lr = 0.0f, li = 0.0f;
                if (!u1) l1 = cb[row] / cb[p1];
                if (!u2) {
                    const float pr = cb[NPB + p2], pi = cb[2 * NPB + p2];
                    const float dd = 1.0f / (pr * pr + pi * pi);
                    const float ir = pr * dd, ii = -pi * dd;
                    const float xr = cb[NPB + row], xi = cb[2 * NPB + row];
                    lr = xr * ir - xi * ii;
                    li = xr * ii + xi * ir;
                }
                if (mine && !u1) e1[(size_t)k * N] = l1;
                if (mine && !u2) {
                    F.re[c] = lr;
                    F.im[c] = li;
                }
                __syncthreads();
                // elimination of the unused rows (columns after k): E2 in
                // registers, then E1 in LDS in batches of 8 columns whose loads
                // all issue before the batch's stores
                if (!u2 && part >= pk) {
                    // the pivot row four entries per LDS read
                    const float4 *pr4 = reinterpret_cast<const float4 *>(pb + NPB + part * CWP);
                    const float4 *pi4 = reinterpret_cast<const float4 *>(pb + 2 * NPB + part * CWP);
#pragma unroll
                    for (int j4 = 0; j4 < (CW + 3) / 4; ++j4) {
                        if (4 * j4 + 3 > c || part > pk) {
                            const float4 a4 = pr4[j4], b4 = pi4[j4];
                            const float urv[4] = {a4.x, a4.y, a4.z, a4.w}, uiv[4] = {b4.x, b4.y, b4.z, b4.w};
#pragma unroll
                            for (int u = 0; u < 4; ++u) {
                                const int j = 4 * j4 + u;
                                if (j < CW && (j > c || part > pk)) {
                                    F.re[j] = fmaf(-lr, urv[u], fmaf(li, uiv[u], F.re[j]));
                                    F.im[j] = fmaf(-lr, uiv[u], fmaf(-li, urv[u], F.im[j]));
                                }
                            }
                        }
                    }
                }
                if (!u1 && part >= pk) {
                    constexpr int UB = 8;
#pragma unroll
                    for (int j0 = 0; j0 < CW; j0 += UB) {
                        float ev[UB], pv[UB];
#pragma unroll
                        for (int u = 0; u < UB; ++u) {
                            const int j = j0 + u;
                            const bool on = j < CW && (j > c || part > pk);
                            ev[u] = on ? e1[(size_t)(part * CW + j) * N] : 0.0f;
                            pv[u] = on ? pb[part * CWP + j] : 0.0f;
                        }
#pragma unroll
                        for (int u = 0; u < UB; ++u) {
                            const int j = j0 + u;
                            if (j < CW && (j > c || part > pk)) e1[(size_t)(part * CW + j) * N] = fmaf(-l1, pv[u], ev[u]);
                        }
                    }
                }
                buf ^= 1;
            }
        }
    }
}

// factor entry widened to double at its point of use
__device__ __forceinline__ double wd(float v) {
    asm volatile("" : "+v"(v));
    return (double)v;
}

// x = E1^-1 b1 and (x2r + i x2i) = E2^-1 (b2r + i b2i): component r in lane r
// in and out (beyond N: 0).  Column-oriented substitutions in elimination
// order; a row's running sum passes from its part-p lane to its part-(p+1)
// lane (forward) or part-(p-1) lane (backward) at the part boundaries.
// two = false skips E2 (the barriers stay).
template <int CW>
__device__ __forceinline__ void bsolve(const BLU<CW> &F, const BL &L, int part, int row, bool active, int N, bool two,
                                       double &b1, double &b2r, double &b2i) {
    const int t = threadIdx.x;
    double a1 = 0.0, ar = 0.0, ai = 0.0;
    if (t < N) {            // part-0 lanes: row t
        a1 = b1 * F.rs1;
        ar = b2r * F.rs2;
        ai = b2i * F.rs2;
    }
    double *y1 = L.yb, *yr = L.yb + NPB, *yi = L.yb + 2 * NPB;
    double *x1 = L.xb, *xr = L.xb + NPB, *xi = L.xb + 2 * NPB;
    double *r1 = L.relay, *rr = L.relay + NPB, *ri = L.relay + 2 * NPB;
    const float *e1r = L.e1 + (active ? row : 0);
    for (int pk = 0; pk < BP; ++pk) {
        if (pk > 0) {
            if (active && part == pk - 1) { r1[row] = a1; rr[row] = ar; ri[row] = ai; }
            __syncthreads();
            if (active && part == pk) { a1 = r1[row]; ar = rr[row]; ai = ri[row]; }
        }
        const bool mine = active && part == pk;
#pragma unroll
        for (int c = 0; c < CW; ++c) {
            const int k = pk * CW + c;
            if (k < N) {
                if (mine && F.pos1 == k) y1[k] = a1;
                if (two && mine && F.pos2 == k) { yr[k] = ar; yi[k] = ai; }
                const float lk = mine ? e1r[(size_t)k * N] : 0.0f;
                __syncthreads();
                if (mine && F.pos1 > k) a1 -= (double)lk * y1[k];
                if (two && mine && F.pos2 > k) {
                    const double lr = wd(F.re[c]), li = wd(F.im[c]), vr = yr[k], vi = yi[k];
                    ar -= lr * vr - li * vi;
                    ai -= lr * vi + li * vr;
                }
            }
        }
    }
    for (int pk = BP - 1; pk >= 0; --pk) {
        if (pk < BP - 1) {
            if (active && part == pk + 1) { r1[row] = a1; rr[row] = ar; ri[row] = ai; }
            __syncthreads();
            if (active && part == pk) { a1 = r1[row]; ar = rr[row]; ai = ri[row]; }
        } else {
            __syncthreads();
            if (active && part == pk) {
                a1 = F.pos1 < N ? y1[F.pos1] : 0.0;
                ar = F.pos2 < N ? yr[F.pos2] : 0.0;
                ai = F.pos2 < N ? yi[F.pos2] : 0.0;
            }
        }
        const bool mine = active && part == pk;
#pragma unroll
        for (int c = CW - 1; c >= 0; --c) {
            const int k = pk * CW + c;
            if (k < N) {
                if (mine && F.pos1 == k) x1[k] = a1 * F.d1;
                if (two && mine && F.pos2 == k) {
                    xr[k] = ar * F.d2r - ai * F.d2i;
                    xi[k] = ar * F.d2i + ai * F.d2r;
                }
                const float uk = mine ? e1r[(size_t)k * N] : 0.0f;
                __syncthreads();
                if (mine && F.pos1 < k) a1 -= (double)uk * x1[k];
                if (two && mine && F.pos2 < k) {
                    const double ur = wd(F.re[c]), ui = wd(F.im[c]), vr = xr[k], vi = xi[k];
                    ar -= ur * vr - ui * vi;
                    ai -= ur * vi + ui * vr;
                }
            }
        }
    }
    __syncthreads();
    if (t < N) {
        const double sc = L.svec[t];
        b1 = x1[t] * sc;
        b2r = two ? xr[t] * sc : 0.0;
        b2i = two ? xi[t] * sc : 0.0;
    } else {
        b1 = b2r = b2i = 0.0;
    }
}

// J v for up to three vectors (component r in lane r), FP64, from the slab
template <int CW>
__device__ __forceinline__ void bjv3(const BL &L, const double *JS, int LDJ, int part, int row, bool active, int N,
                                     int nv, double &v1, double &v2, double &v3) {
    const int t = threadIdx.x;
    double *vx = L.relay;
    if (t < N) { vx[t] = v1; vx[NPB + t] = v2; vx[2 * NPB + t] = v3; }
    __syncthreads();
    double s1 = 0.0, s2 = 0.0, s3 = 0.0;
    if (active) {
        // batches of 17 columns: the loads of a batch issue before its sums
        constexpr int B = 17;
#pragma unroll
        for (int j0 = 0; j0 < CW; j0 += B) {
            double jv[B];
#pragma unroll
            for (int u = 0; u < B; ++u) {
                const int c = part * CW + j0 + u;
                jv[u] = (j0 + u < CW && c < N) ? JS[(size_t)c * LDJ + row] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < B; ++u) {
                const int c = part * CW + j0 + u;
                if (j0 + u < CW && c < N) {
                    s1 += jv[u] * vx[c];
                    if (nv > 1) {
                        s2 += jv[u] * vx[NPB + c];
                        s3 += jv[u] * vx[2 * NPB + c];
                    }
                }
            }
        }
        L.scr[(part * 3) * NPB + row] = s1;
        L.scr[(part * 3 + 1) * NPB + row] = s2;
        L.scr[(part * 3 + 2) * NPB + row] = s3;
    }
    __syncthreads();
    if (t < N) {
        const double *p = L.scr;
        v1 = (p[t] + p[3 * NPB + t]) + p[6 * NPB + t];
        v2 = (p[NPB + t] + p[4 * NPB + t]) + p[7 * NPB + t];
        v3 = (p[2 * NPB + t] + p[5 * NPB + t]) + p[8 * NPB + t];
    } else {
        v1 = v2 = v3 = 0.0;
    }
    __syncthreads();
}

// One state per block, the step sequence of the wavefront kernels: refill,
// Jacobian, factorisation, Newton, error estimate, control.  Every control
// decision is taken on block-uniform values.
template <int CW>
__global__ __launch_bounds__(BT) void radau_block_kernel(DevMech m, RadauParams rp, int64_t n,
                                                         const double *__restrict__ yin, double *__restrict__ yout,
                                                         int32_t *__restrict__ cnt, int *__restrict__ queue,
                                                         const int *__restrict__ order, double *__restrict__ slab,
                                                         int LDJ, const double *__restrict__ pred) {
    extern __shared__ double smem[];
    const BL L = block_lds(smem, m.R, m.n3b, m.N);
    const int t = threadIdx.x, part = t / BRP, row = t - part * BRP;
    const int N = m.N, K = m.K;
    const bool active = part < BP && row < N, comp = t < N;
    double *JS = slab + (size_t)blockIdx.x * N * LDJ;
    const double dt = rp.dt, atol = rp.atol, rtol = rp.rtol, kappa = rp.kappa;
    const int kmax = rp.kmax;
    int ph = 0;
    BLU<CW> F;
    double y = 0.0, h = 0.0, eta = 1.0, theta = 1.0;
    bool last = false, first = true, reject = false, jac_fresh = false, fb = false;
    bool warm = false;     // first attempt starts from the predictor (as the wavefront kernels)
    const int PD = 3 * m.N + 2;
    int action = ACT_JAC, status = 0, nstep = 0, nacc = 0, ndiv_row = 0, flags = 0;
    int64_t s = 0;
    auto scw = [&]() { return comp ? atol + rtol * fabs(y) : 1.0; };
    auto bump = [&](int k, int v) {
        if (t == 0) L.ctr[k] += v;
    };
    bool have = false;
    int qnext = 0, qend = 0;     // queue entries taken by this block and not yet started

    for (;;) {
        if (!have) {
            // the block takes rp.tile consecutive queue entries per atomic
            if (qnext >= qend) {
                if (t == 0) L.bci[0] = atomicAdd(queue, rp.tile);
                __syncthreads();
                qnext = L.bci[0];
                qend = qnext + rp.tile;
            }
            const int qi = qnext++;
            if (qi >= n) break;
            s = order ? (int64_t)order[qi] : (int64_t)qi;
            const double P = yin[(size_t)(K + 1) * n + s];
            y = comp ? yin[(size_t)t * n + s] : 0.0;
            double bad = ((comp && !isfinite(y)) || (t == 0 && !(y > 0.0)) || (t == 0 && !(P > 0.0 && isfinite(P))))
                             ? 1.0 : 0.0, zero = 0.0;
            bsum2(bad, zero, L.red, ph);     // also orders the read of bci before its next write
            nstep = nacc = 0;
            if (t < 8) L.ctr[t] = 0;
            if (bad > 0.0) {
                if (comp) yout[(size_t)t * n + s] = y;
                if (t == 0) {
                    yout[(size_t)(K + 1) * n + s] = P;
                    cnt[(size_t)C_STATUS * n + s] = RK_ST_NONFINITE;
                    for (int c = 1; c < kNumCounters; ++c) cnt[(size_t)c * n + s] = 0;
                }
                __syncthreads();
                continue;
            }
            have = true;
            status = RK_ST_OK;
            flags = rp.fp64_solves ? kFlagFp32Fallback : 0;
            fb = rp.fp64_solves != 0;
            h = rp.h0;
            // warm start: predicted first step (0: the default rule) and stage values
            warm = pred != nullptr && rp.pred_use != 0;
            if (warm && (rp.pred_use & 1) && pred[(size_t)s * PD + 3 * N] > 0.0) h = pred[(size_t)s * PD + 3 * N];
            last = false;
            if (1.0001 * h >= dt) { h = dt; last = true; }
            if (t == 0) { L.hist[3] = P; L.hist[4] = 0.0; }
            __syncthreads();
            const double f0 = rhs_b(m, L, t, y, P, ph);
            if (comp) L.f0s[t] = f0;
            bump(K_NFEV, 1);
            first = true;
            reject = false;
            jac_fresh = false;
            eta = 1.0;
            theta = 1.0;
            if (t == 0) { L.hist[0] = h; L.hist[1] = 1e-2; L.hist[2] = h; }
            ndiv_row = 0;
            action = ACT_JAC;
            __syncthreads();
        }
        const double P = L.hist[3];

        if (action == ACT_JAC) {
            jac_b(m, L, t, y, P, JS, LDJ, ph);
            bump(K_NJEV, 1);
            jac_fresh = true;
            action = ACT_LU;
        }
        if (action == ACT_LU) {
            if (comp) L.svec[t] = scw();
            __syncthreads();
            form_factor<CW>(F, L, JS, LDJ, part, row, active, N, rp.g / h, rp.a / h, rp.b / h);
            bump(K_NLU, 1);
        }
        action = ACT_SAME;
        bool done = false;
        const double tcur = L.hist[4];
        if (nstep >= rp.nmax) {
            status = RK_ST_STEP_LIMIT;
            done = true;
        } else if (0.1 * h <= kU * tcur || h < 1e-300) {
            status = RK_ST_H_UNDERFLOW;
            done = true;
        } else {
            ++nstep;
            double Z1 = 0.0, Z2 = 0.0, Z3 = 0.0;
            if (first) {
                if (warm && comp && (rp.pred_use & 2)) {
                    const double *ps = pred + (size_t)s * PD;
                    Z1 = ps[t];
                    Z2 = ps[N + t];
                    Z3 = ps[2 * N + t];
                }
            } else {
                const double c1 = rp.c1, c2 = rp.c2, q = h / L.hist[2];
                const double Zs1 = comp ? L.zs[t] : 0.0;
                const double Zs2 = comp ? L.zs[NPB + t] : 0.0;
                const double Zs3 = comp ? L.zs[2 * NPB + t] : 0.0;
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
            // refinement sweeps per solve: at least nref, then more while the last
            // correction is above 1e-8 in the error weights (an ill-conditioned
            // iteration matrix needs more than one sweep for an FP64-accurate
            // solve), at most nref_max
            const int nref = fb ? 3 : 1, nref_max = fb ? 6 : 4;
            const double sci = comp ? 1.0 / scw() : 0.0;

            eta = pow(fmax(eta, kU), 0.8);
            bool converged = false, diverged = false;
            int newt = 0;
            double dn_old = 1.0;
            const double gh = rp.g / h, ah = rp.a / h, bh = rp.b / h;
            for (int it = 1; it <= kmax; ++it) {
                double F1 = 0.0, F2 = 0.0, F3 = 0.0;
#pragma nounroll
                for (int i = 0; i < 3; ++i) {
                    const double zi = i == 0 ? Z1 : (i == 1 ? Z2 : Z3);
                    const double fi = rhs_b(m, L, t, y + zi, P, ph);
                    F1 = i == 0 ? fi : F1;
                    F2 = i == 1 ? fi : F2;
                    F3 = i == 2 ? fi : F3;
                }
                bump(K_NFEV, 3);
                const double G1 = rp.Ti[0] * F1 + rp.Ti[1] * F2 + rp.Ti[2] * F3;
                const double G2 = rp.Ti[3] * F1 + rp.Ti[4] * F2 + rp.Ti[5] * F3;
                const double G3 = rp.Ti[6] * F1 + rp.Ti[7] * F2 + rp.Ti[8] * F3;
                const double b1 = comp ? G1 - gh * W1 : 0.0;
                const double b2 = comp ? G2 - (ah * W2 - bh * W3) : 0.0;
                const double b3 = comp ? G3 - (bh * W2 + ah * W3) : 0.0;
                // the solve and its refinement sweeps share one substitution
                // site (rf = -1: the plain solve)
                double dW1 = 0.0, dW2 = 0.0, dW3 = 0.0, cn_prev = 1e300;
#pragma nounroll
                for (int rf = -1; rf < nref_max; ++rf) {
                    double q1 = b1, q2 = b2, q3 = b3;
                    if (rf >= 0) {
                        // refinement against the FP64 matrices
                        double j1 = dW1, j2 = dW2, j3 = dW3;
                        bjv3<CW>(L, JS, LDJ, part, row, active, N, 3, j1, j2, j3);
                        q1 = comp ? b1 - (gh * dW1 - j1) : 0.0;
                        q2 = comp ? b2 - ((ah * dW2 - j2) - bh * dW3) : 0.0;
                        q3 = comp ? b3 - ((ah * dW3 - j3) + bh * dW2) : 0.0;
                    }
                    bsolve<CW>(F, L, part, row, active, N, true, q1, q2, q3);
                    if (rf < 0) {
                        dW1 = q1;
                        dW2 = q2;
                        dW3 = q3;
                        continue;
                    }
                    double cn = ((q1 * sci) * (q1 * sci) + (q2 * sci) * (q2 * sci)) + (q3 * sci) * (q3 * sci), zc = 0.0;
                    bsum2(cn, zc, L.red, ph);
                    if (!(cn < cn_prev)) break;
                    dW1 += q1;
                    dW2 += q2;
                    dW3 += q3;
                    if (rf + 1 >= nref && sqrt(cn / (3 * N)) <= 1e-8) break;
                    cn_prev = cn;
                }
                const double dZ1 = rp.T[0] * dW1 + rp.T[1] * dW2 + rp.T[2] * dW3;
                const double dZ2 = rp.T[3] * dW1 + rp.T[4] * dW2 + rp.T[5] * dW3;
                const double dZ3 = rp.T[6] * dW1 + rp.T[7] * dW2 + rp.T[8] * dW3;
                bump(K_NNEWT, 1);
                newt = it;
                const double sc = scw();
                double ss = comp ? (dZ1 * dZ1 + dZ2 * dZ2 + dZ3 * dZ3) / (sc * sc) : 0.0, zero = 0.0;
                bsum2(ss, zero, L.red, ph);
                const double dn = sqrt(ss / (3 * N));
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
                // the prediction did not converge: restart the state exactly as a
                // cold start (default first step, zero starting values, controller
                // memory); J at y0 stays valid
                bump(K_NNF, 1);
                warm = false;
                flags |= kFlagPredFallback;
                h = rp.h0;
                last = false;
                if (1.0001 * h >= dt) { h = dt; last = true; }
                eta = 1.0;
                theta = 1.0;
                if (t == 0) { L.hist[0] = h; L.hist[1] = 1e-2; L.hist[2] = h; }
                action = ACT_LU;
            } else if (!converged) {
                bump(K_NNF, 1);
                h *= 0.5;
                reject = true;
                last = false;
                action = jac_fresh ? ACT_LU : ACT_JAC;
                ndiv_row = diverged ? ndiv_row + 1 : 0;
                if (!first && ndiv_row >= 2 && !fb) {    // after start-up: FP64-accurate solves from here on
                    fb = true;
                    flags |= kFlagFp32Fallback;
                }
            } else {
                if (warm) {
                    flags |= kFlagPredKept;
                    warm = false;
                }
                const double invh = 1.0 / h;
                const double dz = (rp.d[0] * Z1 + rp.d[1] * Z2 + rp.d[2] * Z3) * invh;
                const double sc2 = comp ? atol + rtol * fmax(fabs(y), fabs(y + Z3)) : 1.0;
                double v = comp ? L.f0s[t] + dz : 0.0;
                double ev = 0.0, err = 1.0;
                // at most two attempts (the second with f(y0 + err) on a first
                // or post-rejection step); one solve-and-refine site for both
#pragma nounroll
                for (int att = 0; att < 2; ++att) {
                    if (att == 1) {
                        const double fe = rhs_b(m, L, t, y + ev, P, ph);
                        bump(K_NFEV, 1);
                        v = comp ? fe + dz : 0.0;
                    }
                    double cn_prev = 1e300;
#pragma nounroll
                    for (int rf = -1; rf < nref_max; ++rf) {
                        double q1 = v, u2 = 0.0, u3 = 0.0;
                        if (rf >= 0) {
                            double j1 = ev, j2 = 0.0, j3 = 0.0;
                            bjv3<CW>(L, JS, LDJ, part, row, active, N, 1, j1, j2, j3);
                            q1 = comp ? v - (gh * ev - j1) : 0.0;
                        }
                        bsolve<CW>(F, L, part, row, active, N, false, q1, u2, u3);
                        if (rf < 0) {
                            ev = q1;
                            continue;
                        }
                        double cn = (q1 * sci) * (q1 * sci), zc = 0.0;
                        bsum2(cn, zc, L.red, ph);
                        if (!(cn < cn_prev)) break;
                        ev += q1;
                        if (rf + 1 >= nref && sqrt(cn / N) <= 1e-8) break;
                        cn_prev = cn;
                    }
                    double e2 = comp ? (ev / sc2) * (ev / sc2) : 0.0, zero = 0.0;
                    bsum2(e2, zero, L.red, ph);
                    err = fmax(sqrt(e2 / N), 1e-10);
                    if (att == 1 || !(err >= 1.0 && (first || reject))) break;
                }
                if (!isfinite(err)) err = 1e300;

                const double fac = fmin(0.9, 0.9 * (2 * kmax + 1) / (double)(2 * kmax + newt));
                double quot = fmax(0.125, fmin(5.0, pow(err, 0.25) / fac));
                double hnew = h / quot;
                if (err < 1.0) {
                    first = false;
                    ndiv_row = 0;
                    ++nacc;
                    if (rp.force_fb && !fb) {    // host-forced switch (tests of the FP64-accurate solves)
                        fb = true;
                        flags |= kFlagFp32Fallback;
                    }
                    const double hacc = L.hist[0], eacc = L.hist[1];
                    if (nacc > 1) {
                        double fg = (hacc / h) * pow(err * err / eacc, 0.25) / 0.9;
                        fg = fmax(0.125, fmin(5.0, fg));
                        quot = fmax(quot, fg);
                        hnew = h / quot;
                    }
                    const double tn = last ? dt : tcur + h;
                    __syncthreads();    // every lane has read hist before lane 0 rewrites it
                    if (t == 0) {
                        L.hist[0] = h;
                        L.hist[1] = fmax(1e-2, err);
                        L.hist[2] = h;
                        L.hist[4] = tn;
                    }
                    if (comp) {
                        L.zs[t] = Z1;
                        L.zs[NPB + t] = Z2;
                        L.zs[2 * NPB + t] = Z3;
                    }
                    y = comp ? y + Z3 : 0.0;
                    jac_fresh = false;
                    if (last) {
                        done = true;
                    } else {
                        const double f0 = rhs_b(m, L, t, y, P, ph);
                        if (comp) L.f0s[t] = f0;
                        bump(K_NFEV, 1);
                        if (reject) hnew = fmin(hnew, h);
                        reject = false;
                        if (tn + 1.0001 * hnew >= dt) {
                            h = dt - tn;
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
            __syncthreads();
            if (comp) yout[(size_t)t * n + s] = y;
            if (t == 0) {
                yout[(size_t)(K + 1) * n + s] = L.hist[3];
                cnt[(size_t)C_STATUS * n + s] = status;
                cnt[(size_t)C_NSTEP * n + s] = nstep;
                cnt[(size_t)C_NACC * n + s] = nacc;
                cnt[(size_t)C_NREJ * n + s] = L.ctr[K_NREJ];
                cnt[(size_t)C_NNEWT * n + s] = L.ctr[K_NNEWT];
                cnt[(size_t)C_NNFAIL * n + s] = L.ctr[K_NNF];
                cnt[(size_t)C_NFEV * n + s] = L.ctr[K_NFEV];
                cnt[(size_t)C_NJEV * n + s] = L.ctr[K_NJEV];
                cnt[(size_t)C_NLU * n + s] = L.ctr[K_NLU];
                cnt[(size_t)C_FLAGS * n + s] = flags;
            }
            __syncthreads();
            have = false;
        }
    }
}

__global__ void reset_block_queue_kernel(int *q) {
    if (threadIdx.x == 0) q[0] = 0;
}

}  // namespace

bool block_supported(int N) { return N > 56 && N <= BP * kCW && N <= BRP; }

int block_ldj(int N) { return N + (N & 1); }

size_t block_lds_bytes(const DevMech &m) { return (size_t)block_layout(m.R, m.n3b, m.N).total * sizeof(double); }

size_t block_slab_doubles(int N, int grid) { return (size_t)grid * N * block_ldj(N); }

int block_max_blocks(const DevMech &m) {
    // more than 64 KB of LDS per block (E1 and its factors live there)
    (void)hipFuncSetAttribute((const void *)radau_block_kernel<kCW>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)block_lds_bytes(m));
    (void)hipGetLastError();
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, radau_block_kernel<kCW>, BT, block_lds_bytes(m)) !=
            hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    int dev = 0, cus = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    return per_cu * std::max(1, cus);
}

hipError_t launch_radau_block(const DevMech &m, const RadauParams &p, int64_t n, const double *yin, double *yout,
                              int32_t *counters, int *queue, const int *order, double *slab, const double *pred,
                              int grid, hipStream_t st) {
    if (n == 0) return hipSuccess;
    if (!block_supported(m.N) || grid < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(reset_block_queue_kernel, dim3(1), dim3(64), 0, st, queue);
    hipLaunchKernelGGL((radau_block_kernel<kCW>), dim3(grid), dim3(BT), block_lds_bytes(m), st, m, p, n, yin, yout,
                       counters, queue, order, slab, block_ldj(m.N), pred);
    return hipGetLastError();
}

}  // namespace rk
