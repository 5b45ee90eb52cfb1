// Host side of the rkchem C ABI: mechanism reader and validation, device
// upload, Radau IIA constants, workspace management, statistics.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "rk_internal.h"

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg) {
    g_err = msg;
    return code;
}

int hip_fail(hipError_t e, const char *what) {
    return fail(RK_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

// ---- tokenizer ----------------------------------------------------------------
struct Tokens {
    std::vector<std::string> t;
    size_t i = 0;
    bool bad = false;
    std::string next() {
        if (i >= t.size()) { bad = true; return ""; }
        return t[i++];
    }
    double num() {
        std::string s = next();
        if (bad) return 0.0;
        char *e = nullptr;
        double v = std::strtod(s.c_str(), &e);
        if (e == s.c_str() || *e) bad = true;
        return v;
    }
    int integer() {
        std::string s = next();
        if (bad) return 0;
        char *e = nullptr;
        long v = std::strtol(s.c_str(), &e, 10);
        if (e == s.c_str() || *e) bad = true;
        return (int)v;
    }
    void word(const char *w) {
        if (next() != w) bad = true;
    }
};

// ---- NASA-7 on the host (validation only) --------------------------------------
void nasa7(const double *a, double T, double &cp, double &h, double &s) {
    cp = a[0] + T * (a[1] + T * (a[2] + T * (a[3] + T * a[4])));
    h = a[0] + T * (a[1] / 2 + T * (a[2] / 3 + T * (a[3] / 4 + T * a[4] / 5))) + a[5] / T;
    s = a[0] * std::log(T) + T * (a[1] + T * (a[2] / 2 + T * (a[3] / 3 + T * a[4] / 4))) + a[6];
}

struct Rx {
    int kind, nr, np, r[2], p[2];
    double A, b, Ea, A0 = 0, b0 = 0, Ea0 = 0, troe[4] = {0, 0, 0, 0};
    std::vector<double> eff;
};

int parse(const char *path, rk_mech *m, std::vector<Rx> &rx, std::vector<double> &alo, std::vector<double> &ahi) {
    std::ifstream in(path);
    if (!in) return fail(RK_EIO, std::string("cannot open mechanism file ") + path);
    Tokens tk;
    std::string line;
    while (std::getline(in, line)) {
        const size_t hash = line.find('#');
        if (hash != std::string::npos) line.resize(hash);
        std::istringstream ls(line);
        std::string w;
        while (ls >> w) tk.t.push_back(w);
    }
    tk.word("rkmech");
    if (tk.integer() != 1) tk.bad = true;
    tk.word("name");
    m->name = tk.next();
    tk.word("elements");
    m->E = tk.integer();
    for (int e = 0; e < m->E && !tk.bad; ++e) tk.next();
    tk.word("species");
    m->K = tk.integer();
    if (tk.bad || m->K <= 0 || m->E <= 0 || m->K > 4096) return fail(RK_EPARSE, "bad header in mechanism file");
    const int K = m->K;
    m->W.assign(K, 0.0);
    m->comp.assign((size_t)K * m->E, 0);
    m->Tmid.assign(K, 0.0);
    alo.assign((size_t)K * 7, 0.0);
    ahi.assign((size_t)K * 7, 0.0);
    for (int k = 0; k < K && !tk.bad; ++k) {
        tk.next();
        m->W[k] = tk.num();
        for (int e = 0; e < m->E; ++e) m->comp[(size_t)k * m->E + e] = tk.integer();
    }
    tk.word("thermo");
    std::vector<int> seen(K, 0);
    for (int i = 0; i < K && !tk.bad; ++i) {
        const int k = tk.integer();
        if (k < 0 || k >= K) { tk.bad = true; break; }
        seen[k] = 1;
        tk.num();                 // T_low (not used: polynomials are evaluated as they are)
        m->Tmid[k] = tk.num();
        tk.num();                 // T_high
        for (int a = 0; a < 7; ++a) alo[(size_t)k * 7 + a] = tk.num();
        for (int a = 0; a < 7; ++a) ahi[(size_t)k * 7 + a] = tk.num();
    }
    tk.word("reactions");
    m->R = tk.integer();
    if (tk.bad || m->R < 0) return fail(RK_EPARSE, "bad species/thermo section in mechanism file");
    rx.resize(m->R);
    for (int j = 0; j < m->R && !tk.bad; ++j) {
        Rx &x = rx[j];
        x.kind = tk.integer();
        x.nr = tk.integer();
        if (x.nr < 1 || x.nr > 2) { tk.bad = true; break; }
        for (int s = 0; s < x.nr; ++s) x.r[s] = tk.integer();
        x.np = tk.integer();
        if (x.np < 1 || x.np > 2) { tk.bad = true; break; }
        for (int s = 0; s < x.np; ++s) x.p[s] = tk.integer();
        x.A = tk.num(); x.b = tk.num(); x.Ea = tk.num();
        if (x.kind == 2) {
            x.A0 = tk.num(); x.b0 = tk.num(); x.Ea0 = tk.num();
            for (double &v : x.troe) v = tk.num();
        }
        if (x.kind == 1 || x.kind == 2) {
            x.eff.assign(K, 1.0);
            const int ne = tk.integer();
            for (int t = 0; t < ne && !tk.bad; ++t) {
                const int k = tk.integer();
                const double a = tk.num();
                if (k < 0 || k >= K) { tk.bad = true; break; }
                x.eff[k] = a;
            }
        } else if (x.kind != 0) {
            tk.bad = true;
        }
        for (int s = 0; s < x.nr; ++s) if (x.r[s] < 0 || x.r[s] >= K) tk.bad = true;
        for (int s = 0; s < x.np; ++s) if (x.p[s] < 0 || x.p[s] >= K) tk.bad = true;
    }
    tk.word("end");
    if (tk.bad) return fail(RK_EPARSE, "malformed reaction section in mechanism file");
    for (int k = 0; k < K; ++k)
        if (!seen[k]) return fail(RK_EPARSE, "species without thermodynamic data");
    return RK_OK;
}

int validate(const rk_mech *m, const std::vector<Rx> &rx, const std::vector<double> &alo, const std::vector<double> &ahi) {
    for (int k = 0; k < m->K; ++k) {
        if (!(m->W[k] > 0.0)) return fail(RK_EINVAL, "non-positive molar mass");
        double c1, h1, s1, c2, h2, s2;
        nasa7(&alo[(size_t)k * 7], m->Tmid[k], c1, h1, s1);
        nasa7(&ahi[(size_t)k * 7], m->Tmid[k], c2, h2, s2);
        auto close = [](double a, double b) { return std::fabs(a - b) <= 1e-6 * std::max(1.0, std::max(std::fabs(a), std::fabs(b))); };
        if (!close(c1, c2) || !close(h1, h2) || !close(s1, s2))
            return fail(RK_EINVAL, "NASA-7 polynomials discontinuous at T_mid for species " + std::to_string(k));
    }
    for (int j = 0; j < m->R; ++j) {
        for (int e = 0; e < m->E; ++e) {
            int bal = 0;
            for (int s = 0; s < rx[j].nr; ++s) bal -= m->comp[(size_t)rx[j].r[s] * m->E + e];
            for (int s = 0; s < rx[j].np; ++s) bal += m->comp[(size_t)rx[j].p[s] * m->E + e];
            if (bal != 0) return fail(RK_EINVAL, "reaction " + std::to_string(j) + " is not element balanced");
        }
        if (!(rx[j].A > 0.0) || (rx[j].kind == 2 && !(rx[j].A0 > 0.0)))
            return fail(RK_EINVAL, "non-positive pre-exponential factor in reaction " + std::to_string(j));
    }
    return RK_OK;
}

int upload(rk_mech *m, const std::vector<Rx> &rx, const std::vector<double> &alo, const std::vector<double> &ahi) {
    const int K = m->K, R = m->R;
    // thermo table: per species and range 16 doubles (cp, h, s polynomial coefficients)
    m->thermo.assign((size_t)K * 32, 0.0);
    for (int k = 0; k < K; ++k)
        for (int r = 0; r < 2; ++r) {
            const double *a = (r == 0 ? &alo[(size_t)k * 7] : &ahi[(size_t)k * 7]);
            double *t = &m->thermo[(size_t)k * 32 + r * 16];
            for (int i = 0; i < 5; ++i) t[i] = a[i];
            for (int i = 0; i < 5; ++i) t[5 + i] = a[i] / (i + 1);
            t[10] = a[5];
            for (int i = 1; i < 5; ++i) t[10 + i] = a[i] / i;
            t[15] = a[6];
        }
    m->rsp.assign(R, int4{-1, -1, -1, -1});
    m->rinfo.assign(R, 0);
    m->rpar.assign((size_t)R * rk::P_NPAR, 0.0);
    m->rhead.assign(std::max(R, 1), double4{0.0, 0.0, 0.0, 0.0});
    m->eff.clear();
    m->n3b = 0;
    for (int j = 0; j < R; ++j) {
        const Rx &x = rx[j];
        m->rsp[j] = int4{x.r[0], x.nr > 1 ? x.r[1] : -1, x.p[0], x.np > 1 ? x.p[1] : -1};
        int info = x.kind | (x.nr << 4) | (x.np << 8);
        if (x.kind != 0) {
            info |= (m->n3b + 1) << 12;
            m->eff.insert(m->eff.end(), x.eff.begin(), x.eff.end());
            ++m->n3b;
        }
        m->rinfo[j] = info;
        double *p = &m->rpar[(size_t)j * rk::P_NPAR];
        p[rk::P_A] = x.A; p[rk::P_B] = x.b; p[rk::P_EAR] = x.Ea / rk::kRu;
        p[rk::P_A0] = x.A0; p[rk::P_B0] = x.b0; p[rk::P_EA0R] = x.Ea0 / rk::kRu;
        p[rk::P_TA] = x.troe[0]; p[rk::P_T3] = x.troe[1]; p[rk::P_T1] = x.troe[2]; p[rk::P_T2] = x.troe[3];
        p[rk::P_DNU] = (double)(x.np - x.nr);
        m->rhead[j] = double4{p[rk::P_A], p[rk::P_B], p[rk::P_EAR], p[rk::P_DNU]};
    }
    if (m->eff.empty()) m->eff.push_back(0.0);
    // species -> (reaction, net nu) lists
    m->sp_off.assign(K + 1, 0);
    m->sp_rx.clear();
    for (int k = 0; k < K; ++k) {
        m->sp_off[k] = (int)m->sp_rx.size();
        for (int j = 0; j < R; ++j) {
            int nu = 0;
            for (int s = 0; s < rx[j].nr; ++s) nu -= rx[j].r[s] == k;
            for (int s = 0; s < rx[j].np; ++s) nu += rx[j].p[s] == k;
            if (nu != 0) m->sp_rx.push_back(int2{j, nu});
        }
    }
    m->sp_off[K] = (int)m->sp_rx.size();
    if (m->sp_rx.empty()) m->sp_rx.push_back(int2{0, 0});
    // species -> reactions with a mass-action slot or a non-default efficiency
    // of that species (the Jacobian's concentration columns)
    m->jl_off.assign(K + 1, 0);
    m->jl.clear();
    for (int k = 0; k < K; ++k) {
        m->jl_off[k] = (int)m->jl.size();
        for (int j = 0; j < R; ++j) {
            const Rx &x = rx[j];
            int e = (x.r[0] == k) | (x.nr > 1 && x.r[1] == k) << 1 | (x.p[0] == k) << 2 | (x.np > 1 && x.p[1] == k) << 3;
            double em1 = 0.0;
            if (x.kind != 0 && x.eff[k] != 1.0) {
                e |= 16;
                em1 = x.eff[k] - 1.0;
            }
            if (e != 0) m->jl.push_back(rk::JlEnt{em1, j << 5 | e, 0});
        }
    }
    m->jl_off[K] = (int)m->jl.size();
    if (m->jl.empty()) m->jl.push_back(rk::JlEnt{0.0, 0, 0});
    // third-body rows: species with a non-default efficiency
    m->tb_off.assign(m->n3b + 1, 0);
    m->tb.clear();
    for (int b = 0; b < m->n3b; ++b) {
        m->tb_off[b] = (int)m->tb.size();
        for (int k = 0; k < K; ++k) {
            const double ef = m->eff[(size_t)b * K + k];
            if (ef != 1.0) m->tb.push_back(rk::TbEnt{ef - 1.0, k, 0});
        }
    }
    m->tb_off[m->n3b] = (int)m->tb.size();
    if (m->tb.empty()) m->tb.push_back(rk::TbEnt{0.0, 0, 0});
    // per reaction: its third-body row's range in tb (read with the reaction's
    // other table entries, so the row offset is not a dependent load)
    m->tbr.assign(std::max(R, 1), int2{0, 0});
    for (int j = 0; j < R; ++j) {
        const int row = (m->rinfo[j] >> 12) - 1;
        if ((m->rinfo[j] & 15) != 0 && row >= 0) m->tbr[j] = int2{m->tb_off[row], m->tb_off[row + 1]};
    }
    std::vector<double> invW(K);
    for (int k = 0; k < K; ++k) invW[k] = 1.0 / m->W[k];

    // one device block, each table 256-byte aligned
    struct Part { const void *src; size_t bytes; size_t off; };
    std::vector<Part> parts = {
        {m->W.data(), K * sizeof(double), 0}, {invW.data(), K * sizeof(double), 0},
        {m->Tmid.data(), K * sizeof(double), 0}, {m->thermo.data(), m->thermo.size() * sizeof(double), 0},
        {m->rsp.data(), std::max(R, 1) * sizeof(int4), 0}, {m->rinfo.data(), std::max(R, 1) * sizeof(int), 0},
        {m->rpar.data(), std::max<size_t>(m->rpar.size(), 1) * sizeof(double), 0},
        {m->eff.data(), m->eff.size() * sizeof(double), 0},
        {m->sp_off.data(), m->sp_off.size() * sizeof(int), 0}, {m->sp_rx.data(), m->sp_rx.size() * sizeof(int2), 0},
        {m->jl_off.data(), m->jl_off.size() * sizeof(int), 0}, {m->jl.data(), m->jl.size() * sizeof(rk::JlEnt), 0},
        {m->tb_off.data(), m->tb_off.size() * sizeof(int), 0}, {m->tb.data(), m->tb.size() * sizeof(rk::TbEnt), 0},
        {m->rhead.data(), m->rhead.size() * sizeof(double4), 0},
        {m->tbr.data(), m->tbr.size() * sizeof(int2), 0}};
    size_t total = 0;
    for (Part &p : parts) { p.off = total; total += (p.bytes + 255) / 256 * 256; }
    std::vector<char> host(total, 0);
    for (Part &p : parts) if (p.src && p.bytes) std::memcpy(host.data() + p.off, p.src, p.bytes);
    hipError_t e = hipGetDevice(&m->device);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    e = hipMalloc(&m->dev_block, total);
    if (e != hipSuccess) return fail(RK_ENOMEM, "hipMalloc of mechanism tables failed");
    e = hipMemcpy(m->dev_block, host.data(), total, hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy of mechanism tables");
    char *b = static_cast<char *>(m->dev_block);
    rk::DevMech &d = m->dev;
    d.K = K; d.R = R; d.N = K + 1; d.n3b = m->n3b;
    d.nsp = m->sp_off[K];
    d.W = reinterpret_cast<const double *>(b + parts[0].off);
    d.invW = reinterpret_cast<const double *>(b + parts[1].off);
    d.Tmid = reinterpret_cast<const double *>(b + parts[2].off);
    d.thermo = reinterpret_cast<const double *>(b + parts[3].off);
    d.rsp = reinterpret_cast<const int4 *>(b + parts[4].off);
    d.rinfo = reinterpret_cast<const int *>(b + parts[5].off);
    d.rpar = reinterpret_cast<const double *>(b + parts[6].off);
    d.eff = reinterpret_cast<const double *>(b + parts[7].off);
    d.sp_off = reinterpret_cast<const int *>(b + parts[8].off);
    d.sp_rx = reinterpret_cast<const int2 *>(b + parts[9].off);
    d.jl_off = reinterpret_cast<const int *>(b + parts[10].off);
    d.jl = reinterpret_cast<const rk::JlEnt *>(b + parts[11].off);
    d.tb_off = reinterpret_cast<const int *>(b + parts[12].off);
    d.tb = reinterpret_cast<const rk::TbEnt *>(b + parts[13].off);
    d.rhead = reinterpret_cast<const double4 *>(b + parts[14].off);
    d.tbr = reinterpret_cast<const int2 *>(b + parts[15].off);
    e = hipEventCreate(&m->ev0);
    if (e == hipSuccess) e = hipEventCreate(&m->ev1);
    if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
    return RK_OK;
}

// ---- Radau IIA constants (three-stage, order five) ------------------------------
// A^-1 has one real eigenvalue g and a complex pair a +- i b.  T is built from
// an eigenvector for g and the real and imaginary parts of an eigenvector for
// a - i b, each normalised to last component 1, which gives
// T^-1 A^-1 T = [[g,0,0],[0,a,-b],[0,b,a]].
template <class S>
void null_vec_last1(const S B[3][3], S v[3]) {
    // rows 0 and 1 of B v = 0 with v2 = 1 (Cramer's rule)
    const S det = B[0][0] * B[1][1] - B[0][1] * B[1][0];
    v[0] = (-B[0][2] * B[1][1] + B[0][1] * B[1][2]) / det;
    v[1] = (-B[0][0] * B[1][2] + B[1][0] * B[0][2]) / det;
    v[2] = S(1.0);
}

void invert3(const double A[9], double R[9]) {
    // Gauss-Jordan with partial pivoting
    double a[3][6];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 6; ++j) a[i][j] = j < 3 ? A[i * 3 + j] : (j - 3 == i ? 1.0 : 0.0);
    for (int c = 0; c < 3; ++c) {
        int p = c;
        for (int i = c + 1; i < 3; ++i) if (std::fabs(a[i][c]) > std::fabs(a[p][c])) p = i;
        for (int j = 0; j < 6; ++j) std::swap(a[c][j], a[p][j]);
        const double d = a[c][c];
        for (int j = 0; j < 6; ++j) a[c][j] /= d;
        for (int i = 0; i < 3; ++i)
            if (i != c) {
                const double f = a[i][c];
                for (int j = 0; j < 6; ++j) a[i][j] -= f * a[c][j];
            }
    }
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) R[i * 3 + j] = a[i][j + 3];
}

void radau_constants(rk::RadauParams &p) {
    const double r6 = std::sqrt(6.0);
    const double A[9] = {(88.0 - 7.0 * r6) / 360.0, (296.0 - 169.0 * r6) / 1800.0, (-2.0 + 3.0 * r6) / 225.0,
                         (296.0 + 169.0 * r6) / 1800.0, (88.0 + 7.0 * r6) / 360.0, (-2.0 - 3.0 * r6) / 225.0,
                         (16.0 - r6) / 36.0, (16.0 + r6) / 36.0, 1.0 / 9.0};
    p.c1 = (4.0 - r6) / 10.0;
    p.c2 = (4.0 + r6) / 10.0;
    const double q81 = std::cbrt(81.0), q9 = std::cbrt(9.0);
    p.g = 30.0 / (6.0 + q81 - q9);
    const double al = (12.0 - q81 + q9) / 60.0, be = (q81 + q9) * std::sqrt(3.0) / 60.0;
    p.a = al / (al * al + be * be);
    p.b = be / (al * al + be * be);
    double Ai[9];
    invert3(A, Ai);
    double Br[3][3];
    std::complex<double> Bc[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            Br[i][j] = Ai[i * 3 + j] - (i == j ? p.g : 0.0);
            Bc[i][j] = Ai[i * 3 + j] - (i == j ? std::complex<double>(p.a, -p.b) : 0.0);
        }
    double v1[3];
    std::complex<double> v2[3];
    null_vec_last1(Br, v1);
    null_vec_last1(Bc, v2);
    for (int i = 0; i < 3; ++i) {
        p.T[i * 3 + 0] = v1[i];
        p.T[i * 3 + 1] = v2[i].real();
        p.T[i * 3 + 2] = v2[i].imag();
    }
    invert3(p.T, p.Ti);
    p.d[0] = -(13.0 + 7.0 * r6) / 3.0;
    p.d[1] = (-13.0 + 7.0 * r6) / 3.0;
    p.d[2] = -1.0 / 3.0;
}

bool is_device_ptr(const void *ptr) {
    hipPointerAttribute_t a;
    if (hipPointerGetAttributes(&a, ptr) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

// per-lane working set of the lane-per-state kernel and the debug kernels
// (only they use it: the group kernels keep everything on chip)
int ensure_lane_scratch(rk_mech *m, int64_t n) {
    const size_t need = rk::lane_scratch_doubles(m->K, std::max<int64_t>(n, 1));
    if (need > m->scratch_cap) {
        if (m->scratch) { (void)hipDeviceSynchronize(); (void)hipFree(m->scratch); m->scratch = nullptr; m->scratch_cap = 0; }
        if (hipMalloc(&m->scratch, need * sizeof(double)) != hipSuccess) {
            (void)hipGetLastError();
            return fail(RK_ENOMEM, "cannot allocate the lane-kernel workspace");
        }
        m->scratch_cap = need;
    }
    return RK_OK;
}

// Jacobian slabs of the block kernel, one per resident block
int ensure_block_slab(rk_mech *m) {
    if (m->block_blocks == 0) m->block_blocks = rk::block_max_blocks(m->dev);
    const size_t need = rk::block_slab_doubles(m->K + 1, m->block_blocks);
    if (need > m->block_slab_cap) {
        if (m->block_slab) { (void)hipDeviceSynchronize(); (void)hipFree(m->block_slab); m->block_slab = nullptr; m->block_slab_cap = 0; }
        if (hipMalloc(&m->block_slab, need * sizeof(double)) != hipSuccess) {
            (void)hipGetLastError();
            return fail(RK_ENOMEM, "cannot allocate the block-kernel Jacobian slabs");
        }
        m->block_slab_cap = need;
    }
    return RK_OK;
}

int ensure_workspace(rk_mech *m, int64_t n) {
    if (!m->queue && hipMalloc(&m->queue, 256) != hipSuccess) {
        (void)hipGetLastError();
        return fail(RK_ENOMEM, "cannot allocate the work queue");
    }
    if (n > m->fb_cap) {
        if (m->fb_list) { (void)hipDeviceSynchronize(); (void)hipFree(m->fb_list); m->fb_list = nullptr; m->fb_cap = 0; }
        if (hipMalloc(&m->fb_list, (size_t)n * sizeof(int)) != hipSuccess) {
            (void)hipGetLastError();
            return fail(RK_ENOMEM, "cannot allocate the fallback list");
        }
        m->fb_cap = n;
    }
    if (m->nbins > 0 || m->autotune) {
        if (n > m->bin_cap) {
            if (m->bins) { (void)hipDeviceSynchronize(); (void)hipFree(m->bins); (void)hipFree(m->order); }
            m->bins = m->order = nullptr;
            m->bin_cap = 0;
            if (hipMalloc(&m->bins, (size_t)n * sizeof(int)) != hipSuccess ||
                hipMalloc(&m->order, (size_t)n * sizeof(int)) != hipSuccess) {
                (void)hipGetLastError();
                return fail(RK_ENOMEM, "cannot allocate the binning workspace");
            }
            m->bin_cap = n;
        }
        if (!m->hist && (hipMalloc(&m->hist, 128 * sizeof(int)) != hipSuccess ||
                         hipMalloc(&m->proxy_scratch, rk::proxy_scratch_doubles(m->K) * sizeof(double)) != hipSuccess)) {
            (void)hipGetLastError();
            return fail(RK_ENOMEM, "cannot allocate the binning workspace");
        }
    }
    if (n > m->counters_cap) {
        if (m->counters) { (void)hipDeviceSynchronize(); (void)hipFree(m->counters); m->counters = nullptr; m->counters_cap = 0; }
        if (hipMalloc(&m->counters, (size_t)n * rk::kNumCounters * sizeof(int32_t)) != hipSuccess) {
            (void)hipGetLastError();
            return fail(RK_ENOMEM, "cannot allocate per-state counters");
        }
        m->counters_cap = n;
    }
    return RK_OK;
}

}  // namespace

rk::Predictor::~Predictor() {
    for (void *q : {(void *)in_shift, (void *)in_scale, (void *)out_shift, (void *)out_scale, (void *)X, (void *)pred})
        if (q) (void)hipFree(q);
    delete net;
}

hipError_t rk::Predictor::ensure(int64_t n) {
    if (n <= cap) return hipSuccess;
    if (X) { (void)hipDeviceSynchronize(); (void)hipFree(X); (void)hipFree(pred); X = nullptr; pred = nullptr; }
    hipError_t e = hipMalloc(&X, (size_t)n * (K + 2) * sizeof(float));
    if (e == hipSuccess) e = hipMalloc(&pred, (size_t)n * (3 * (K + 1) + 2) * sizeof(double));
    if (e == hipSuccess) cap = n;
    return e;
}

namespace {

// ---- predictor files -----------------------------------------------------------
// Text format: "rkpred 1", "mech <name> K <K> dt <dt>", "dims <L> <w0..>",
// "in_shift"/"in_scale" (K+2 values), "out_shift"/"out_scale" (3N+2 values),
// "params <count>" values, "end".
int load_predictor(rk_mech *m, const char *path) {
    std::ifstream in(path);
    if (!in) return fail(RK_EIO, std::string("cannot open predictor file ") + path);
    Tokens tk;
    std::string w;
    while (in >> w) tk.t.push_back(w);
    tk.word("rkpred");
    if (tk.integer() != 1) tk.bad = true;
    tk.word("mech");
    tk.next();
    tk.word("K");
    const int K = tk.integer();
    tk.word("dt");
    const double dt = tk.num();
    tk.word("dims");
    const int L = tk.integer();
    if (tk.bad || K != m->K || L < 2 || L > 8 || !(dt > 0.0)) return fail(RK_EINVAL, "predictor does not fit this mechanism");
    std::vector<int> dims(L);
    for (int &d : dims) {
        d = tk.integer();
        if (d < 1 || d > 4096) tk.bad = true;
    }
    const int N = K + 1, Din = K + 2, Dout = 3 * N + 2;
    if (tk.bad || dims.front() != Din || dims.back() != Dout) return fail(RK_EINVAL, "predictor widths do not fit this mechanism");
    auto vec = [&](const char *name, int cnt) {
        tk.word(name);
        std::vector<float> v(cnt);
        for (float &x : v) x = (float)tk.num();
        return v;
    };
    std::vector<float> ish = vec("in_shift", Din), isc = vec("in_scale", Din);
    std::vector<float> osh = vec("out_shift", Dout), osc = vec("out_scale", Dout);
    tk.word("params");
    const int64_t cnt = tk.integer();
    std::vector<float> params(cnt > 0 && cnt < (1 << 26) ? cnt : 0);
    for (float &x : params) x = (float)tk.num();
    tk.word("end");
    if (tk.bad) return fail(RK_EPARSE, "malformed predictor file");
    auto *pr = new rk::Predictor();
    pr->dt = dt;
    pr->K = K;
    pr->dims = dims;
    pr->net = new rk::Mlp();
    hipError_t e = pr->net->init(dims);
    if (e == hipSuccess && pr->net->count() != cnt) {
        delete pr;
        return fail(RK_EINVAL, "predictor parameter count does not match its widths");
    }
    for (auto pp : {&pr->in_shift, &pr->in_scale})
        if (e == hipSuccess) e = hipMalloc(pp, Din * sizeof(float));
    for (auto pp : {&pr->out_shift, &pr->out_scale})
        if (e == hipSuccess) e = hipMalloc(pp, Dout * sizeof(float));
    if (e == hipSuccess) e = hipMemcpy(pr->in_shift, ish.data(), Din * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(pr->in_scale, isc.data(), Din * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(pr->out_shift, osh.data(), Dout * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(pr->out_scale, osc.data(), Dout * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(pr->net->params, params.data(), cnt * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = pr->net->refresh_bf16(nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        delete pr;
        return hip_fail(e, "predictor upload");
    }
    for (auto &q : m->predictors)
        if (q->dt == dt) { delete q; q = pr; return RK_OK; }
    m->predictors.push_back(pr);
    return RK_OK;
}

rk::Predictor *predictor_for(rk_mech *m, double dt) {
    for (auto *q : m->predictors)
        if (std::fabs(q->dt - dt) <= 1e-12 * dt) return q;
    return nullptr;
}

rk::Work handle_work(rk_mech *m) {
    rk::Work w;
    w.counters = m->counters;
    w.queue = m->queue;
    w.fb_list = m->fb_list;
    w.bins = m->bins;
    w.order = m->order;
    w.hist = m->hist;
    w.proxy = m->proxy_scratch;
    w.lane = m->scratch;
    w.slab = m->block_slab;
    w.allow_predictor = true;
    return w;
}

// Enqueue the flag clear, the optional cost binning and the integrator.
// w names the device buffers: the handle's workspaces, or the caller-free
// static array of the no-allocation entry (no predictor, no bins there).
hipError_t launch_integrator(rk_mech *m, const rk::RadauParams &p, int64_t n, const double *yin, double *yout,
                             double atol, double rtol, int variant, int nbins, int gpct, hipStream_t st,
                             const rk::Work &w) {
    hipError_t e = rk::launch_zero_i32(w.counters + (size_t)rk::C_FLAGS * n, n, st);
    if (e != hipSuccess) return e;
    const int *order = nullptr;
    const double *pred = nullptr;
    // the network keys the bins and, unless predictor_use is "bins", warm-starts
    // the first step attempt (wavefront and block variants)
    const bool use_net = w.allow_predictor && (variant == 1 || variant == 2 ||
                                               (variant == 3 && (nbins > 0 || p.pred_use != 0)));
    rk::Predictor *pr = use_net ? predictor_for(m, p.dt) : nullptr;
    if (pr) {
        e = pr->ensure(n);
        if (e != hipSuccess) return e;
        // network inference; with bins, the key is the predicted step count
        e = rk::launch_predictor(*pr, n, yin, p.dt, atol, rtol, nbins, nbins > 0 ? w.bins : nullptr, st);
        if (e != hipSuccess) return e;
        pred = pr->pred;
        if (nbins > 0) {
            e = rk::launch_sort_bins(w.bins, n, nbins, w.order, w.hist, st);
            if (e != hipSuccess) return e;
            order = w.order;
        }
    } else if (nbins > 0) {
        e = rk::launch_binning(m->dev, n, yin, p.dt, atol, rtol, nbins, w.bins, w.order, w.hist, w.proxy, st);
        if (e != hipSuccess) return e;
        order = w.order;
    }
    m->last_nbins = nbins;
    m->last_order = nbins > 0 ? w.order : nullptr;
    if (variant == 3) {
        // one block per state; the slabs were sized for block_blocks blocks
        const int64_t cap = std::max<int64_t>(1, (int64_t)m->block_blocks * gpct / 100);
        const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(n, cap));
        m->last_grid = grid;
        return rk::launch_radau_block(m->dev, p, n, yin, yout, w.counters, w.queue, order, w.slab,
                                      p.pred_use != 0 ? pred : nullptr, grid, st);
    }
    if (variant == 1 || variant == 2) {
        if (m->group_blocks == 0) m->group_blocks = rk::group_max_blocks(m->dev);
        if (p.method == 1) {
            const int spb = rk::group_states_per_block(m->K + 1);
            const int64_t need = (n + spb - 1) / spb;
            const int64_t cap = std::max<int64_t>(1, (int64_t)m->group_blocks * gpct / 100);
            const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(need, cap));
            m->last_grid = grid;
            return rk::launch_rodas3_group(m->dev, p, n, yin, yout, w.counters, w.queue, order, grid, st);
        }
        const int spb = rk::group_states_per_block(m->K + 1);
        const int64_t need = (n + spb - 1) / spb;
        const int64_t cap = std::max<int64_t>(1, (int64_t)m->group_blocks * gpct / 100);
        const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(need, cap));
        m->last_grid = grid;
        return rk::launch_radau_group(m->dev, p, n, yin, yout, w.counters, w.queue, w.fb_list, order, pred,
                                      variant == 2, grid, st);
    }
    m->last_grid = (int)((n + rk::kWave - 1) / rk::kWave);
    return rk::launch_radau_lane(m->dev, p, n, yin, yout, w.lane, w.counters, order, st);
}

// Scheduling autotuner: times the integrator on a bounded sample (the first
// min(n, S) states, compacted: S = 32768 for N <= 16, 8192 for N <= 56, 1024
// for the block kernel) and keeps the fastest schedule for this dt.  A
// coordinate search: cost-bin count x persistent-grid share at one state per
// queue grab, then larger grabs at the best of those.  One warm-up run, then
// one timed run per candidate.  Runs once per (handle, dt); blocks the host.
int autotune(rk_mech *m, int64_t n, double dt, const double *yin, double atol, double rtol, hipStream_t st,
             rk::RadauParams p, int variant, int &nbins, int &gpct, int &tile) {
    for (auto &t : m->tuned)
        if (t.dt == dt) { nbins = t.bins; gpct = t.grid_pct; tile = t.tile; return RK_OK; }
    const int64_t cap = variant == 3 ? 1024 : (m->K + 1 <= 16 ? 32768 : 8192);
    const int64_t ms = std::min<int64_t>(n, cap);
    const int rows = m->K + 2;
    const size_t need = (size_t)ms * rows * 2;
    if (need > m->tune_cap) {
        if (m->tune_buf) { (void)hipDeviceSynchronize(); (void)hipFree(m->tune_buf); m->tune_buf = nullptr; }
        if (hipMalloc(&m->tune_buf, need * sizeof(double)) != hipSuccess) {
            (void)hipGetLastError();
            return fail(RK_ENOMEM, "cannot allocate autotuner buffers");
        }
        m->tune_cap = need;
    }
    double *ys = m->tune_buf, *yo = m->tune_buf + (size_t)ms * rows;
    hipError_t e = rk::launch_gather_head(yin, n, ms, rows, ys, st);
    if (e != hipSuccess) return hip_fail(e, "autotune gather");
    struct Cand { int bins, grid, tile; };
    std::vector<Cand> first;
    if (variant == 3) {
        for (int b : {0, 16}) first.push_back({b, 100, 1});
    } else if (variant == 0) {
        for (int b : {0, 8, 16, 32}) first.push_back({b, 100, 1});   // the lane kernel is not persistent
    } else {
        for (int b : {0, 8, 16, 32})
            for (int g : {100, 75, 50}) first.push_back({b, g, 1});
    }
    auto time_one = [&](const Cand &c, float &ms_t) -> int {
        p.tile = c.tile;
        e = hipEventRecord(m->ev0, st);
        if (e == hipSuccess) e = launch_integrator(m, p, ms, ys, yo, atol, rtol, variant, c.bins, c.grid, st, handle_work(m));
        if (e == hipSuccess) e = hipEventRecord(m->ev1, st);
        if (e == hipSuccess) e = hipEventSynchronize(m->ev1);
        if (e != hipSuccess) return hip_fail(e, "autotune trial");
        (void)hipEventElapsedTime(&ms_t, m->ev0, m->ev1);
        return RK_OK;
    };
    float t_warm = 0.0f, best = 1e30f;
    int rc = time_one(first[0], t_warm);     // warms caches and code
    if (rc != RK_OK) return rc;
    Cand bc = first[0];
    for (const Cand &c : first) {
        float t = 0.0f;
        if ((rc = time_one(c, t)) != RK_OK) return rc;
        if (t < best) { best = t; bc = c; }
    }
    if (variant != 0) {
        for (int tl : {2, 4}) {
            const Cand c{bc.bins, bc.grid, tl};
            float t = 0.0f;
            if ((rc = time_one(c, t)) != RK_OK) return rc;
            if (t < best) { best = t; bc = c; }
        }
    }
    m->tuned.push_back({dt, bc.bins, bc.grid, bc.tile, best});
    nbins = bc.bins;
    gpct = bc.grid;
    tile = bc.tile;
    return RK_OK;
}

}  // namespace

// The integration call on the handle's workspaces (w == nullptr: allocated
// here as needed; predictor, bins and autotuner as set) or on caller-free
// buffers (the no-allocation entry: wave and mixed variants only, input
// order, cold starts, nothing allocated).
int rk_integrate_common(rk_mech *m, int64_t n, double dt, const double *yin, double *yout, double atol, double rtol,
                        void *stream, const rk::Work *w) {
    if (!m) return fail(RK_EINVAL, "radau_integrate: NULL handle");
    if (n < 0 || !(dt > 0.0) || !std::isfinite(dt) || !(atol >= 0.0) || !(rtol > 0.0))
        return fail(RK_EINVAL, "radau_integrate: need n >= 0, dt > 0, atol >= 0, rtol > 0");
    if (n > 0 && (!yin || !yout)) return fail(RK_EINVAL, "radau_integrate: NULL state pointer");
    if (n > 0 && (!is_device_ptr(yin) || !is_device_ptr(yout)))
        return fail(RK_EINVAL, "radau_integrate: state arrays must be device memory");
    const bool group_ok = rk::group_supported(m->K + 1) && rk::group_lds_bytes(m->dev) <= 65536;
    const bool block_ok = rk::block_supported(m->K + 1) && rk::block_lds_bytes(m->dev) <= 163840;
    const int variant = m->variant >= 0 ? m->variant : (group_ok ? 1 : (block_ok ? 3 : 0));
    if ((variant == 1 || variant == 2) && !group_ok)
        return fail(RK_EINVAL, "radau_integrate: the wave and mixed variants need K + 1 <= 56");
    if (variant == 3 && !block_ok)
        return fail(RK_EINVAL, "radau_integrate: the block variant needs 57 <= K + 1 <= 153 and at most 160 KB of LDS per block");
    if (m->method == 1 && (variant != 1 || m->fd_jac))
        return fail(RK_EINVAL, "radau_integrate: the Rodas3 method runs with the wave variant and the analytical Jacobian");
    if (m->fd_jac && variant != 0 && variant != 1)
        return fail(RK_EINVAL, "radau_integrate: the forward-difference Jacobian runs with the lane and wave variants");
    if (w && variant != 1 && variant != 2)
        return fail(RK_EINVAL, "radau_integrate_noalloc: only the wave and mixed variants (K + 1 <= 56)");
    if (!w) {
        int rc = ensure_workspace(m, std::max<int64_t>(n, 1));
        if (rc == RK_OK && variant == 0) rc = ensure_lane_scratch(m, n);
        if (rc == RK_OK && variant == 3) rc = ensure_block_slab(m);
        if (rc != RK_OK) return rc;
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    rk::RadauParams p{};
    radau_constants(p);
    p.dt = dt;
    p.atol = atol;
    p.rtol = rtol;
    p.kmax = m->kmax;
    p.nmax = m->nmax;
    p.pred_use = m->pred_use;
    p.tile = m->tile;
    p.force_fb = m->force_fb;
    p.fd_jac = m->fd_jac;
    p.method = m->method;
    p.fp64_solves = m->fp64_solves;
    p.kappa = m->kappa > 0.0 ? m->kappa : std::max(10.0 * 2.220446049250313e-16 / rtol, std::min(0.03, std::sqrt(rtol)));
    p.h0 = m->h0 > 0.0 ? m->h0 : std::min(dt, 1e-6);
    int nbins = w ? 0 : m->nbins, gpct = m->grid_pct, tile = m->tile;
    if (!w && m->autotune && n >= (variant == 3 ? 1024 : 4096)) {
        int rc2 = autotune(m, n, dt, yin, atol, rtol, st, p, variant, nbins, gpct, tile);
        if (rc2 != RK_OK) return rc2;
    }
    p.tile = tile;
    m->last_tile = tile;
    hipError_t e = hipEventRecord(m->ev0, st);
    if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
    const rk::Work work = w ? *w : handle_work(m);
    e = launch_integrator(m, p, n, yin, yout, atol, rtol, variant, nbins, gpct, st, work);
    if (e != hipSuccess) return hip_fail(e, "radau kernel launch");
    e = hipEventRecord(m->ev1, st);
    if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
    m->last_n = n;
    m->last_counters = work.counters;
    m->last_stream = st;
    m->have_run = true;
    return RK_OK;
}


int rk_fail(int code, const char *msg) { return fail(code, msg); }

// =============================================================================
// C ABI
// =============================================================================
extern "C" {

const char *rk_last_error(void) { return g_err.c_str(); }

int mech_load(const char *path, rk_mech **out) {
    if (!out || !path) return fail(RK_EINVAL, "mech_load: NULL argument");
    *out = nullptr;
    rk_mech *m = new rk_mech();
    std::vector<Rx> rx;
    std::vector<double> alo, ahi;
    int rc = parse(path, m, rx, alo, ahi);
    if (rc == RK_OK) rc = validate(m, rx, alo, ahi);
    if (rc == RK_OK) rc = upload(m, rx, alo, ahi);
    if (rc != RK_OK) {
        mech_free(m);
        return rc;
    }
    *out = m;
    g_err.clear();
    return RK_OK;
}

void mech_free(rk_mech *m) {
    if (!m) return;
    if (m->have_run && m->last_stream) (void)hipStreamSynchronize(m->last_stream);
    if (m->have_run) (void)hipDeviceSynchronize();
    if (m->dev_block) (void)hipFree(m->dev_block);
    if (m->scratch) (void)hipFree(m->scratch);
    if (m->counters) (void)hipFree(m->counters);
    if (m->queue) (void)hipFree(m->queue);
    if (m->fb_list) (void)hipFree(m->fb_list);
    if (m->block_slab) (void)hipFree(m->block_slab);
    if (m->bins) (void)hipFree(m->bins);
    if (m->order) (void)hipFree(m->order);
    if (m->hist) (void)hipFree(m->hist);
    if (m->proxy_scratch) (void)hipFree(m->proxy_scratch);
    if (m->tune_buf) (void)hipFree(m->tune_buf);
    for (auto *q : m->predictors) delete q;
    if (m->ev0) (void)hipEventDestroy(m->ev0);
    if (m->ev1) (void)hipEventDestroy(m->ev1);
    delete m;
}

int mech_dims(const rk_mech *m, int32_t *K, int32_t *R) {
    if (!m || !K || !R) return fail(RK_EINVAL, "mech_dims: NULL argument");
    *K = m->K;
    *R = m->R;
    return RK_OK;
}

int radau_set_option(rk_mech *m, const char *key, const char *value) {
    if (!m || !key || !value) return fail(RK_EINVAL, "radau_set_option: NULL argument");
    std::string k(key), v(value);
    char *e = nullptr;
    if (k == "variant") {
        if (v == "lane") m->variant = 0;
        else if (v == "wave") m->variant = 1;
        else if (v == "mixed") m->variant = 2;
        else if (v == "block") m->variant = 3;
        else if (v == "auto") m->variant = -1;
        else return fail(RK_EINVAL, "unknown variant " + v);
        return RK_OK;
    }
    if (k == "kmax" || k == "nmax") {
        const long x = std::strtol(value, &e, 10);
        if (e == value || *e || x < 1 || x > 100000000) return fail(RK_EINVAL, "bad integer for " + k);
        (k == "kmax" ? m->kmax : m->nmax) = (int)x;
        return RK_OK;
    }
    if (k == "binning") {
        const long x = std::strtol(value, &e, 10);
        if (e == value || *e || x < 0 || x > 64) return fail(RK_EINVAL, "binning: number of bins 0..64");
        m->nbins = (int)x;
        return RK_OK;
    }
    if (k == "grid_pct") {
        const long x = std::strtol(value, &e, 10);
        if (e == value || *e || x < 10 || x > 100) return fail(RK_EINVAL, "grid_pct: 10..100");
        m->grid_pct = (int)x;
        return RK_OK;
    }
    if (k == "predictor") {
        if (v.empty() || v == "none") {
            if (m->have_run) (void)hipDeviceSynchronize();
            for (auto *q : m->predictors) delete q;
            m->predictors.clear();
            return RK_OK;
        }
        return load_predictor(m, value);
    }
    if (k == "predictor_use") {
        if (v == "both") m->pred_use = 3;
        else if (v == "h0") m->pred_use = 1;
        else if (v == "z0") m->pred_use = 2;
        else if (v == "bins") m->pred_use = 0;
        else return fail(RK_EINVAL, "predictor_use: both | h0 | z0 | bins");
        return RK_OK;
    }
    if (k == "autotune") {
        if (v != "0" && v != "1") return fail(RK_EINVAL, "autotune: 0 or 1");
        m->autotune = v == "1";
        if (!m->autotune) m->tuned.clear();
        return RK_OK;
    }
    if (k == "tile") {
        const long x = std::strtol(value, &e, 10);
        if (e == value || *e || x < 1 || x > 64) return fail(RK_EINVAL, "tile: states per queue grab, 1..64");
        m->tile = (int)x;
        return RK_OK;
    }
    if (k == "method") {
        if (v == "radau") m->method = 0;
        else if (v == "rodas3") m->method = 1;
        else return fail(RK_EINVAL, "method: radau | rodas3");
        return RK_OK;
    }
    if (k == "jacobian") {
        if (v == "analytical") m->fd_jac = 0;
        else if (v == "fd") m->fd_jac = 1;
        else return fail(RK_EINVAL, "jacobian: analytical | fd");
        return RK_OK;
    }
    if (k == "force_fallback") {
        if (v != "0" && v != "1") return fail(RK_EINVAL, "force_fallback: 0 or 1");
        m->force_fb = v == "1";
        return RK_OK;
    }
    if (k == "block_solves") {
        if (v == "fp32_refined") m->fp64_solves = 0;
        else if (v == "fp64_accurate") m->fp64_solves = 1;
        else return fail(RK_EINVAL, "block_solves: fp32_refined | fp64_accurate");
        return RK_OK;
    }
    if (k == "kappa" || k == "h0") {
        const double x = std::strtod(value, &e);
        if (e == value || *e || !(x >= 0.0) || !std::isfinite(x)) return fail(RK_EINVAL, "bad number for " + k);
        (k == "kappa" ? m->kappa : m->h0) = x;
        return RK_OK;
    }
    return fail(RK_EINVAL, "unknown option " + k);
}

int radau_integrate(rk_mech *m, int64_t n, double dt, const double *yin, double *yout, double atol, double rtol,
                    void *stream) {
    return rk_integrate_common(m, n, dt, yin, yout, atol, rtol, stream, nullptr);
}

int stats_get(rk_mech *m, rk_stats *out, int32_t *steps, int32_t *status) {
    if (!m || !out) return fail(RK_EINVAL, "stats_get: NULL argument");
    std::memset(out, 0, sizeof *out);
    if (!m->have_run) return RK_OK;
    hipError_t e = hipEventSynchronize(m->ev1);
    if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, m->ev0, m->ev1) == hipSuccess) out->kernel_ms = ms;
    const int64_t n = m->last_n;
    out->n_states = n;
    if (n == 0) return RK_OK;
    std::vector<int32_t> c((size_t)n * rk::kNumCounters);
    e = hipMemcpy(c.data(), m->last_counters, c.size() * sizeof(int32_t), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy of counters");
    const int32_t *st = &c[(size_t)rk::C_STATUS * n];
    const int32_t *ns = &c[(size_t)rk::C_NSTEP * n];
    out->max_steps = 0;
    out->min_steps = ns[0];
    for (int64_t i = 0; i < n; ++i) {
        out->steps += ns[i];
        out->accepted += c[(size_t)rk::C_NACC * n + i];
        out->rejected += c[(size_t)rk::C_NREJ * n + i];
        out->newton_iters += c[(size_t)rk::C_NNEWT * n + i];
        out->newton_fail += c[(size_t)rk::C_NNFAIL * n + i];
        out->f_evals += c[(size_t)rk::C_NFEV * n + i];
        out->jac_evals += c[(size_t)rk::C_NJEV * n + i];
        out->lu_factor += c[(size_t)rk::C_NLU * n + i];
        const int32_t fl = c[(size_t)rk::C_FLAGS * n + i];
        out->fp32_fallback += (fl & rk::kFlagFp32Fallback) != 0;
        out->predictor_kept += (fl & rk::kFlagPredKept) != 0;
        out->predictor_fallback += (fl & rk::kFlagPredFallback) != 0;
        out->n_failed += st[i] != RK_ST_OK;
        out->max_steps = std::max(out->max_steps, ns[i]);
        out->min_steps = std::min(out->min_steps, ns[i]);
    }
    // divergence measure over groups of w consecutive states
    auto hist = [&](int w, int64_t *h, double *mean) {
        int64_t groups = 0;
        double sum = 0.0;
        for (int64_t g0 = 0; g0 < n; g0 += w) {
            const int64_t g1 = std::min<int64_t>(n, g0 + w);
            int64_t tot = 0;
            int32_t mx = 0;
            for (int64_t i = g0; i < g1; ++i) { tot += ns[i]; mx = std::max(mx, ns[i]); }
            const double D = mx > 0 ? 1.0 - (double)tot / ((double)(g1 - g0) * mx) : 0.0;
            int b = (int)(D / 0.05);
            b = std::min(19, std::max(0, b));
            ++h[b];
            sum += D;
            ++groups;
        }
        *mean = groups ? sum / groups : 0.0;
    };
    hist(64, out->d_hist64, &out->d_mean64);
    hist(32, out->d_hist32, &out->d_mean32);
    // the same measure over the work-queue order the integrator drew states in
    // (how well the cost bins put states of equal step counts next to each other)
    if (m->last_nbins > 0 && m->last_order) {
        std::vector<int32_t> ord((size_t)n), qs((size_t)n);
        e = hipMemcpy(ord.data(), m->last_order, (size_t)n * sizeof(int32_t), hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_fail(e, "hipMemcpy of the queue order");
        for (int64_t q = 0; q < n; ++q) qs[q] = ns[ord[q]];
        const int32_t *keep = ns;
        ns = qs.data();
        hist(64, out->d_hist64_queue, &out->d_mean64_queue);
        ns = keep;
    } else {
        std::memcpy(out->d_hist64_queue, out->d_hist64, sizeof out->d_hist64);
        out->d_mean64_queue = out->d_mean64;
    }
    out->nbins_used = m->last_nbins;
    out->grid_used = m->last_grid;
    out->tile_used = m->last_tile;
    if (steps) std::memcpy(steps, &c[(size_t)rk::C_NSTEP * n], (size_t)n * sizeof(int32_t));
    if (status) std::memcpy(status, st, (size_t)n * sizeof(int32_t));
    return RK_OK;
}

static int dbg_common(rk_mech *m, int64_t n, const void *a, const void *b) {
    if (!m) return fail(RK_EINVAL, "NULL handle");
    if (n < 0) return fail(RK_EINVAL, "n < 0");
    if (n > 0 && (!a || !b || !is_device_ptr(a) || !is_device_ptr(b)))
        return fail(RK_EINVAL, "arrays must be device memory");
    const int rc = ensure_workspace(m, std::max<int64_t>(n, 1));
    return rc != RK_OK ? rc : ensure_lane_scratch(m, n);
}

int rk_dbg_rhs(rk_mech *m, int64_t n, const double *y, double *f, void *stream) {
    int rc = dbg_common(m, n, y, f);
    if (rc != RK_OK) return rc;
    hipError_t e = rk::launch_rhs(m->dev, n, y, f, m->scratch, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? RK_OK : hip_fail(e, "rhs kernel launch");
}

int rk_dbg_jacobian(rk_mech *m, int64_t n, const double *y, double *J, void *stream) {
    int rc = dbg_common(m, n, y, J);
    if (rc != RK_OK) return rc;
    hipError_t e = rk::launch_jac(m->dev, n, y, J, m->scratch, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? RK_OK : hip_fail(e, "jacobian kernel launch");
}

int rk_dbg_lu_solve(rk_mech *m, int64_t n, int fp32, double h, const double *J, const double *sc, const double *b,
                    double *x, void *stream) {
    if (!m) return fail(RK_EINVAL, "NULL handle");
    if (n < 0 || !(h > 0.0) || !std::isfinite(h) || (fp32 != 0 && fp32 != 1))
        return fail(RK_EINVAL, "rk_dbg_lu_solve: need n >= 0, h > 0, fp32 in {0, 1}");
    if (!rk::group_supported(m->K + 1))
        return fail(RK_EINVAL, "rk_dbg_lu_solve: the wavefront factorisation covers K + 1 <= 56");
    if (n > 0) {
        for (const void *q : {(const void *)J, (const void *)sc, (const void *)b, (const void *)x})
            if (!q || !is_device_ptr(q)) return fail(RK_EINVAL, "rk_dbg_lu_solve: arrays must be device memory");
    }
    rk::RadauParams p{};
    radau_constants(p);
    hipError_t e = rk::launch_lu_solve(m->K + 1, fp32 == 1, n, p.g / h, p.a / h, p.b / h, J, sc, b, x,
                                       static_cast<hipStream_t>(stream));
    return e == hipSuccess ? RK_OK : hip_fail(e, "lu_solve kernel launch");
}

}  // extern "C"
