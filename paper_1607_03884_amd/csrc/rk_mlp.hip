// Multilayer perceptron for the learned stage/step predictor: training and
// inference kernels for gfx950.  Weights are held as FP32 master copies and
// used as BF16 (round-to-nearest-even) in every product; products accumulate
// in FP32.  Hidden layers use GELU (x * Phi(x), erf form); the output layer
// is linear.  Loss: weighted, masked mean squared error.  Optimiser: Adam.
//
// Layer l maps [B, d_l] -> [B, d_(l+1)] with W_l [d_(l+1), d_l] (row-major)
// and bias b_l.  The flat parameter vector stores, per layer, W_l then b_l.
#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "rk_internal.h"

namespace rk {

namespace {

__device__ __forceinline__ float bf16_round(float x) {
    // round to nearest even at 16 mantissa bits of FP32 (the BF16 value, kept in FP32)
    uint32_t u = __builtin_bit_cast(uint32_t, x);
    if ((u & 0x7f800000u) == 0x7f800000u) return x;      // inf / nan unchanged
    u += 0x7fffu + ((u >> 16) & 1u);
    u &= 0xffff0000u;
    return __builtin_bit_cast(float, u);
}

__device__ __forceinline__ float gelu(float x) { return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f)); }

__device__ __forceinline__ float gelu_grad(float x) {
    return 0.5f * (1.0f + erff(x * 0.70710678118654752f)) + x * 0.39894228040143268f * expf(-0.5f * x * x);
}

// Z = X W^T + b (pre-activation), A = act(Z) on the matrix cores: each
// wavefront computes a 16 (rows of X) x 16 (outputs) tile with
// v_mfma_f32_16x16x4_f32, k in steps of 4.  The BF16 weights are exact in
// FP32, so the products are BF16 weight x FP32 activation, accumulated in
// FP32.  Operand layout of the 16x16x4 FP32 MFMA (lane l = 16 q + i):
// A[i][q] and B[q][i] in, D[4 q + v][i] (v = 0..3) out.  A block of four
// wavefronts covers 16 rows x 64 outputs; din and dout need not be
// multiples of 4 or 16 (out-of-range operands are zero, results not stored).
typedef float f32x4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void layer_fwd_kernel(int64_t B, int din, int dout, const float *__restrict__ X,
                                                        const uint16_t *__restrict__ Wb, const float *__restrict__ bias,
                                                        float *__restrict__ Z, float *__restrict__ A, int act) {
    const int lane = threadIdx.x & 63;
    const int i = lane & 15, q = lane >> 4;
    const int o0 = blockIdx.x * 64 + (threadIdx.x >> 6) * 16;
    const int64_t b0 = (int64_t)blockIdx.y * 16;
    if (o0 >= dout) return;                       // whole wavefront: no MFMA with partial exec
    const int64_t row = b0 + i;                    // A operand: X[row][k + q]
    const int oc = o0 + i;                         // B operand: W[oc][k + q]
    const bool rok = row < B, ook = oc < dout;
    const float *x = X + (rok ? row : 0) * din;
    const uint16_t *w = Wb + (size_t)(ook ? oc : 0) * din;
    f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
    for (int k = 0; k < din; k += 4) {
        const int kk = k + q;
        const float a = (rok && kk < din) ? x[kk] : 0.0f;
        const float b = (ook && kk < din) ? __builtin_bit_cast(float, (uint32_t)w[kk] << 16) : 0.0f;
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
    }
    // this lane holds D[4 q + v][i]: rows b0 + 4 q + v, output o0 + i
    if (!ook) return;
    const float bo = bias[oc];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int64_t r = b0 + 4 * q + v;
        if (r < B) {
            const float zz = acc[v] + bo;
            Z[r * dout + oc] = zz;
            if (A) A[r * dout + oc] = act ? gelu(zz) : zz;
        }
    }
}

// dZ = dA * act'(Z) (in place on dA when act)
__global__ void act_bwd_kernel(int64_t n, const float *__restrict__ Z, float *__restrict__ dA) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dA[i] *= gelu_grad(Z[i]);
}

// dX = dZ W  ([B, dout] x [dout, din])
__global__ __launch_bounds__(256) void layer_bwd_x_kernel(int64_t B, int din, int dout, const float *__restrict__ dZ,
                                                          const uint16_t *__restrict__ Wb, float *__restrict__ dX) {
    const int i = blockIdx.x * 64 + (threadIdx.x & 63);
    const int64_t b = (int64_t)blockIdx.y * 4 + (threadIdx.x >> 6);
    if (i >= din || b >= B) return;
    const float *dz = dZ + b * dout;
    float acc = 0.0f;
    for (int o = 0; o < dout; ++o) acc += dz[o] * __builtin_bit_cast(float, (uint32_t)Wb[(size_t)o * din + i] << 16);
    dX[b * din + i] = acc;
}

// dW[o, i] = sum_b dZ[b, o] X[b, i]; db[o] = sum_b dZ[b, o].  One block per
// output o, threads over inputs (+1 for the bias), loop over the batch.
__global__ __launch_bounds__(256) void layer_bwd_w_kernel(int64_t B, int din, int dout, const float *__restrict__ dZ,
                                                          const float *__restrict__ X, float *__restrict__ dW,
                                                          float *__restrict__ db) {
    const int o = blockIdx.x;
    for (int i = threadIdx.x; i <= din; i += blockDim.x) {
        float acc = 0.0f;
        if (i < din)
            for (int64_t b = 0; b < B; ++b) acc += dZ[b * dout + o] * X[b * din + i];
        else
            for (int64_t b = 0; b < B; ++b) acc += dZ[b * dout + o];
        if (i < din) dW[(size_t)o * din + i] = acc;
        else db[o] = acc;
    }
}

// masked weighted MSE: loss = sum_b mask_b sum_o w_o (y - t)^2 / sum_b mask_b;
// dY = dloss/dy.  Partial sums per block into part[blockIdx] (loss, mask).
__global__ __launch_bounds__(256) void mse_kernel(int64_t B, int dout, const float *__restrict__ Y,
                                                  const float *__restrict__ T, const float *__restrict__ mask,
                                                  const float *__restrict__ w, float inv_count, float *__restrict__ dY,
                                                  float *__restrict__ part) {
    __shared__ float red[256];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    float l = 0.0f;
    if (i < B * dout) {
        const int64_t b = i / dout;
        const int o = (int)(i % dout);
        const float d = Y[i] - T[i];
        const float mw = mask[b] * w[o];
        l = mw * d * d;
        dY[i] = 2.0f * mw * d * inv_count;
    }
    red[threadIdx.x] = l;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void sum_kernel(int n, const float *__restrict__ part, float scale, float *__restrict__ out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        float s = 0.0f;
        for (int i = 0; i < n; ++i) s += part[i];
        *out = s * scale;
    }
}

// Adam on the FP32 masters, then the BF16 copy of the weights
__global__ void adam_kernel(int64_t n, float *__restrict__ p, float *__restrict__ m, float *__restrict__ v,
                            const float *__restrict__ g, float lr, float b1, float b2, float eps, float c1, float c2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__global__ void to_bf16_kernel(int64_t n, const float *__restrict__ p, uint16_t *__restrict__ q) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) q[i] = (uint16_t)(__builtin_bit_cast(uint32_t, bf16_round(p[i])) >> 16);
}

unsigned blocks(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

// ---------------------------------------------------------------------------
// host object
// ---------------------------------------------------------------------------
Mlp::~Mlp() {
    for (void *p : {(void *)params, (void *)wbf, (void *)grads, (void *)adam_m, (void *)adam_v, (void *)part})
        if (p) (void)hipFree(p);
    for (float *p : acts) if (p) (void)hipFree(p);
    for (float *p : pre) if (p) (void)hipFree(p);
    for (float *p : dacts) if (p) (void)hipFree(p);
}

int64_t Mlp::count() const {
    int64_t c = 0;
    for (size_t l = 0; l + 1 < dims.size(); ++l) c += (int64_t)dims[l + 1] * dims[l] + dims[l + 1];
    return c;
}

hipError_t Mlp::init(const std::vector<int> &d) {
    dims = d;
    const int64_t c = count();
    hipError_t e = hipSuccess;
    for (auto pp : {(void **)&params, (void **)&grads, (void **)&adam_m, (void **)&adam_v}) {
        if (e == hipSuccess) e = hipMalloc(pp, c * sizeof(float));
        if (e == hipSuccess) e = hipMemset(*pp, 0, c * sizeof(float));
    }
    if (e == hipSuccess) e = hipMalloc(&wbf, c * sizeof(uint16_t));
    if (e == hipSuccess) e = hipMalloc(&part, 65536 * sizeof(float));
    return e;
}

hipError_t Mlp::ensure_batch(int64_t B) {
    if (B <= cap_b) return hipSuccess;
    for (float *p : acts) if (p) (void)hipFree(p);
    for (float *p : pre) if (p) (void)hipFree(p);
    for (float *p : dacts) if (p) (void)hipFree(p);
    const size_t L = dims.size();
    acts.assign(L, nullptr);
    pre.assign(L, nullptr);
    dacts.assign(L, nullptr);
    hipError_t e = hipSuccess;
    for (size_t l = 1; l < L && e == hipSuccess; ++l) {
        e = hipMalloc(&acts[l], (size_t)B * dims[l] * sizeof(float));
        if (e == hipSuccess) e = hipMalloc(&pre[l], (size_t)B * dims[l] * sizeof(float));
        if (e == hipSuccess) e = hipMalloc(&dacts[l], (size_t)B * dims[l] * sizeof(float));
    }
    if (e == hipSuccess) e = hipMalloc(&dacts[0], (size_t)B * dims[0] * sizeof(float));
    if (e == hipSuccess) cap_b = B;
    return e;
}

hipError_t Mlp::refresh_bf16(hipStream_t st) {
    const int64_t c = count();
    hipLaunchKernelGGL(to_bf16_kernel, dim3(blocks(c, 256)), dim3(256), 0, st, c, params, wbf);
    return hipGetLastError();
}

// forward pass; the output layer's values land in pre[L-1] (linear)
hipError_t Mlp::forward(int64_t B, const float *x, hipStream_t st) {
    hipError_t e = ensure_batch(B);
    if (e != hipSuccess) return e;
    const size_t L = dims.size();
    const float *in = x;
    int64_t off = 0;
    for (size_t l = 0; l + 1 < L; ++l) {
        const int din = dims[l], dout = dims[l + 1];
        const bool hidden = l + 2 < L;
        if (blocks(B, 16) > 0x7fffffffu) return hipErrorInvalidValue;
        hipLaunchKernelGGL(layer_fwd_kernel, dim3(blocks(dout, 64), blocks(B, 16)), dim3(256), 0, st, B, din, dout, in,
                           wbf + off, params + off + (int64_t)dout * din, pre[l + 1], hidden ? acts[l + 1] : nullptr,
                           hidden ? 1 : 0);
        in = acts[l + 1];
        off += (int64_t)dout * din + dout;
    }
    return hipGetLastError();
}

// loss and gradients into grads (no update)
hipError_t Mlp::backward(int64_t B, const float *x, const float *t, const float *mask, const float *wout,
                         float inv_count, float *loss, hipStream_t st) {
    hipError_t e = forward(B, x, st);
    if (e != hipSuccess) return e;
    const size_t L = dims.size();
    const int dlast = dims[L - 1];
    const int64_t nout = B * dlast;
    const unsigned nb = blocks(nout, 256);
    if (nb > 65536) return hipErrorInvalidValue;
    hipLaunchKernelGGL(mse_kernel, dim3(nb), dim3(256), 0, st, B, dlast, pre[L - 1], t, mask, wout, inv_count,
                       dacts[L - 1], part);
    hipLaunchKernelGGL(sum_kernel, dim3(1), dim3(1), 0, st, (int)nb, part, inv_count, loss);
    // parameter offsets per layer
    std::vector<int64_t> off(L, 0);
    for (size_t l = 0; l + 1 < L; ++l) off[l + 1] = off[l] + (int64_t)dims[l + 1] * dims[l] + dims[l + 1];
    for (size_t l = L - 1; l >= 1; --l) {
        const int dout = dims[l], din = dims[l - 1];
        float *dZ = dacts[l];
        if (l + 1 < L) {      // hidden layer: through GELU
            const int64_t n = B * dout;
            hipLaunchKernelGGL(act_bwd_kernel, dim3(blocks(n, 256)), dim3(256), 0, st, n, pre[l], dZ);
        }
        const float *Xin = l >= 2 ? acts[l - 1] : x;
        hipLaunchKernelGGL(layer_bwd_w_kernel, dim3(dout), dim3(256), 0, st, B, din, dout, dZ, Xin,
                           grads + off[l - 1], grads + off[l - 1] + (int64_t)dout * din);
        if (l >= 2)
            hipLaunchKernelGGL(layer_bwd_x_kernel, dim3(blocks(din, 64), blocks(B, 4)), dim3(256), 0, st, B, din, dout,
                               dZ, wbf + off[l - 1], dacts[l - 1]);
    }
    return hipGetLastError();
}

hipError_t Mlp::adam(float lr, hipStream_t st) {
    ++steps;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.0f - std::pow(b1, (float)steps), c2 = 1.0f - std::pow(b2, (float)steps);
    const int64_t c = count();
    hipLaunchKernelGGL(adam_kernel, dim3(blocks(c, 256)), dim3(256), 0, st, c, params, adam_m, adam_v, grads, lr, b1, b2,
                       1e-8f, c1, c2);
    return refresh_bf16(st);
}

}  // namespace rk

// =============================================================================
// C ABI of the predictor network
// =============================================================================
namespace {
thread_local std::string g_mlp_err;
int mfail(int code, const std::string &m) {
    g_mlp_err = m;
    return code;
}
}  // namespace

extern "C" {

const char *rk_mlp_last_error(void) { return g_mlp_err.c_str(); }

int rk_mlp_create(int32_t n_dims, const int32_t *dims, rk_mlp **out) {
    if (!out || !dims || n_dims < 2 || n_dims > 8) return mfail(RK_EINVAL, "rk_mlp_create: 2..8 layer widths");
    for (int i = 0; i < n_dims; ++i)
        if (dims[i] < 1 || dims[i] > 4096) return mfail(RK_EINVAL, "rk_mlp_create: widths 1..4096");
    auto *m = new rk::Mlp();
    if (m->init(std::vector<int>(dims, dims + n_dims)) != hipSuccess) {
        delete m;
        (void)hipGetLastError();
        return mfail(RK_ENOMEM, "rk_mlp_create: device allocation failed");
    }
    *out = reinterpret_cast<rk_mlp *>(m);
    return RK_OK;
}

void rk_mlp_free(rk_mlp *h) {
    if (!h) return;
    (void)hipDeviceSynchronize();
    delete reinterpret_cast<rk::Mlp *>(h);
}

int64_t rk_mlp_param_count(const rk_mlp *h) { return h ? reinterpret_cast<const rk::Mlp *>(h)->count() : -1; }

int rk_mlp_set_params(rk_mlp *h, const float *host, int64_t count) {
    auto *m = reinterpret_cast<rk::Mlp *>(h);
    if (!m || !host || count != m->count()) return mfail(RK_EINVAL, "rk_mlp_set_params: size mismatch");
    if (hipMemcpy(m->params, host, count * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(m->adam_m, 0, count * sizeof(float)) != hipSuccess ||
        hipMemset(m->adam_v, 0, count * sizeof(float)) != hipSuccess)
        return mfail(RK_EHIP, "rk_mlp_set_params: copy failed");
    m->steps = 0;
    if (m->refresh_bf16(nullptr) != hipSuccess || hipDeviceSynchronize() != hipSuccess)
        return mfail(RK_EHIP, "rk_mlp_set_params: conversion failed");
    return RK_OK;
}

int rk_mlp_get_params(const rk_mlp *h, float *host, int64_t count) {
    auto *m = reinterpret_cast<const rk::Mlp *>(h);
    if (!m || !host || count != m->count()) return mfail(RK_EINVAL, "rk_mlp_get_params: size mismatch");
    if (hipMemcpy(host, m->params, count * sizeof(float), hipMemcpyDeviceToHost) != hipSuccess)
        return mfail(RK_EHIP, "rk_mlp_get_params: copy failed");
    return RK_OK;
}

int rk_mlp_forward(rk_mlp *h, int64_t B, const float *d_x, float *d_y, void *stream) {
    auto *m = reinterpret_cast<rk::Mlp *>(h);
    if (!m || B < 1 || !d_x || !d_y) return mfail(RK_EINVAL, "rk_mlp_forward: bad arguments");
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (m->forward(B, d_x, st) != hipSuccess) return mfail(RK_EHIP, "rk_mlp_forward: launch failed");
    const int dl = m->dims.back();
    if (hipMemcpyAsync(d_y, m->pre.back(), (size_t)B * dl * sizeof(float), hipMemcpyDeviceToDevice, st) != hipSuccess)
        return mfail(RK_EHIP, "rk_mlp_forward: copy failed");
    return RK_OK;
}

int rk_mlp_grads(rk_mlp *h, int64_t B, const float *d_x, const float *d_t, const float *d_mask, const float *d_wout,
                 float *d_grad, float *d_loss, void *stream) {
    auto *m = reinterpret_cast<rk::Mlp *>(h);
    if (!m || B < 1 || !d_x || !d_t || !d_mask || !d_wout || !d_loss) return mfail(RK_EINVAL, "rk_mlp_grads: bad arguments");
    hipStream_t st = static_cast<hipStream_t>(stream);
    std::vector<float> mk(B);
    if (hipMemcpy(mk.data(), d_mask, B * sizeof(float), hipMemcpyDeviceToHost) != hipSuccess)
        return mfail(RK_EHIP, "rk_mlp_grads: mask copy failed");
    double cnt = 0.0;
    for (float v : mk) cnt += v;
    const float inv = cnt > 0 ? (float)(1.0 / cnt) : 0.0f;
    if (m->backward(B, d_x, d_t, d_mask, d_wout, inv, d_loss, st) != hipSuccess)
        return mfail(RK_EHIP, "rk_mlp_grads: launch failed");
    if (d_grad && hipMemcpyAsync(d_grad, m->grads, m->count() * sizeof(float), hipMemcpyDeviceToDevice, st) != hipSuccess)
        return mfail(RK_EHIP, "rk_mlp_grads: copy failed");
    return RK_OK;
}

int rk_mlp_train_step(rk_mlp *h, int64_t B, const float *d_x, const float *d_t, const float *d_mask,
                      const float *d_wout, float inv_count, float lr, float *d_loss, void *stream) {
    auto *m = reinterpret_cast<rk::Mlp *>(h);
    if (!m || B < 1 || !d_x || !d_t || !d_mask || !d_wout || !d_loss || !(lr > 0.0f))
        return mfail(RK_EINVAL, "rk_mlp_train_step: bad arguments");
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (m->backward(B, d_x, d_t, d_mask, d_wout, inv_count, d_loss, st) != hipSuccess || m->adam(lr, st) != hipSuccess)
        return mfail(RK_EHIP, "rk_mlp_train_step: launch failed");
    return RK_OK;
}

}  // extern "C"
