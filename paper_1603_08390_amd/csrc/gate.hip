// Learned initial gate on gfx950: query features, a 64-128-128-1 MLP
// (bf16 weights, fp32 arithmetic), its backward pass and Adam.
//
// The paper starts the AuditThreshold at 1 (Algorithm 1).  Theorem 3.1 says
// AT - 1 ends at the query's k-th match count; a model that predicts that
// count lets the scan start AT close to it, so that far fewer increments pass
// the gate.  The search stays exact: a prediction that is too high is
// detected after the scan and the query is answered again with AT = 1.
//
// Every sum below runs in a fixed order, so a query's features and
// prediction do not depend on the other queries of the batch, and gradients
// do not depend on timing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "internal.h"

namespace genie {
namespace {

constexpr int kF = GENIE_GATE_FEATURES;   // 64
constexpr int kH = 128;                   // both hidden layers
constexpr int kOffW1 = 0, kOffB1 = kH * kF, kOffW2 = kOffB1 + kH, kOffB2 = kOffW2 + kH * kH;
constexpr int kOffW3 = kOffB2 + kH, kOffB3 = kOffW3 + kH, kParams = kOffB3 + 1;
static_assert(kParams == GENIE_GATE_PARAMS, "parameter layout");
constexpr int kQB = 32;                   // samples per workgroup in the MLP kernels

// ---------------------------------------------------------------------------
// features: see genie.h (genie_gate_features_async) for the list
// ---------------------------------------------------------------------------

struct FeatParams {
    const uint64_t *kcum;
    uint64_t n;
    uint32_t d, V;
    const uint64_t *q_off;
    const uint32_t *items;
    uint64_t n_items;
    uint32_t nq;
    double z;
    float *out;
};

__global__ __launch_bounds__(256) void gate_features_kernel(FeatParams p) {
    __shared__ uint64_t Ls[GENIE_MAX_ITEMS];
    __shared__ double red[4][256];
    __shared__ uint32_t hist[16], nzero, nbig;
    const uint32_t q = blockIdx.x, tid = threadIdx.x;
    const uint64_t i0 = p.q_off[q], i1 = p.q_off[q + 1];
    const bool bad = i1 < i0 || i1 > p.n_items || i1 - i0 > GENIE_MAX_ITEMS;
    const uint32_t s = bad ? 0u : (uint32_t)(i1 - i0);
    if (tid < 16)
        hist[tid] = 0;
    if (tid == 0) {
        nzero = 0;
        nbig = 0;
    }
    __syncthreads();
    const double n = (double)p.n;
    double a0 = 0, a1 = 0, a2 = 0, a3 = 0;
    for (uint32_t i = tid; i < s; i += 256) {
        const uint32_t *it = p.items + 3 * (i0 + i);
        const uint32_t dim = it[0], lo = it[1];
        const uint32_t hi = min(it[2], p.V - 1);
        uint64_t L = 0;
        if (dim < p.d && lo <= hi) {
            const uint64_t key = (uint64_t)dim * p.V;
            L = p.kcum[key + hi + 1] - p.kcum[key + lo];
        }
        Ls[i] = L;
        const double pi = (double)L / n;
        a0 += pi;
        a1 += pi * (1.0 - pi);
        a2 += pi * pi;
        a3 += pi * pi * pi;
        if (L == 0) {
            atomicAdd(&nzero, 1u);
        } else {
            uint32_t b = 0;   // largest b <= 15 with L * 2^b <= n
            while (b < 15 && (L << (b + 1)) <= p.n)
                b++;
            atomicAdd(&hist[b], 1u);
        }
        if (4 * L >= p.n)
            atomicAdd(&nbig, 1u);
    }
    red[0][tid] = a0;
    red[1][tid] = a1;
    red[2][tid] = a2;
    red[3][tid] = a3;
    uint32_t np2 = 1;
    while (np2 < s)
        np2 <<= 1;
    for (uint32_t i = s + tid; i < np2; i += 256)
        Ls[i] = 0;
    __syncthreads();
    for (uint32_t w = 128; w > 0; w >>= 1) {   // fixed-order tree
        if (tid < w)
            for (int c = 0; c < 4; c++)
                red[c][tid] += red[c][tid + w];
        __syncthreads();
    }
    // bitonic sort of the posting counts, descending
    for (uint32_t size = 2; size <= np2; size <<= 1)
        for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
            for (uint32_t i = tid; i < np2 / 2; i += 256) {
                const uint32_t lo = 2 * i - (i & (stride - 1)), hi = lo + stride;
                const bool desc = (lo & size) == 0;
                const uint64_t x = Ls[lo], y = Ls[hi];
                if ((x < y) == desc) {
                    Ls[lo] = y;
                    Ls[hi] = x;
                }
            }
            __syncthreads();
        }
    float *f = p.out + (uint64_t)q * kF;
    if (tid == 0) {
        const double mu = red[0][0], sigma = sqrt(red[1][0]);
        f[0] = (float)(s / 512.0);
        f[1] = (float)(mu / 64.0);
        f[2] = (float)(sigma / 8.0);
        f[3] = (float)((mu + p.z * sigma) / 64.0);
        f[4] = s ? (float)((double)Ls[0] / n) : 0.0f;
        f[5] = (float)(red[2][0] / 64.0);
        f[6] = (float)(red[3][0] / 64.0);
        f[7] = (float)(p.z / 8.0);
        f[56] = (float)(nzero / 64.0);
        f[57] = (float)(nbig / 64.0);
    }
    if (tid < 16)
        f[8 + tid] = (float)(hist[tid] / 64.0);
    if (tid < 32)
        f[24 + tid] = tid < s ? (float)((double)Ls[tid] / n) : 0.0f;
    if (tid >= 58 && tid < 64)
        f[tid] = 0.0f;
}

// ---------------------------------------------------------------------------
// MLP
// ---------------------------------------------------------------------------

__device__ __forceinline__ float wload(const uint16_t *w, int i) {
    return __uint_as_float((uint32_t)w[i] << 16);
}
__device__ __forceinline__ float wload(const float *w, int i) { return w[i]; }

// Forward for QB samples; thread j owns hidden unit j.  Leaves the hidden
// activations in h1s / h2s and the outputs in outs.
template <typename WT, int QB>
__device__ void mlp_forward_block(const WT *w, const float (*xs)[kF + 1], float (*h1s)[kH + 1],
                                  float (*h2s)[kH + 1], float *outs) {
    const int j = threadIdx.x;
    // Every output is the same fixed-order chain: bias, then one fma per
    // input in ascending order (batch-invariant); the loops run over the
    // inputs outside the samples, so each weight is read once per workgroup.
    {
        float acc[QB];
        const float b = wload(w, kOffB1 + j);
#pragma unroll
        for (int q = 0; q < QB; q++)
            acc[q] = b;
#pragma unroll 8
        for (int i = 0; i < kF; i++) {
            const float wi = wload(w, kOffW1 + j * kF + i);
#pragma unroll
            for (int q = 0; q < QB; q++)
                acc[q] = fmaf(wi, xs[q][i], acc[q]);
        }
#pragma unroll
        for (int q = 0; q < QB; q++)
            h1s[q][j] = fmaxf(acc[q], 0.0f);
    }
    __syncthreads();
    {
        float acc[QB];
        const float b = wload(w, kOffB2 + j);
#pragma unroll
        for (int q = 0; q < QB; q++)
            acc[q] = b;
#pragma unroll 8
        for (int i = 0; i < kH; i++) {
            const float wi = wload(w, kOffW2 + j * kH + i);
#pragma unroll
            for (int q = 0; q < QB; q++)
                acc[q] = fmaf(wi, h1s[q][i], acc[q]);
        }
#pragma unroll
        for (int q = 0; q < QB; q++)
            h2s[q][j] = fmaxf(acc[q], 0.0f);
    }
    __syncthreads();
    if (j < QB) {
        float acc = wload(w, kOffB3);
        for (int i = 0; i < kH; i++)
            acc = fmaf(wload(w, kOffW3 + i), h2s[j][i], acc);
        outs[j] = acc;
    }
    __syncthreads();
}

// Prediction: kQF samples per workgroup, so that a batch of about a thousand
// queries spreads over the device.
constexpr int kQF = 4;
template <typename WT>
__global__ __launch_bounds__(kH) void gate_forward_kernel(const WT *w, const float *x, uint32_t n,
                                                          float *out) {
    __shared__ float xs[kQF][kF + 1];
    __shared__ float h1s[kQF][kH + 1];
    __shared__ float h2s[kQF][kH + 1];
    __shared__ float outs[kQF];
    const uint64_t q0 = (uint64_t)blockIdx.x * kQF;
    for (int e = threadIdx.x; e < kQF * kF; e += kH) {
        const int q = e / kF, i = e % kF;
        xs[q][i] = q0 + q < n ? x[(q0 + q) * kF + i] : 0.0f;
    }
    __syncthreads();
    mlp_forward_block<WT, kQF>(w, xs, h1s, h2s, outs);
    if (threadIdx.x < kQF && q0 + threadIdx.x < n)
        out[q0 + threadIdx.x] = outs[threadIdx.x];
}

// Gradient of the mean pinball loss over n samples, for the kQB samples of
// this workgroup, written to partial[blockIdx.x][*] (summed in a fixed order
// by gate_reduce_kernel).
template <typename WT>
__global__ __launch_bounds__(kH) void gate_backward_kernel(const WT *w, const float *x,
                                                           const float *y, uint32_t n, float tau,
                                                           float *partial, float *partial_loss) {
    __shared__ float xs[kQB][kF + 1];
    __shared__ float h1s[kQB][kH + 1];
    __shared__ float h2s[kQB][kH + 1];
    __shared__ float d2s[kQB][kH + 1];
    __shared__ float outs[kQB], gs[kQB];
    const int j = threadIdx.x;
    const uint64_t q0 = (uint64_t)blockIdx.x * kQB;
    const uint32_t nb = (uint32_t)min<uint64_t>(kQB, n - q0);
    for (int e = j; e < kQB * kF; e += kH) {
        const int q = e / kF, i = e % kF;
        xs[q][i] = (uint32_t)q < nb ? x[(q0 + q) * kF + i] : 0.0f;
    }
    __syncthreads();
    mlp_forward_block<WT, kQB>(w, xs, h1s, h2s, outs);
    if (j < kQB) {
        float g = 0.0f;
        if ((uint32_t)j < nb) {
            const float r = y[q0 + j] - outs[j];
            g = (r >= 0.0f ? -tau : 1.0f - tau) / (float)n;
        }
        gs[j] = g;
    }
    __syncthreads();
    if (j == 0) {
        float l = 0.0f;
        for (uint32_t q = 0; q < nb; q++) {
            const float r = y[q0 + q] - outs[q];
            l += (r >= 0.0f ? tau * r : (tau - 1.0f) * r) / (float)n;
        }
        partial_loss[blockIdx.x] = l;
    }
    float *P = partial + (uint64_t)blockIdx.x * kParams;
    // output layer, and the error at the second hidden layer
    {
        const float w3 = wload(w, kOffW3 + j);
        float gw3 = 0.0f;
        for (int q = 0; q < kQB; q++) {
            gw3 = fmaf(gs[q], h2s[q][j], gw3);
            d2s[q][j] = h2s[q][j] > 0.0f ? gs[q] * w3 : 0.0f;
        }
        P[kOffW3 + j] = gw3;
        if (j == 0) {
            float gb = 0.0f;
            for (int q = 0; q < kQB; q++)
                gb += gs[q];
            P[kOffB3] = gb;
        }
    }
    __syncthreads();
    // second layer: row j of W2
    {
        float gb = 0.0f;
        for (int q = 0; q < kQB; q++)
            gb += d2s[q][j];
        P[kOffB2 + j] = gb;
        for (int i = 0; i < kH; i++) {
            float acc = 0.0f;
            for (int q = 0; q < kQB; q++)
                acc = fmaf(d2s[q][j], h1s[q][i], acc);
            P[kOffW2 + j * kH + i] = acc;
        }
    }
    // error at the first hidden layer (unit i = j): reuse h1s for it
    float d1[kQB];
    for (int q = 0; q < kQB; q++) {
        float acc = 0.0f;
        for (int jj = 0; jj < kH; jj++)
            acc = fmaf(d2s[q][jj], wload(w, kOffW2 + jj * kH + j), acc);
        d1[q] = h1s[q][j] > 0.0f ? acc : 0.0f;
    }
    {
        float gb = 0.0f;
        for (int q = 0; q < kQB; q++)
            gb += d1[q];
        P[kOffB1 + j] = gb;
        for (int c = 0; c < kF; c++) {
            float acc = 0.0f;
            for (int q = 0; q < kQB; q++)
                acc = fmaf(d1[q], xs[q][c], acc);
            P[kOffW1 + j * kF + c] = acc;
        }
    }
}

__global__ void gate_reduce_kernel(const float *partial, const float *partial_loss, uint32_t nwg,
                                   float *grad, float *loss) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < (uint32_t)kParams) {
        float acc = 0.0f;
        for (uint32_t b = 0; b < nwg; b++)
            acc += partial[(uint64_t)b * kParams + i];
        grad[i] = acc;
    }
    if (i == 0 && loss) {
        float l = 0.0f;
        for (uint32_t b = 0; b < nwg; b++)
            l += partial_loss[b];
        *loss = l;
    }
}

__device__ __forceinline__ uint16_t to_bf16_bits(float v) {
    const uint32_t b = __float_as_uint(v);
    return (uint16_t)((b + 0x7FFFu + ((b >> 16) & 1u)) >> 16);   // nearest, ties to even
}

__global__ void gate_adam_kernel(float *master, uint16_t *wbf, const float *grad, float *m,
                                 float *v, float lr, float beta1, float beta2, float eps,
                                 float c1, float c2) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (uint32_t)kParams)
        return;
    const float g = grad[i];
    const float mi = beta1 * m[i] + (1.0f - beta1) * g;
    const float vi = beta2 * v[i] + (1.0f - beta2) * g * g;
    m[i] = mi;
    v[i] = vi;
    const float th = master[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    master[i] = th;
    if (wbf)
        wbf[i] = to_bf16_bits(th);
}

int check_weights(const uint16_t *wb, const float *wf) {
    if ((wb == nullptr) == (wf == nullptr)) {
        set_error("pass exactly one of the bf16 and fp32 weight pointers");
        return GENIE_EINVAL;
    }
    return GENIE_OK;
}

}  // namespace
}  // namespace genie

using namespace genie;

extern "C" int genie_gate_features_async(const genie_index *ix, const uint64_t *d_q_offsets,
                                         const genie_item *d_items, uint64_t n_items,
                                         uint32_t n_queries, uint32_t k, float *d_features,
                                         void *stream) {
    clear_error();
    if (!ix || (n_queries && (!d_q_offsets || !d_items || !d_features)) || k == 0) {
        set_error("bad arguments");
        return GENIE_EINVAL;
    }
    if (n_queries == 0)
        return GENIE_OK;
    FeatParams p{};
    p.kcum = ix->kcum;
    p.n = ix->n;
    p.d = ix->d;
    p.V = ix->V;
    p.q_off = d_q_offsets;
    p.items = reinterpret_cast<const uint32_t *>(d_items);
    p.n_items = n_items;
    p.nq = n_queries;
    // upper k/n quantile of the standard normal (k < n; clamped otherwise)
    double qk = std::min(std::max((double)k / (double)ix->n, 1e-12), 1.0 - 1e-12);
    {
        // invert the upper tail by bisection on erfc: P(Z > z) = erfc(z/sqrt2)/2
        double lo = -40.0, hi = 40.0;
        for (int it = 0; it < 200; it++) {
            const double mid = 0.5 * (lo + hi);
            if (0.5 * std::erfc(mid / std::sqrt(2.0)) > qk)
                lo = mid;
            else
                hi = mid;
        }
        p.z = 0.5 * (lo + hi);
    }
    p.out = d_features;
    hipLaunchKernelGGL(gate_features_kernel, dim3(n_queries), dim3(256), 0, (hipStream_t)stream, p);
    GENIE_HIP(hipGetLastError());
    return GENIE_OK;
}

extern "C" int genie_gate_forward_async(const uint16_t *d_w_bf16, const float *d_w_f32,
                                        const float *d_x, uint32_t n, float *d_out, void *stream) {
    clear_error();
    int rc = check_weights(d_w_bf16, d_w_f32);
    if (rc)
        return rc;
    if (n == 0)
        return GENIE_OK;
    if (!d_x || !d_out) {
        set_error("null pointer");
        return GENIE_EINVAL;
    }
    dim3 grid((n + kQF - 1) / kQF);
    if (d_w_bf16)
        hipLaunchKernelGGL(gate_forward_kernel<uint16_t>, grid, dim3(kH), 0, (hipStream_t)stream,
                           d_w_bf16, d_x, n, d_out);
    else
        hipLaunchKernelGGL(gate_forward_kernel<float>, grid, dim3(kH), 0, (hipStream_t)stream,
                           d_w_f32, d_x, n, d_out);
    GENIE_HIP(hipGetLastError());
    return GENIE_OK;
}

extern "C" size_t genie_gate_workspace_size(uint32_t n) {
    const size_t nwg = (n + kQB - 1) / kQB;
    return nwg * kParams * sizeof(float) + ((nwg * sizeof(float) + 255) & ~size_t(255)) + 256;
}

extern "C" int genie_gate_backward_async(const uint16_t *d_w_bf16, const float *d_w_f32,
                                         const float *d_x, const float *d_y, uint32_t n, float tau,
                                         float *d_grad, float *d_loss, void *d_workspace,
                                         size_t workspace_bytes, void *stream) {
    clear_error();
    int rc = check_weights(d_w_bf16, d_w_f32);
    if (rc)
        return rc;
    if (n == 0 || !d_x || !d_y || !d_grad || !d_workspace || !(tau > 0.0f && tau < 1.0f)) {
        set_error("bad arguments");
        return GENIE_EINVAL;
    }
    if (workspace_bytes < genie_gate_workspace_size(n)) {
        set_error("workspace too small");
        return GENIE_EINVAL;
    }
    const uint32_t nwg = (n + kQB - 1) / kQB;
    float *partial_loss = static_cast<float *>(d_workspace);
    float *partial = reinterpret_cast<float *>(static_cast<char *>(d_workspace) +
                                               ((nwg * sizeof(float) + 255) & ~size_t(255)));
    hipStream_t st = (hipStream_t)stream;
    if (d_w_bf16)
        hipLaunchKernelGGL(gate_backward_kernel<uint16_t>, dim3(nwg), dim3(kH), 0, st, d_w_bf16,
                           d_x, d_y, n, tau, partial, partial_loss);
    else
        hipLaunchKernelGGL(gate_backward_kernel<float>, dim3(nwg), dim3(kH), 0, st, d_w_f32, d_x,
                           d_y, n, tau, partial, partial_loss);
    GENIE_HIP(hipGetLastError());
    hipLaunchKernelGGL(gate_reduce_kernel, dim3((kParams + 255) / 256), dim3(256), 0, st, partial,
                       partial_loss, nwg, d_grad, d_loss);
    GENIE_HIP(hipGetLastError());
    return GENIE_OK;
}

extern "C" int genie_gate_adam_async(float *d_master, uint16_t *d_w_bf16, const float *d_grad,
                                     float *d_m, float *d_v, uint32_t step, float lr, float beta1,
                                     float beta2, float eps, void *stream) {
    clear_error();
    if (!d_master || !d_grad || !d_m || !d_v || step == 0) {
        set_error("bad arguments");
        return GENIE_EINVAL;
    }
    const float c1 = 1.0f - std::pow(beta1, (float)step);
    const float c2 = 1.0f - std::pow(beta2, (float)step);
    hipLaunchKernelGGL(gate_adam_kernel, dim3((kParams + 255) / 256), dim3(256), 0,
                       (hipStream_t)stream, d_master, d_w_bf16, d_grad, d_m, d_v, lr, beta1, beta2,
                       eps, c1, c2);
    GENIE_HIP(hipGetLastError());
    return GENIE_OK;
}
