// LSH signatures on gfx950: the object transform of Section 4.1.2 with the
// E2LSH family of Section 4.2.3.
//
//   h_i(p) = floor((a_i . p + b_i) / w)                       (float32)
//   r_i(h) = ((A_i * u + B_i) mod 2^64) >> (64 - log2 D),      u = (uint32)h
//
// Each projection a_i . p is one fma chain over the coordinates in
// ascending order, so a point's signature does not depend on which other
// points share the launch or how the grid is cut.  A workgroup computes a
// 64 x 64 block of (point, function) pairs from 32-coordinate slices of the
// points and of the projection vectors staged in LDS.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "internal.h"

namespace genie {
namespace {

constexpr int kLshTile = 64;   // points and functions per workgroup
constexpr int kLshSlice = 32;  // coordinates staged per step

struct LshParams {
    const float *points, *a, *b;
    const uint64_t *rehash;
    uint64_t n;
    uint32_t dim, m, shift;
    float w;
    uint32_t *out;
};

__global__ __launch_bounds__(256) void lsh_kernel(LshParams p) {
    __shared__ float ps[kLshTile][kLshSlice + 1];
    __shared__ float as[kLshTile][kLshSlice + 1];
    const uint32_t tid = threadIdx.x;
    const uint32_t tx = tid & 15, ty = tid >> 4;
    const uint32_t f0 = blockIdx.y * kLshTile;
    const uint64_t i0 = (uint64_t)blockIdx.x * kLshTile;
    float acc[4][4];
#pragma unroll
    for (int r = 0; r < 4; r++)
#pragma unroll
        for (int c = 0; c < 4; c++)
            acc[r][c] = 0.0f;

    for (uint32_t j0 = 0; j0 < p.dim; j0 += kLshSlice) {
        for (uint32_t e = tid; e < kLshTile * kLshSlice; e += 256) {
            const uint32_t r = e / kLshSlice, c = e % kLshSlice;
            const uint32_t j = j0 + c;
            const uint64_t i = i0 + r;
            const uint32_t f = f0 + r;
            ps[r][c] = (i < p.n && j < p.dim) ? p.points[i * p.dim + j] : 0.0f;
            as[r][c] = (f < p.m && j < p.dim) ? p.a[(uint64_t)f * p.dim + j] : 0.0f;
        }
        __syncthreads();
        const uint32_t jn = min<uint32_t>(kLshSlice, p.dim - j0);
        for (uint32_t c = 0; c < jn; c++) {
            float pv[4], av[4];
#pragma unroll
            for (int r = 0; r < 4; r++) {
                pv[r] = ps[ty * 4 + r][c];
                av[r] = as[tx * 4 + r][c];
            }
#pragma unroll
            for (int r = 0; r < 4; r++)
#pragma unroll
                for (int cc = 0; cc < 4; cc++)
                    acc[r][cc] = fmaf(pv[r], av[cc], acc[r][cc]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < 4; r++) {
        const uint64_t i = i0 + ty * 4 + r;
        if (i >= p.n)
            continue;
#pragma unroll
        for (int c = 0; c < 4; c++) {
            const uint32_t f = f0 + tx * 4 + c;
            if (f >= p.m)
                continue;
            const float hv = floorf((acc[r][c] + p.b[f]) / p.w);
            // clamp to the int32 range before the conversion
            const float lo = -2147483648.0f, hi = 2147483520.0f;
            const int32_t h = (int32_t)fminf(fmaxf(hv, lo), hi);
            const uint64_t u = (uint64_t)(uint32_t)h;
            const uint64_t x = p.rehash[2 * f] * u + p.rehash[2 * f + 1];
            p.out[i * p.m + f] = (uint32_t)(x >> p.shift);
        }
    }
}

// Random binning hashing for the Laplacian kernel (Section 4.1.3): function
// f puts point p in the bin floor((p_j - u_fj) / g_fj) on every dimension
// j (float32, correctly rounded division), and the bin vector, as int32
// blocks in ascending j, is re-hashed by MurmurHash3_x86_32 seeded with
// seed_f (the hash's public description: per block k *= c1, k = rotl(k, 15),
// k *= c2, h ^= k, h = rotl(h, 13), h = 5 h + 0xe6546b64; then h ^= bytes
// and fmix32); the bucket is its top log2 D bits.  The hash state of each
// (point, function) pair is carried through the coordinate slices, so the
// result does not depend on the launch.  Same 64 x 64 blocking as
// lsh_kernel, with the pitches and shifts of the functions staged in LDS.
struct RbhParams {
    const float *points, *g, *u;
    const uint32_t *seeds;
    uint64_t n;
    uint32_t dim, m, shift;
    uint32_t *out;
};

__device__ __forceinline__ uint32_t rotl32(uint32_t x, int r) {
    return (x << r) | (x >> (32 - r));
}

__global__ __launch_bounds__(256) void rbh_kernel(RbhParams p) {
    __shared__ float ps[kLshTile][kLshSlice + 1];
    __shared__ float gs[kLshTile][kLshSlice + 1];
    __shared__ float us[kLshTile][kLshSlice + 1];
    const uint32_t tid = threadIdx.x;
    const uint32_t tx = tid & 15, ty = tid >> 4;
    const uint32_t f0 = blockIdx.y * kLshTile;
    const uint64_t i0 = (uint64_t)blockIdx.x * kLshTile;
    uint32_t h[4][4];
#pragma unroll
    for (int c = 0; c < 4; c++) {
        const uint32_t f = f0 + tx * 4 + c;
        const uint32_t seed = f < p.m ? p.seeds[f] : 0u;
#pragma unroll
        for (int r = 0; r < 4; r++)
            h[r][c] = seed;
    }
    for (uint32_t j0 = 0; j0 < p.dim; j0 += kLshSlice) {
        for (uint32_t e = tid; e < kLshTile * kLshSlice; e += 256) {
            const uint32_t r = e / kLshSlice, c = e % kLshSlice;
            const uint32_t j = j0 + c;
            const uint64_t i = i0 + r;
            const uint32_t f = f0 + r;
            const bool fj = f < p.m && j < p.dim;
            ps[r][c] = (i < p.n && j < p.dim) ? p.points[i * p.dim + j] : 0.0f;
            gs[r][c] = fj ? p.g[(uint64_t)f * p.dim + j] : 1.0f;
            us[r][c] = fj ? p.u[(uint64_t)f * p.dim + j] : 0.0f;
        }
        __syncthreads();
        const uint32_t jn = min<uint32_t>(kLshSlice, p.dim - j0);
        for (uint32_t c = 0; c < jn; c++) {
            float pv[4], gv[4], uv[4];
#pragma unroll
            for (int r = 0; r < 4; r++) {
                pv[r] = ps[ty * 4 + r][c];
                gv[r] = gs[tx * 4 + r][c];
                uv[r] = us[tx * 4 + r][c];
            }
#pragma unroll
            for (int r = 0; r < 4; r++)
#pragma unroll
                for (int cc = 0; cc < 4; cc++) {
                    const float bv = floorf((pv[r] - uv[cc]) / gv[cc]);
                    const float lo = -2147483648.0f, hi = 2147483520.0f;
                    uint32_t k = (uint32_t)(int32_t)fminf(fmaxf(bv, lo), hi);
                    k *= 0xCC9E2D51u;
                    k = rotl32(k, 15);
                    k *= 0x1B873593u;
                    uint32_t x = h[r][cc] ^ k;
                    x = rotl32(x, 13);
                    h[r][cc] = x * 5u + 0xE6546B64u;
                }
        }
        __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < 4; r++) {
        const uint64_t i = i0 + ty * 4 + r;
        if (i >= p.n)
            continue;
#pragma unroll
        for (int c = 0; c < 4; c++) {
            const uint32_t f = f0 + tx * 4 + c;
            if (f >= p.m)
                continue;
            uint32_t x = h[r][c] ^ (4u * p.dim);
            x ^= x >> 16;
            x *= 0x85EBCA6Bu;
            x ^= x >> 13;
            x *= 0xC2B2AE35u;
            x ^= x >> 16;
            p.out[i * p.m + f] = p.shift >= 32 ? 0u : (x >> p.shift);
        }
    }
}

__global__ void lsh_items_kernel(const uint32_t *sig, uint32_t nq, uint32_t m, uint32_t *items,
                                 uint64_t *q_off) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t total = (uint64_t)nq * m;
    if (i < total) {
        const uint32_t f = (uint32_t)(i % m);
        const uint32_t v = sig[i];
        items[3 * i] = f;
        items[3 * i + 1] = v;
        items[3 * i + 2] = v;
    }
    if (i <= nq)
        q_off[i] = i * m;
}

}  // namespace
}  // namespace genie

using namespace genie;

extern "C" int genie_lsh_items_async(const uint32_t *d_sig, uint32_t n_queries, uint32_t m,
                                     genie_item *d_items, uint64_t *d_q_offsets, void *stream) {
    clear_error();
    if (!d_items || !d_q_offsets || (n_queries && !d_sig) || m == 0) {
        set_error("bad arguments");
        return GENIE_EINVAL;
    }
    const uint64_t total = std::max<uint64_t>((uint64_t)n_queries * m, (uint64_t)n_queries + 1);
    const uint64_t blocks = (total + 255) / 256;
    if (blocks > 0x7FFFFFFFull) {
        set_error("too many items");
        return GENIE_EINVAL;
    }
    hipLaunchKernelGGL(lsh_items_kernel, dim3((uint32_t)blocks), dim3(256), 0, (hipStream_t)stream,
                       d_sig, n_queries, m, reinterpret_cast<uint32_t *>(d_items), d_q_offsets);
    GENIE_HIP(hipGetLastError());
    return GENIE_OK;
}

extern "C" int genie_lsh_signatures(const float *d_points, uint64_t n, uint32_t dim,
                                    const float *d_a, const float *d_b, float w, uint32_t m,
                                    const uint64_t *d_rehash, uint32_t log2_buckets,
                                    uint32_t *d_out_sig, void *stream) {
    clear_error();
    if (n == 0)
        return GENIE_OK;
    if (!d_points || !d_a || !d_b || !d_rehash || !d_out_sig) {
        set_error("null pointer");
        return GENIE_EINVAL;
    }
    if (dim == 0 || m == 0 || !(w > 0.0f) || !std::isfinite(w) || log2_buckets < 1 ||
        log2_buckets > 32) {
        set_error("bad arguments dim=%u m=%u w=%g log2_buckets=%u", dim, m, (double)w,
                  log2_buckets);
        return GENIE_EINVAL;
    }
    uint64_t gx = (n + kLshTile - 1) / kLshTile;
    uint32_t gy = (m + kLshTile - 1) / kLshTile;
    if (gx > 0x7FFFFFFFull || gy > 65535) {
        set_error("too many points in one call");
        return GENIE_EINVAL;
    }
    LshParams p{d_points, d_a, d_b, d_rehash, n, dim, m, 64u - log2_buckets, w, d_out_sig};
    dim3 grid((uint32_t)gx, gy);
    hipLaunchKernelGGL(lsh_kernel, grid, dim3(256), 0, (hipStream_t)stream, p);
    GENIE_HIP(hipGetLastError());
    return GENIE_OK;
}

extern "C" int genie_rbh_signatures(const float *d_points, uint64_t n, uint32_t dim,
                                    const float *d_g, const float *d_u, const uint32_t *d_seeds,
                                    uint32_t m, uint32_t log2_buckets, uint32_t *d_out_sig,
                                    void *stream) {
    clear_error();
    if (n == 0)
        return GENIE_OK;
    if (!d_points || !d_g || !d_u || !d_seeds || !d_out_sig) {
        set_error("null pointer");
        return GENIE_EINVAL;
    }
    if (dim == 0 || m == 0 || log2_buckets < 1 || log2_buckets > 32) {
        set_error("bad arguments dim=%u m=%u log2_buckets=%u", dim, m, log2_buckets);
        return GENIE_EINVAL;
    }
    uint64_t gx = (n + kLshTile - 1) / kLshTile;
    uint32_t gy = (m + kLshTile - 1) / kLshTile;
    if (gx > 0x7FFFFFFFull || gy > 65535) {
        set_error("too many points in one call");
        return GENIE_EINVAL;
    }
    RbhParams p{d_points, d_g, d_u, d_seeds, n, dim, m, 32u - log2_buckets, d_out_sig};
    dim3 grid((uint32_t)gx, gy);
    hipLaunchKernelGGL(rbh_kernel, grid, dim3(256), 0, (hipStream_t)stream, p);
    GENIE_HIP(hipGetLastError());
    return GENIE_OK;
}
