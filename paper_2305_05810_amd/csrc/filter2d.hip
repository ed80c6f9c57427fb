// filter2d.hip -- bilinear / bicubic B-spline filtering of dense 2D textures,
// deterministic (all 4 / 16 taps, Eq. filtered-texture with tensor-product
// weights) and stochastic (one tap per query, Eq. stochastic-sum with the
// per-axis draw of Eq. stochastic-bilerp / the bicubic sampling of section
// "B-Spline and Anisotropic Filters").
//
// The interpolating cubics (Keys, Mitchell) filter deterministically with
// their 16 weights and stochastically by positivization: one tap from the
// positive and one from the negative weights (interp.h).
//
// Raster position: x = uv.x * W - 0.5 (texel centres at half-integers of
// uv * W); taps are clamped to the texture.
#include <math.h>

#include "device_common.h"
#include "interp.h"
#include "stf_internal.h"

using namespace stf;

namespace {

constexpr int BLOCK = 256;

__device__ __forceinline__ int clampi(int v, int hi)
{
    return v < 0 ? 0 : (v > hi ? hi : v);
}

// All C channels of texel (x, y) (already clamped).
template <int FMT, int C>
__device__ __forceinline__ void load_rgba(const TexLevel& L, int x, int y, float (&v)[C])
{
    int64_t e = ((int64_t)y * L.w + x) * C;
    if constexpr (FMT == F32 && C == 4) {
        float4 f = reinterpret_cast<const float4*>(L.texels)[e >> 2];
        v[0] = f.x; v[1] = f.y; v[2] = f.z; v[3] = f.w;
    } else if constexpr (FMT == F32 && C == 2) {
        float2 f = reinterpret_cast<const float2*>(L.texels)[e >> 1];
        v[0] = f.x; v[1] = f.y;
    } else {
#pragma unroll
        for (int c = 0; c < C; ++c) v[c] = load_texel<FMT>(L.texels, e + c);
    }
}

// Query i of a batch of n, drawn with id qid0 + i.
template <int FMT, int C, bool CUBIC>
__device__ __forceinline__ void tex2d_stochastic_one(const TexLevel& L, const float* __restrict__ q, int32_t n,
                                                     int32_t i, uint32_t key, uint32_t qid0, float* __restrict__ out,
                                                     int32_t* __restrict__ idx, const int32_t* __restrict__ order,
                                                     int scatter)
{
    if (i >= n) return;
    const int32_t id = order ? order[i] : (int32_t)(qid0 + (uint32_t)i);
    const int64_t oi = (order && scatter) ? (int64_t)id : (int64_t)i;
    float2 uv = reinterpret_cast<const float2*>(q)[i];
    float x = uv.x * (float)L.w - 0.5f;
    float y = uv.y * (float)L.h - 0.5f;
    int cx, cy;
    float tx, ty;
    bool ok = cell_of(x, cx, tx) & cell_of(y, cy, ty);
    float v[C];
    int sx = BAD_INDEX, sy = BAD_INDEX;
    if (ok) {
        uint32_t b = pcg(key ^ (uint32_t)id);
        float ux = axis_uniform(b, 0), uy = axis_uniform(b, 1);
        if constexpr (CUBIC) {
            sx = cx + choose_cubic(tx, ux);
            sy = cy + choose_cubic(ty, uy);
        } else {
            sx = cx + choose_linear(tx, ux);
            sy = cy + choose_linear(ty, uy);
        }
        sx = clampi(sx, L.w - 1);
        sy = clampi(sy, L.h - 1);
        load_rgba<FMT, C>(L, sx, sy, v);
    } else {
#pragma unroll
        for (int c = 0; c < C; ++c) v[c] = __builtin_nanf("");
    }
#pragma unroll
    for (int c = 0; c < C; ++c) out[oi * C + c] = v[c];
    if (idx) {
        idx[2 * oi] = sx;
        idx[2 * oi + 1] = sy;
    }
}

template <int FMT, int C, bool CUBIC>
__global__ __launch_bounds__(BLOCK) void k_tex2d_stochastic(TexLevel L, const float* __restrict__ q, int32_t n,
                                                            uint32_t key, float* __restrict__ out,
                                                            int32_t* __restrict__ idx, const int32_t* __restrict__ order,
                                                            int scatter)
{
    tex2d_stochastic_one<FMT, C, CUBIC>(L, q, n, blockIdx.x * BLOCK + threadIdx.x, key, 0u, out, idx, order, scatter);
}

// Positivized estimate of an interpolating cubic for query i: two clamped
// taps, value (S+ t(j+) - S- t(j-)) / scale^2; index (x+, y+, x-, y-), the
// negative tap INT32_MIN when S- = 0.
template <int FMT, int C, int KIND>
__global__ __launch_bounds__(BLOCK) void k_tex2d_positivized(TexLevel L, const float* __restrict__ q, int32_t n,
                                                             uint32_t key, float* __restrict__ out,
                                                             int32_t* __restrict__ idx,
                                                             const int32_t* __restrict__ order, int scatter)
{
    const int32_t i = blockIdx.x * BLOCK + threadIdx.x;
    if (i >= n) return;
    const int32_t id = order ? order[i] : i;
    const int64_t oi = (order && scatter) ? (int64_t)id : (int64_t)i;
    float2 uv = reinterpret_cast<const float2*>(q)[i];
    float x = uv.x * (float)L.w - 0.5f;
    float y = uv.y * (float)L.h - 0.5f;
    int cx, cy;
    float tx, ty;
    bool ok = cell_of(x, cx, tx) & cell_of(y, cy, ty);
    float v[C];
    int ix[4] = {BAD_INDEX, BAD_INDEX, BAD_INDEX, BAD_INDEX};
    if (ok) {
        const float t[2] = {tx, ty};
        const PosDraw<2> d = positivized_draw<2, KIND>(t, pcg(key ^ (uint32_t)id));
        ix[0] = clampi(cx + d.op[0], L.w - 1);
        ix[1] = clampi(cy + d.op[1], L.h - 1);
        float vp[C], vn[C];
        load_rgba<FMT, C>(L, ix[0], ix[1], vp);
        if (d.neg) {
            ix[2] = clampi(cx + d.on[0], L.w - 1);
            ix[3] = clampi(cy + d.on[1], L.h - 1);
            load_rgba<FMT, C>(L, ix[2], ix[3], vn);
        }
        constexpr float inv = inv_scale<2, KIND>();
#pragma unroll
        for (int c = 0; c < C; ++c) v[c] = (d.neg ? d.sp * vp[c] - d.sn * vn[c] : d.sp * vp[c]) * inv;
    } else {
#pragma unroll
        for (int c = 0; c < C; ++c) v[c] = __builtin_nanf("");
    }
#pragma unroll
    for (int c = 0; c < C; ++c) out[oi * C + c] = v[c];
    if (idx) {
#pragma unroll
        for (int k = 0; k < 4; ++k) idx[4 * oi + k] = ix[k];
    }
}

// Serving: block b serves chunk c with start[c] <= b < start[c + 1].
template <int FMT, int C, bool CUBIC>
__global__ __launch_bounds__(BLOCK) void k_tex2d_serve(TexLevel L, const ServeChunk* __restrict__ chunks,
                                                       int32_t nchunks)
{
    int lo = 0, hi = nchunks - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) / 2;
        if (chunks[mid].block0 <= (int32_t)blockIdx.x) lo = mid;
        else hi = mid - 1;
    }
    const ServeChunk c = chunks[lo];
    tex2d_stochastic_one<FMT, C, CUBIC>(L, c.q, c.count, ((int32_t)blockIdx.x - c.block0) * BLOCK + threadIdx.x, c.key,
                                        c.qid0, c.out, c.idx, nullptr, 0);
}

template <int FMT, int C, int KIND>
__global__ __launch_bounds__(BLOCK) void k_tex2d_deterministic(TexLevel L, const float* __restrict__ q, int32_t n,
                                                               float* __restrict__ out, const int32_t* __restrict__ order,
                                                               int scatter)
{
    constexpr int NT = KIND == KIND_LINEAR ? 2 : 4;
    int32_t i = blockIdx.x * BLOCK + threadIdx.x;
    if (i >= n) return;
    const int64_t oi = (order && scatter) ? (int64_t)order[i] : (int64_t)i;
    float2 uv = reinterpret_cast<const float2*>(q)[i];
    float x = uv.x * (float)L.w - 0.5f;
    float y = uv.y * (float)L.h - 0.5f;
    int cx, cy;
    float tx, ty;
    bool ok = cell_of(x, cx, tx) & cell_of(y, cy, ty);
    float acc[C];
    if (!ok) {
#pragma unroll
        for (int c = 0; c < C; ++c) out[oi * C + c] = __builtin_nanf("");
        return;
    }
    float wx[4], wy[4];
    cx += axis_weights_scaled<KIND>(tx, wx);
    cy += axis_weights_scaled<KIND>(ty, wy);
#pragma unroll
    for (int c = 0; c < C; ++c) acc[c] = 0.0f;
#pragma unroll
    for (int b = 0; b < NT; ++b) {
        int yy = clampi(cy + b, L.h - 1);
        float row[C];
#pragma unroll
        for (int c = 0; c < C; ++c) row[c] = 0.0f;
#pragma unroll
        for (int a = 0; a < NT; ++a) {
            float v[C];
            load_rgba<FMT, C>(L, clampi(cx + a, L.w - 1), yy, v);
#pragma unroll
            for (int c = 0; c < C; ++c) row[c] = __builtin_fmaf(wx[a], v[c], row[c]);
        }
#pragma unroll
        for (int c = 0; c < C; ++c) acc[c] = __builtin_fmaf(wy[b], row[c], acc[c]);
    }
    constexpr float S2 = axis_scale<KIND>() * axis_scale<KIND>();   // 36 (B-spline), 4 (Keys), 324 (Mitchell)
#pragma unroll
    for (int c = 0; c < C; ++c) out[oi * C + c] = KIND == KIND_LINEAR ? acc[c] : acc[c] / S2;
}

// channel-0 moments of the stochastic estimator over many seeds
template <int FMT, int C, int KIND>
__global__ __launch_bounds__(BLOCK) void k_tex2d_moments(TexLevel L, const float* __restrict__ q, int32_t n,
                                                         uint64_t seed_base, int32_t n_seeds,
                                                         double* __restrict__ sum, double* __restrict__ sumsq)
{
    __shared__ double s1[BLOCK], s2[BLOCK];
    int32_t i = blockIdx.x;
    float2 uv = reinterpret_cast<const float2*>(q)[i];
    float x = uv.x * (float)L.w - 0.5f;
    float y = uv.y * (float)L.h - 0.5f;
    int cx, cy;
    float tx, ty;
    bool ok = cell_of(x, cx, tx) & cell_of(y, cy, ty);
    double a1 = 0.0, a2 = 0.0;
    if (ok) {
        for (int32_t k = threadIdx.x; k < n_seeds; k += BLOCK) {
            uint32_t b = pcg(seed_key(seed_base + (uint64_t)k) ^ (uint32_t)i);
            float e;
            if constexpr (KIND == KIND_KEYS || KIND == KIND_MITCHELL) {
                const float t[2] = {tx, ty};
                const PosDraw<2> d = positivized_draw<2, KIND>(t, b);
                float vp[C], vn[C];
                load_rgba<FMT, C>(L, clampi(cx + d.op[0], L.w - 1), clampi(cy + d.op[1], L.h - 1), vp);
                e = d.sp * vp[0];
                if (d.neg) {
                    load_rgba<FMT, C>(L, clampi(cx + d.on[0], L.w - 1), clampi(cy + d.on[1], L.h - 1), vn);
                    e = e - d.sn * vn[0];
                }
                e = e * inv_scale<2, KIND>();
            } else {
                float ux = axis_uniform(b, 0), uy = axis_uniform(b, 1);
                int sx, sy;
                if constexpr (KIND == KIND_BSPLINE) {
                    sx = cx + choose_cubic(tx, ux); sy = cy + choose_cubic(ty, uy);
                } else {
                    sx = cx + choose_linear(tx, ux); sy = cy + choose_linear(ty, uy);
                }
                float v[C];
                load_rgba<FMT, C>(L, clampi(sx, L.w - 1), clampi(sy, L.h - 1), v);
                e = v[0];
            }
            double d = (double)e;
            a1 += d;
            a2 += d * d;
        }
    } else {
        a1 = a2 = __builtin_nan("");
    }
    s1[threadIdx.x] = a1;
    s2[threadIdx.x] = a2;
    __syncthreads();
    for (int stride = BLOCK / 2; stride > 0; stride >>= 1) {
        if (threadIdx.x < stride) {
            s1[threadIdx.x] += s1[threadIdx.x + stride];
            s2[threadIdx.x] += s2[threadIdx.x + stride];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        sum[i] = s1[0];
        sumsq[i] = s2[0];
    }
}

template <int FMT, int C, int KIND>
void launch2d_kind(const TexLevel& L, const float* q, int32_t n, int mode, uint32_t key, float* out, int32_t* idx,
                   const int32_t* order, int scatter, hipStream_t stream)
{
    dim3 grid((n + BLOCK - 1) / BLOCK), block(BLOCK);
    if (mode == STF_STOCHASTIC) {
        if constexpr (KIND == KIND_KEYS || KIND == KIND_MITCHELL)
            hipLaunchKernelGGL((k_tex2d_positivized<FMT, C, KIND>), grid, block, 0, stream, L, q, n, key, out, idx,
                               order, scatter);
        else
            hipLaunchKernelGGL((k_tex2d_stochastic<FMT, C, KIND == KIND_BSPLINE>), grid, block, 0, stream, L, q, n, key,
                               out, idx, order, scatter);
    } else {
        hipLaunchKernelGGL((k_tex2d_deterministic<FMT, C, KIND>), grid, block, 0, stream, L, q, n, out, order, scatter);
    }
}

template <int FMT, int C>
hipError_t launch2d_fc(const TexLevel& L, const float* q, int32_t n, int filter, int mode, uint32_t key, float* out,
                       int32_t* idx, const int32_t* order, int scatter, hipStream_t stream)
{
    switch (filter) {
    case KIND_LINEAR: launch2d_kind<FMT, C, KIND_LINEAR>(L, q, n, mode, key, out, idx, order, scatter, stream); break;
    case KIND_BSPLINE: launch2d_kind<FMT, C, KIND_BSPLINE>(L, q, n, mode, key, out, idx, order, scatter, stream); break;
    case KIND_KEYS: launch2d_kind<FMT, C, KIND_KEYS>(L, q, n, mode, key, out, idx, order, scatter, stream); break;
    case KIND_MITCHELL: launch2d_kind<FMT, C, KIND_MITCHELL>(L, q, n, mode, key, out, idx, order, scatter, stream); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int FMT, int C>
hipError_t serve2d_fc(const TexLevel& L, int filter, const ServeChunk* chunks, int32_t nchunks, int32_t nblocks,
                      hipStream_t s)
{
    if (filter == STF_CUBIC_BSPLINE)
        hipLaunchKernelGGL((k_tex2d_serve<FMT, C, true>), dim3(nblocks), dim3(BLOCK), 0, s, L, chunks, nchunks);
    else
        hipLaunchKernelGGL((k_tex2d_serve<FMT, C, false>), dim3(nblocks), dim3(BLOCK), 0, s, L, chunks, nchunks);
    return hipGetLastError();
}

template <int FMT>
hipError_t serve2d_f(const stf_texture* t, int filter, const ServeChunk* chunks, int32_t nchunks, int32_t nblocks,
                     hipStream_t s)
{
    const TexLevel& L = t->level[0];
    switch (t->channels) {
    case 1: return serve2d_fc<FMT, 1>(L, filter, chunks, nchunks, nblocks, s);
    case 2: return serve2d_fc<FMT, 2>(L, filter, chunks, nchunks, nblocks, s);
    case 3: return serve2d_fc<FMT, 3>(L, filter, chunks, nchunks, nblocks, s);
    case 4: return serve2d_fc<FMT, 4>(L, filter, chunks, nchunks, nblocks, s);
    }
    return hipErrorInvalidValue;
}

template <int FMT, int C>
hipError_t moments2d_fc(const TexLevel& L, const float* q, int32_t n, int filter, uint64_t seed_base,
                        int32_t n_seeds, double* sum, double* sumsq, hipStream_t stream)
{
    dim3 grid(n), block(BLOCK);
    switch (filter) {
    case KIND_LINEAR:
        hipLaunchKernelGGL((k_tex2d_moments<FMT, C, KIND_LINEAR>), grid, block, 0, stream, L, q, n, seed_base, n_seeds,
                           sum, sumsq);
        break;
    case KIND_BSPLINE:
        hipLaunchKernelGGL((k_tex2d_moments<FMT, C, KIND_BSPLINE>), grid, block, 0, stream, L, q, n, seed_base, n_seeds,
                           sum, sumsq);
        break;
    case KIND_KEYS:
        hipLaunchKernelGGL((k_tex2d_moments<FMT, C, KIND_KEYS>), grid, block, 0, stream, L, q, n, seed_base, n_seeds,
                           sum, sumsq);
        break;
    case KIND_MITCHELL:
        hipLaunchKernelGGL((k_tex2d_moments<FMT, C, KIND_MITCHELL>), grid, block, 0, stream, L, q, n, seed_base,
                           n_seeds, sum, sumsq);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int FMT>
hipError_t launch2d_f(const stf_texture* t, const float* q, int32_t n, int filter, int mode, uint32_t key,
                      float* out, int32_t* idx, const int32_t* order, int scatter, hipStream_t s)
{
    const TexLevel& L = t->level[0];
    switch (t->channels) {
    case 1: return launch2d_fc<FMT, 1>(L, q, n, filter, mode, key, out, idx, order, scatter, s);
    case 2: return launch2d_fc<FMT, 2>(L, q, n, filter, mode, key, out, idx, order, scatter, s);
    case 3: return launch2d_fc<FMT, 3>(L, q, n, filter, mode, key, out, idx, order, scatter, s);
    case 4: return launch2d_fc<FMT, 4>(L, q, n, filter, mode, key, out, idx, order, scatter, s);
    }
    return hipErrorInvalidValue;
}

template <int FMT>
hipError_t moments2d_f(const stf_texture* t, const float* q, int32_t n, int filter, uint64_t seed_base,
                       int32_t n_seeds, double* sum, double* sumsq, hipStream_t s)
{
    const TexLevel& L = t->level[0];
    switch (t->channels) {
    case 1: return moments2d_fc<FMT, 1>(L, q, n, filter, seed_base, n_seeds, sum, sumsq, s);
    case 2: return moments2d_fc<FMT, 2>(L, q, n, filter, seed_base, n_seeds, sum, sumsq, s);
    case 3: return moments2d_fc<FMT, 3>(L, q, n, filter, seed_base, n_seeds, sum, sumsq, s);
    case 4: return moments2d_fc<FMT, 4>(L, q, n, filter, seed_base, n_seeds, sum, sumsq, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_filter2d(const stf_texture* t, const float* q, int32_t n, int filter, int mode, uint32_t key,
                           float* out, int32_t* idx, const int32_t* order, int scatter, hipStream_t s)
{
    switch (t->fmt) {
    case F32: return launch2d_f<F32>(t, q, n, filter, mode, key, out, idx, order, scatter, s);
    case F16: return launch2d_f<F16>(t, q, n, filter, mode, key, out, idx, order, scatter, s);
    case BF16: return launch2d_f<BF16>(t, q, n, filter, mode, key, out, idx, order, scatter, s);
    case FP8_E4M3: return launch2d_f<FP8_E4M3>(t, q, n, filter, mode, key, out, idx, order, scatter, s);
    case U8: return launch2d_f<U8>(t, q, n, filter, mode, key, out, idx, order, scatter, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_moments2d(const stf_texture* t, const float* q, int32_t n, int filter, uint64_t seed_base,
                            int32_t n_seeds, double* sum, double* sumsq, hipStream_t s)
{
    switch (t->fmt) {
    case F32: return moments2d_f<F32>(t, q, n, filter, seed_base, n_seeds, sum, sumsq, s);
    case F16: return moments2d_f<F16>(t, q, n, filter, seed_base, n_seeds, sum, sumsq, s);
    case BF16: return moments2d_f<BF16>(t, q, n, filter, seed_base, n_seeds, sum, sumsq, s);
    case FP8_E4M3: return moments2d_f<FP8_E4M3>(t, q, n, filter, seed_base, n_seeds, sum, sumsq, s);
    case U8: return moments2d_f<U8>(t, q, n, filter, seed_base, n_seeds, sum, sumsq, s);
    }
    return hipErrorInvalidValue;
}

int32_t serve2d_queries_per_block()
{
    return BLOCK;
}

hipError_t launch_serve2d(const stf_texture* t, int filter, const ServeChunk* chunks, int32_t nchunks, int32_t nblocks,
                          hipStream_t s)
{
    switch (t->fmt) {
    case F32: return serve2d_f<F32>(t, filter, chunks, nchunks, nblocks, s);
    case F16: return serve2d_f<F16>(t, filter, chunks, nchunks, nblocks, s);
    case BF16: return serve2d_f<BF16>(t, filter, chunks, nchunks, nblocks, s);
    case FP8_E4M3: return serve2d_f<FP8_E4M3>(t, filter, chunks, nchunks, nblocks, s);
    case U8: return serve2d_f<U8>(t, filter, chunks, nchunks, nblocks, s);
    }
    return hipErrorInvalidValue;
}
