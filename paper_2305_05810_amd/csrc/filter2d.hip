// filter2d.hip -- filtering of 2D textures: bilinear / bicubic B-spline,
// deterministic (all 4 / 16 taps, Eq. filtered-texture with tensor-product
// weights) and stochastic (one tap per query, Eq. stochastic-sum with the
// per-axis draw of Eq. stochastic-bilerp / the bicubic sampling of section
// "B-Spline and Anisotropic Filters").  The interpolating cubics (Keys,
// Mitchell) filter deterministically with their 16 weights and
// stochastically by positivization: one tap from the positive and one from
// the negative weights (interp.h).
//
// Every kernel is generic over its texel source: stored texels of a format
// (DenseSrc), or DCT-compressed blocks decoded one texel at a time
// (DctSrc; the stochastic filters decode one texel per lookup instead of
// 4 or 16, the case the paper makes for compressed formats).
//
// Raster position: x = uv.x * W - 0.5 (texel centres at half-integers of
// uv * W); taps are clamped to the texture.
#include <limits.h>
#include <math.h>

#include "dct_decode.h"
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

// Stored texels: C channels of format FMT.
template <int FMT, int C>
struct DenseSrc {
    static constexpr int CAP = C;
    static constexpr bool DECODES = false;   // a texel is a plain load
    TexLevel L;
    __device__ int w() const { return L.w; }
    __device__ int h() const { return L.h; }
    __device__ int channels() const { return C; }
    __device__ void load(int x, int y, float (&v)[CAP]) const { load_rgba<FMT, C>(L, x, y, v); }
};

// Material texels (8 bytes: albedo RGB UNORM8, roughness UNORM8, tangent
// normal x and y binary16; stored in 4x4-texel tiles, material_index) of
// level 0, decoded exactly to six channels.
struct MaterialSrc {
    static constexpr int CAP = 6;
    static constexpr bool DECODES = false;
    TexLevel L;
    __device__ int w() const { return L.w; }
    __device__ int h() const { return L.h; }
    __device__ int channels() const { return 6; }
    __device__ void load(int x, int y, float (&v)[CAP]) const
    {
        const uint2 t = reinterpret_cast<const uint2*>(L.texels)[material_index(x, y, L.w)];
        v[0] = dec_u8(t.x & 0xffu);
        v[1] = dec_u8((t.x >> 8) & 0xffu);
        v[2] = dec_u8((t.x >> 16) & 0xffu);
        v[3] = dec_u8(t.x >> 24);
        v[4] = dec_f16((uint16_t)(t.y & 0xffffu));
        v[5] = dec_f16((uint16_t)(t.y >> 16));
    }
};

// DCT blocks: CAP words per block (a multiple of 4), C <= CAP channels used.
template <int CAP_>
struct DctSrc {
    static constexpr int CAP = CAP_;
    static constexpr bool DECODES = true;   // a texel costs an inverse DCT per channel
    const uint32_t* blocks;
    int32_t W, H, BW, C;
    __device__ int w() const { return W; }
    __device__ int h() const { return H; }
    __device__ int channels() const { return C; }
    __device__ void load(int x, int y, float (&v)[CAP]) const
    {
        const uint4* b = reinterpret_cast<const uint4*>(blocks + ((int64_t)(y >> 3) * BW + (x >> 3)) * CAP);
        const DctBasis B = dct_basis(x & 7, y & 7);
#pragma unroll
        for (int g = 0; g < CAP / 4; ++g) {
            const uint4 q = b[g];
            v[4 * g] = dct_decode_word(q.x, B);
            v[4 * g + 1] = dct_decode_word(q.y, B);
            v[4 * g + 2] = dct_decode_word(q.z, B);
            v[4 * g + 3] = dct_decode_word(q.w, B);
        }
    }
};

template <class Src>
__device__ __forceinline__ void store_channels(const Src& S, float* __restrict__ out, int64_t oi, const float* v)
{
    const int C = S.channels();
#pragma unroll
    for (int c = 0; c < Src::CAP; ++c)
        if (c < C) out[oi * C + c] = v[c];
}

// Stores the C results of every live query of the block.  In batch order the
// block's results are one contiguous span of cnt * C floats: each thread
// stages its values in LDS and the block writes the span with consecutive
// 16-byte stores (4-byte ones if the span is not 16-byte aligned), instead of
// C strided 4-byte stores per lane.  Scattered results (an ordered stream
// with STF_ORDER_SCATTER) are stored directly.  Every thread of the block
// must call this (it synchronises the block).
template <class Src>
__device__ __forceinline__ void block_store_via(const Src& S, float* __restrict__ out, int32_t n, bool live, int64_t oi,
                                                const float (&v)[Src::CAP], bool scattered, float* stage)
{
    const int C = S.channels();
    if (scattered) {
        if (live) store_channels(S, out, oi, v);
        return;
    }
#pragma unroll
    for (int c = 0; c < Src::CAP; ++c)
        if (c < C) stage[threadIdx.x * C + c] = v[c];
    __syncthreads();
    const int64_t first = (int64_t)blockIdx.x * BLOCK;
    const int cnt = (int)((int64_t)n - first < BLOCK ? (int64_t)n - first : BLOCK);
    const int total = cnt * C;
    float* dst = out + first * C;
    int k0 = 0;
    // the results are streamed out: nontemporal stores (1.37x on the DCT
    // set's stochastic bilinear, whose 36 bytes of results per lookup are
    // most of its traffic)
    typedef float f32x4_nt __attribute__((ext_vector_type(4)));
    if ((reinterpret_cast<uintptr_t>(dst) & 15u) == 0) {
        const int n4 = total >> 2;
        for (int k = threadIdx.x; k < n4; k += BLOCK)
            __builtin_nontemporal_store(reinterpret_cast<const f32x4_nt*>(stage)[k],
                                        reinterpret_cast<f32x4_nt*>(dst) + k);
        k0 = n4 << 2;
    }
    for (int k = k0 + threadIdx.x; k < total; k += BLOCK) __builtin_nontemporal_store(stage[k], dst + k);
}

// block_store_via with LDS of its own (BLOCK * CAP floats, 16-byte aligned).
template <class Src>
__device__ __forceinline__ void block_store(const Src& S, float* __restrict__ out, int32_t n, bool live, int64_t oi,
                                            const float (&v)[Src::CAP], bool scattered)
{
    __shared__ __align__(16) float stage[BLOCK * Src::CAP];
    block_store_via(S, out, n, live, oi, v, scattered, stage);
}

// Query i of a batch (i valid), drawn with id qid0 + i (or order[i]): its
// values, its tap (INT32_MIN for a non-finite query) and where its results go.
template <class Src, bool CUBIC, bool FIS = false>
__device__ __forceinline__ void tex2d_stochastic_eval(const Src& S, const float* __restrict__ q, int32_t i, uint32_t key,
                                                      uint32_t qid0, const int32_t* __restrict__ order, int scatter,
                                                      float (&v)[Src::CAP], int& sx, int& sy, int64_t& oi)
{
    const int32_t id = order ? order[i] : (int32_t)(qid0 + (uint32_t)i);
    oi = (order && scatter) ? (int64_t)id : (int64_t)i;
    float2 uv = reinterpret_cast<const float2*>(q)[i];
    float x = uv.x * (float)S.w() - 0.5f;
    float y = uv.y * (float)S.h() - 0.5f;
    int cx, cy;
    float tx, ty;
    bool ok = cell_of(x, cx, tx) & cell_of(y, cy, ty);
    sx = BAD_INDEX;
    sy = BAD_INDEX;
    if (ok) {
        uint32_t b = pcg(key ^ (uint32_t)id);
        if constexpr (FIS) {
            sx = fis_tap<CUBIC>(x, b, 0);
            sy = fis_tap<CUBIC>(y, b, 1);
        } else {
            float ux = axis_uniform(b, 0), uy = axis_uniform(b, 1);
            if constexpr (CUBIC) {
                sx = cx + choose_cubic(tx, ux);
                sy = cy + choose_cubic(ty, uy);
            } else {
                sx = cx + choose_linear(tx, ux);
                sy = cy + choose_linear(ty, uy);
            }
        }
        sx = clampi(sx, S.w() - 1);
        sy = clampi(sy, S.h() - 1);
        S.load(sx, sy, v);
    } else {
#pragma unroll
        for (int c = 0; c < Src::CAP; ++c) v[c] = __builtin_nanf("");
    }
}

template <class Src, bool CUBIC, bool FIS>
__global__ __launch_bounds__(BLOCK) void k_tex2d_stochastic(Src S, const float* __restrict__ q, int32_t n,
                                                            uint32_t key, float* __restrict__ out,
                                                            int32_t* __restrict__ idx, const int32_t* __restrict__ order,
                                                            int scatter)
{
    const int32_t i = blockIdx.x * BLOCK + threadIdx.x;
    const bool live = i < n;
    float v[Src::CAP];
    int sx, sy;
    int64_t oi;
    tex2d_stochastic_eval<Src, CUBIC, FIS>(S, q, live ? i : 0, key, 0u, order, scatter, v, sx, sy, oi);
    block_store(S, out, n, live, oi, v, order && scatter);
    if (live && idx) {
        idx[2 * oi] = sx;
        idx[2 * oi + 1] = sy;
    }
}

// Positivized estimate of an interpolating cubic for query i: two clamped
// taps, value (S+ t(j+) - S- t(j-)) / scale^2; index (x+, y+, x-, y-), the
// negative tap INT32_MIN when S- = 0.
template <class Src, int KIND>
__global__ __launch_bounds__(BLOCK) void k_tex2d_positivized(Src S, const float* __restrict__ q, int32_t n,
                                                             uint32_t key, float* __restrict__ out,
                                                             int32_t* __restrict__ idx,
                                                             const int32_t* __restrict__ order, int scatter)
{
    constexpr int CAP = Src::CAP;
    const int32_t i0 = blockIdx.x * BLOCK + threadIdx.x;
    const bool live = i0 < n;
    const int32_t i = live ? i0 : 0;
    const int32_t id = order ? order[i] : i;
    const int64_t oi = (order && scatter) ? (int64_t)id : (int64_t)i;
    float2 uv = reinterpret_cast<const float2*>(q)[i];
    float x = uv.x * (float)S.w() - 0.5f;
    float y = uv.y * (float)S.h() - 0.5f;
    int cx, cy;
    float tx, ty;
    bool ok = cell_of(x, cx, tx) & cell_of(y, cy, ty);
    float v[CAP];
    int ix[4] = {BAD_INDEX, BAD_INDEX, BAD_INDEX, BAD_INDEX};
    if (ok) {
        const float t[2] = {tx, ty};
        const PosDraw<2> d = positivized_draw<2, KIND>(t, pcg(key ^ (uint32_t)id));
        ix[0] = clampi(cx + d.op[0], S.w() - 1);
        ix[1] = clampi(cy + d.op[1], S.h() - 1);
        float vp[CAP], vn[CAP];
        S.load(ix[0], ix[1], vp);
        if (d.neg) {
            ix[2] = clampi(cx + d.on[0], S.w() - 1);
            ix[3] = clampi(cy + d.on[1], S.h() - 1);
            S.load(ix[2], ix[3], vn);
        }
        constexpr float inv = inv_scale<2, KIND>();
#pragma unroll
        for (int c = 0; c < CAP; ++c) v[c] = (d.neg ? d.sp * vp[c] - d.sn * vn[c] : d.sp * vp[c]) * inv;
    } else {
#pragma unroll
        for (int c = 0; c < CAP; ++c) v[c] = __builtin_nanf("");
    }
    block_store(S, out, n, live, oi, v, order && scatter);
    if (live && idx) {
#pragma unroll
        for (int k = 0; k < 4; ++k) idx[4 * oi + k] = ix[k];
    }
}

// Serving: block b serves chunk c with start[c] <= b < start[c + 1].
template <class Src, bool CUBIC>
__global__ __launch_bounds__(BLOCK) void k_tex2d_serve(Src S, const ServeChunk* __restrict__ chunks, int32_t nchunks)
{
    int lo = 0, hi = nchunks - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) / 2;
        if (chunks[mid].block0 <= (int32_t)blockIdx.x) lo = mid;
        else hi = mid - 1;
    }
    const ServeChunk c = chunks[lo];
    const int32_t i = ((int32_t)blockIdx.x - c.block0) * BLOCK + threadIdx.x;
    if (i >= c.count) return;
    float v[Src::CAP];
    int sx, sy;
    int64_t oi;
    tex2d_stochastic_eval<Src, CUBIC>(S, c.q, i, c.key, c.qid0, nullptr, 0, v, sx, sy, oi);
    store_channels(S, c.out, oi, v);
    if (c.idx) {
        c.idx[2 * oi] = sx;
        c.idx[2 * oi + 1] = sy;
    }
}

template <class Src, int KIND>
__global__ __launch_bounds__(BLOCK) void k_tex2d_deterministic(Src S, const float* __restrict__ q, int32_t n,
                                                               float* __restrict__ out, const int32_t* __restrict__ order,
                                                               int scatter)
{
    constexpr int NT = KIND == KIND_LINEAR ? 2 : 4;
    constexpr int CAP = Src::CAP;
    const int32_t i0 = blockIdx.x * BLOCK + threadIdx.x;
    const bool live = i0 < n;
    const int32_t i = live ? i0 : 0;
    const int64_t oi = (order && scatter) ? (int64_t)order[i] : (int64_t)i;
    float2 uv = reinterpret_cast<const float2*>(q)[i];
    float x = uv.x * (float)S.w() - 0.5f;
    float y = uv.y * (float)S.h() - 0.5f;
    int cx = 0, cy = 0;
    float tx = 0.0f, ty = 0.0f;
    const bool ok = cell_of(x, cx, tx) & cell_of(y, cy, ty);
    float acc[CAP];
    float wx[4], wy[4];
    cx += axis_weights_scaled<KIND>(tx, wx);
    cy += axis_weights_scaled<KIND>(ty, wy);
#pragma unroll
    for (int c = 0; c < CAP; ++c) acc[c] = 0.0f;
    // Wide sources (DCT blocks of 8+ channels) keep one row of taps in
    // flight: unrolling all rows would hold every tap's words at once.
    constexpr int ROWS_UNROLLED = CAP > 4 ? 1 : NT;
#pragma unroll ROWS_UNROLLED
    for (int b = 0; b < NT; ++b) {
        int yy = clampi(cy + b, S.h() - 1);
        float row[CAP];
#pragma unroll
        for (int c = 0; c < CAP; ++c) row[c] = 0.0f;
#pragma unroll
        for (int a = 0; a < NT; ++a) {
            float v[CAP];
            S.load(clampi(cx + a, S.w() - 1), yy, v);
#pragma unroll
            for (int c = 0; c < CAP; ++c) row[c] = __builtin_fmaf(wx[a], v[c], row[c]);
        }
#pragma unroll
        for (int c = 0; c < CAP; ++c) acc[c] = __builtin_fmaf(wy[b], row[c], acc[c]);
    }
    constexpr float S2 = axis_scale<KIND>() * axis_scale<KIND>();   // 36 (B-spline), 4 (Keys), 324 (Mitchell)
#pragma unroll
    for (int c = 0; c < CAP; ++c) acc[c] = !ok ? __builtin_nanf("") : (KIND == KIND_LINEAR ? acc[c] : acc[c] / S2);
    block_store(S, out, n, live, oi, acc, order && scatter);
}

// Deterministic bicubic filtering of a Morton-sorted stream (neighbouring
// queries close in the texture) of a source whose texels cost a decode.  The block decodes every texel of the bounding
// box of its queries' clamped taps once into LDS and filters each query from
// there; a block whose box exceeds STAGE_FLOATS values, or whose queries
// would read fewer than STAGE_REUSE taps per decoded texel, decodes per tap
// like k_tex2d_deterministic.  Both paths see the same decoded values and sum
// them in the same order, so the results are the same.
constexpr int STAGE_FLOATS = 8192;   // 32 KiB per block
constexpr int STAGE_REUSE = 4;

__device__ __forceinline__ int block_reduce_min(int v, int* red)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = min(v, __shfl_xor(v, off, 64));
    if (threadIdx.x % 64 == 0) red[threadIdx.x / 64] = v;
    __syncthreads();
    int r = red[0];
#pragma unroll
    for (int k = 1; k < BLOCK / 64; ++k) r = min(r, red[k]);
    __syncthreads();
    return r;
}

// Discrete Gaussian weights of the 4x4 window i-1..i+2 (binary64, unnormalised).
__device__ __forceinline__ void gauss_discrete_weights(double t, double inv2s2, double (&w)[4])
{
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const double d = (double)(k - 1) - t;
        w[k] = exp(-(d * d) * inv2s2);
    }
}

// The discrete Gaussian mean (normalised 4x4 window) as a staged kind.
constexpr int KIND_GAUSS_MEAN = 100;

template <class Src, int KIND>
__global__ __launch_bounds__(BLOCK) void k_tex2d_det_staged(Src S, const float* __restrict__ q, int32_t n,
                                                            float* __restrict__ out, const int32_t* __restrict__ order,
                                                            int scatter, unsigned long long* __restrict__ counters,
                                                            float sigma)
{
    constexpr int NT = KIND == KIND_LINEAR ? 2 : 4;
    constexpr int CAP = Src::CAP;
    static_assert(BLOCK * CAP <= STAGE_FLOATS, "the tile also stages the block's results");
    __shared__ __align__(16) float tile[STAGE_FLOATS];
    __shared__ int red[BLOCK / 64];
    const int32_t i0 = blockIdx.x * BLOCK + threadIdx.x;
    const bool live = i0 < n;
    const int32_t i = live ? i0 : 0;
    const int64_t oi = (order && scatter) ? (int64_t)order[i] : (int64_t)i;
    float2 uv = reinterpret_cast<const float2*>(q)[i];
    float x = uv.x * (float)S.w() - 0.5f;
    float y = uv.y * (float)S.h() - 0.5f;
    int cx = 0, cy = 0;
    float tx = 0.0f, ty = 0.0f;
    const bool ok = cell_of(x, cx, tx) & cell_of(y, cy, ty);
    float wx[4], wy[4];
    if constexpr (KIND == KIND_GAUSS_MEAN) {
        // as k_tex2d_gauss's discrete mean: binary64 weights, normalised, in binary32
        const double sg = (double)sigma, inv2s2 = 1.0 / (2.0 * sg * sg);
        const double xe = (double)x, ye = (double)y;
        double dx[4], dy[4];
        gauss_discrete_weights(xe - floor(xe), inv2s2, dx);
        gauss_discrete_weights(ye - floor(ye), inv2s2, dy);
        const double nx = ((dx[0] + dx[1]) + dx[2]) + dx[3], ny = ((dy[0] + dy[1]) + dy[2]) + dy[3];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            wx[k] = (float)(dx[k] / nx);
            wy[k] = (float)(dy[k] / ny);
        }
        cx -= 1;
        cy -= 1;
    } else {
        cx += axis_weights_scaled<KIND>(tx, wx);
        cy += axis_weights_scaled<KIND>(ty, wy);
    }
    // box of the clamped taps of the block's queries (clamping is monotone)
    const bool in = live && ok;
    const int W1 = S.w() - 1, H1 = S.h() - 1;
    const int x0 = block_reduce_min(in ? clampi(cx, W1) : INT_MAX, red);
    const int x1 = -block_reduce_min(in ? -clampi(cx + NT - 1, W1) : INT_MAX, red);
    const int y0 = block_reduce_min(in ? clampi(cy, H1) : INT_MAX, red);
    const int y1 = -block_reduce_min(in ? -clampi(cy + NT - 1, H1) : INT_MAX, red);
    const int nin = __syncthreads_count(in);
    const int C = S.channels();
    const int ew = nin ? x1 - x0 + 1 : 0, eh = nin ? y1 - y0 + 1 : 0;   // both within the texture
    const int64_t ntex = (int64_t)ew * eh;
    float acc[CAP];
#pragma unroll
    for (int c = 0; c < CAP; ++c) acc[c] = 0.0f;
    const bool stage = nin && ntex * C <= STAGE_FLOATS && ntex * STAGE_REUSE <= (int64_t)nin * NT * NT;
    if (counters && threadIdx.x == 0) {   // {blocks that staged, blocks}, when counting is on
        if (stage) atomicAdd(&counters[0], 1ull);
        atomicAdd(&counters[1], 1ull);
    }
    if (stage) {
        for (int t = threadIdx.x; t < (int)ntex; t += BLOCK) {
            float v[CAP];
            S.load(x0 + t % ew, y0 + t / ew, v);
#pragma unroll
            for (int c = 0; c < CAP; ++c)
                if (c < C) tile[t * C + c] = v[c];
        }
        __syncthreads();
        // tap offsets in the box (a query without a cell reads texel 0)
        int ix[NT];
#pragma unroll
        for (int a = 0; a < NT; ++a) ix[a] = in ? (clampi(cx + a, W1) - x0) * C : 0;
        // wide sources keep one row of taps in registers at a time
        constexpr int ROWS = CAP > 4 ? 1 : NT;
#pragma unroll ROWS
        for (int b = 0; b < NT; ++b) {
            const int iy = in ? (clampi(cy + b, H1) - y0) * ew * C : 0;
            float row[CAP];
#pragma unroll
            for (int c = 0; c < CAP; ++c) row[c] = 0.0f;
#pragma unroll
            for (int a = 0; a < NT; ++a) {
                const float* e = tile + iy + ix[a];
#pragma unroll
                for (int c = 0; c < CAP; ++c) row[c] = __builtin_fmaf(wx[a], c < C ? e[c] : 0.0f, row[c]);
            }
#pragma unroll
            for (int c = 0; c < CAP; ++c) acc[c] = __builtin_fmaf(wy[b], row[c], acc[c]);
        }
    } else {
        constexpr int ROWS_UNROLLED = CAP > 4 ? 1 : NT;
#pragma unroll ROWS_UNROLLED
        for (int b = 0; b < NT; ++b) {
            int yy = clampi(cy + b, H1);
            float row[CAP];
#pragma unroll
            for (int c = 0; c < CAP; ++c) row[c] = 0.0f;
#pragma unroll
            for (int a = 0; a < NT; ++a) {
                float v[CAP];
                S.load(clampi(cx + a, W1), yy, v);
#pragma unroll
                for (int c = 0; c < CAP; ++c) row[c] = __builtin_fmaf(wx[a], v[c], row[c]);
            }
#pragma unroll
            for (int c = 0; c < CAP; ++c) acc[c] = __builtin_fmaf(wy[b], row[c], acc[c]);
        }
    }
    constexpr float S2 = axis_scale<KIND>() * axis_scale<KIND>();
#pragma unroll
    for (int c = 0; c < CAP; ++c) acc[c] = !ok ? __builtin_nanf("") : (KIND == KIND_LINEAR ? acc[c] : acc[c] / S2);
    __syncthreads();   // every thread is done with the tile: it now stages the results
    block_store_via(S, out, n, live, oi, acc, order && scatter, tile);
}

// channel-0 moments of the stochastic estimator over many seeds
template <class Src, int KIND>
__global__ __launch_bounds__(BLOCK) void k_tex2d_moments(Src S, const float* __restrict__ q, int32_t n,
                                                         uint64_t seed_base, int32_t n_seeds,
                                                         double* __restrict__ sum, double* __restrict__ sumsq)
{
    constexpr int CAP = Src::CAP;
    __shared__ double s1[BLOCK], s2[BLOCK];
    int32_t i = blockIdx.x;
    float2 uv = reinterpret_cast<const float2*>(q)[i];
    float x = uv.x * (float)S.w() - 0.5f;
    float y = uv.y * (float)S.h() - 0.5f;
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
                float vp[CAP], vn[CAP];
                S.load(clampi(cx + d.op[0], S.w() - 1), clampi(cy + d.op[1], S.h() - 1), vp);
                e = d.sp * vp[0];
                if (d.neg) {
                    S.load(clampi(cx + d.on[0], S.w() - 1), clampi(cy + d.on[1], S.h() - 1), vn);
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
                float v[CAP];
                S.load(clampi(sx, S.w() - 1), clampi(sy, S.h() - 1), v);
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

// ---------------------------------------------------------------------------
// Gaussian filters (sections "Filter Importance Sampling" and "Results",
// magnification).  Decisions and weights in binary64; sigma in texels.
//   GAUSS_FIS: offset sigma (r cos 2 pi u1, r sin 2 pi u1), r = sqrt(-2 ln(1 -
//     u0)) (Box-Muller of hash indices 0, 1), nearest texel floor(x' + 1/2).
//   GAUSS_FIS_MEAN: the Gaussian convolved with the nearest-texel box (what
//     GAUSS_FIS estimates): per-axis weights Phi((k + 1/2 - x)/sigma) -
//     Phi((k - 1/2 - x)/sigma) over |k - floor(x)| <= R = ceil(6 sigma) + 1.
//   GAUSS_DISCRETE: window i-1..i+2, per-axis weights exp(-(d - t)^2 /
//     (2 sigma^2)), one tap per axis by the cumulative rule (hash index a).
//   GAUSS_DISCRETE_MEAN: the normalised sum over that window.
// ---------------------------------------------------------------------------
enum GaussMode { GAUSS_FIS = 0, GAUSS_FIS_MEAN = 1, GAUSS_DISCRETE = 2, GAUSS_DISCRETE_MEAN = 3 };
constexpr int GAUSS_MAX_TAPS = 52;   // 2 R + 2 for sigma <= 4 (GAUSS_FIS_MEAN)

__device__ __forceinline__ double gauss_phi(double z)
{
    return 0.5 * erfc(-z * 0.70710678118654752440);
}

__device__ __forceinline__ int gauss_pick(const double (&m)[4], double u)
{
    const double total = ((m[0] + m[1]) + m[2]) + m[3];
    const int last = m[3] > 0.0 ? 3 : (m[2] > 0.0 ? 2 : (m[1] > 0.0 ? 1 : 0));
    const double T = u * total;
    int j = (T >= m[0]) + (T >= m[0] + m[1]) + (T >= (m[0] + m[1]) + m[2]);
    return j > last ? last : j;
}

// The discrete pick with binary32 weights, for sigma >= 1/4 (every weight is
// then at least e^-32: none underflows and none is clamped).  A weight is
// 2^(a log2 e) with a = -d^2 / (2 sigma^2), |a| <= 32, by the hardware's 2^x.
// The exponent carries a few ulps from d^2, 1/(2 sigma^2) and the scaling by
// log2 e (at most 1.4e-5 + 4.2e-6 absolute), and 2^x is within 8.5e-8
// relative over [-64, 0] (measured on every binary32 value there against
// binary64), so each weight is within 2e-5 relative of its binary64 value,
// and u * total and the cumulative sums lie within 4e-5 total of theirs;
// where u * total is at least total 2^-12 from every cumulative sum, the pick
// is the binary64 pick.  Returns -1 otherwise.
__device__ __forceinline__ int gauss_pick_fast(float t, float inv2s2, float u)
{
    float m[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const float d = (float)(k - 1) - t;
        m[k] = __builtin_amdgcn_exp2f((-(d * d) * inv2s2) * 1.44269504088896341f);
    }
    const float c1 = m[0], c2 = m[0] + m[1], c3 = (m[0] + m[1]) + m[2];
    const float total = c3 + m[3];
    const float T = u * total;
    if (fminf(fminf(fabsf(T - c1), fabsf(T - c2)), fabsf(T - c3)) < total * 0x1p-12f) return -1;
    return (T >= c1) + (T >= c2) + (T >= c3);
}

template <class Src, int GMODE>
__global__ __launch_bounds__(BLOCK) void k_tex2d_gauss(Src S, const float* __restrict__ q, int32_t n, float sigma,
                                                       int32_t radius, uint32_t key, float* __restrict__ out,
                                                       int32_t* __restrict__ idx)
{
    constexpr int CAP = Src::CAP;
    const int32_t i0 = blockIdx.x * BLOCK + threadIdx.x;
    const bool live = i0 < n;
    const int32_t i = live ? i0 : 0;
    float2 uv = reinterpret_cast<const float2*>(q)[i];
    const float x = uv.x * (float)S.w() - 0.5f;
    const float y = uv.y * (float)S.h() - 0.5f;
    int cx = 0, cy = 0;
    float tx = 0.0f, ty = 0.0f;
    const bool ok = cell_of(x, cx, tx) & cell_of(y, cy, ty);
    const double xe = (double)x, ye = (double)y, sg = (double)sigma;
    float v[CAP];
    int sx = BAD_INDEX, sy = BAD_INDEX;
    if constexpr (GMODE == GAUSS_FIS || GMODE == GAUSS_DISCRETE) {
        if (ok) {
            const uint32_t b = pcg(key ^ (uint32_t)i);
            const float u0f = axis_uniform(b, 0), u1f = axis_uniform(b, 1);
            const double u0 = (double)u0f, u1 = (double)u1f;
            if constexpr (GMODE == GAUSS_FIS) {
                // The offset is first formed in binary32 with the hardware's
                // log2, square root, sine and cosine (the last two take the
                // angle in turns, so u1 needs no scaling by 2 pi).  1 - u0 is
                // exact, and over all 2^24 values a uniform can take, r is
                // within 4.9e-7 of sqrt(-2 ln(1 - u0)) and the sine and cosine
                // within 1.3e-7 of sin and cos(2 pi u1) (measured exhaustively
                // against binary64), so with the products' rounding the offset
                // lies within 2e-6 sigma texels of the binary64 offset
                // (r <= 5.8).  A sample at least sigma 2^-14 from a texel edge
                // therefore takes the same texel as the binary64 sample;
                // nearer ones (about one query in 4,000 per unit sigma) redo
                // the offset in binary64.
                const float rf = __builtin_amdgcn_sqrtf(-1.38629436112f * __builtin_amdgcn_logf(1.0f - u0f));
                const float sf = __builtin_amdgcn_sinf(u1f), cf = __builtin_amdgcn_cosf(u1f);
                const double zx = (xe + (double)(sigma * (rf * cf))) + 0.5;
                const double zy = (ye + (double)(sigma * (rf * sf))) + 0.5;
                double fx = floor(zx), fy = floor(zy);
                const double margin = sg * 0x1p-14;
                if (fmin(fmin(zx - fx, (fx + 1.0) - zx), fmin(zy - fy, (fy + 1.0) - zy)) < margin) {
                    const double r = sqrt(-2.0 * log(1.0 - u0));
                    const double a = 6.28318530717958647692 * u1;
                    double sa, ca;
                    sincos(a, &sa, &ca);   // one argument reduction for both
                    const double xs = xe + sg * (r * ca), ys = ye + sg * (r * sa);
                    fx = floor(xs + 0.5);
                    fy = floor(ys + 0.5);
                }
                sx = (int)fmin(fmax(fx, -1.0), (double)S.w());
                sy = (int)fmin(fmax(fy, -1.0), (double)S.h());
            } else {
                const double inv2s2 = 1.0 / (2.0 * sg * sg);
                int jx = -1, jy = -1;
                if (sigma >= 0.25f) {
                    jx = gauss_pick_fast(x - floorf(x), (float)inv2s2, u0f);
                    jy = gauss_pick_fast(y - floorf(y), (float)inv2s2, u1f);
                }
                if (jx < 0) {
                    double wx[4];
                    gauss_discrete_weights(xe - floor(xe), inv2s2, wx);
                    jx = gauss_pick(wx, u0);
                }
                if (jy < 0) {
                    double wy[4];
                    gauss_discrete_weights(ye - floor(ye), inv2s2, wy);
                    jy = gauss_pick(wy, u1);
                }
                sx = cx - 1 + jx;
                sy = cy - 1 + jy;
            }
            sx = clampi(sx, S.w() - 1);
            sy = clampi(sy, S.h() - 1);
            S.load(sx, sy, v);
        } else {
#pragma unroll
            for (int c = 0; c < CAP; ++c) v[c] = __builtin_nanf("");
        }
    } else if constexpr (GMODE == GAUSS_DISCRETE_MEAN) {
        const double inv2s2 = 1.0 / (2.0 * sg * sg);
        double dx[4], dy[4];
        gauss_discrete_weights(xe - floor(xe), inv2s2, dx);
        gauss_discrete_weights(ye - floor(ye), inv2s2, dy);
        const double nx = ((dx[0] + dx[1]) + dx[2]) + dx[3], ny = ((dy[0] + dy[1]) + dy[2]) + dy[3];
        float wx[4], wy[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            wx[k] = (float)(dx[k] / nx);
            wy[k] = (float)(dy[k] / ny);
        }
        float acc[CAP];
#pragma unroll
        for (int c = 0; c < CAP; ++c) acc[c] = 0.0f;
        for (int b = 0; b < 4; ++b) {
            const int yy = clampi(cy - 1 + b, S.h() - 1);
            float row[CAP];
#pragma unroll
            for (int c = 0; c < CAP; ++c) row[c] = 0.0f;
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                float t[CAP];
                S.load(clampi(cx - 1 + a, S.w() - 1), yy, t);
#pragma unroll
                for (int c = 0; c < CAP; ++c) row[c] = __builtin_fmaf(wx[a], t[c], row[c]);
            }
#pragma unroll
            for (int c = 0; c < CAP; ++c) acc[c] = __builtin_fmaf(wy[b], row[c], acc[c]);
        }
#pragma unroll
        for (int c = 0; c < CAP; ++c) v[c] = ok ? acc[c] : __builtin_nanf("");
    } else {   // GAUSS_FIS_MEAN
        // The x weights of the window are kept in LDS, one column per thread
        // (a run-time sized array in registers would live in scratch), in
        // 2R + 2 rows of BLOCK floats sized at launch, so that the block
        // takes no more LDS than its radius needs; the y weights follow as
        // running differences in the row loop.
        extern __shared__ float wxs[];
        const int nt = 2 * radius + 2;
        double px = gauss_phi(((double)(cx - radius) - xe - 0.5) / sg);
        double py = gauss_phi(((double)(cy - radius) - ye - 0.5) / sg);
        for (int k = 0; k < nt; ++k) {
            const double qx = gauss_phi(((double)(cx - radius + k) - xe + 0.5) / sg);
            wxs[k * BLOCK + threadIdx.x] = (float)(qx - px);
            px = qx;
        }
        float acc[CAP];
#pragma unroll
        for (int c = 0; c < CAP; ++c) acc[c] = 0.0f;
        for (int b = 0; b < nt; ++b) {
            const double qy = gauss_phi(((double)(cy - radius + b) - ye + 0.5) / sg);
            const float wyb = (float)(qy - py);
            py = qy;
            const int yy = clampi(cy - radius + b, S.h() - 1);
            float row[CAP];
#pragma unroll
            for (int c = 0; c < CAP; ++c) row[c] = 0.0f;
            for (int a = 0; a < nt; ++a) {
                float t[CAP];
                S.load(clampi(cx - radius + a, S.w() - 1), yy, t);
                const float wxa = wxs[a * BLOCK + threadIdx.x];
#pragma unroll
                for (int c = 0; c < CAP; ++c) row[c] = __builtin_fmaf(wxa, t[c], row[c]);
            }
#pragma unroll
            for (int c = 0; c < CAP; ++c) acc[c] = __builtin_fmaf(wyb, row[c], acc[c]);
        }
#pragma unroll
        for (int c = 0; c < CAP; ++c) v[c] = ok ? acc[c] : __builtin_nanf("");
    }
    block_store(S, out, n, live, (int64_t)i, v, false);
    if (live && idx && (GMODE == GAUSS_FIS || GMODE == GAUSS_DISCRETE)) {
        idx[2 * (int64_t)i] = sx;
        idx[2 * (int64_t)i + 1] = sy;
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <class Src, int KIND>
void launch2d_kind(const Src& S, const float* q, int32_t n, int mode, uint32_t key, float* out, int32_t* idx,
                   const int32_t* order, int scatter, hipStream_t stream)
{
    dim3 grid((n + BLOCK - 1) / BLOCK), block(BLOCK);
    if (mode == STF_STOCHASTIC) {
        if constexpr (KIND == KIND_KEYS || KIND == KIND_MITCHELL)
            hipLaunchKernelGGL((k_tex2d_positivized<Src, KIND>), grid, block, 0, stream, S, q, n, key, out, idx, order,
                               scatter);
        else
            hipLaunchKernelGGL((k_tex2d_stochastic<Src, KIND == KIND_BSPLINE, false>), grid, block, 0, stream, S, q, n,
                               key, out, idx, order, scatter);
    } else if (mode == STF_STOCHASTIC_FIS) {
        if constexpr (KIND == KIND_LINEAR || KIND == KIND_BSPLINE)
            hipLaunchKernelGGL((k_tex2d_stochastic<Src, KIND == KIND_BSPLINE, true>), grid, block, 0, stream, S, q, n,
                               key, out, idx, order, scatter);
    } else {
        if constexpr (Src::DECODES && KIND != KIND_LINEAR) {
            // a decoded source: neighbouring queries of a sorted stream or of
            // a frame in pixel order share most of their 16 taps, so a block
            // decodes its tap box once when the box is small enough (the
            // kernel decides per block and otherwise decodes per tap)
            hipLaunchKernelGGL((k_tex2d_det_staged<Src, KIND>), grid, block, 0, stream, S, q, n, out, order, scatter,
                               stage_counters(), 0.0f);
            return;
        }
        hipLaunchKernelGGL((k_tex2d_deterministic<Src, KIND>), grid, block, 0, stream, S, q, n, out, order, scatter);
    }
}

template <class Src>
hipError_t launch2d_src(const Src& S, const float* q, int32_t n, int filter, int mode, uint32_t key, float* out,
                        int32_t* idx, const int32_t* order, int scatter, hipStream_t stream)
{
    switch (filter) {
    case KIND_LINEAR: launch2d_kind<Src, KIND_LINEAR>(S, q, n, mode, key, out, idx, order, scatter, stream); break;
    case KIND_BSPLINE: launch2d_kind<Src, KIND_BSPLINE>(S, q, n, mode, key, out, idx, order, scatter, stream); break;
    case KIND_KEYS: launch2d_kind<Src, KIND_KEYS>(S, q, n, mode, key, out, idx, order, scatter, stream); break;
    case KIND_MITCHELL: launch2d_kind<Src, KIND_MITCHELL>(S, q, n, mode, key, out, idx, order, scatter, stream); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <class Src>
hipError_t moments2d_src(const Src& S, const float* q, int32_t n, int filter, uint64_t seed_base, int32_t n_seeds,
                         double* sum, double* sumsq, hipStream_t stream)
{
    dim3 grid(n), block(BLOCK);
    switch (filter) {
    case KIND_LINEAR:
        hipLaunchKernelGGL((k_tex2d_moments<Src, KIND_LINEAR>), grid, block, 0, stream, S, q, n, seed_base, n_seeds, sum,
                           sumsq);
        break;
    case KIND_BSPLINE:
        hipLaunchKernelGGL((k_tex2d_moments<Src, KIND_BSPLINE>), grid, block, 0, stream, S, q, n, seed_base, n_seeds,
                           sum, sumsq);
        break;
    case KIND_KEYS:
        hipLaunchKernelGGL((k_tex2d_moments<Src, KIND_KEYS>), grid, block, 0, stream, S, q, n, seed_base, n_seeds, sum,
                           sumsq);
        break;
    case KIND_MITCHELL:
        hipLaunchKernelGGL((k_tex2d_moments<Src, KIND_MITCHELL>), grid, block, 0, stream, S, q, n, seed_base, n_seeds,
                           sum, sumsq);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int FMT, class F>
hipError_t with_dense(const stf_texture* t, F&& f)
{
    const TexLevel& L = t->level[0];
    switch (t->channels) {
    case 1: return f(DenseSrc<FMT, 1>{L});
    case 2: return f(DenseSrc<FMT, 2>{L});
    case 3: return f(DenseSrc<FMT, 3>{L});
    case 4: return f(DenseSrc<FMT, 4>{L});
    }
    return hipErrorInvalidValue;
}

// Calls f with the texel source of a 2D texture: a dense format and channel
// count, or DCT blocks and their padded word count.
template <class F>
hipError_t with_src(const stf_texture* t, F&& f)
{
    if (t->kind == STF_KIND_MATERIAL) return f(MaterialSrc{t->level[0]});
    if (t->kind == STF_KIND_DCT2D) {
        const TexLevel& L = t->level[0];
        const uint32_t* b = static_cast<const uint32_t*>(L.texels);
        switch (t->dct_wpb) {
        case 4: return f(DctSrc<4>{b, L.w, L.h, L.w / 8, t->channels});
        case 8: return f(DctSrc<8>{b, L.w, L.h, L.w / 8, t->channels});
        case 12: return f(DctSrc<12>{b, L.w, L.h, L.w / 8, t->channels});
        case 16: return f(DctSrc<16>{b, L.w, L.h, L.w / 8, t->channels});
        }
        return hipErrorInvalidValue;
    }
    switch (t->fmt) {
    case F32: return with_dense<F32>(t, f);
    case F16: return with_dense<F16>(t, f);
    case BF16: return with_dense<BF16>(t, f);
    case FP8_E4M3: return with_dense<FP8_E4M3>(t, f);
    case U8: return with_dense<U8>(t, f);
    }
    return hipErrorInvalidValue;
}

template <class Src>
hipError_t gauss2d_src(const Src& S, const float* q, int32_t n, float sigma, int gmode, uint32_t key, float* out,
                       int32_t* idx, hipStream_t stream)
{
    dim3 grid((n + BLOCK - 1) / BLOCK), block(BLOCK);
    const int32_t radius = (int32_t)ceilf(6.0f * sigma) + 1;
    switch (gmode) {
    case GAUSS_FIS:
        hipLaunchKernelGGL((k_tex2d_gauss<Src, GAUSS_FIS>), grid, block, 0, stream, S, q, n, sigma, radius, key, out,
                           idx);
        break;
    case GAUSS_FIS_MEAN:
        if (2 * radius + 2 > GAUSS_MAX_TAPS) return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_tex2d_gauss<Src, GAUSS_FIS_MEAN>), grid, block,
                           (size_t)(2 * radius + 2) * BLOCK * sizeof(float), stream, S, q, n, sigma, radius, key,
                           out, idx);
        break;
    case GAUSS_DISCRETE:
        hipLaunchKernelGGL((k_tex2d_gauss<Src, GAUSS_DISCRETE>), grid, block, 0, stream, S, q, n, sigma, radius, key,
                           out, idx);
        break;
    case GAUSS_DISCRETE_MEAN:
        if constexpr (Src::DECODES)   // decoded sources: each block decodes its taps' box once (when it pays)
            hipLaunchKernelGGL((k_tex2d_det_staged<Src, KIND_GAUSS_MEAN>), grid, block, 0, stream, S, q, n, out,
                               nullptr, 0, stage_counters(), sigma);
        else
            hipLaunchKernelGGL((k_tex2d_gauss<Src, GAUSS_DISCRETE_MEAN>), grid, block, 0, stream, S, q, n, sigma,
                               radius, key, out, idx);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_gauss2d(const stf_texture* t, const float* q, int32_t n, float sigma, int gmode, uint32_t key,
                          float* out, int32_t* idx, hipStream_t s)
{
    return with_src(t, [&](auto S) { return gauss2d_src(S, q, n, sigma, gmode, key, out, idx, s); });
}

hipError_t launch_filter2d(const stf_texture* t, const float* q, int32_t n, int filter, int mode, uint32_t key,
                           float* out, int32_t* idx, const int32_t* order, int scatter, hipStream_t s)
{
    return with_src(t, [&](auto S) { return launch2d_src(S, q, n, filter, mode, key, out, idx, order, scatter, s); });
}

hipError_t launch_moments2d(const stf_texture* t, const float* q, int32_t n, int filter, uint64_t seed_base,
                            int32_t n_seeds, double* sum, double* sumsq, hipStream_t s)
{
    return with_src(t, [&](auto S) { return moments2d_src(S, q, n, filter, seed_base, n_seeds, sum, sumsq, s); });
}

int32_t serve2d_queries_per_block()
{
    return BLOCK;
}

hipError_t launch_serve2d(const stf_texture* t, int filter, const ServeChunk* chunks, int32_t nchunks, int32_t nblocks,
                          hipStream_t s)
{
    if (t->kind != STF_KIND_TEX2D && t->kind != STF_KIND_MATERIAL) return hipErrorInvalidValue;
    return with_src(t, [&](auto S) {
        using Src = decltype(S);
        if (filter == STF_CUBIC_BSPLINE)
            hipLaunchKernelGGL((k_tex2d_serve<Src, true>), dim3(nblocks), dim3(BLOCK), 0, s, S, chunks, nchunks);
        else
            hipLaunchKernelGGL((k_tex2d_serve<Src, false>), dim3(nblocks), dim3(BLOCK), 0, s, S, chunks, nchunks);
        return hipGetLastError();
    });
}
