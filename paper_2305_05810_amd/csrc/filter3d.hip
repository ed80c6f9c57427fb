// filter3d.hip -- trilinear / tricubic B-spline filtering of sparse voxel
// grids, deterministic (all 8 / 64 taps, Eq. filtered-texture) and stochastic
// (one tap drawn with probability equal to its weight, Eq. stochastic-sum;
// the per-axis draw of section "B-Spline and Anisotropic Filters").
//
// The interpolating cubics (Keys, Mitchell) filter deterministically with
// their 64 weights and stochastically by positivization: one tap from the
// positive and one from the negative weights (interp.h).
//
// Grid walk: root slot (128^3 voxels) -> internal node child (8^3 voxels) ->
// dense 8^3 leaf, x fastest.  Voxels outside the domain or in empty slots read
// as the grid's background value.
#include <limits.h>
#include <math.h>

#include <type_traits>

#include "device_common.h"
#include "interp.h"
#include "stf_internal.h"

using namespace stf;

namespace {

constexpr int BLOCK = 256;
#ifndef STOCH_Q
#define STOCH_Q 4   // queries per thread in the stochastic kernel
#endif

// Leaf id holding voxel (x, y, z), which must lie in the domain; -1 if none.
__device__ __forceinline__ int32_t grid_leaf(const GridView& g, int x, int y, int z)
{
    int32_t node = g.root[((z >> 7) * g.ry + (y >> 7)) * g.rx + (x >> 7)];
    if (node < 0) return -1;
    return g.nodes[(int64_t)node * 4096 + (((z >> 3) & 15) * 16 + ((y >> 3) & 15)) * 16 + ((x >> 3) & 15)];
}

__device__ __forceinline__ bool in_domain(const GridView& g, int x, int y, int z)
{
    return (unsigned)x < (unsigned)g.dx && (unsigned)y < (unsigned)g.dy && (unsigned)z < (unsigned)g.dz;
}

template <int FMT>
__device__ __forceinline__ float grid_voxel(const GridView& g, int x, int y, int z)
{
    if (!in_domain(g, x, y, z)) return g.background;
    int32_t leaf = grid_leaf(g, x, y, z);
    if (leaf < 0) return g.background;
    return load_texel<FMT>(g.leaves, (int64_t)leaf * 512 + leaf_offset(FMT, x & 7, y & 7, z & 7));
}

// ---------------------------------------------------------------------------
// stochastic: one tap per query.
//
// Each thread takes Q queries (block-strided, so every load and store
// instruction of a wave covers one contiguous span) and walks their grid
// paths in lock step: the Q root loads are issued together, then the Q node
// loads, then the Q leaf loads, which keeps Q dependent-load chains in flight
// per lane.  Lanes whose query is out of the domain or in an empty slot load
// from offset 0 and discard the value, so the walk has no divergent branches;
// a level is skipped only when no lane of the wave needs it.  Table offsets
// are 32-bit (the library rejects grids whose tables exceed 4 GiB), so every
// gather is a scalar-base + 32-bit vector-offset load.
// ---------------------------------------------------------------------------
template <int FMT>
__device__ __forceinline__ float leaf_value(const void* __restrict__ leaves, uint32_t elem)
{
    const char* p = reinterpret_cast<const char*>(leaves) + (size_t)(elem * (uint32_t)fmt_bytes(FMT));
    if constexpr (FMT == F32) return *reinterpret_cast<const float*>(p);
    if constexpr (FMT == F16) return dec_f16(*reinterpret_cast<const uint16_t*>(p));
    if constexpr (FMT == BF16) return dec_bf16(*reinterpret_cast<const uint16_t*>(p));
    if constexpr (FMT == FP8_E4M3) return dec_e4m3(*reinterpret_cast<const uint8_t*>(p));
    if constexpr (FMT == U8) return dec_u8(*reinterpret_cast<const uint8_t*>(p));
    return 0.0f;
}

__device__ __forceinline__ int32_t table_load(const int32_t* __restrict__ t, uint32_t elem)
{
    return *reinterpret_cast<const int32_t*>(reinterpret_cast<const char*>(t) + (size_t)(elem * 4u));
}

// One block's share: queries first + k*BLOCK (k < Q) of a batch of n, whose
// random draw uses the id qid0 + index.
template <int FMT, bool CUBIC, int Q, bool FIS = false>
__device__ __forceinline__ void grid_stochastic_block(const GridView& g, const float* __restrict__ q, int32_t n,
                                                      int32_t first, uint32_t key, uint32_t qid0,
                                                      float* __restrict__ out, int32_t* __restrict__ idx,
                                                      const int32_t* __restrict__ order, int scatter)
{
    float p[Q][3];
    bool live[Q];
    uint32_t qid[Q];   // id of the draw: the query's place in the caller's batch
    int64_t oi[Q];     // where its result goes
#pragma unroll
    for (int k = 0; k < Q; ++k) {   // all query loads first
        int32_t i = first + k * BLOCK;
        live[k] = i < n;
        int32_t src = live[k] ? i : 0;
        int32_t id = order ? order[src] : (int32_t)(qid0 + (uint32_t)i);
        qid[k] = (uint32_t)id;
        oi[k] = (order && scatter) ? (int64_t)id : (int64_t)i;
        const float* e = q + 3 * (int64_t)src;
        p[k][0] = __builtin_nontemporal_load(e);
        p[k][1] = __builtin_nontemporal_load(e + 1);
        p[k][2] = __builtin_nontemporal_load(e + 2);
    }
    int vx[Q], vy[Q], vz[Q];
    bool fin[Q], ok[Q];
    uint32_t roff[Q];
#pragma unroll
    for (int k = 0; k < Q; ++k) {
        int c0 = 0, c1 = 0, c2 = 0;
        float t0 = 0.0f, t1 = 0.0f, t2 = 0.0f;
        fin[k] = cell_of(p[k][0], c0, t0) & cell_of(p[k][1], c1, t1) & cell_of(p[k][2], c2, t2);
        const uint32_t b = pcg(key ^ qid[k]);
        uint32_t h0, h1, h2;
        pcg_axes3(b, h0, h1, h2);
        float m0 = hash_m(h0), m1 = hash_m(h1), m2 = hash_m(h2);
        if constexpr (FIS) {
            vx[k] = fis_tap<CUBIC>(p[k][0], b, 0);
            vy[k] = fis_tap<CUBIC>(p[k][1], b, 1);
            vz[k] = fis_tap<CUBIC>(p[k][2], b, 2);
        } else if constexpr (CUBIC) {
            vx[k] = c0 + choose_cubic_m(t0, m0);
            vy[k] = c1 + choose_cubic_m(t1, m1);
            vz[k] = c2 + choose_cubic_m(t2, m2);
        } else {
            vx[k] = c0 + choose_linear_m(t0, m0);
            vy[k] = c1 + choose_linear_m(t1, m1);
            vz[k] = c2 + choose_linear_m(t2, m2);
        }
        ok[k] = live[k] && fin[k] && in_domain(g, vx[k], vy[k], vz[k]);
        roff[k] = ok[k] ? (uint32_t)(((vz[k] >> 7) * g.ry + (vy[k] >> 7)) * g.rx + (vx[k] >> 7)) : 0u;
    }
    int32_t node[Q];
#pragma unroll
    for (int k = 0; k < Q; ++k) node[k] = table_load(g.root, roff[k]);
    bool any = false;
#pragma unroll
    for (int k = 0; k < Q; ++k) {
        ok[k] = ok[k] && node[k] >= 0;
        any |= ok[k];
    }
    float v[Q];
#pragma unroll
    for (int k = 0; k < Q; ++k) v[k] = g.background;
    if (__any(any)) {
        int32_t leaf[Q];
#pragma unroll
        for (int k = 0; k < Q; ++k) {
            uint32_t child = ((((uint32_t)vz[k] >> 3) & 15u) * 16u + (((uint32_t)vy[k] >> 3) & 15u)) * 16u +
                             (((uint32_t)vx[k] >> 3) & 15u);
            leaf[k] = table_load(g.nodes, ok[k] ? (uint32_t)node[k] * 4096u + child : 0u);
        }
        any = false;
#pragma unroll
        for (int k = 0; k < Q; ++k) {
            ok[k] = ok[k] && leaf[k] >= 0;
            any |= ok[k];
        }
        if (__any(any)) {
#pragma unroll
            for (int k = 0; k < Q; ++k) {
                uint32_t vox = leaf_offset(FMT, (uint32_t)vx[k] & 7u, (uint32_t)vy[k] & 7u, (uint32_t)vz[k] & 7u);
                float t = leaf_value<FMT>(g.leaves, ok[k] ? (uint32_t)leaf[k] * 512u + vox : 0u);
                v[k] = ok[k] ? t : g.background;
            }
        }
    }
#pragma unroll
    for (int k = 0; k < Q; ++k) {
        if (!live[k]) continue;
        __builtin_nontemporal_store(fin[k] ? v[k] : __builtin_nanf(""), out + oi[k]);
        if (idx) {
            idx[3 * oi[k]] = fin[k] ? vx[k] : BAD_INDEX;
            idx[3 * oi[k] + 1] = fin[k] ? vy[k] : BAD_INDEX;
            idx[3 * oi[k] + 2] = fin[k] ? vz[k] : BAD_INDEX;
        }
    }
}

template <int FMT, bool CUBIC, int Q>
__global__ __launch_bounds__(BLOCK) void k_grid_stochastic(GridView g, const float* __restrict__ q, int32_t n,
                                                           uint32_t key, float* __restrict__ out,
                                                           int32_t* __restrict__ idx, const int32_t* __restrict__ order,
                                                           int scatter)
{
    grid_stochastic_block<FMT, CUBIC, Q>(g, q, n, blockIdx.x * (BLOCK * Q) + threadIdx.x, key, 0u, out, idx, order,
                                         scatter);
}

// ---------------------------------------------------------------------------
// positivized interpolating cubics: two taps per query.
//
// Each thread takes Q queries (block-strided like the single-tap kernel) and
// walks the 2Q voxel paths of their positive and negative taps in lock step.
// ---------------------------------------------------------------------------
// Values of T voxels, walked in lock step: root loads, then node loads, then
// leaf loads; a voxel with ok[k] false (or outside the domain, or in an empty
// slot) reads as background and loads from offset 0.
template <int FMT, int T>
__device__ __forceinline__ void grid_fetch(const GridView& g, const int (&vx)[T], const int (&vy)[T],
                                           const int (&vz)[T], bool (&ok)[T], float (&v)[T])
{
    uint32_t roff[T];
#pragma unroll
    for (int k = 0; k < T; ++k) {
        ok[k] = ok[k] && in_domain(g, vx[k], vy[k], vz[k]);
        roff[k] = ok[k] ? (uint32_t)(((vz[k] >> 7) * g.ry + (vy[k] >> 7)) * g.rx + (vx[k] >> 7)) : 0u;
        v[k] = g.background;
    }
    int32_t node[T];
#pragma unroll
    for (int k = 0; k < T; ++k) node[k] = table_load(g.root, roff[k]);
    bool any = false;
#pragma unroll
    for (int k = 0; k < T; ++k) {
        ok[k] = ok[k] && node[k] >= 0;
        any |= ok[k];
    }
    if (!__any(any)) return;
    int32_t leaf[T];
#pragma unroll
    for (int k = 0; k < T; ++k) {
        uint32_t child = ((((uint32_t)vz[k] >> 3) & 15u) * 16u + (((uint32_t)vy[k] >> 3) & 15u)) * 16u +
                         (((uint32_t)vx[k] >> 3) & 15u);
        leaf[k] = table_load(g.nodes, ok[k] ? (uint32_t)node[k] * 4096u + child : 0u);
    }
    any = false;
#pragma unroll
    for (int k = 0; k < T; ++k) {
        ok[k] = ok[k] && leaf[k] >= 0;
        any |= ok[k];
    }
    if (!__any(any)) return;
#pragma unroll
    for (int k = 0; k < T; ++k) {
        uint32_t vox = leaf_offset(FMT, (uint32_t)vx[k] & 7u, (uint32_t)vy[k] & 7u, (uint32_t)vz[k] & 7u);
        float t = leaf_value<FMT>(g.leaves, ok[k] ? (uint32_t)leaf[k] * 512u + vox : 0u);
        v[k] = ok[k] ? t : g.background;
    }
}

// Value (S+ t(j+) - S- t(j-)) / scale^3; index (x+, y+, z+, x-, y-, z-), the
// negative tap INT32_MIN when S- = 0.
template <int FMT, int KIND, int Q>
__global__ __launch_bounds__(BLOCK) void k_grid_positivized(GridView g, const float* __restrict__ q, int32_t n,
                                                            uint32_t key, float* __restrict__ out,
                                                            int32_t* __restrict__ idx,
                                                            const int32_t* __restrict__ order, int scatter)
{
    const int32_t first = blockIdx.x * (BLOCK * Q) + threadIdx.x;
    float p[Q][3];
    bool live[Q];
    int64_t oi[Q];
    uint32_t qid[Q];
#pragma unroll
    for (int k = 0; k < Q; ++k) {
        int32_t i = first + k * BLOCK;
        live[k] = i < n;
        int32_t src = live[k] ? i : 0;
        int32_t id = order ? order[src] : i;
        qid[k] = (uint32_t)id;
        oi[k] = (order && scatter) ? (int64_t)id : (int64_t)i;
        const float* e = q + 3 * (int64_t)src;
        p[k][0] = __builtin_nontemporal_load(e);
        p[k][1] = __builtin_nontemporal_load(e + 1);
        p[k][2] = __builtin_nontemporal_load(e + 2);
    }
    int vx[2 * Q], vy[2 * Q], vz[2 * Q];
    bool ok[2 * Q], fin[Q], neg[Q];
    float sp[Q], sn[Q];
#pragma unroll
    for (int k = 0; k < Q; ++k) {
        int c[3] = {0, 0, 0};
        float t[3] = {0.0f, 0.0f, 0.0f};
        fin[k] = cell_of(p[k][0], c[0], t[0]) & cell_of(p[k][1], c[1], t[1]) & cell_of(p[k][2], c[2], t[2]);
        const PosDraw<3> d = positivized_draw<3, KIND>(t, pcg(key ^ qid[k]));
        vx[2 * k] = c[0] + d.op[0];
        vy[2 * k] = c[1] + d.op[1];
        vz[2 * k] = c[2] + d.op[2];
        vx[2 * k + 1] = c[0] + d.on[0];
        vy[2 * k + 1] = c[1] + d.on[1];
        vz[2 * k + 1] = c[2] + d.on[2];
        neg[k] = d.neg;
        sp[k] = d.sp;
        sn[k] = d.sn;
        ok[2 * k] = live[k] && fin[k];
        ok[2 * k + 1] = live[k] && fin[k] && d.neg;
    }
    float v[2 * Q];
    grid_fetch<FMT, 2 * Q>(g, vx, vy, vz, ok, v);
    constexpr float inv = inv_scale<3, KIND>();
#pragma unroll
    for (int k = 0; k < Q; ++k) {
        if (!live[k]) continue;
        float r = (neg[k] ? sp[k] * v[2 * k] - sn[k] * v[2 * k + 1] : sp[k] * v[2 * k]) * inv;
        __builtin_nontemporal_store(fin[k] ? r : __builtin_nanf(""), out + oi[k]);
        if (idx) {
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const int pv = a == 0 ? vx[2 * k] : (a == 1 ? vy[2 * k] : vz[2 * k]);
                const int nv = a == 0 ? vx[2 * k + 1] : (a == 1 ? vy[2 * k + 1] : vz[2 * k + 1]);
                idx[6 * oi[k] + a] = fin[k] ? pv : BAD_INDEX;
                idx[6 * oi[k] + 3 + a] = (fin[k] && neg[k]) ? nv : BAD_INDEX;
            }
        }
    }
}

// Filter importance sampling of the same filters: jittered position, nearest
// voxel (fis_tap); otherwise the single-tap kernel.
template <int FMT, bool CUBIC, int Q>
__global__ __launch_bounds__(BLOCK) void k_grid_fis(GridView g, const float* __restrict__ q, int32_t n, uint32_t key,
                                                    float* __restrict__ out, int32_t* __restrict__ idx,
                                                    const int32_t* __restrict__ order, int scatter)
{
    grid_stochastic_block<FMT, CUBIC, Q, true>(g, q, n, blockIdx.x * (BLOCK * Q) + threadIdx.x, key, 0u, out, idx,
                                               order, scatter);
}

// Serving: one launch over many requests' chunks (same grid and filter).
// Block b serves chunk c with start[c] <= b < start[c + 1].
template <int FMT, bool CUBIC, int Q>
__global__ __launch_bounds__(BLOCK) void k_grid_serve(GridView g, const ServeChunk* __restrict__ chunks, int32_t nchunks)
{
    int lo = 0, hi = nchunks - 1;
    while (lo < hi) {   // last chunk whose first block is <= blockIdx.x
        int mid = (lo + hi + 1) / 2;
        if (chunks[mid].block0 <= (int32_t)blockIdx.x) lo = mid;
        else hi = mid - 1;
    }
    const ServeChunk c = chunks[lo];
    grid_stochastic_block<FMT, CUBIC, Q>(g, c.q, c.count, ((int32_t)blockIdx.x - c.block0) * (BLOCK * Q) + threadIdx.x,
                                         c.key, c.qid0, c.out, c.idx, nullptr, 0);
}

// ---------------------------------------------------------------------------
// deterministic: all taps.  The taps of one axis span at most two leaves, so
// the (up to) 2x2x2 leaves are resolved once and each tap picks its leaf by
// the bit that says which side of the leaf boundary it lies on.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int32_t pick8(const int32_t (&l)[8], bool kx, bool ky, bool kz)
{
    int32_t a = kx ? l[1] : l[0], b = kx ? l[3] : l[2], c = kx ? l[5] : l[4], d = kx ? l[7] : l[6];
    int32_t e = ky ? b : a, f = ky ? d : c;
    return kz ? f : e;
}

// The unscaled sum over the NT^3 taps starting at voxel base, from global
// memory (weights scaled by axis_scale per axis).
// The value itself, opaque to the optimizer (an empty asm statement, no
// instruction): a byte offset selected against 0 otherwise becomes a select
// of 64-bit addresses, and the loads lose the uniform-base-plus-32-bit-offset
// form (two VGPRs of address per load in flight instead of one).
__device__ __forceinline__ uint32_t vgpr_u32(uint32_t v)
{
    asm volatile("" : "+v"(v));
    return v;
}

// As vgpr_u32, and ordered after `dep` is known: loads addressed by the
// result wait for the value (a partial sum) that `dep` carries.
__device__ __forceinline__ uint32_t vgpr_u32_after(uint32_t v, float dep)
{
    asm volatile("" : "+v"(v) : "v"(dep));
    return v;
}

// The NT taps of a row from its two-chunk window (uint4 chunks: 4 binary32
// or 8 16-bit values; uint2 chunks: 8 8-bit values), starting at voxel p of
// the window.  Selection is branch-free on the bits of p, then each tap is
// decoded exactly as a single-texel load would.
template <int FMT, int NT>
__device__ __forceinline__ void window_taps(const uint4& c0, const uint4& c1, int p, float (&t)[NT])
{
    // (named registers, not an indexed array: the selection stays in VGPRs)
    if constexpr (FMT == F32) {
        // p in 0..3: tap j is dword p + j of the window
        const bool b0 = p & 1, b1 = p & 2;
        const uint32_t s0 = b0 ? c0.y : c0.x, s1 = b0 ? c0.z : c0.y, s2 = b0 ? c0.w : c0.z,
                       s3 = b0 ? c1.x : c0.w;
        t[0] = __builtin_bit_cast(float, b1 ? s2 : s0);
        t[1] = __builtin_bit_cast(float, b1 ? s3 : s1);
        if constexpr (NT == 4) {
            const uint32_t s4 = b0 ? c1.y : c1.x, s5 = b0 ? c1.z : c1.y;
            t[2] = __builtin_bit_cast(float, b1 ? s4 : s2);
            t[3] = __builtin_bit_cast(float, b1 ? s5 : s3);
        }
    } else {
        // p in 0..7: tap j is half p + j; the taps' dwords start at p >> 1
        const bool b1 = p & 2, b2 = p & 4;
        const uint32_t s0 = b1 ? c0.y : c0.x, s1 = b1 ? c0.z : c0.y, s2 = b1 ? c0.w : c0.z,
                       s3 = b1 ? c1.x : c0.w;
        const uint32_t e0 = b2 ? s2 : s0, e1 = b2 ? s3 : s1;
        const uint32_t sh = (uint32_t)(p & 1) * 16u;
        uint32_t wd[NT / 2];
        wd[0] = __builtin_amdgcn_alignbit(e1, e0, sh);
        if constexpr (NT == 4) {
            const uint32_t s4 = b1 ? c1.y : c1.x;
            const uint32_t e2 = b2 ? s4 : s2;
            wd[1] = __builtin_amdgcn_alignbit(e2, e1, sh);
        }
#pragma unroll
        for (int k = 0; k < NT / 2; ++k) {
            if constexpr (FMT == F16) {
                t[2 * k] = dec_f16((uint16_t)wd[k]);
                t[2 * k + 1] = dec_f16((uint16_t)(wd[k] >> 16));
            } else {
                t[2 * k] = dec_bf16((uint16_t)wd[k]);
                t[2 * k + 1] = dec_bf16((uint16_t)(wd[k] >> 16));
            }
        }
    }
}

template <int FMT, int NT>
__device__ __forceinline__ void window_taps(const uint2& c0, const uint2& c1, int p, float (&t)[NT])
{
    // p in 0..7: tap j is byte p + j of the 16-byte window
    const uint32_t lo = (p & 4) ? c0.y : c0.x, hi = (p & 4) ? c1.x : c0.y;
    const uint32_t wd = __builtin_amdgcn_alignbit(hi, lo, (uint32_t)(p & 3) * 8u);
    if constexpr (FMT == FP8_E4M3) {
        t[0] = dec_e4m3_byte<0>(wd);
        t[1] = dec_e4m3_byte<1>(wd);
        if constexpr (NT == 4) {
            t[2] = dec_e4m3_byte<2>(wd);
            t[3] = dec_e4m3_byte<3>(wd);
        }
    } else {
#pragma unroll
        for (int j = 0; j < NT; ++j) t[j] = dec_u8((wd >> (8 * j)) & 0xffu);
    }
}

// The at most 2x2x2 leaves that a query's tap block (NT^3 voxels from base)
// meets, low/high side per axis in bits 0/1/2 of k; -1 where no stored leaf
// is (empty slot, outside the domain) or where no tap lies.  True if any
// holds texels.
template <int KIND>
__device__ __forceinline__ bool det_leaves(const GridView& g, const int (&base)[3], int32_t (&leaf)[8])
{
    constexpr int NT = KIND == KIND_LINEAR ? 2 : 4;
    int lo[3];
    bool nb[3];   // the second leaf along an axis is resolved only when a tap lies in it
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        lo[a] = base[a] >> 3;   // leaf coordinate of the first tap (floor for negatives)
        nb[a] = ((base[a] + NT - 1) >> 3) != lo[a];
    }
    // the walks in lock step, without branches: the root entries of all
    // leaves are loaded together, then their node entries (a leaf that is
    // not needed, or outside the domain, loads entry 0 and is discarded), so
    // a query waits for two loads instead of two per leaf
    bool use[8];
    uint32_t roff[8], child[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const bool used = (!(k & 1) || nb[0]) && (!(k & 2) || nb[1]) && (!(k & 4) || nb[2]);
        const int x = (lo[0] + (k & 1)) * 8, y = (lo[1] + ((k >> 1) & 1)) * 8, z = (lo[2] + (k >> 2)) * 8;
        use[k] = used && in_domain(g, x, y, z);
        roff[k] = vgpr_u32(use[k] ? (uint32_t)(((z >> 7) * g.ry + (y >> 7)) * g.rx + (x >> 7)) : 0u);
        child[k] = ((((uint32_t)z >> 3) & 15u) * 16u + (((uint32_t)y >> 3) & 15u)) * 16u + (((uint32_t)x >> 3) & 15u);
    }
    int32_t node[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) node[k] = table_load(g.root, roff[k]);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        use[k] = use[k] && node[k] >= 0;
        leaf[k] = table_load(g.nodes, vgpr_u32(use[k] ? (uint32_t)node[k] * 4096u + child[k] : 0u));
    }
    bool live = false;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        leaf[k] = use[k] ? leaf[k] : -1;
        live = live || leaf[k] >= 0;
    }
    return live;
}

// Empty space: every tap reads the background, so the nested sums of
// det_taps reduce to one row, one plane and one volume sum of it (the same
// operations in the same order, so the same binary32 result).
template <int KIND>
__device__ __forceinline__ float det_background(const GridView& g, const float (&w)[3][4])
{
    constexpr int NT = KIND == KIND_LINEAR ? 2 : 4;
    float row = 0.0f, plane = 0.0f, acc = 0.0f;
#pragma unroll
    for (int cx = 0; cx < NT; ++cx) row = __builtin_fmaf(w[0][cx], g.background, row);
#pragma unroll
    for (int cy = 0; cy < NT; ++cy) plane = __builtin_fmaf(w[1][cy], row, plane);
#pragma unroll
    for (int cz = 0; cz < NT; ++cz) acc = __builtin_fmaf(w[2][cz], plane, acc);
    return acc;
}

// The separable tap sum (x innermost, then y, then z) over the query's leaves.
template <int FMT, int KIND>
__device__ __forceinline__ float det_taps(const GridView& g, const int (&base)[3], const int32_t (&leaf)[8],
                                          const float (&w)[3][4])
{
    constexpr int NT = KIND == KIND_LINEAR ? 2 : 4;
    int lo[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) lo[a] = base[a] >> 3;
    float acc = 0.0f;
    // Per axis and tap: whether the tap lies in the second leaf along
    // the axis and inside the domain; row offsets within a leaf.
    bool ky[NT], kz[NT], inx[NT], iny[NT], inz[NT];
    uint32_t oy[NT], oz[NT];
#pragma unroll
    for (int k = 0; k < NT; ++k) {
        const int vx = base[0] + k, vy = base[1] + k, vz = base[2] + k;
        ky[k] = (vy >> 3) != lo[1];
        kz[k] = (vz >> 3) != lo[2];
        inx[k] = (unsigned)vx < (unsigned)g.dx;
        iny[k] = (unsigned)vy < (unsigned)g.dy;
        inz[k] = (unsigned)vz < (unsigned)g.dz;
        oy[k] = leaf_oy(FMT, (uint32_t)(vy & 7));
        oz[k] = leaf_oz(FMT, (uint32_t)(vz & 7));
    }
    // A row's taps are read as one window of two aligned chunks along x
    // (16 bytes each: half a leaf row of binary32, a whole row of 16-bit
    // values; 8 bytes, a whole row, of 8-bit values), one vector load per
    // chunk instead of one load per tap.  The taps start at voxel p of the
    // window; the second chunk is loaded only when a tap reaches it, and
    // lies in the x-neighbour leaf when the first ends a leaf row.
    constexpr uint32_t TB = FMT == F32 ? 4u : (FMT == F16 || FMT == BF16 ? 2u : 1u);
    constexpr int CV = FMT == F32 ? 4 : 8;
    using Chunk = typename std::conditional<TB == 1u, uint2, uint4>::type;
    const int p = base[0] & (CV - 1);
    const uint32_t xo0 = (uint32_t)(base[0] & 7 & ~(CV - 1));   // first chunk's offset in its leaf row
    const bool c1b = xo0 + CV == 8;                             // second chunk in the x-neighbour leaf
    const uint32_t xo1 = c1b ? 0u : xo0 + CV;
    const uint32_t ox0 = leaf_ox(FMT, xo0), ox1 = leaf_ox(FMT, xo1);   // the chunks' places in the leaf
    const bool two = p + NT > CV;
    const char* __restrict__ leaves = reinterpret_cast<const char*>(g.leaves);
    // the leaves as values, so that selecting a row's pair stays a register
    // select rather than becoming an indexed read of a local array
    const int32_t L0 = leaf[0], L1 = leaf[1], L2 = leaf[2], L3 = leaf[3], L4 = leaf[4], L5 = leaf[5],
                  L6 = leaf[6], L7 = leaf[7];
#pragma unroll
    for (int cz = 0; cz < NT; ++cz) {
        float plane = 0.0f;
#pragma unroll
        for (int cy = 0; cy < NT; ++cy) {
            // the row's leaves on the low and high side along x, and
            // whether each chunk holds texels; a chunk with none (or not
            // needed) loads from offset 0, shared by all such lanes
            const int32_t la = kz[cz] ? (ky[cy] ? L6 : L4) : (ky[cy] ? L2 : L0);
            const int32_t lb = kz[cz] ? (ky[cy] ? L7 : L5) : (ky[cy] ? L3 : L1);
            const int32_t l1 = c1b ? lb : la;
            const bool ryz = iny[cy] && inz[cz];
            const bool ok0 = ryz && la >= 0, ok1 = ryz && l1 >= 0;
            const uint32_t roff = oz[cz] + oy[cy];
            // the second half of the rows is addressed after the first half
            // is summed: half the loads in flight, half the registers
            const float gate = 2 * cz < NT ? 0.0f : acc;
            const uint32_t a0 = vgpr_u32_after(ok0 ? ((uint32_t)la * 512u + roff + ox0) * TB : 0u, gate);
            const uint32_t a1 = vgpr_u32_after((ok1 && two) ? ((uint32_t)l1 * 512u + roff + ox1) * TB : 0u, gate);
            const Chunk v0 = *reinterpret_cast<const Chunk*>(leaves + a0);
            const Chunk v1 = *reinterpret_cast<const Chunk*>(leaves + a1);
            float t[NT];
            window_taps<FMT>(v0, v1, p, t);
            float row = 0.0f;
#pragma unroll
            for (int cx = 0; cx < NT; ++cx) {
                const bool tap = (p + cx >= CV ? ok1 : ok0) && inx[cx];
                row = __builtin_fmaf(w[0][cx], tap ? t[cx] : g.background, row);
            }
            plane = __builtin_fmaf(w[1][cy], row, plane);
        }
        acc = __builtin_fmaf(w[2][cz], plane, acc);
    }
    return acc;
}

template <int FMT, int KIND>
__device__ __forceinline__ float det_sum_global(const GridView& g, const int (&base)[3], const float (&w)[3][4])
{
    int32_t leaf[8];
    return det_leaves<KIND>(g, base, leaf) ? det_taps<FMT, KIND>(g, base, leaf, w) : det_background<KIND>(g, w);
}

// Cell, first tap and scaled per-axis weights of a query; false if the
// position has no cell (R10: non-finite or too large).
template <int KIND>
__device__ __forceinline__ bool det_setup(const float (&p)[3], int (&base)[3], float (&w)[3][4])
{
    int c[3];
    float t[3];
    const bool ok = cell_of(p[0], c[0], t[0]) & cell_of(p[1], c[1], t[1]) & cell_of(p[2], c[2], t[2]);
#pragma unroll
    for (int a = 0; a < 3; ++a) base[a] = c[a] + axis_weights_scaled<KIND>(t[a], w[a]);
    return ok;
}

// The three per-axis scale factors (216, 8 or 5832) divided out.
template <int KIND>
__device__ __forceinline__ float det_unscale(float acc)
{
    constexpr float S3 = axis_scale<KIND>() * axis_scale<KIND>() * axis_scale<KIND>();
    if constexpr (KIND != KIND_LINEAR) acc = acc / S3;
    return acc;
}

// Deterministic filtering from global memory, one query per thread, at 8
// waves per SIMD (64 VGPRs) where that fits without spilling, else 7 (72
// VGPRs; the binary32 cubics): the dependent leaf walks of
// empty-space queries need the waves to hide their latency, and the tap rows
// of a query are loaded in two halves to fit.
template <int FMT, int KIND>
constexpr int det_waves()
{
    return (FMT == F32 && KIND != KIND_LINEAR) ? 7 : 8;
}

template <int FMT, int KIND>
__global__ __launch_bounds__(BLOCK, (det_waves<FMT, KIND>())) void k_grid_deterministic(
    GridView g, const float* __restrict__ q, int32_t n, float* __restrict__ out, const int32_t* __restrict__ order,
    int scatter)
{
    int32_t i = blockIdx.x * BLOCK + threadIdx.x;
    if (i >= n) return;
    const float p[3] = {q[3 * (int64_t)i], q[3 * (int64_t)i + 1], q[3 * (int64_t)i + 2]};
    int base[3];
    float w[3][4];
    const bool ok = det_setup<KIND>(p, base, w);
    __builtin_nontemporal_store(ok ? det_unscale<KIND>(det_sum_global<FMT, KIND>(g, base, w))
                                                : __builtin_nanf(""), out + ((order && scatter) ? order[i] : i));
}

// ---------------------------------------------------------------------------
// deterministic filtering of a sorted stream with the block's taps staged in
// LDS.  Queries that are neighbours in Morton order share most of their tap
// blocks, so a block reads every voxel of the bounding box of its queries'
// tap blocks once and then filters each query from LDS: the box's leaf slots
// are resolved first (one walk per slot), then each voxel is one load.  A
// block stages only when that pays: the box holds at most STAGE_VOXELS
// voxels in at most STAGE_SLOTS leaf slots, its queries read at least
// STAGE_REUSE taps per staged voxel, and some slot holds a leaf; otherwise it
// filters from global memory (where all-empty tap blocks cost no loads).
// Both paths read the same texel values and sum them in the same order, so
// the results are the same.
// ---------------------------------------------------------------------------
constexpr int STAGE_VOXELS = 4096;   // 16 KiB of binary32 per block
constexpr int STAGE_SLOTS = 64;
constexpr int STAGE_REUSE = 4;

__device__ __forceinline__ int wave_min(int v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = min(v, __shfl_xor(v, off, 64));
    return v;
}

__device__ __forceinline__ int wave_max(int v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off, 64));
    return v;
}

template <int FMT, int KIND>
__global__ __launch_bounds__(BLOCK) void k_grid_det_staged(GridView g, const float* __restrict__ q, int32_t n,
                                                           float* __restrict__ out, const int32_t* __restrict__ order,
                                                           int scatter, unsigned long long* __restrict__ counters)
{
    constexpr int NT = KIND == KIND_LINEAR ? 2 : 4;
    __shared__ float tile[STAGE_VOXELS];
    __shared__ int32_t slot_leaf[STAGE_SLOTS];
    __shared__ int box[6][BLOCK / 64];
    const int32_t i = blockIdx.x * BLOCK + threadIdx.x;
    const bool live = i < n;
    float p[3] = {0.0f, 0.0f, 0.0f};
    if (live) {
        p[0] = q[3 * (int64_t)i];
        p[1] = q[3 * (int64_t)i + 1];
        p[2] = q[3 * (int64_t)i + 2];
    }
    int base[3];
    float w[3][4];
    const bool ok = live && det_setup<KIND>(p, base, w);
    // bounding box of the block's tap blocks (queries with a cell only)
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int mn = wave_min(ok ? base[a] : INT_MAX), mx = wave_max(ok ? base[a] + NT - 1 : INT_MIN);
        if (lane == 0) {
            box[a][wave] = mn;
            box[3 + a][wave] = mx;
        }
    }
    const int nok = __syncthreads_count(ok);
    int lo[3], ext[3], l0[3], nl[3];
    bool fits = nok > 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        int mn = box[a][0], mx = box[3 + a][0];
#pragma unroll
        for (int k = 1; k < BLOCK / 64; ++k) {
            mn = min(mn, box[a][k]);
            mx = max(mx, box[3 + a][k]);
        }
        lo[a] = mn;
        ext[a] = fits ? mx - mn + 1 : 0;   // at most 2^25 + 4: coordinates with a cell are below 2^24
        l0[a] = mn >> 3;
        nl[a] = fits ? (mx >> 3) - l0[a] + 1 : 0;
        fits = fits && ext[a] <= STAGE_VOXELS && nl[a] <= STAGE_SLOTS;
    }
    const int64_t vol = (int64_t)ext[0] * ext[1] * ext[2];
    const int nslot = nl[0] * nl[1] * nl[2];
    // the same decision in every thread of the block
    bool stage = fits && vol <= STAGE_VOXELS && nslot <= STAGE_SLOTS &&
                 vol * STAGE_REUSE <= (int64_t)nok * NT * NT * NT;
    bool taps = false;   // this query's tap block meets a stored leaf
    if (stage) {
        if ((int)threadIdx.x < nslot) {
            const int sx = l0[0] + (int)threadIdx.x % nl[0], sy = l0[1] + ((int)threadIdx.x / nl[0]) % nl[1],
                      sz = l0[2] + (int)threadIdx.x / (nl[0] * nl[1]);
            slot_leaf[threadIdx.x] = in_domain(g, sx * 8, sy * 8, sz * 8) ? grid_leaf(g, sx * 8, sy * 8, sz * 8) : -1;
        }
        __syncthreads();
        if (ok) {
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const int sx = ((base[0] + ((k & 1) ? NT - 1 : 0)) >> 3) - l0[0];
                const int sy = ((base[1] + ((k & 2) ? NT - 1 : 0)) >> 3) - l0[1];
                const int sz = ((base[2] + ((k & 4) ? NT - 1 : 0)) >> 3) - l0[2];
                taps = taps || slot_leaf[(sz * nl[1] + sy) * nl[0] + sx] >= 0;
            }
        }
        // staging pays only for the queries that read texels; the others
        // (empty space) sum the background either way
        stage = (int64_t)__syncthreads_count(taps) * NT * NT * NT >= vol * STAGE_REUSE;
    }
    if (counters && threadIdx.x == 0) {   // {blocks that staged, blocks}, when counting is on
        if (stage) atomicAdd(&counters[0], 1ull);
        atomicAdd(&counters[1], 1ull);
    }
    if (stage) {
        // voxel v = threadIdx.x + k BLOCK of the box, x fastest; its
        // coordinates advance by those of BLOCK (one carry per axis at most)
        const int e01 = ext[0] * ext[1];
        const int sx = BLOCK % ext[0], sy = (BLOCK / ext[0]) % ext[1], sz = BLOCK / e01;
        int x = (int)threadIdx.x % ext[0], y = ((int)threadIdx.x / ext[0]) % ext[1], z = (int)threadIdx.x / e01;
        for (int v = threadIdx.x; v < (int)vol; v += BLOCK) {
            const int vx = lo[0] + x, vy = lo[1] + y, vz = lo[2] + z;
            const int32_t lf = slot_leaf[((vz >> 3) - l0[2]) * nl[1] * nl[0] + ((vy >> 3) - l0[1]) * nl[0] +
                                         (vx >> 3) - l0[0]];
            tile[v] = (lf >= 0 && in_domain(g, vx, vy, vz))
                          ? load_texel<FMT>(g.leaves, (int64_t)lf * 512 + leaf_offset(FMT, vx & 7, vy & 7, vz & 7))
                          : g.background;
            x += sx;
            y += sy;
            z += sz;
            if (x >= ext[0]) {
                x -= ext[0];
                ++y;
            }
            if (y >= ext[1]) {
                y -= ext[1];
                ++z;
            }
        }
        __syncthreads();
        if (!live) return;
        float acc = 0.0f;
        if (ok && !taps) {   // empty space
            acc = det_background<KIND>(g, w);
        } else if (ok) {
#pragma unroll
            for (int cz = 0; cz < NT; ++cz) {
                float plane = 0.0f;
#pragma unroll
                for (int cy = 0; cy < NT; ++cy) {
                    const float* r = tile + ((base[2] + cz - lo[2]) * ext[1] + (base[1] + cy - lo[1])) * ext[0] +
                                     (base[0] - lo[0]);
                    float row = 0.0f;
#pragma unroll
                    for (int cx = 0; cx < NT; ++cx) row = __builtin_fmaf(w[0][cx], r[cx], row);
                    plane = __builtin_fmaf(w[1][cy], row, plane);
                }
                acc = __builtin_fmaf(w[2][cz], plane, acc);
            }
        }
        __builtin_nontemporal_store(ok ? det_unscale<KIND>(acc) : __builtin_nanf(""), out + ((order && scatter) ? order[i] : i));
    } else {
        if (!live) return;
        __builtin_nontemporal_store(ok ? det_unscale<KIND>(det_sum_global<FMT, KIND>(g, base, w))
                                                    : __builtin_nanf(""), out + ((order && scatter) ? order[i] : i));
    }
}

// ---------------------------------------------------------------------------
// moments of the stochastic estimator over many seeds (binary64 sums)
// ---------------------------------------------------------------------------
template <int FMT, int KIND>
__global__ __launch_bounds__(BLOCK) void k_grid_moments(GridView g, const float* __restrict__ q, int32_t n,
                                                        uint64_t seed_base, int32_t n_seeds,
                                                        double* __restrict__ sum, double* __restrict__ sumsq)
{
    // one block per query; the seeds are split over the block's lanes and the
    // partial sums reduced in a fixed order (bitwise reproducible).
    __shared__ double s1[BLOCK], s2[BLOCK];
    int32_t i = blockIdx.x;
    float p0 = q[3 * (int64_t)i], p1 = q[3 * (int64_t)i + 1], p2 = q[3 * (int64_t)i + 2];
    int c0, c1, c2;
    float t0, t1, t2;
    bool ok = cell_of(p0, c0, t0) & cell_of(p1, c1, t1) & cell_of(p2, c2, t2);
    double a1 = 0.0, a2 = 0.0;
    if (ok) {
        for (int32_t k = threadIdx.x; k < n_seeds; k += BLOCK) {
            uint32_t b = pcg(seed_key(seed_base + (uint64_t)k) ^ (uint32_t)i);
            float e;
            if constexpr (KIND == KIND_KEYS || KIND == KIND_MITCHELL) {
                const float t[3] = {t0, t1, t2};
                const PosDraw<3> d = positivized_draw<3, KIND>(t, b);
                e = d.sp * grid_voxel<FMT>(g, c0 + d.op[0], c1 + d.op[1], c2 + d.op[2]);
                if (d.neg) e = e - d.sn * grid_voxel<FMT>(g, c0 + d.on[0], c1 + d.on[1], c2 + d.on[2]);
                e = e * inv_scale<3, KIND>();
            } else {
                float u0 = axis_uniform(b, 0), u1 = axis_uniform(b, 1), u2 = axis_uniform(b, 2);
                int v0, v1, v2;
                if constexpr (KIND == KIND_BSPLINE) {
                    v0 = c0 + choose_cubic(t0, u0); v1 = c1 + choose_cubic(t1, u1); v2 = c2 + choose_cubic(t2, u2);
                } else {
                    v0 = c0 + choose_linear(t0, u0); v1 = c1 + choose_linear(t1, u1); v2 = c2 + choose_linear(t2, u2);
                }
                e = grid_voxel<FMT>(g, v0, v1, v2);
            }
            double v = (double)e;
            a1 += v;
            a2 += v * v;
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

template <int FMT, int KIND>
void launch3d_kind(const GridView& g, const float* q, int32_t n, int mode, uint32_t key, float* out, int32_t* idx,
                   const int32_t* order, int scatter, hipStream_t stream)
{
    dim3 block(BLOCK);
    if (mode == STF_STOCHASTIC) {
        if constexpr (KIND == KIND_KEYS || KIND == KIND_MITCHELL) {
            constexpr int Q = 2;   // two taps per query: 2Q = 4 walks in lock step
            dim3 pgrid((unsigned)(((int64_t)n + BLOCK * Q - 1) / (BLOCK * Q)));
            hipLaunchKernelGGL((k_grid_positivized<FMT, KIND, Q>), pgrid, block, 0, stream, g, q, n, key, out, idx,
                               order, scatter);
        } else {
            constexpr int Q = STOCH_Q;
            dim3 sgrid((unsigned)(((int64_t)n + BLOCK * Q - 1) / (BLOCK * Q)));
            hipLaunchKernelGGL((k_grid_stochastic<FMT, KIND == KIND_BSPLINE, Q>), sgrid, block, 0, stream, g, q, n, key,
                               out, idx, order, scatter);
        }
    } else if (mode == STF_STOCHASTIC_FIS) {
        if constexpr (KIND == KIND_LINEAR || KIND == KIND_BSPLINE) {
            constexpr int Q = STOCH_Q;
            dim3 sgrid((unsigned)(((int64_t)n + BLOCK * Q - 1) / (BLOCK * Q)));
            hipLaunchKernelGGL((k_grid_fis<FMT, KIND == KIND_BSPLINE, Q>), sgrid, block, 0, stream, g, q, n, key, out,
                               idx, order, scatter);
        }
    } else {
        dim3 grid((n + BLOCK - 1) / BLOCK);
        if (order && KIND != KIND_LINEAR)   // a sorted stream: neighbouring queries share their 64 taps
            hipLaunchKernelGGL((k_grid_det_staged<FMT, KIND>), grid, block, 0, stream, g, q, n, out, order, scatter,
                               stage_counters());
        else
            hipLaunchKernelGGL((k_grid_deterministic<FMT, KIND>), grid, block, 0, stream, g, q, n, out, order, scatter);
    }
}

template <int FMT>
hipError_t launch3d_fmt(const GridView& g, const float* q, int32_t n, int filter, int mode, uint32_t key, float* out,
                        int32_t* idx, const int32_t* order, int scatter, hipStream_t stream)
{
    switch (filter) {
    case KIND_LINEAR: launch3d_kind<FMT, KIND_LINEAR>(g, q, n, mode, key, out, idx, order, scatter, stream); break;
    case KIND_BSPLINE: launch3d_kind<FMT, KIND_BSPLINE>(g, q, n, mode, key, out, idx, order, scatter, stream); break;
    case KIND_KEYS: launch3d_kind<FMT, KIND_KEYS>(g, q, n, mode, key, out, idx, order, scatter, stream); break;
    case KIND_MITCHELL: launch3d_kind<FMT, KIND_MITCHELL>(g, q, n, mode, key, out, idx, order, scatter, stream); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int FMT>
hipError_t moments3d_fmt(const GridView& g, const float* q, int32_t n, int filter, uint64_t seed_base,
                         int32_t n_seeds, double* sum, double* sumsq, hipStream_t stream)
{
    dim3 grid(n), block(BLOCK);
    switch (filter) {
    case KIND_LINEAR:
        hipLaunchKernelGGL((k_grid_moments<FMT, KIND_LINEAR>), grid, block, 0, stream, g, q, n, seed_base, n_seeds, sum,
                           sumsq);
        break;
    case KIND_BSPLINE:
        hipLaunchKernelGGL((k_grid_moments<FMT, KIND_BSPLINE>), grid, block, 0, stream, g, q, n, seed_base, n_seeds,
                           sum, sumsq);
        break;
    case KIND_KEYS:
        hipLaunchKernelGGL((k_grid_moments<FMT, KIND_KEYS>), grid, block, 0, stream, g, q, n, seed_base, n_seeds, sum,
                           sumsq);
        break;
    case KIND_MITCHELL:
        hipLaunchKernelGGL((k_grid_moments<FMT, KIND_MITCHELL>), grid, block, 0, stream, g, q, n, seed_base, n_seeds,
                           sum, sumsq);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int FMT>
hipError_t serve3d_fmt(const GridView& g, int filter, const ServeChunk* chunks, int32_t nchunks, int32_t nblocks,
                       hipStream_t s)
{
    if (filter == STF_CUBIC_BSPLINE)
        hipLaunchKernelGGL((k_grid_serve<FMT, true, STOCH_Q>), dim3(nblocks), dim3(BLOCK), 0, s, g, chunks, nchunks);
    else
        hipLaunchKernelGGL((k_grid_serve<FMT, false, STOCH_Q>), dim3(nblocks), dim3(BLOCK), 0, s, g, chunks, nchunks);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_filter3d(const stf_texture* tex, const float* q, int32_t n, int filter, int mode, uint32_t key,
                           float* out, int32_t* idx, const int32_t* order, int scatter, hipStream_t stream)
{
    const GridView& g = tex->grid;
    switch (tex->fmt) {
    case F32: return launch3d_fmt<F32>(g, q, n, filter, mode, key, out, idx, order, scatter, stream);
    case F16: return launch3d_fmt<F16>(g, q, n, filter, mode, key, out, idx, order, scatter, stream);
    case BF16: return launch3d_fmt<BF16>(g, q, n, filter, mode, key, out, idx, order, scatter, stream);
    case FP8_E4M3: return launch3d_fmt<FP8_E4M3>(g, q, n, filter, mode, key, out, idx, order, scatter, stream);
    case U8: return launch3d_fmt<U8>(g, q, n, filter, mode, key, out, idx, order, scatter, stream);
    }
    return hipErrorInvalidValue;
}

int32_t serve3d_queries_per_block()
{
    return BLOCK * STOCH_Q;
}

hipError_t launch_serve3d(const stf_texture* tex, int filter, const ServeChunk* chunks, int32_t nchunks,
                          int32_t nblocks, hipStream_t s)
{
    const GridView& g = tex->grid;
    switch (tex->fmt) {
    case F32: return serve3d_fmt<F32>(g, filter, chunks, nchunks, nblocks, s);
    case F16: return serve3d_fmt<F16>(g, filter, chunks, nchunks, nblocks, s);
    case BF16: return serve3d_fmt<BF16>(g, filter, chunks, nchunks, nblocks, s);
    case FP8_E4M3: return serve3d_fmt<FP8_E4M3>(g, filter, chunks, nchunks, nblocks, s);
    case U8: return serve3d_fmt<U8>(g, filter, chunks, nchunks, nblocks, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_moments3d(const stf_texture* tex, const float* q, int32_t n, int filter, uint64_t seed_base,
                            int32_t n_seeds, double* sum, double* sumsq, hipStream_t stream)
{
    const GridView& g = tex->grid;
    switch (tex->fmt) {
    case F32: return moments3d_fmt<F32>(g, q, n, filter, seed_base, n_seeds, sum, sumsq, stream);
    case F16: return moments3d_fmt<F16>(g, q, n, filter, seed_base, n_seeds, sum, sumsq, stream);
    case BF16: return moments3d_fmt<BF16>(g, q, n, filter, seed_base, n_seeds, sum, sumsq, stream);
    case FP8_E4M3: return moments3d_fmt<FP8_E4M3>(g, q, n, filter, seed_base, n_seeds, sum, sumsq, stream);
    case U8: return moments3d_fmt<U8>(g, q, n, filter, seed_base, n_seeds, sum, sumsq, stream);
    }
    return hipErrorInvalidValue;
}
