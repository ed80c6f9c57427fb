// ewa.hip -- elliptically weighted average filtering over a MIP pyramid,
// deterministic and stochastic (section "B-Spline and Anisotropic Filters":
// a stochastic choice of MIP level from the ellipse's extent, then one tap
// drawn in proportion to the EWA weights; supplement, "Stochastic sampling of
// the EWA kernel", which follows pbrt's EWA lookup).
//
// A query is (s, t, ds/dx, dt/dx, ds/dy, dt/dy) in [0, 1] texture units.
//  - Axes (binary32): the longer derivative vector is the major axis; the
//    shorter is raised to longer / max_aniso if it is shorter than that.
//  - lod = max(0, (levels - 1) + log2(shorter)) in binary64; deterministic:
//    lerp(lod - floor(lod), EWA(floor(lod)), EWA(floor(lod) + 1)); stochastic:
//    level floor(lod) + [u0 < lod - floor(lod)] (hash index 0), then one tap.
//  - EWA on a level (binary32, each operation rounded once in this order):
//    A = (d0y^2 + d1y^2) + 1, B = -2 (d0x d0y + d1x d1y), C = (d0x^2 + d1x^2)
//    + 1 with the derivatives in texels; A, B, C divided by F = A C -
//    B^2 / 4; the bounding box st +- 2 sqrt(det C) / det (x), +- 2 sqrt(A det)
//    / det (y), det = -B^2 + 4 A C; taps with r2 = A ss^2 + B ss tt + C tt^2
//    < 1 weigh LUT[min(floor(128 r2), 127)], LUT[i] = exp(-2 i/127) -
//    exp(-2).  The stochastic tap: a row by weighted reservoir sampling over
//    the row sums, then a tap of the row by the cumulative rule (ewa_draw).
//    The kernels keep 128 A, 128 B and 128 C, so that each tap forms 128 r2
//    directly: every operation's result is 128 times the unscaled one,
//    exactly (the scale is a power of two, and no intermediate comes near the
//    subnormal or overflow range on a scanned level, where the coefficients
//    are at most 1 in magnitude and the box at most a few hundred texels).
//  - A zero footprint reads bilinearly from level 0 (stochastic: the linear
//    draw with hash indices 2, 3).  The pyramid ends at one texel, and a
//    level at or past that last one yields that texel (pbrt's rule): the
//    ellipse is only scanned on levels where its minor axis spans fewer
//    than 4 texels, so a query's box holds O(max_aniso) taps.
// Taps are clamped to their level.
#include <math.h>

#include <new>

#include "device_common.h"
#include "interp.h"
#include "stf_internal.h"

using namespace stf;

namespace {

constexpr int BLOCK = 256;
constexpr int LUT_SIZE = 129;   // 128 weights, then +0 for taps outside the ellipse

struct EwaLevels {
    TexLevel level[STF_MAX_LEVELS];
    int32_t levels;
};

struct EwaLut {
    float v[LUT_SIZE];
};

EwaLut make_lut()
{
    EwaLut L;
    for (int i = 0; i < 128; ++i) L.v[i] = (float)(std::exp(-2.0 * i / 127.0) - std::exp(-2.0));
    L.v[128] = 0.0f;
    return L;
}

__device__ __forceinline__ int clampi(int v, int hi)
{
    return v < 0 ? 0 : (v > hi ? hi : v);
}

template <int FMT, int C>
__device__ __forceinline__ void texel(const TexLevel& L, int x, int y, float (&v)[C])
{
    const int64_t e = ((int64_t)clampi(y, L.h - 1) * L.w + clampi(x, L.w - 1)) * C;
    if constexpr (FMT == F32 && C == 4) {
        const float4 f = reinterpret_cast<const float4*>(L.texels)[e >> 2];
        v[0] = f.x; v[1] = f.y; v[2] = f.z; v[3] = f.w;
    } else {
#pragma unroll
        for (int c = 0; c < C; ++c) v[c] = load_texel<FMT>(L.texels, e + c);
    }
}

// The ellipse of one level in texel units: coefficients and bounding box.
struct Ellipse {
    float stx, sty, A, B, C;
    int s0, s1, t0, t1;
};

__device__ __forceinline__ Ellipse ellipse(const TexLevel& L, float s, float t, const float (&d0)[2],
                                           const float (&d1)[2])
{
    Ellipse e;
    const float W = (float)L.w, H = (float)L.h;
    e.stx = s * W - 0.5f;
    e.sty = t * H - 0.5f;
    const float d0x = d0[0] * W, d0y = d0[1] * H, d1x = d1[0] * W, d1y = d1[1] * H;
    float A = (d0y * d0y + d1y * d1y) + 1.0f;
    float B = -2.0f * (d0x * d0y + d1x * d1y);
    float C = (d0x * d0x + d1x * d1x) + 1.0f;
    const float invF = 1.0f / (A * C - (B * B) * 0.25f);
    A *= invF;
    B *= invF;
    C *= invF;
    const float det = -(B * B) + 4.0f * A * C;
    const float invDet = 1.0f / det;
    const float us = sqrtf(fmaxf(det * C, 0.0f)), vs = sqrtf(fmaxf(A * det, 0.0f));
    e.s0 = (int)ceilf(e.stx - 2.0f * invDet * us);
    e.s1 = (int)floorf(e.stx + 2.0f * invDet * us);
    e.t0 = (int)ceilf(e.sty - 2.0f * invDet * vs);
    e.t1 = (int)floorf(e.sty + 2.0f * invDet * vs);
    e.A = A * 128.0f;   // exact: the taps form 128 r2
    e.B = B * 128.0f;
    e.C = C * 128.0f;
    return e;
}

// The weight of a tap whose quadratic form is r2, given r2s = 128 r2, without
// a branch: min(r2s, 128) (NaN gives 128), then max with 0 (r2 is never
// negative beyond rounding; trunc of a value in (-1, 0) is 0 as well),
// truncated: 0..127 inside the ellipse, 128 -- the entry +0 -- outside.
// Every LUT entry is >= +0, so adding a weight of +0 leaves a running sum's
// bits unchanged.
__device__ __forceinline__ int lut_index(float r2s)
{
    return (int)fmaxf(fminf(r2s, 128.0f), 0.0f);
}

__device__ __forceinline__ float lut_weight(const float* lut, float r2s)
{
    return lut[lut_index(r2s)];
}

__device__ __forceinline__ float ewa_weight(const Ellipse& e, const float* lut, int is, int it)
{
    const float ss = (float)is - e.stx, tt = (float)it - e.sty;
    return lut_weight(lut, (e.A * (ss * ss) + (e.B * ss) * tt) + e.C * (tt * tt));
}

// The EWA mean of one level: sum w t / sum w over the taps of the box with
// w > 0, two rows at a time (a column's A ss^2 and B ss serve both rows;
// every weight keeps its order of operations, the sums interleave the two
// rows' taps).
template <int FMT, int C>
__device__ __forceinline__ void ewa_mean(const TexLevel& L, const Ellipse& e, const float* lut, float (&v)[C])
{
    float acc[C], wsum = 0.0f;
#pragma unroll
    for (int c = 0; c < C; ++c) acc[c] = 0.0f;
    for (int it = e.t0; it <= e.t1; it += 2) {
        const bool two = it + 1 <= e.t1;
        const float ta = (float)it - e.sty, tb = (float)(it + 1) - e.sty;
        const float ca = e.C * (ta * ta), cb = e.C * (tb * tb);
        for (int is = e.s0; is <= e.s1; ++is) {
            const float ss = (float)is - e.stx;
            const float P = e.A * (ss * ss), Q = e.B * ss;
            const float wa = lut_weight(lut, (P + Q * ta) + ca);
            const float wb = two ? lut_weight(lut, (P + Q * tb) + cb) : 0.0f;
            if (wa > 0.0f) {
                float t[C];
                texel<FMT, C>(L, is, it, t);
                wsum += wa;
#pragma unroll
                for (int c = 0; c < C; ++c) acc[c] = __builtin_fmaf(wa, t[c], acc[c]);
            }
            if (wb > 0.0f) {
                float t[C];
                texel<FMT, C>(L, is, it + 1, t);
                wsum += wb;
#pragma unroll
                for (int c = 0; c < C; ++c) acc[c] = __builtin_fmaf(wb, t[c], acc[c]);
            }
        }
    }
#pragma unroll
    for (int c = 0; c < C; ++c) v[c] = acc[c] / wsum;
}

// The stochastic tap: a row of the box by weighted reservoir sampling over
// the row sums R_k (binary32, scan order; row k replaces the choice iff
// u_(16+k) * S < R_k, S the running sum of row sums), then a tap of that row
// by the cumulative rule (T = u1 R, the first tap whose running sum exceeds
// T).  The box is scanned two rows at a time: a column's A ss^2 and B ss
// serve both rows (each tap's r2 keeps its order of operations, so every
// weight and every row sum has the bits of a row-by-row scan).
__device__ __forceinline__ void ewa_draw(const Ellipse& e, const float* lut, uint32_t b, float u1, int& tx, int& ty)
{
    const uint32_t base = pcg_base(b);
    float S = 0.0f, Rsel = 0.0f;
    int rsel = e.t0;
    bool found = false;
    auto offer = [&](int it, float R) {   // row `it` with sum R enters the reservoir
        if (!(R > 0.0f)) return;
        S += R;
        if (uniform_from_base(base, 16u + (uint32_t)(it - e.t0)) * S < R) {
            rsel = it;
            Rsel = R;
            found = true;
        }
    };
    for (int it = e.t0; it <= e.t1; it += 2) {
        const float ta = (float)it - e.sty, tb = (float)(it + 1) - e.sty;
        const float ca = e.C * (ta * ta), cb = e.C * (tb * tb);
        // Two columns at a time, software-pipelined: the LUT indices of the
        // next pair of columns are formed while this pair's four LDS reads
        // are in flight.  A column past the box gets P = +inf, hence the
        // weight +0, which leaves the sums' bits unchanged.
        auto indices = [&](int is, int (&k)[4]) {
            const float ss0 = (float)is - e.stx, ss1 = (float)(is + 1) - e.stx;
            const float P0 = is <= e.s1 ? e.A * (ss0 * ss0) : __builtin_inff(), Q0 = e.B * ss0;
            const float P1 = is + 1 <= e.s1 ? e.A * (ss1 * ss1) : __builtin_inff(), Q1 = e.B * ss1;
            k[0] = lut_index((P0 + Q0 * ta) + ca);
            k[1] = lut_index((P0 + Q0 * tb) + cb);
            k[2] = lut_index((P1 + Q1 * ta) + ca);
            k[3] = lut_index((P1 + Q1 * tb) + cb);
        };
        int k[4];
        indices(e.s0, k);
        float w0 = lut[k[0]], w1 = lut[k[1]], w2 = lut[k[2]], w3 = lut[k[3]];
        float Ra = 0.0f, Rb = 0.0f;
        for (int is = e.s0 + 2; is <= e.s1; is += 2) {
            int kn[4];
            indices(is, kn);
            Ra += w0;   // column is - 2, then is - 1, of each row: scan order
            Rb += w1;
            Ra += w2;
            Rb += w3;
            w0 = lut[kn[0]];
            w1 = lut[kn[1]];
            w2 = lut[kn[2]];
            w3 = lut[kn[3]];
        }
        Ra += w0;
        Rb += w1;
        Ra += w2;
        Rb += w3;
        offer(it, Ra);
        if (it + 1 <= e.t1) offer(it + 1, Rb);
    }
    tx = e.s0;
    ty = rsel;
    if (!found) return;
    const float T = u1 * Rsel;
    float run = 0.0f;
    for (int is = e.s0; is <= e.s1; ++is) {
        const float w = ewa_weight(e, lut, is, rsel);
        if (!(w > 0.0f)) continue;
        run += w;
        tx = is;   // the last tap with weight, if the running sum never exceeds T
        if (T < run) return;
    }
}

// Loads query i and forms its axes (binary32): the longer derivative is d0,
// the shorter d1 is raised to |d0| / max_aniso when it is shorter than that
// (and not zero); sh = |d1|.  False for a record with a non-finite entry or
// one of magnitude >= 65536, and for one whose raster position on level 0
// (s W0 - 1/2, t H0 - 1/2) is not below 2^24 in magnitude, the bound of
// every 2D filter: the coarser levels' positions are no larger, so every
// cell, box bound and tap column of the query fits an int.
__device__ __forceinline__ bool ewa_axes(const float* __restrict__ q, int32_t i, const TexLevel& L0,
                                         float max_aniso, float (&r)[6], float (&d0)[2], float (&d1)[2], float& sh)
{
#pragma unroll
    for (int j = 0; j < 6; ++j) r[j] = q[6 * (int64_t)i + j];
    bool ok = true;
#pragma unroll
    for (int j = 0; j < 6; ++j) ok = ok && (__builtin_fabsf(r[j]) < 65536.0f);
    ok = ok && __builtin_fabsf(r[0] * (float)L0.w - 0.5f) < 16777216.0f &&
         __builtin_fabsf(r[1] * (float)L0.h - 0.5f) < 16777216.0f;
    if (!ok) return false;
    d0[0] = r[2]; d0[1] = r[3];
    d1[0] = r[4]; d1[1] = r[5];
    if (d0[0] * d0[0] + d0[1] * d0[1] < d1[0] * d1[0] + d1[1] * d1[1]) {
        const float a = d0[0], b = d0[1];
        d0[0] = d1[0]; d0[1] = d1[1];
        d1[0] = a; d1[1] = b;
    }
    const float longer = sqrtf(d0[0] * d0[0] + d0[1] * d0[1]);
    sh = sqrtf(d1[0] * d1[0] + d1[1] * d1[1]);
    if (sh * max_aniso < longer && sh > 0.0f) {
        const float scale = longer / (sh * max_aniso);
        d1[0] *= scale;
        d1[1] *= scale;
        sh *= scale;
    }
    return true;
}

__device__ __forceinline__ double ewa_lod(int levels, float sh)
{
    const double lod = (double)(levels - 1) + log2((double)sh);
    return lod < 0.0 ? 0.0 : lod;
}

// The stochastic level: floor(lod) + [u0 < lod - floor(lod)] with lod of
// binary64 (ewa_lod), capped at the last level.  The hardware binary32 log2
// (error below 1e-5 in lod here) settles both decisions -- the floor and the
// comparison with u0 -- whenever lod, its fraction and u0 - fraction are more
// than 1e-4 away from a decision boundary; the rest (about 5e-4 of the
// queries) takes the binary64 path, so the level is the binary64 rule's.
__device__ __forceinline__ int ewa_draw_level(int levels, float sh, float u0)
{
    const float lod32 = (float)(levels - 1) + __builtin_amdgcn_logf(sh);
    const float fl = floorf(lod32), fr = lod32 - fl;
    int l;
    if (lod32 < -1e-4f) {
        l = 0;
    } else if (lod32 > 1e-4f && fr > 1e-4f && fr < 1.0f - 1e-4f && __builtin_fabsf(u0 - fr) > 1e-4f) {
        l = (int)fl + (u0 < fr ? 1 : 0);
    } else {
        const double lod = ewa_lod(levels, sh);
        const int il = (int)floor(lod);
        l = il + ((double)u0 < lod - (double)il ? 1 : 0);
    }
    return l > levels - 1 ? levels - 1 : l;
}

// Deterministic EWA: lerp of the EWA means of levels floor(lod) and
// floor(lod) + 1 (a level at or past the last reads its single texel); a
// zero footprint reads bilinearly from level 0.
template <int FMT, int C>
__global__ __launch_bounds__(BLOCK) void k_ewa_det(EwaLevels P, EwaLut lut_in, const float* __restrict__ q,
                                                   int32_t n, float max_aniso, float* __restrict__ out)
{
    __shared__ float lut[LUT_SIZE];
    for (int k = threadIdx.x; k < LUT_SIZE; k += BLOCK) lut[k] = lut_in.v[k];
    __syncthreads();
    const int32_t i = blockIdx.x * BLOCK + threadIdx.x;
    if (i >= n) return;
    float r[6], d0[2], d1[2], sh = 0.0f;
    float v[C];
    if (!ewa_axes(q, i, P.level[0], max_aniso, r, d0, d1, sh)) {
#pragma unroll
        for (int c = 0; c < C; ++c) v[c] = __builtin_nanf("");
    } else if (!(sh > 0.0f)) {
        const TexLevel& T0 = P.level[0];
        const float x = r[0] * (float)T0.w - 0.5f, y = r[1] * (float)T0.h - 0.5f;
        int cx = 0, cy = 0;
        float tx = 0.0f, ty = 0.0f;
        (void)cell_of(x, cx, tx);   // inside the raster bound ewa_axes checked
        (void)cell_of(y, cy, ty);
        float a[C], b[C], c2[C], d[C];
        texel<FMT, C>(T0, cx, cy, a);
        texel<FMT, C>(T0, cx + 1, cy, b);
        texel<FMT, C>(T0, cx, cy + 1, c2);
        texel<FMT, C>(T0, cx + 1, cy + 1, d);
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const float r0 = __builtin_fmaf(tx, b[c], (1.0f - tx) * a[c]);
            const float r1 = __builtin_fmaf(tx, d[c], (1.0f - tx) * c2[c]);
            v[c] = __builtin_fmaf(ty, r1, (1.0f - ty) * r0);
        }
    } else {
        const int L = P.levels;
        const double lod = ewa_lod(L, sh);
        const int il = (int)floor(lod);
        const double frac = lod - (double)il;
        const int l0 = il < L ? il : L - 1, l1 = il + 1 < L ? il + 1 : L - 1;
        float a[C], c1[C];
        if (l0 < L - 1)
            ewa_mean<FMT, C>(P.level[l0], ellipse(P.level[l0], r[0], r[1], d0, d1), lut, a);
        else
            texel<FMT, C>(P.level[l0], 0, 0, a);
        if (l1 < L - 1)
            ewa_mean<FMT, C>(P.level[l1], ellipse(P.level[l1], r[0], r[1], d0, d1), lut, c1);
        else
            texel<FMT, C>(P.level[l1], 0, 0, c1);
#pragma unroll
        for (int c = 0; c < C; ++c) v[c] = (float)((1.0 - frac) * (double)a[c] + frac * (double)c1[c]);
    }
#pragma unroll
    for (int c = 0; c < C; ++c) __builtin_nontemporal_store(v[c], out + (int64_t)i * C + c);   // streamed out
}

// Stochastic EWA in two phases.  Phase 1 (a thread per query): the level
// draw (hash index 0) and the ellipse of the drawn level; queries with no
// ellipse to scan (non-finite, zero footprint, last level) finish here.
// Neighbouring pixels draw different levels, whose boxes differ about 4x in
// size, so a wave scanning its own queries' boxes idles about half its lanes.
// Phase 2 regroups the block's scans by box height (a counting sort over LDS
// slots; the slot a query lands in does not change its result) so that each
// wave scans boxes of similar size, then draws the tap (ewa_draw) and reads
// it; the results go back through LDS to their queries' threads, which write
// them in query order.
constexpr int EWA_HEIGHT_KEYS = 64;   // box heights 0..62, 63 and more share the last key

struct EwaScanSlots {
    float stx[BLOCK], sty[BLOCK], A[BLOCK], B[BLOCK], C[BLOCK];
    int s0[BLOCK], s1[BLOCK], t0[BLOCK], t1[BLOCK], level[BLOCK], query[BLOCK];
    uint32_t b[BLOCK];
};

// A scanned query's result, returned to the query's own thread.
template <int C>
struct EwaResults {
    float v[BLOCK * C];
    int ix[BLOCK], iy[BLOCK], il[BLOCK];
};

template <int C>
__device__ __forceinline__ void ewa_store(float* __restrict__ out, int32_t* __restrict__ idx, int32_t i,
                                          const float (&v)[C], const int (&ix)[3])
{
#pragma unroll
    for (int c = 0; c < C; ++c) __builtin_nontemporal_store(v[c], out + (int64_t)i * C + c);   // streamed out
    if (idx) {
#pragma unroll
        for (int k = 0; k < 3; ++k) idx[3 * (int64_t)i + k] = ix[k];
    }
}

template <int FMT, int C>
__global__ __launch_bounds__(BLOCK) void k_ewa_stoch(EwaLevels P, EwaLut lut_in, const float* __restrict__ q,
                                                     int32_t n, float max_aniso, uint32_t key, float* __restrict__ out,
                                                     int32_t* __restrict__ idx)
{
    __shared__ float lut[LUT_SIZE];
    __shared__ int bucket[EWA_HEIGHT_KEYS];
    __shared__ EwaScanSlots S;
    __shared__ EwaResults<C> R;
    for (int k = threadIdx.x; k < LUT_SIZE; k += BLOCK) lut[k] = lut_in.v[k];
    if (threadIdx.x < EWA_HEIGHT_KEYS) bucket[threadIdx.x] = 0;
    __syncthreads();

    // phase 1
    const int32_t i = blockIdx.x * BLOCK + threadIdx.x;
    bool scan = false;
    Ellipse e{};
    int l = 0;
    uint32_t b = 0;
    if (i < n) {
        float r[6], d0[2], d1[2], sh = 0.0f;
        float v[C];
        int ix[3] = {BAD_INDEX, BAD_INDEX, BAD_INDEX};
        if (!ewa_axes(q, i, P.level[0], max_aniso, r, d0, d1, sh)) {
#pragma unroll
            for (int c = 0; c < C; ++c) v[c] = __builtin_nanf("");
        } else {
            b = pcg(key ^ (uint32_t)i);
            const int L = P.levels;
            if (!(sh > 0.0f)) {   // degenerate footprint: the bilinear draw on level 0
                const TexLevel& T0 = P.level[0];
                const float x = r[0] * (float)T0.w - 0.5f, y = r[1] * (float)T0.h - 0.5f;
                int cx = 0, cy = 0;
                float tx = 0.0f, ty = 0.0f;
                (void)cell_of(x, cx, tx);   // inside the raster bound ewa_axes checked
                (void)cell_of(y, cy, ty);
                ix[0] = clampi(cx + choose_linear(tx, axis_uniform(b, 2)), T0.w - 1);
                ix[1] = clampi(cy + choose_linear(ty, axis_uniform(b, 3)), T0.h - 1);
                ix[2] = 0;
                texel<FMT, C>(T0, ix[0], ix[1], v);
            } else {
                l = ewa_draw_level(L, sh, axis_uniform(b, 0));
                if (l < L - 1) {
                    e = ellipse(P.level[l], r[0], r[1], d0, d1);
                    scan = true;
                } else {   // the last level: its single texel
                    ix[0] = 0;
                    ix[1] = 0;
                    ix[2] = l;
                    texel<FMT, C>(P.level[l], 0, 0, v);
                }
            }
        }
        if (!scan) ewa_store<C>(out, idx, i, v, ix);
    }

    // phase 2: counting sort of the block's queries by box height
    int k = 0;
    if (scan) {
        const int rows = e.t1 - e.t0 + 1;
        k = rows < 0 ? 0 : (rows > EWA_HEIGHT_KEYS - 1 ? EWA_HEIGHT_KEYS - 1 : rows);
    }
    const int rank = atomicAdd(&bucket[k], 1);
    __syncthreads();
    if (threadIdx.x < EWA_HEIGHT_KEYS) {   // wave 0: exclusive prefix of the bucket sizes
        const int c = bucket[threadIdx.x];
        int x = c;
#pragma unroll
        for (int d = 1; d < EWA_HEIGHT_KEYS; d <<= 1) {
            const int y = __shfl_up(x, d, EWA_HEIGHT_KEYS);
            if ((int)threadIdx.x >= d) x += y;
        }
        bucket[threadIdx.x] = x - c;
    }
    __syncthreads();
    const int slot = bucket[k] + rank;   // a permutation of 0..BLOCK-1
    S.query[slot] = scan ? i : -1;
    if (scan) {
        S.stx[slot] = e.stx; S.sty[slot] = e.sty;
        S.A[slot] = e.A; S.B[slot] = e.B; S.C[slot] = e.C;
        S.s0[slot] = e.s0; S.s1[slot] = e.s1; S.t0[slot] = e.t0; S.t1[slot] = e.t1;
        S.level[slot] = l;
        S.b[slot] = b;
    }
    __syncthreads();
    const int t = threadIdx.x;
    const int32_t j = S.query[t];
    if (j >= 0) {
        Ellipse f;
        f.stx = S.stx[t]; f.sty = S.sty[t];
        f.A = S.A[t]; f.B = S.B[t]; f.C = S.C[t];
        f.s0 = S.s0[t]; f.s1 = S.s1[t]; f.t0 = S.t0[t]; f.t1 = S.t1[t];
        const int lj = S.level[t];
        const uint32_t bj = S.b[t];
        int tx = 0, ty = 0;
        ewa_draw(f, lut, bj, axis_uniform(bj, 1), tx, ty);
        const int tx_c = clampi(tx, P.level[lj].w - 1), ty_c = clampi(ty, P.level[lj].h - 1);
        float v[C];
        texel<FMT, C>(P.level[lj], tx_c, ty_c, v);
        // back to the query's own thread, so that the block's results are
        // written in query order (one contiguous span, full lines)
        const int o = j - (int32_t)blockIdx.x * BLOCK;
#pragma unroll
        for (int c = 0; c < C; ++c) R.v[o * C + c] = v[c];
        R.ix[o] = tx_c;
        R.iy[o] = ty_c;
        R.il[o] = lj;
    }
    __syncthreads();
    if (scan) {
        const int o = threadIdx.x;
        float v[C];
#pragma unroll
        for (int c = 0; c < C; ++c) v[c] = R.v[o * C + c];
        const int ix[3] = {R.ix[o], R.iy[o], R.il[o]};
        ewa_store<C>(out, idx, i, v, ix);
    }
}

template <int FMT, int C>
hipError_t launch_ewa_fc(const EwaLevels& P, const float* q, int32_t n, float max_aniso, int mode, uint32_t key,
                         float* out, int32_t* idx, hipStream_t s)
{
    static const EwaLut lut = make_lut();
    dim3 grid((n + BLOCK - 1) / BLOCK), block(BLOCK);
    if (mode == STF_STOCHASTIC)
        hipLaunchKernelGGL((k_ewa_stoch<FMT, C>), grid, block, 0, s, P, lut, q, n, max_aniso, key, out, idx);
    else
        hipLaunchKernelGGL((k_ewa_det<FMT, C>), grid, block, 0, s, P, lut, q, n, max_aniso, out);
    return hipGetLastError();
}

template <int FMT>
hipError_t launch_ewa_f(const EwaLevels& P, int C, const float* q, int32_t n, float max_aniso, int mode, uint32_t key,
                        float* out, int32_t* idx, hipStream_t s)
{
    switch (C) {
    case 1: return launch_ewa_fc<FMT, 1>(P, q, n, max_aniso, mode, key, out, idx, s);
    case 2: return launch_ewa_fc<FMT, 2>(P, q, n, max_aniso, mode, key, out, idx, s);
    case 3: return launch_ewa_fc<FMT, 3>(P, q, n, max_aniso, mode, key, out, idx, s);
    case 4: return launch_ewa_fc<FMT, 4>(P, q, n, max_aniso, mode, key, out, idx, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace

extern "C" stf_status stf_filter_ewa(const stf_texture* tex, const float* queries_dev, int64_t n, float max_anisotropy,
                                     stf_mode mode, uint64_t seed, float* out_dev, int32_t* out_index_dev,
                                     void* hip_stream)
{
    stf_clear_error();
    if (!tex) return stf_fail(STF_E_INVALID, "texture is NULL");
    if (tex->kind != STF_KIND_TEX2D) return stf_fail(STF_E_INVALID, "stf_filter_ewa needs a 2D texture (with levels)");
    if (n < 0 || n > 0x7fffffff) return stf_fail(STF_E_INVALID, "n = %lld out of range", (long long)n);
    if (!(max_anisotropy >= 1.0f && max_anisotropy <= 64.0f))
        return stf_fail(STF_E_INVALID, "max_anisotropy = %g out of range [1, 64]", (double)max_anisotropy);
    if (tex->level[tex->levels - 1].w != 1 || tex->level[tex->levels - 1].h != 1)
        return stf_fail(STF_E_INVALID, "stf_filter_ewa needs the full MIP pyramid (its last level %dx%d is not 1x1)",
                        tex->level[tex->levels - 1].w, tex->level[tex->levels - 1].h);
    if (mode != STF_DETERMINISTIC && mode != STF_STOCHASTIC) return stf_fail(STF_E_INVALID, "unknown mode %d", (int)mode);
    if (mode == STF_DETERMINISTIC && out_index_dev)
        return stf_fail(STF_E_INVALID, "out_index_dev must be NULL in deterministic mode");
    if (n == 0) return STF_OK;
    hipPointerAttribute_t attr;
    for (const void* p : {(const void*)queries_dev, (const void*)out_dev, (const void*)out_index_dev}) {
        if (!p) continue;
        if ((uintptr_t)p % 4) return stf_fail(STF_E_INVALID, "a device buffer is not 4-byte aligned");
        if (hipPointerGetAttributes(&attr, p) != hipSuccess ||
            (attr.type != hipMemoryTypeDevice && attr.type != hipMemoryTypeManaged)) {
            (void)hipGetLastError();
            return stf_fail(STF_E_INVALID, "queries, out and out_index must be device memory");
        }
    }
    if (!queries_dev || !out_dev) return stf_fail(STF_E_INVALID, "queries_dev or out_dev is NULL");
    EwaLevels P;
    for (int l = 0; l < STF_MAX_LEVELS; ++l) P.level[l] = tex->level[l];
    P.levels = tex->levels;
    hipStream_t st = (hipStream_t)hip_stream;
    const uint32_t key = seed_key(seed);
    hipError_t e = hipErrorInvalidValue;
    switch (tex->fmt) {
    case F32: e = launch_ewa_f<F32>(P, tex->channels, queries_dev, (int32_t)n, max_anisotropy, mode, key, out_dev, out_index_dev, st); break;
    case F16: e = launch_ewa_f<F16>(P, tex->channels, queries_dev, (int32_t)n, max_anisotropy, mode, key, out_dev, out_index_dev, st); break;
    case BF16: e = launch_ewa_f<BF16>(P, tex->channels, queries_dev, (int32_t)n, max_anisotropy, mode, key, out_dev, out_index_dev, st); break;
    case FP8_E4M3: e = launch_ewa_f<FP8_E4M3>(P, tex->channels, queries_dev, (int32_t)n, max_anisotropy, mode, key, out_dev, out_index_dev, st); break;
    case U8: e = launch_ewa_f<U8>(P, tex->channels, queries_dev, (int32_t)n, max_anisotropy, mode, key, out_dev, out_index_dev, st); break;
    }
    if (e != hipSuccess) return stf_fail(STF_E_DEVICE, "kernel launch failed: %s", hipGetErrorString(e));
    return STF_OK;
}
