// interp.h -- interpolating cubic filters with negative lobes and their
// positivized stochastic estimate (section "Sampling Techniques", paragraph
// on positivization; supplement, "The interpolating (negative lobe) bicubic
// filter" and "Filter Kernels").
//
// Kernels: KEYS is the cubic polynomial kernel K_3 with a = -1/2 (the
// Catmull-Rom spline; interpolating), MITCHELL the Mitchell-Netravali cubic
// with B = C = 1/3.  Taps i-1..i+2 of cell i sit at distances t+1, t, 1-t,
// 2-t from the sample.
//
// Estimate: the tensor-product weights w split into positive weights w+ and
// the magnitudes w- of the negative ones, masses S+ and S-.  One tap j+ is
// drawn with probability w+/S+ and one tap j- with probability w-/S-, and
// the result is S+ t(j+) - S- t(j-) (without the second term when S- = 0).
//
// Drawing: a tap is positive exactly when an even number of its per-axis
// weights is negative.  So w+ is a mixture, over the sign patterns with an
// even number of "negative" axes, of products of per-axis parts (positive
// part p_k = max(w_k, 0), negative part n_k = max(-w_k, 0)); w- is the same
// over the odd patterns.  A draw picks a pattern in proportion to the product
// of the per-axis masses of its parts, then one tap per axis in proportion to
// that axis's part: 4*D weights instead of 4^D.  Every choice among masses
// m_0..m_{k-1} uses one uniform u: T = u * M, M = ((m_0 + m_1) + ...), and
// the choice is the number of partial sums m_0 + ... + m_i (i < k-1) that are
// <= T, lowered to the last nonzero mass.  Patterns are numbered by their
// bits (bit a set: axis a takes its negative part), visited in increasing
// order, and a pattern's mass multiplies the axis masses from axis 0 up.
// Uniforms of a query: positive draw axes 0..D-1 and 4 (pattern), negative
// draw axes 5..5+D-1 and 8 (pattern).  Every decision is binary32 with one
// rounding per operation, so it has a unique answer for a given query and
// seed.
#pragma once

#include "device_common.h"

namespace stf {

enum FilterKind { KIND_LINEAR = 0, KIND_BSPLINE = 1, KIND_KEYS = 2, KIND_MITCHELL = 3 };

// The four per-axis weights of an interpolating cubic scaled by 2 (KEYS) or
// 18 (MITCHELL), in factored forms that keep a small relative error near
// every zero of a weight (s = 1 - t):
//   KEYS:      -(t s) s,  s (2 + t (2 - 3t)),  t (2 + s (2 - 3s)),  -(t t) s
//   MITCHELL:  (s s) fma(-7, t, 1),  1 + s (9 + s (27 - 21 s)),
//              1 + t (9 + t (27 - 21 t)),  (t t) fma(-7, s, 1)
template <int KIND>
__device__ __forceinline__ void interp_weights(float t, float (&w)[4])
{
    const float s = 1.0f - t;
    if constexpr (KIND == KIND_KEYS) {
        w[0] = -((t * s) * s);
        w[1] = s * (2.0f + t * (2.0f - 3.0f * t));
        w[2] = t * (2.0f + s * (2.0f - 3.0f * s));
        w[3] = -((t * t) * s);
    } else {
        w[0] = (s * s) * __builtin_fmaf(-7.0f, t, 1.0f);
        w[1] = 1.0f + s * (9.0f + s * (27.0f - 21.0f * s));
        w[2] = 1.0f + t * (9.0f + t * (27.0f - 21.0f * t));
        w[3] = (t * t) * __builtin_fmaf(-7.0f, s, 1.0f);
    }
}

// Scale of interp_weights (and of cubic6 for the B-spline) per axis.
template <int KIND>
constexpr float axis_scale()
{
    return KIND == KIND_KEYS ? 2.0f : (KIND == KIND_MITCHELL ? 18.0f : (KIND == KIND_BSPLINE ? 6.0f : 1.0f));
}

// Deterministic per-axis weights (scaled by axis_scale) and the offset of
// the first tap from the cell.
template <int KIND>
__device__ __forceinline__ int axis_weights_scaled(float t, float (&w)[4])
{
    if constexpr (KIND == KIND_LINEAR) {
        w[0] = 1.0f - t; w[1] = t; w[2] = 0.0f; w[3] = 0.0f;
        return 0;
    } else if constexpr (KIND == KIND_BSPLINE) {
        Cubic6 c = cubic6(t);
        w[0] = c.a0; w[1] = c.a1; w[2] = c.a2; w[3] = c.a3;
        return -1;
    } else {
        interp_weights<KIND>(t, w);
        return -1;
    }
}

// The cumulative choice among k masses (see the header comment).
template <int K>
__device__ __forceinline__ int cumulative_pick(const float (&m)[K], float u)
{
    float total = m[0];
    int last = 0;
#pragma unroll
    for (int i = 1; i < K; ++i) {
        total += m[i];
        if (m[i] > 0.0f) last = i;
    }
    const float T = u * total;
    float c = 0.0f;
    int j = 0;
#pragma unroll
    for (int i = 0; i < K - 1; ++i) {
        c += m[i];
        j += (T >= c) ? 1 : 0;
    }
    return j > last ? last : j;
}

template <int D>
struct PosDraw {
    int op[D];     // positive tap, offset -1..2 from the cell per axis
    int on[D];     // negative tap
    bool neg;      // a negative tap was drawn (S- > 0)
    float sp, sn;  // binary32 masses S+ and S-, scaled by axis_scale^D
};

// Sign patterns of each set in increasing order (bit a set: axis a takes
// its negative part): even patterns for w+, odd ones for w-.
template <int D>
__device__ __forceinline__ int pattern_bits(int set, int j)
{
    if constexpr (D == 2) return set == 0 ? (j == 0 ? 0 : 3) : (j == 0 ? 1 : 2);
    else
        return set == 0 ? (j == 0 ? 0 : (j == 1 ? 3 : (j == 2 ? 5 : 6)))
                        : (j == 0 ? 1 : (j == 1 ? 2 : (j == 2 ? 4 : 7)));
}

// Mass of pattern b: the per-axis masses multiplied from axis 0 up.
template <int D>
__device__ __forceinline__ float pattern_mass(const float (&P)[D], const float (&N)[D], int b)
{
    float m = (b & 1) ? N[0] : P[0];
#pragma unroll
    for (int a = 1; a < D; ++a) m = m * (((b >> a) & 1) ? N[a] : P[a]);
    return m;
}

// Per-axis draws from the positive and the negative part of the weights w
// (scaled), each the cumulative rule over the four taps, returning the tap
// offset -1..2.  Both kernels have positive inner weights (taps i, i+1), so
// the negative part lives on the outer taps only; with its zero middle
// masses the four-tap rule reduces exactly to a two-way choice between
// offsets -1 and +2 (the partial sums n0, n0 + 0, n0 + 0 coincide).  For
// KEYS the outer weights are never positive, and the positive part likewise
// reduces to a two-way choice between offsets 0 and +1.
template <int KIND>
__device__ __forceinline__ int pick_positive(const float (&w)[4], float P, float u)
{
    if constexpr (KIND == KIND_KEYS) {
        const float T = u * P;
        const int j = (T >= w[1]) ? 1 : 0;
        return (w[2] > 0.0f) ? j : 0;
    } else {
        float m[4] = {w[0] > 0.0f ? w[0] : 0.0f, w[1], w[2], w[3] > 0.0f ? w[3] : 0.0f};
        return cumulative_pick<4>(m, u) - 1;
    }
}

__device__ __forceinline__ int pick_negative(float n0, float n3, float N, float u)
{
    const float T = u * N;
    const bool upper = (T >= n0) && (n3 > 0.0f);
    return upper ? 2 : -1;
}

// The uniform of hash index a of a query, pcg(b + a), from base = pcg_base(b).
__device__ __forceinline__ float uniform_from_base(uint32_t base, uint32_t a)
{
    return hash_uniform(pcg_from_base(base, a));
}

// Both draws of one query; b = pcg(key ^ qid) is the query's base hash.
// All array indices are compile-time constants after unrolling; the pattern
// picked at run time only steers selects.
template <int D, int KIND>
__device__ __forceinline__ PosDraw<D> positivized_draw(const float (&t)[D], uint32_t b)
{
    constexpr int NP = 1 << (D - 1);   // patterns per sign set
    float w[D][4], n0[D], n3[D], P[D], N[D];
#pragma unroll
    for (int a = 0; a < D; ++a) {
        interp_weights<KIND>(t[a], w[a]);
        n0[a] = w[a][0] < 0.0f ? -w[a][0] : 0.0f;
        n3[a] = w[a][3] < 0.0f ? -w[a][3] : 0.0f;
        // masses in tap order, zero terms included where they can be nonzero
        if constexpr (KIND == KIND_KEYS) {
            P[a] = w[a][1] + w[a][2];
        } else {
            P[a] = (((w[a][0] > 0.0f ? w[a][0] : 0.0f) + w[a][1]) + w[a][2]) + (w[a][3] > 0.0f ? w[a][3] : 0.0f);
        }
        N[a] = n0[a] + n3[a];
    }
    const uint32_t base = pcg_base(b);
    PosDraw<D> r;
#pragma unroll
    for (int set = 0; set < 2; ++set) {
        float pm[NP];
#pragma unroll
        for (int j = 0; j < NP; ++j) pm[j] = pattern_mass<D>(P, N, pattern_bits<D>(set, j));
        float total = pm[0];
#pragma unroll
        for (int j = 1; j < NP; ++j) total += pm[j];
        const uint32_t ubase = set == 0 ? 0u : 5u, ucomp = set == 0 ? 4u : 8u;
        const int pat = pattern_bits<D>(set, cumulative_pick<NP>(pm, uniform_from_base(base, ucomp)));
#pragma unroll
        for (int a = 0; a < D; ++a) {
            const float u = uniform_from_base(base, ubase + (uint32_t)a);
            const int o = ((pat >> a) & 1) ? pick_negative(n0[a], n3[a], N[a], u) : pick_positive<KIND>(w[a], P[a], u);
            if (set == 0) r.op[a] = o;
            else r.on[a] = o;
        }
        if (set == 0) {
            r.sp = total;
        } else {
            r.sn = total;
            r.neg = total > 0.0f;
        }
    }
    return r;
}

// Filter importance sampling of the tent / cubic B-spline (section "Filter
// Importance Sampling"): jitter the position by a draw of the B-spline one
// degree lower -- a box (u - 1/2) for the tent, a quadratic B-spline (the sum
// of three uniforms minus 3/2) for the cubic -- and read the nearest texel
// floor(x' + 1/2), x' + 1/2 = x + s + 1/2 summed in binary64 in that order.
// Uniforms of axis a: hash index a (tent); a, 4 + a, 8 + a (cubic).
//
// With the uniforms as integers m = u 2^24 and K their sum (one uniform for
// the tent), s + 1/2 = K 2^-24 - c, c = 1 (cubic) or 0 (tent).  For |x| >=
// 2^-29 the binary64 sum is exact (x is binary32, K 2^-24 lies on the 2^-24
// grid and the result needs at most 53 bits), so the tap is floor(x + K 2^-24)
// - c, formed in binary32 and integers: with Y = x 2^24 (exact) and H =
// floor(x), R = floor(Y) - H 2^24 is an integer in [0, 2^24) that one fused
// multiply-add gives exactly, and floor(x + K 2^-24) = H + floor((R + K) /
// 2^24).  Below 2^-29 the binary64 sum can round x away, so it is evaluated
// as written.
template <bool CUBIC>
__device__ __forceinline__ int fis_tap(float x, uint32_t b, int a)
{
    const uint32_t base = pcg_base(b);
    const uint32_t ua = (uint32_t)a;
    auto m = [&](uint32_t k) { return pcg_from_base(base, k) >> 8; };
    const uint32_t K = CUBIC ? (m(ua) + m(4u + ua)) + m(8u + ua) : m(ua);
    if (__builtin_fabsf(x) >= 0x1p-29f) {
        const float yi = __builtin_floorf(x * 16777216.0f), h = __builtin_floorf(x);
        const uint32_t r = (uint32_t)__builtin_fmaf(h, -16777216.0f, yi);
        return (int)h - (CUBIC ? 1 : 0) + (int)((r + K) >> 24);
    }
    const double s = (double)K * 0x1p-24 - (CUBIC ? 1.5 : 0.5);   // exact: the rounded sums of the uniforms are too
    return (int)__builtin_floor((double)x + s + 0.5);
}

// 1 / axis_scale^D as a binary32 constant.
template <int D, int KIND>
constexpr float inv_scale()
{
    return D == 2 ? 1.0f / (axis_scale<KIND>() * axis_scale<KIND>())
                  : 1.0f / (axis_scale<KIND>() * axis_scale<KIND>() * axis_scale<KIND>());
}

}  // namespace stf
