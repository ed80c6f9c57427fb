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

// Both draws of one query; h0 = pcg(key ^ qid) is the query's first hash.
template <int D, int KIND>
__device__ __forceinline__ PosDraw<D> positivized_draw(const float (&t)[D], uint32_t h0)
{
    constexpr int NP = 1 << (D - 1);   // patterns per sign set
    float part[2][D][4], mass[2][D];
#pragma unroll
    for (int a = 0; a < D; ++a) {
        float w[4];
        interp_weights<KIND>(t[a], w);
        mass[0][a] = 0.0f;
        mass[1][a] = 0.0f;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            part[0][a][k] = w[k] > 0.0f ? w[k] : 0.0f;
            part[1][a][k] = w[k] < 0.0f ? -w[k] : 0.0f;
            mass[0][a] += part[0][a][k];
            mass[1][a] += part[1][a][k];
        }
    }
    PosDraw<D> r;
#pragma unroll
    for (int set = 0; set < 2; ++set) {
        int pat[NP];
        float pm[NP];
        int np = 0;
#pragma unroll
        for (int b = 0; b < (1 << D); ++b) {
            if ((__builtin_popcount((unsigned)b) & 1) != set) continue;
            float m = mass[b & 1][0];
#pragma unroll
            for (int a = 1; a < D; ++a) m = m * mass[(b >> a) & 1][a];
            pat[np] = b;
            pm[np] = m;
            ++np;
        }
        float total = pm[0];
#pragma unroll
        for (int i = 1; i < NP; ++i) total += pm[i];
        const uint32_t ubase = set == 0 ? 0u : 5u, ucomp = set == 0 ? 4u : 8u;
        const int b = pat[cumulative_pick<NP>(pm, axis_uniform(h0, ucomp))];
#pragma unroll
        for (int a = 0; a < D; ++a) {
            const int sel = (b >> a) & 1;
            float pa[4] = {part[sel][a][0], part[sel][a][1], part[sel][a][2], part[sel][a][3]};
            const int o = cumulative_pick<4>(pa, axis_uniform(h0, ubase + (uint32_t)a)) - 1;
            if (set == 0) r.op[a] = o;
            else r.on[a] = o;
        }
        if (set == 0) r.sp = total;
        else {
            r.sn = total;
            r.neg = total > 0.0f;
        }
    }
    return r;
}

// 1 / axis_scale^D as a binary32 constant.
template <int D, int KIND>
constexpr float inv_scale()
{
    return D == 2 ? 1.0f / (axis_scale<KIND>() * axis_scale<KIND>())
                  : 1.0f / (axis_scale<KIND>() * axis_scale<KIND>() * axis_scale<KIND>());
}

}  // namespace stf
