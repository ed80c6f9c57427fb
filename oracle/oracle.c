/*
 * oracle.c -- plain, slow, obviously-correct CPU reference for stochastic
 * texture filtering (Fajardo, Wronski, Salvi, Pharr, "Stochastic Texture
 * Filtering", 2023).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * includes this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark load it.  It shares no code, header, table or constant
 * generator with the HIP path.
 *
 * Arithmetic conventions
 *   - Every filtered *value* (weights, sums, variances) is computed in IEEE
 *     binary64 from the exact binary32 query coordinate.
 *   - Every sampling *decision* (which tap is taken) is computed in pinned
 *     binary32: each operation rounded to nearest-even, subnormals kept, and
 *     no fused multiply-add except where fmaf() is written out (this file is
 *     compiled with -ffp-contract=off).  The decision therefore has one unique
 *     answer for a given query and seed.
 *   - Texels are decoded exactly from their storage format.
 *
 * Conventions where the paper leaves a choice (each is listed with its reason
 * in the design notes of the repository):
 *   - 2D raster position x = fl32(fl32(uv * W) - 0.5): texel centres sit at
 *     half-integers of uv*W, as in the paper's discrete Gaussian listing
 *     (supplement, "Real-time discrete and filter importance sampling").
 *   - 3D positions are already in voxel index space, voxel k centred at k, as
 *     in the tricubic listing (supplement, "Sampling a cubic B-spline kernel
 *     in 3D").
 *   - Cubic B-spline taps of cell i are i-1..i+2 (Eq. bicubic-bspline-texfilt
 *     read with the offset K_bs(x - (i+k)) that the weight polynomials of the
 *     bicubic listing imply).
 *   - One fresh uniform per axis from a counter-based hash (no sample reuse;
 *     reuse, Eq. uniform-sample-reuse, is an optimisation of the same
 *     distribution and is kept here as the `reuse' variant for distribution
 *     tests only).
 *   - 2D addressing clamps each tap to the texture; 3D addressing returns the
 *     grid's background value outside the domain and in inactive leaves.
 *   - The interpolating cubics (negative lobes) are the paper's cubic
 *     polynomial kernel K_3 with a = -1/2 ("Keys") and the Mitchell-Netravali
 *     cubic with B = C = 1/3; both are estimated by positivization with one
 *     tap drawn from the positive and one from the negative weights.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* storage formats */
enum { ORC_F32 = 0, ORC_F16 = 1, ORC_BF16 = 2, ORC_FP8_E4M3 = 3, ORC_U8 = 4 };
/* filters and modes */
enum { ORC_LINEAR = 0, ORC_CUBIC = 1, ORC_KEYS = 2, ORC_MITCHELL = 3 };
enum { ORC_DET = 0, ORC_STOCH = 1, ORC_STOCH_REUSE = 2, ORC_DET_ABS = 3, ORC_STOCH_FIS = 4 };
/* ORC_DET_ABS: sum_k |w_k| |t_k|, the scale of the deterministic tolerance. */

#define ORC_BAD_INDEX ((int32_t)0x80000000)

/* ------------------------------------------------------------------------ */
/* Counter-based random numbers.                                             */
/* The paper draws its per-lookup uniforms from white or blue noise (Results, */
/* real-time section).  A counter-based generator makes the draw a pure       */
/* function of (seed, query, hash index): the one-round PCG hash "pcg"        */
/* published by Jarzynski and Olano (JCGT 9(3), 2020), chained as             */
/*   s = pcg(seed_lo ^ pcg(seed_hi)),  b = pcg(s ^ qid),                      */
/*   h_a = pcg(b + a) for every hash index a >= 0 (a = 0, 1, 2: axes x, y, z),*/
/*   u_a = (h_a >> 8) * 2^-24  in [0, 1 - 2^-24].                             */
/* ------------------------------------------------------------------------ */
uint32_t orc_pcg(uint32_t x)
{
    uint32_t state = x * 747796405u + 2891336453u;
    uint32_t word = ((state >> ((state >> 28u) + 4u)) ^ state) * 277803737u;
    return (word >> 22u) ^ word;
}

uint32_t orc_seed_key(uint64_t seed)
{
    return orc_pcg((uint32_t)seed ^ orc_pcg((uint32_t)(seed >> 32)));
}

float orc_uniform(uint64_t seed, uint32_t qid, uint32_t axis)
{
    uint32_t b = orc_pcg(orc_seed_key(seed) ^ qid);
    uint32_t h = orc_pcg(b + axis);
    return (float)(h >> 8) * 0x1p-24f;
}

/* ------------------------------------------------------------------------ */
/* Exact texel decoding from the storage format to binary64.                 */
/* ------------------------------------------------------------------------ */
static double orc_half_to_double(uint16_t h)
{
    int sign = (h >> 15) & 1, e = (h >> 10) & 31, m = h & 1023;
    double v;
    if (e == 0)
        v = ldexp((double)m, -24);                 /* subnormal: m * 2^-24 */
    else if (e == 31)
        v = m ? NAN : INFINITY;
    else
        v = ldexp((double)(1024 + m), e - 25);     /* (1 + m/1024) * 2^(e-15) */
    return sign ? -v : v;
}

static double orc_bf16_to_double(uint16_t b)
{
    /* bfloat16 is the upper half of a binary32 word */
    uint32_t w = (uint32_t)b << 16;
    float f;
    memcpy(&f, &w, 4);
    return (double)f;
}

static double orc_e4m3_to_double(uint8_t q)
{
    /* OCP 8-bit E4M3 ("FN"): bias 7, no infinities, S.1111.111 is NaN */
    int sign = (q >> 7) & 1, e = (q >> 3) & 15, m = q & 7;
    double v;
    if (e == 15 && m == 7)
        v = NAN;
    else if (e == 0)
        v = ldexp((double)m, -9);                  /* m/8 * 2^-6 */
    else
        v = ldexp((double)(8 + m), e - 10);        /* (1 + m/8) * 2^(e-7) */
    return sign ? -v : v;
}

double orc_decode(int fmt, const void* base, int64_t i)
{
    switch (fmt) {
    case ORC_F32: { float f; memcpy(&f, (const char*)base + 4 * i, 4); return (double)f; }
    case ORC_F16: { uint16_t h; memcpy(&h, (const char*)base + 2 * i, 2); return orc_half_to_double(h); }
    case ORC_BF16: { uint16_t h; memcpy(&h, (const char*)base + 2 * i, 2); return orc_bf16_to_double(h); }
    case ORC_FP8_E4M3: return orc_e4m3_to_double(((const uint8_t*)base)[i]);
    case ORC_U8: return (double)((const uint8_t*)base)[i] / 255.0;   /* UNORM */
    }
    return NAN;
}

/* ------------------------------------------------------------------------ */
/* Filter kernels (supplement, "Filter Kernels"), binary64.                  */
/* ------------------------------------------------------------------------ */
double orc_kernel_tent(double d)   /* K_1 */
{
    d = fabs(d);
    return d < 1.0 ? 1.0 - d : 0.0;
}

double orc_kernel_bspline(double d)   /* K_bs, Eq. cubic-bspline */
{
    d = fabs(d);
    if (d <= 1.0) return (4.0 - 3.0 * d * d * (2.0 - d)) / 6.0;
    if (d <= 2.0) return (2.0 - d) * (2.0 - d) * (2.0 - d) / 6.0;
    return 0.0;
}

/* The cubic polynomial kernel K_3 of the supplement ("Filter Kernels") with
 * the free parameter a = -1/2 that the paper recommends: the interpolating
 * (negative lobe) cubic of its real-time results. */
double orc_kernel_keys(double d)
{
    const double a = -0.5;
    d = fabs(d);
    if (d < 1.0) return (a + 2.0) * d * d * d - (a + 3.0) * d * d + 1.0;
    if (d < 2.0) return a * d * d * d - 5.0 * a * d * d + 8.0 * a * d - 4.0 * a;
    return 0.0;
}

/* Mitchell and Netravali's cubic (SIGGRAPH 1988) with B = C = 1/3, the other
 * filter the name "Mitchell" can mean; it also has negative lobes. */
double orc_kernel_mitchell(double d)
{
    const double B = 1.0 / 3.0, C = 1.0 / 3.0;
    d = fabs(d);
    if (d < 1.0) return ((12.0 - 9.0 * B - 6.0 * C) * d * d * d + (-18.0 + 12.0 * B + 6.0 * C) * d * d + (6.0 - 2.0 * B)) / 6.0;
    if (d < 2.0)
        return ((-B - 6.0 * C) * d * d * d + (6.0 * B + 30.0 * C) * d * d + (-12.0 * B - 48.0 * C) * d + (8.0 * B + 24.0 * C)) / 6.0;
    return 0.0;
}

/* The kernel of a filter, evaluated at a signed distance (brute-force paths). */
double orc_kernel(int filter, double d)
{
    switch (filter) {
    case ORC_LINEAR: return orc_kernel_tent(d);
    case ORC_CUBIC: return orc_kernel_bspline(d);
    case ORC_KEYS: return orc_kernel_keys(d);
    case ORC_MITCHELL: return orc_kernel_mitchell(d);
    }
    return NAN;
}

/* Per-axis weights of the taps of cell i for the fractional offset t.
 * Linear: taps i, i+1 with (1-t, t) -- the lerp of section "Linear Filters".
 * Cubic:  taps i-1..i+2 with the B-spline weights of the bicubic listing,
 * i.e. K_bs(t+1), K_bs(t), K_bs(1-t), K_bs(2-t); the first is written as
 * (1-t)^3/6 rather than the listing's expanded polynomial (same value).
 * Keys / Mitchell: taps i-1..i+2 with the kernel at the same four distances. */
void orc_axis_weights(int filter, double t, double w[4])
{
    if (filter == ORC_LINEAR) {
        w[0] = 1.0 - t; w[1] = t; w[2] = 0.0; w[3] = 0.0;
    } else if (filter == ORC_KEYS || filter == ORC_MITCHELL) {
        w[0] = orc_kernel(filter, t + 1.0);
        w[1] = orc_kernel(filter, t);
        w[2] = orc_kernel(filter, 1.0 - t);
        w[3] = orc_kernel(filter, 2.0 - t);
    } else {
        double t2 = t * t, t3 = t2 * t, s = 1.0 - t;
        w[0] = s * s * s / 6.0;
        w[1] = (3.0 * t3 - 6.0 * t2 + 4.0) / 6.0;
        w[2] = (-3.0 * t3 + 3.0 * t2 + 3.0 * t + 1.0) / 6.0;
        w[3] = t3 / 6.0;
    }
}

/* ------------------------------------------------------------------------ */
/* Cell of a binary32 coordinate.  A coordinate that is NaN, infinite or has */
/* magnitude >= 2^24 has no cell (the query then yields NaN and the index    */
/* INT32_MIN).  Otherwise i = floor(x) and t = x - floor(x) in binary32.     */
/* ------------------------------------------------------------------------ */
static int orc_cell(float x, int* i, float* t)
{
    if (!(fabsf(x) < 16777216.0f)) return 0;
    float f = floorf(x);
    *i = (int)f;
    *t = x - f;
    return 1;
}

/* Pinned binary32 tap choice on one axis: the "sampling arrays" rule of the  */
/* Sampling Techniques section -- the first j whose cumulative weight exceeds */
/* u -- applied to the per-axis filter weights.                               */
/*   Linear: the upper tap iff u < t (the strict comparison of the bilinear   */
/*           listing; P(upper) = t, Eq. stochastic-lerp).                     */
/*   Cubic:  breakpoints at the cumulative B-spline weights of Eq.            */
/*           cubic-bspline, c1 = w0, c2 = w0 + w1, c3 = 1 - w3, with          */
/*           w0 = s^3/6, w1 = (4 + 3 t^2 (t - 2))/6, w3 = t^3/6, s = 1 - t,    */
/*           evaluated in binary32 as written, each operation rounded once:  */
/*             c1 = ((s*s)*s)*K6,                                             */
/*             c2 = c1 + (4 + (3*(t*t))*(t - 2))*K6,                          */
/*             c3 = 1 - ((t*t)*t)*K6,          K6 = fl32(1/6);                */
/*           j = [u>=c1] + [u>=c2] + [u>=c3].                                 */
/* Returns the offset of the chosen tap from cell i (0/1 linear, -1..2 cubic).*/
void orc_cubic_breakpoints(float t, float c[3])
{
    const float K6 = 0x1.555556p-3f;   /* (float)(1/6) */
    float s = 1.0f - t;
    c[0] = ((s * s) * s) * K6;
    c[1] = c[0] + (4.0f + (3.0f * (t * t)) * (t - 2.0f)) * K6;
    c[2] = 1.0f - ((t * t) * t) * K6;
}

int orc_select(int filter, float t, float u)
{
    if (filter == ORC_LINEAR)
        return (u < t) ? 1 : 0;
    float c[3];
    orc_cubic_breakpoints(t, c);
    int j = (u >= c[0]) + (u >= c[1]) + (u >= c[2]);
    return j - 1;
}

/* Number of binary32 values t in [0, 1) whose breakpoints are out of order
 * (c1 > c2 or c2 > c3); the cumulative-weight rule needs none. */
int64_t orc_cubic_breakpoints_disorder(void)
{
    int64_t bad = 0;
    const uint32_t end = 0x3f800000u;   /* bits of 1.0f */
#pragma omp parallel for reduction(+ : bad) schedule(static)
    for (int64_t b = 0; b < (int64_t)end; ++b) {
        uint32_t w = (uint32_t)b;
        float t, c[3];
        memcpy(&t, &w, 4);
        orc_cubic_breakpoints(t, c);
        bad += (c[0] > c[1]) || (c[1] > c[2]);
    }
    return bad;
}

/* The paper's own sampler, for distribution tests only: the weights are     */
/* visited in order with weighted reservoir sampling and the single uniform  */
/* is re-used from axis to axis by the remapping of Eq.                      */
/* uniform-sample-reuse (tricubic listing; for two taps this reduces to the  */
/* bilinear listing).  The remapped uniform is kept below 1, which the       */
/* binary32 remap otherwise reaches by rounding.  Arithmetic is binary32.    */
static int orc_select_reuse(int filter, float t, float* u)
{
    float w[4];
    int n, k, chosen;
    if (filter == ORC_LINEAR) {
        /* two taps: upper with probability t */
        float p = t;
        if (*u < p) { chosen = 1; *u = *u / p; }
        else { chosen = 0; *u = (*u - p) / (1.0f - p); }
        if (!(*u < 1.0f)) *u = 0x1.fffffep-1f;
        return chosen;
    }
    float t2 = t * t;
    w[0] = (1.0f / 6.0f) * (-t * t2 + 3 * t2 - 3 * t + 1);
    w[1] = (1.0f / 6.0f) * (3 * t * t2 - 6 * t2 + 4);
    w[2] = (1.0f / 6.0f) * (-3 * t * t2 + 3 * t2 + 3 * t + 1);
    w[3] = (1.0f / 6.0f) * t * t2;
    n = 4;
    float sum = w[0];
    chosen = 0;
    for (k = 1; k < n; ++k) {
        sum += w[k];
        float p = w[k] / sum;
        if (*u < p) { chosen = k; *u = *u / p; }
        else *u = (*u - p) / (1.0f - p);
        if (!(*u < 1.0f)) *u = 0x1.fffffep-1f;
        if (!(*u >= 0.0f)) *u = 0.0f;
    }
    return chosen - 1;
}

/* ------------------------------------------------------------------------ */
/* Positivization (section "Sampling Techniques", paragraph on               */
/* positivization; supplement, "The interpolating (negative lobe) bicubic    */
/* filter").  The tensor-product weights w of an interpolating cubic are     */
/* split into the positive weights w+ and the magnitudes w- of the negative  */
/* ones, with masses S+ = sum w+ and S- = sum w-.  One tap j+ is drawn with  */
/* probability w+_j / S+ and, independently, one tap j- with probability     */
/* w-_j / S-; the estimate is                                                */
/*     <F> = S+ t(j+) - S- t(j-),                                            */
/* whose mean is sum w t (the estimator of the positivization paragraph with */
/* both sums weighted, as the paper prescribes for a normalised filter).     */
/* When S- = 0 there is no negative tap.                                     */
/*                                                                           */
/* Drawing (pinned binary32, decisions only).  Per axis the four weights are */
/* split into positive parts p_k and negative parts n_k with masses P and N. */
/* A tap of the tensor product is positive exactly when an even number of    */
/* its axis factors is negative, so w+ is the sum over the sign patterns     */
/* with an even number of N axes of the products of the chosen per-axis      */
/* parts, and w- the same over the odd patterns.  A draw from w+ picks a     */
/* pattern in proportion to the product of its per-axis masses and then, on  */
/* each axis, a tap in proportion to that axis's chosen part.                */
/*   - Patterns are numbered by their bits (bit a set = axis a takes its      */
/*     negative part) and visited in increasing order; a pattern's mass is   */
/*     the product of the axis masses from axis 0 up.                        */
/*   - Every choice among masses m_0..m_{k-1} uses one uniform u and the      */
/*     cumulative rule: T = u * M with M = ((m_0 + m_1) + ...) + m_{k-1};     */
/*     the choice is the number of partial sums m_0 + ... + m_i (i < k-1)     */
/*     that are <= T, lowered to the last nonzero mass if it lands past it.   */
/*   - Uniforms: the positive draw takes axes 0..D-1 and 4 (pattern), the     */
/*     negative draw axes 5..5+D-1 and 8 (pattern).                          */
/* Per-axis weights in binary32 (scaled: Keys by 2, Mitchell by 18), in      */
/* factored forms whose relative error stays small near their zeros, with    */
/* s = 1 - t and every operation rounded once:                               */
/*   Keys:      2w0 = -((t*s)*s)              2w3 = -((t*t)*s)                */
/*              2w1 = s*(2 + t*(2 - 3*t))     2w2 = t*(2 + s*(2 - 3*s))       */
/*   Mitchell: 18w0 = (s*s)*fma(-7, t, 1)    18w3 = (t*t)*fma(-7, s, 1)       */
/*             18w1 = 1 + s*(9 + s*(27 - 21*s))                              */
/*             18w2 = 1 + t*(9 + t*(27 - 21*t))                              */
/* (These are the kernels at distances t+1, t, 1-t, 2-t, factored.)          */
/* ------------------------------------------------------------------------ */
void orc_interp_weights32(int filter, float t, float w[4])
{
    float s = 1.0f - t;
    if (filter == ORC_KEYS) {
        w[0] = -((t * s) * s);
        w[1] = s * (2.0f + t * (2.0f - 3.0f * t));
        w[2] = t * (2.0f + s * (2.0f - 3.0f * s));
        w[3] = -((t * t) * s);
    } else {
        w[0] = (s * s) * fmaf(-7.0f, t, 1.0f);
        w[1] = 1.0f + s * (9.0f + s * (27.0f - 21.0f * s));
        w[2] = 1.0f + t * (9.0f + t * (27.0f - 21.0f * t));
        w[3] = (t * t) * fmaf(-7.0f, s, 1.0f);
    }
}

/* The cumulative rule over k masses (see above). */
int orc_cumulative_choice(const float* m, int k, float u)
{
    float total = 0.0f;
    int last = 0;
    for (int i = 0; i < k; ++i) {
        total += m[i];
        if (m[i] > 0.0f) last = i;
    }
    float T = u * total, c = 0.0f;
    int j = 0;
    for (int i = 0; i < k - 1; ++i) {
        c += m[i];
        j += (T >= c);
    }
    return j > last ? last : j;
}

/* Tap offsets (relative to the cell, -1..2 per axis) of the positive draw
 * and, when the negative weights have mass, the negative draw; returns
 * whether a negative tap was drawn. */
int orc_positivized_taps(int filter, int D, const float* t, uint64_t seed, uint32_t qid, int* off_pos, int* off_neg)
{
    float part[2][3][4], mass[2][3];   /* [positive/negative][axis][tap] */
    for (int a = 0; a < D; ++a) {
        float w[4];
        orc_interp_weights32(filter, t[a], w);
        mass[0][a] = mass[1][a] = 0.0f;
        for (int k = 0; k < 4; ++k) {
            part[0][a][k] = w[k] > 0.0f ? w[k] : 0.0f;
            part[1][a][k] = w[k] < 0.0f ? -w[k] : 0.0f;
            mass[0][a] += part[0][a][k];
            mass[1][a] += part[1][a][k];
        }
    }
    int has_neg = 0;
    for (int set = 0; set < 2; ++set) {   /* 0: positive (even patterns), 1: negative (odd) */
        int pat[4], np = 0;
        float pm[4];
        for (int b = 0; b < (1 << D); ++b) {
            int odd = __builtin_popcount((unsigned)b) & 1;
            if (odd != set) continue;
            float m = mass[b & 1][0];
            for (int a = 1; a < D; ++a) m = m * mass[(b >> a) & 1][a];
            pat[np] = b;
            pm[np++] = m;
        }
        float total = 0.0f;
        for (int i = 0; i < np; ++i) total += pm[i];
        if (set == 1 && !(total > 0.0f)) break;
        uint32_t ubase = set == 0 ? 0u : 5u, ucomp = set == 0 ? 4u : 8u;
        int b = pat[orc_cumulative_choice(pm, np, orc_uniform(seed, qid, ucomp))];
        int* off = set == 0 ? off_pos : off_neg;
        for (int a = 0; a < D; ++a)
            off[a] = orc_cumulative_choice(part[(b >> a) & 1][a], 4, orc_uniform(seed, qid, ubase + (uint32_t)a)) - 1;
        if (set == 1) has_neg = 1;
    }
    return has_neg;
}

/* Exact masses S+ and S- of the tensor-product weights (binary64, from the
 * exact fractional offsets). */
void orc_positivized_masses(int filter, int D, const double* t, double* Sp, double* Sn)
{
    double w[3][4];
    for (int a = 0; a < D; ++a) orc_axis_weights(filter, t[a], w[a]);
    *Sp = *Sn = 0.0;
    int ntap = 1;
    for (int a = 0; a < D; ++a) ntap *= 4;
    for (int k = 0; k < ntap; ++k) {
        double wt = 1.0;
        for (int a = 0, r = k; a < D; ++a, r /= 4) wt *= w[a][r % 4];
        if (wt > 0.0) *Sp += wt;
        else *Sn -= wt;
    }
}

/* The paper's own sampler for the interpolating bicubic, for distribution
 * tests only: the 16 weights are visited row by row (y outer, x inner) and
 * fed to two weighted reservoirs, one per sign, that share one uniform
 * re-used by the warping of Eq. uniform-sample-reuse.  Zero weights are not
 * offered to either reservoir (the first one would divide zero by zero).
 * Binary64 throughout.  Returns whether a negative tap was chosen. */
int orc_positivized_wrs2d(int filter, double tx, double ty, double u, int* off_pos, int* off_neg)
{
    double wx[4], wy[4], sum[2] = {0.0, 0.0};
    int chosen[2][2] = {{0, 0}, {0, 0}}, any[2] = {0, 0};
    orc_axis_weights(filter, tx, wx);
    orc_axis_weights(filter, ty, wy);
    for (int b = 0; b < 4; ++b)
        for (int a = 0; a < 4; ++a) {
            double w = wx[a] * wy[b];
            if (w == 0.0) continue;
            int r = w < 0.0;
            sum[r] += fabs(w);
            double p = fabs(w) / sum[r];
            if (u < p) {
                chosen[r][0] = a - 1;
                chosen[r][1] = b - 1;
                any[r] = 1;
                u = u / p;
            } else {
                u = (u - p) / (1.0 - p);
            }
            if (!(u < 1.0)) u = 0x1.fffffffffffffp-1;
        }
    off_pos[0] = chosen[0][0]; off_pos[1] = chosen[0][1];
    off_neg[0] = chosen[1][0]; off_neg[1] = chosen[1][1];
    return any[1];
}

/* ------------------------------------------------------------------------ */
/* Filter importance sampling of the tent and cubic B-spline filters        */
/* (section "Filter Importance Sampling"): a B-spline of degree n is the     */
/* box-convolution of one of degree n - 1, so the position is jittered by a  */
/* draw of the degree n - 1 spline -- a box (one uniform minus 1/2) for the  */
/* tent, a quadratic B-spline (three uniforms minus 3/2, the Cox-de Boor     */
/* sum) for the cubic -- and the nearest texel floor(x' + 1/2) is read.      */
/* Binary64, summed in the order written: exact for |x| >= 2^-29 (x is       */
/* binary32 and the uniforms lie on the 2^-24 grid); nearer 0 the sum x + s  */
/* can round x's lowest bits away, and the tap is that of the rounded sum.   */
/* Uniforms of axis a: hash index a (tent); a, 4 + a, 8 + a (cubic).         */
/* ------------------------------------------------------------------------ */
int orc_fis_tap(int filter, double x, uint64_t seed, uint32_t qid, int a)
{
    double s;
    if (filter == ORC_LINEAR)
        s = (double)orc_uniform(seed, qid, (uint32_t)a) - 0.5;
    else
        s = ((double)orc_uniform(seed, qid, (uint32_t)a) + (double)orc_uniform(seed, qid, 4u + (uint32_t)a)) +
            (double)orc_uniform(seed, qid, 8u + (uint32_t)a) - 1.5;
    return (int)floor(x + s + 0.5);
}

/* ------------------------------------------------------------------------ */
/* 2D textures: row-major texels, channels interleaved; tap indices clamped. */
/* ------------------------------------------------------------------------ */
static int orc_clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

/* A 2D texel source: stored texels of a format, DCT-compressed blocks
 * (dct.c), or 8-byte material texels (shade.c: albedo RGB, roughness, normal
 * x and y, six channels).  Taps are clamped to the texture before they are
 * read. */
typedef struct orc_src2d {
    const void* tex;
    int W, H, C, fmt;   /* fmt: a storage format, ORC_FMT_DCT or ORC_FMT_MATERIAL */
} orc_src2d;

#define ORC_FMT_DCT 100
#define ORC_FMT_MATERIAL 101
double orc_dct_texel(const uint32_t* blocks, int W, int C, int x, int y, int c);
void orc_material_decode(const uint8_t* texel, double out[6]);

static double orc_src_texel(const orc_src2d* s, int x, int y, int c)
{
    x = orc_clampi(x, 0, s->W - 1);
    y = orc_clampi(y, 0, s->H - 1);
    if (s->fmt == ORC_FMT_DCT) return orc_dct_texel((const uint32_t*)s->tex, s->W, s->C, x, y, c);
    if (s->fmt == ORC_FMT_MATERIAL) {
        double m[6];
        orc_material_decode((const uint8_t*)s->tex + 8 * ((int64_t)y * s->W + x), m);
        return m[c];
    }
    return orc_decode(s->fmt, s->tex, ((int64_t)y * s->W + x) * s->C + c);
}

static double orc_texel2d(const void* tex, int W, int H, int C, int fmt, int x, int y, int c)
{
    orc_src2d s = {tex, W, H, C, fmt};
    return orc_src_texel(&s, x, y, c);
}

static int orc_raster2d(const float* uv, int W, int H, float* x, float* y)
{
    *x = uv[0] * (float)W - 0.5f;   /* two binary32 roundings, no fma */
    *y = uv[1] * (float)H - 0.5f;
    return 1;
}

static void orc_nan_out(double* out, int C, int32_t* idx, int dims)
{
    for (int c = 0; c < C; ++c) out[c] = NAN;
    if (idx) for (int a = 0; a < dims; ++a) idx[a] = ORC_BAD_INDEX;
}

static int orc_positivized(int filter) { return filter == ORC_KEYS || filter == ORC_MITCHELL; }

/* Index entries per query: the chosen tap, or for positivized filters the
 * positive tap followed by the negative one. */
static int orc_index_width(int filter, int dims) { return orc_positivized(filter) ? 2 * dims : dims; }

/* One 2D query.  mode: ORC_DET (separable weighted sum, Eq. filtered-texture
 * with the tensor-product weights), ORC_STOCH (one tap per Eq.
 * stochastic-sum, or the two taps of positivization), ORC_STOCH_REUSE (the
 * paper's listing samplers). */
static void orc_query2d(const orc_src2d* src, const float* uv, int filter, int mode, uint64_t seed, uint32_t qid,
                        double* out, int32_t* idx)
{
    const int W = src->W, H = src->H, C = src->C;
    float x, y, tx, ty;
    int ix, iy;
    orc_raster2d(uv, W, H, &x, &y);
    if (!orc_cell(x, &ix, &tx) || !orc_cell(y, &iy, &ty)) {
        orc_nan_out(out, C, idx, orc_index_width(filter, 2));
        return;
    }
    int base = (filter == ORC_LINEAR) ? 0 : -1;
    int ntap = (filter == ORC_LINEAR) ? 2 : 4;
    if (mode == ORC_DET || mode == ORC_DET_ABS) {
        double wx[4], wy[4];
        orc_axis_weights(filter, (double)x - floor((double)x), wx);
        orc_axis_weights(filter, (double)y - floor((double)y), wy);
        int ab = mode == ORC_DET_ABS;
        for (int c = 0; c < C; ++c) {
            double acc = 0.0;
            for (int b = 0; b < ntap; ++b) {
                double row = 0.0;
                for (int a = 0; a < ntap; ++a) {
                    double v = orc_src_texel(src, ix + base + a, iy + base + b, c);
                    row += ab ? fabs(wx[a]) * fabs(v) : wx[a] * v;
                }
                acc += (ab ? fabs(wy[b]) : wy[b]) * row;
            }
            out[c] = acc;
        }
        return;
    }
    if (orc_positivized(filter)) {
        int op[2], on[2], neg;
        float t2[2] = {tx, ty};
        if (mode == ORC_STOCH)
            neg = orc_positivized_taps(filter, 2, t2, seed, qid, op, on);
        else
            neg = orc_positivized_wrs2d(filter, (double)tx, (double)ty, (double)orc_uniform(seed, qid, 0), op, on);
        double tt[2] = {(double)x - floor((double)x), (double)y - floor((double)y)}, Sp, Sn;   /* exact offsets */
        orc_positivized_masses(filter, 2, tt, &Sp, &Sn);
        int px = orc_clampi(ix + op[0], 0, W - 1), py = orc_clampi(iy + op[1], 0, H - 1);
        int nx = orc_clampi(ix + on[0], 0, W - 1), ny = orc_clampi(iy + on[1], 0, H - 1);
        for (int c = 0; c < C; ++c) {
            double v = Sp * orc_src_texel(src, px, py, c);
            if (neg) v -= Sn * orc_src_texel(src, nx, ny, c);
            out[c] = v;
        }
        if (idx) {
            idx[0] = px; idx[1] = py;
            idx[2] = neg ? nx : ORC_BAD_INDEX;
            idx[3] = neg ? ny : ORC_BAD_INDEX;
        }
        return;
    }
    int jx, jy;
    if (mode == ORC_STOCH_FIS) {
        jx = orc_fis_tap(filter, (double)x, seed, qid, 0) - ix;
        jy = orc_fis_tap(filter, (double)y, seed, qid, 1) - iy;
    } else if (mode == ORC_STOCH) {
        jx = orc_select(filter, tx, orc_uniform(seed, qid, 0));
        jy = orc_select(filter, ty, orc_uniform(seed, qid, 1));
    } else {
        float u = orc_uniform(seed, qid, 0);
        jx = orc_select_reuse(filter, tx, &u);
        jy = orc_select_reuse(filter, ty, &u);
    }
    int sx = orc_clampi(ix + jx, 0, W - 1), sy = orc_clampi(iy + jy, 0, H - 1);
    for (int c = 0; c < C; ++c) out[c] = orc_src_texel(src, sx, sy, c);
    if (idx) { idx[0] = sx; idx[1] = sy; }
}

static int orc_threads(int nthreads)
{
#ifdef _OPENMP
    return nthreads > 0 ? nthreads : omp_get_max_threads();
#else
    (void)nthreads;
    return 1;
#endif
}

int orc_max_threads(void) { return orc_threads(0); }

/* Queries k = 0..n-1 of a batch, or, with qids, the queries qids[k] of a
 * batch evaluated as members of it (a draw depends on the query's index);
 * result k goes to out[k]. */
static int orc_filter_src2d(const orc_src2d* src, const float* uv, const int64_t* qids, int64_t n, int filter,
                            int mode, uint64_t seed, double* out, int32_t* idx, int nthreads)
{
    if (mode < ORC_DET || mode > ORC_STOCH_FIS || (orc_positivized(filter) && mode == ORC_STOCH_FIS)) return -1;
    int nt = orc_threads(nthreads), iw = orc_index_width(filter, 2), C = src->C;
    (void)nt;
#pragma omp parallel for schedule(static) num_threads(nt)
    for (int64_t k = 0; k < n; ++k) {
        int64_t q = qids ? qids[k] : k;
        orc_query2d(src, uv + 2 * q, filter, mode, seed, (uint32_t)q, out + k * C, idx ? idx + iw * k : NULL);
    }
    return 0;
}

/* DCT-compressed textures (blocks as written by orc_dct_encode). */
int orc_dct_filter2d(const uint32_t* blocks, int W, int H, int C, const float* uv, int64_t n, int filter, int mode,
                     uint64_t seed, double* out, int32_t* idx, int nthreads)
{
    if (W <= 0 || H <= 0 || W % 8 || H % 8 || C <= 0 || C > 16 || n < 0 || filter < ORC_LINEAR || filter > ORC_MITCHELL)
        return -1;
    orc_src2d src = {blocks, W, H, C, ORC_FMT_DCT};
    return orc_filter_src2d(&src, uv, NULL, n, filter, mode, seed, out, idx, nthreads);
}

int orc_dct_filter2d_at(const uint32_t* blocks, int W, int H, int C, const float* uv, const int64_t* qids, int64_t m,
                        int filter, int mode, uint64_t seed, double* out, int32_t* idx, int nthreads)
{
    if (W <= 0 || H <= 0 || W % 8 || H % 8 || C <= 0 || C > 16 || m < 0 || filter < ORC_LINEAR || filter > ORC_MITCHELL)
        return -1;
    orc_src2d src = {blocks, W, H, C, ORC_FMT_DCT};
    return orc_filter_src2d(&src, uv, qids, m, filter, mode, seed, out, idx, nthreads);
}

/* Material textures (W x H texels of 8 bytes), filtered as six channels. */
int orc_material_filter2d_at(const uint8_t* tex, int W, int H, const float* uv, const int64_t* qids, int64_t m,
                             int filter, int mode, uint64_t seed, double* out, int32_t* idx, int nthreads)
{
    if (W <= 0 || H <= 0 || m < 0 || filter < ORC_LINEAR || filter > ORC_MITCHELL) return -1;
    orc_src2d src = {tex, W, H, 6, ORC_FMT_MATERIAL};
    return orc_filter_src2d(&src, uv, qids, m, filter, mode, seed, out, idx, nthreads);
}

int orc_filter2d(const void* tex, int W, int H, int C, int fmt, const float* uv, int64_t n,
                 int filter, int mode, uint64_t seed, double* out, int32_t* idx, int nthreads)
{
    if (W <= 0 || H <= 0 || C <= 0 || C > 16 || n < 0 || filter < ORC_LINEAR || filter > ORC_MITCHELL) return -1;
    orc_src2d src = {tex, W, H, C, fmt};
    return orc_filter_src2d(&src, uv, NULL, n, filter, mode, seed, out, idx, nthreads);
}

/* Brute-force deterministic 2D filter: every texel of a 6x6 window around the
 * cell, weighted by the kernel itself evaluated at the texel's distance
 * (Eq. filter-function restricted to texel centres); kernels with zero weight
 * contribute nothing.  Independent of orc_axis_weights. */
int orc_filter2d_brute(const void* tex, int W, int H, int C, int fmt, const float* uv, int64_t n,
                       int filter, double* out)
{
    for (int64_t q = 0; q < n; ++q) {
        float x, y;
        orc_raster2d(uv + 2 * q, W, H, &x, &y);
        double* o = out + q * C;
        if (!(fabsf(x) < 16777216.0f) || !(fabsf(y) < 16777216.0f)) { orc_nan_out(o, C, NULL, 0); continue; }
        int ix = (int)floor((double)x), iy = (int)floor((double)y);
        for (int c = 0; c < C; ++c) {
            double acc = 0.0;
            for (int b = iy - 2; b <= iy + 3; ++b)
                for (int a = ix - 2; a <= ix + 3; ++a) {
                    double w = orc_kernel(filter, (double)x - a) * orc_kernel(filter, (double)y - b);
                    if (w != 0.0) acc += w * orc_texel2d(tex, W, H, C, fmt, a, b, c);
                }
            o[c] = acc;
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* 3D sparse grids.  The oracle keeps the simplest possible structure: a     */
/* dense table, one entry per 8^3 brick of the domain, holding the index of  */
/* the stored leaf or -1.                                                    */
/* ------------------------------------------------------------------------ */
typedef struct orc_grid {
    int dim[3];
    int nb[3];             /* bricks per axis */
    int fmt;
    double background;
    int32_t* brick;        /* nb[0]*nb[1]*nb[2] entries */
    const void* values;    /* leaf values, 512 per leaf, x fastest (borrowed) */
} orc_grid;

orc_grid* orc_grid_create(int dx, int dy, int dz, int fmt, int64_t nleaves,
                          const int32_t* origins, const void* values, double background)
{
    if (dx <= 0 || dy <= 0 || dz <= 0 || nleaves < 0) return NULL;
    orc_grid* g = (orc_grid*)calloc(1, sizeof(orc_grid));
    if (!g) return NULL;
    g->dim[0] = dx; g->dim[1] = dy; g->dim[2] = dz;
    for (int a = 0; a < 3; ++a) g->nb[a] = (g->dim[a] + 7) / 8;
    g->fmt = fmt;
    g->background = background;
    g->values = values;
    int64_t nbt = (int64_t)g->nb[0] * g->nb[1] * g->nb[2];
    g->brick = (int32_t*)malloc(sizeof(int32_t) * (size_t)nbt);
    if (!g->brick) { free(g); return NULL; }
    for (int64_t k = 0; k < nbt; ++k) g->brick[k] = -1;
    for (int64_t l = 0; l < nleaves; ++l) {
        int bx = origins[3 * l] / 8, by = origins[3 * l + 1] / 8, bz = origins[3 * l + 2] / 8;
        if (origins[3 * l] % 8 || origins[3 * l + 1] % 8 || origins[3 * l + 2] % 8 ||
            bx < 0 || by < 0 || bz < 0 || bx >= g->nb[0] || by >= g->nb[1] || bz >= g->nb[2]) {
            free(g->brick); free(g); return NULL;
        }
        int64_t k = ((int64_t)bz * g->nb[1] + by) * g->nb[0] + bx;
        if (g->brick[k] >= 0) { free(g->brick); free(g); return NULL; }
        g->brick[k] = (int32_t)l;
    }
    return g;
}

void orc_grid_destroy(orc_grid* g)
{
    if (g) { free(g->brick); free(g); }
}

/* Texel at integer voxel (x,y,z): background outside the domain or in an
 * inactive brick. */
double orc_grid_texel(const orc_grid* g, int x, int y, int z)
{
    if (x < 0 || y < 0 || z < 0 || x >= g->dim[0] || y >= g->dim[1] || z >= g->dim[2])
        return g->background;
    int64_t k = ((int64_t)(z / 8) * g->nb[1] + (y / 8)) * g->nb[0] + (x / 8);
    int32_t l = g->brick[k];
    if (l < 0) return g->background;
    return orc_decode(g->fmt, g->values, (int64_t)l * 512 + ((z % 8) * 8 + (y % 8)) * 8 + (x % 8));
}

static void orc_query3d(const orc_grid* g, const float* p, int filter, int mode, uint64_t seed,
                        uint32_t qid, double* out, int32_t* idx)
{
    int i[3];
    float t[3];
    for (int a = 0; a < 3; ++a)
        if (!orc_cell(p[a], &i[a], &t[a])) { orc_nan_out(out, 1, idx, orc_index_width(filter, 3)); return; }
    int base = (filter == ORC_LINEAR) ? 0 : -1;
    int ntap = (filter == ORC_LINEAR) ? 2 : 4;
    if (mode == ORC_DET || mode == ORC_DET_ABS) {
        double w[3][4];
        for (int a = 0; a < 3; ++a) orc_axis_weights(filter, (double)p[a] - floor((double)p[a]), w[a]);
        if (mode == ORC_DET_ABS)
            for (int a = 0; a < 3; ++a)
                for (int k = 0; k < 4; ++k) w[a][k] = fabs(w[a][k]);
        double acc = 0.0;
        for (int cz = 0; cz < ntap; ++cz) {
            double plane = 0.0;
            for (int cy = 0; cy < ntap; ++cy) {
                double row = 0.0;
                for (int cx = 0; cx < ntap; ++cx) {
                    double v = orc_grid_texel(g, i[0] + base + cx, i[1] + base + cy, i[2] + base + cz);
                    row += w[0][cx] * (mode == ORC_DET_ABS ? fabs(v) : v);
                }
                plane += w[1][cy] * row;
            }
            acc += w[2][cz] * plane;
        }
        out[0] = acc;
        return;
    }
    if (orc_positivized(filter)) {
        int op[3], on[3];
        int neg = orc_positivized_taps(filter, 3, t, seed, qid, op, on);
        double tt[3], Sp, Sn;   /* exact offsets */
        for (int a = 0; a < 3; ++a) tt[a] = (double)p[a] - floor((double)p[a]);
        orc_positivized_masses(filter, 3, tt, &Sp, &Sn);
        double v = Sp * orc_grid_texel(g, i[0] + op[0], i[1] + op[1], i[2] + op[2]);
        if (neg) v -= Sn * orc_grid_texel(g, i[0] + on[0], i[1] + on[1], i[2] + on[2]);
        out[0] = v;
        if (idx)
            for (int a = 0; a < 3; ++a) {
                idx[a] = i[a] + op[a];
                idx[3 + a] = neg ? i[a] + on[a] : ORC_BAD_INDEX;
            }
        return;
    }
    int v[3];
    if (mode == ORC_STOCH_FIS) {
        for (int a = 0; a < 3; ++a) v[a] = orc_fis_tap(filter, (double)p[a], seed, qid, a);
    } else if (mode == ORC_STOCH) {
        for (int a = 0; a < 3; ++a) v[a] = i[a] + orc_select(filter, t[a], orc_uniform(seed, qid, (uint32_t)a));
    } else {
        float u = orc_uniform(seed, qid, 0);
        for (int a = 0; a < 3; ++a) v[a] = i[a] + orc_select_reuse(filter, t[a], &u);
    }
    out[0] = orc_grid_texel(g, v[0], v[1], v[2]);
    if (idx) { idx[0] = v[0]; idx[1] = v[1]; idx[2] = v[2]; }
}

static int orc_filter3d_args_ok(const orc_grid* g, int64_t n, int filter, int mode)
{
    if (!g || n < 0 || filter < ORC_LINEAR || filter > ORC_MITCHELL || mode < ORC_DET || mode > ORC_STOCH_FIS) return 0;
    if (orc_positivized(filter) && mode == ORC_STOCH_FIS) return 0;    /* FIS covers the B-spline family */
    return !(orc_positivized(filter) && mode == ORC_STOCH_REUSE);   /* the paper's listing is 2D */
}

int orc_filter3d(const orc_grid* g, const float* p, int64_t n, int filter, int mode, uint64_t seed,
                 double* out, int32_t* idx, int nthreads)
{
    if (!orc_filter3d_args_ok(g, n, filter, mode)) return -1;
    int nt = orc_threads(nthreads), iw = orc_index_width(filter, 3);
    (void)nt;
#pragma omp parallel for schedule(static) num_threads(nt)
    for (int64_t q = 0; q < n; ++q)
        orc_query3d(g, p + 3 * q, filter, mode, seed, (uint32_t)q, out + q, idx ? idx + iw * q : NULL);
    return 0;
}

/* Stochastic samples for an explicit list of query ids (used to check a     */
/* large GPU batch at sampled positions: the draw depends on the query's     */
/* index within its batch).                                                   */
int orc_filter3d_at(const orc_grid* g, const float* p, const int64_t* qids, int64_t m, int filter,
                    int mode, uint64_t seed, double* out, int32_t* idx, int nthreads)
{
    if (!orc_filter3d_args_ok(g, m, filter, mode)) return -1;
    int nt = orc_threads(nthreads), iw = orc_index_width(filter, 3);
    (void)nt;
#pragma omp parallel for schedule(static) num_threads(nt)
    for (int64_t k = 0; k < m; ++k)
        orc_query3d(g, p + 3 * qids[k], filter, mode, seed, (uint32_t)qids[k], out + k,
                    idx ? idx + iw * k : NULL);
    return 0;
}

/* Brute-force deterministic 3D filter over a 6^3 window with the kernel
 * evaluated at each voxel's distance. */
int orc_filter3d_brute(const orc_grid* g, const float* p, int64_t n, int filter, double* out)
{
    for (int64_t q = 0; q < n; ++q) {
        const float* pq = p + 3 * q;
        if (!(fabsf(pq[0]) < 16777216.0f) || !(fabsf(pq[1]) < 16777216.0f) || !(fabsf(pq[2]) < 16777216.0f)) {
            out[q] = NAN; continue;
        }
        int i0 = (int)floor((double)pq[0]), i1 = (int)floor((double)pq[1]), i2 = (int)floor((double)pq[2]);
        double acc = 0.0;
        for (int z = i2 - 2; z <= i2 + 3; ++z)
            for (int y = i1 - 2; y <= i1 + 3; ++y)
                for (int x = i0 - 2; x <= i0 + 3; ++x) {
                    double w = orc_kernel(filter, (double)pq[0] - x) * orc_kernel(filter, (double)pq[1] - y) *
                               orc_kernel(filter, (double)pq[2] - z);
                    if (w != 0.0) acc += w * orc_grid_texel(g, x, y, z);
                }
        out[q] = acc;
    }
    return 0;
}

/* Exact mean and variance of the stochastic estimator of one query from its
 * taps (weights w, texels v):
 *   single tap (Eqs. filtered-texture and stochastic-sum; the tap
 *   probabilities are the normalised weights): E = sum w v,
 *   Var = sum w v^2 - E^2;
 *   positivized (two independent draws, see above): with A = sum_{w>0} w v,
 *   B = sum_{w<0} |w| v, E = A - B and
 *   Var = S+ sum_{w>0} w v^2 + S- sum_{w<0} |w| v^2 - A^2 - B^2. */
typedef struct orc_moment_acc { double A, B, A2, B2, Sp, Sn; } orc_moment_acc;

static void orc_moment_add(orc_moment_acc* m, double w, double v)
{
    if (w > 0.0) { m->A += w * v; m->A2 += w * v * v; m->Sp += w; }
    else if (w < 0.0) { m->B -= w * v; m->B2 -= w * v * v; m->Sn -= w; }
}

static void orc_moment_finish(const orc_moment_acc* m, int filter, double* mean, double* var)
{
    *mean = m->A - m->B;
    if (orc_positivized(filter))
        *var = m->Sp * m->A2 + m->Sn * m->B2 - m->A * m->A - m->B * m->B;
    else
        *var = m->A2 - m->A * m->A;   /* weights are non-negative */
}

int orc_filter3d_moments(const orc_grid* g, const float* p, int64_t n, int filter,
                         double* mean, double* var, int nthreads)
{
    if (!orc_filter3d_args_ok(g, n, filter, ORC_STOCH)) return -1;
    int nt = orc_threads(nthreads);
    (void)nt;
#pragma omp parallel for schedule(static) num_threads(nt)
    for (int64_t q = 0; q < n; ++q) {
        const float* pq = p + 3 * q;
        int i[3];
        float t[3];
        int ok = 1;
        for (int a = 0; a < 3; ++a) ok &= orc_cell(pq[a], &i[a], &t[a]);
        if (!ok) { mean[q] = NAN; var[q] = NAN; continue; }
        double w[3][4];
        for (int a = 0; a < 3; ++a) orc_axis_weights(filter, (double)pq[a] - floor((double)pq[a]), w[a]);
        int base = (filter == ORC_LINEAR) ? 0 : -1, ntap = (filter == ORC_LINEAR) ? 2 : 4;
        orc_moment_acc m = {0, 0, 0, 0, 0, 0};
        for (int cz = 0; cz < ntap; ++cz)
            for (int cy = 0; cy < ntap; ++cy)
                for (int cx = 0; cx < ntap; ++cx)
                    orc_moment_add(&m, w[0][cx] * w[1][cy] * w[2][cz],
                                   orc_grid_texel(g, i[0] + base + cx, i[1] + base + cy, i[2] + base + cz));
        orc_moment_finish(&m, filter, &mean[q], &var[q]);
    }
    return 0;
}

/* The same for 2D textures, per channel (n x C outputs). */
static int orc_moments_src2d(const orc_src2d* src, const float* uv, int64_t n, int filter, double* mean, double* var,
                             int nthreads)
{
    const int W = src->W, H = src->H, C = src->C;
    int nt = orc_threads(nthreads);
    (void)nt;
#pragma omp parallel for schedule(static) num_threads(nt)
    for (int64_t q = 0; q < n; ++q) {
        float x, y, tx, ty;
        int ix, iy;
        orc_raster2d(uv + 2 * q, W, H, &x, &y);
        if (!orc_cell(x, &ix, &tx) || !orc_cell(y, &iy, &ty)) {
            for (int c = 0; c < C; ++c) mean[q * C + c] = var[q * C + c] = NAN;
            continue;
        }
        double wx[4], wy[4];
        orc_axis_weights(filter, (double)x - floor((double)x), wx);   /* exact offsets */
        orc_axis_weights(filter, (double)y - floor((double)y), wy);
        int base = (filter == ORC_LINEAR) ? 0 : -1, ntap = (filter == ORC_LINEAR) ? 2 : 4;
        for (int c = 0; c < C; ++c) {
            orc_moment_acc m = {0, 0, 0, 0, 0, 0};
            for (int b = 0; b < ntap; ++b)
                for (int a = 0; a < ntap; ++a)
                    orc_moment_add(&m, wx[a] * wy[b], orc_src_texel(src, ix + base + a, iy + base + b, c));
            orc_moment_finish(&m, filter, &mean[q * C + c], &var[q * C + c]);
        }
    }
    return 0;
}

int orc_filter2d_moments(const void* tex, int W, int H, int C, int fmt, const float* uv, int64_t n, int filter,
                         double* mean, double* var, int nthreads)
{
    if (W <= 0 || H <= 0 || C <= 0 || C > 16 || n < 0 || filter < ORC_LINEAR || filter > ORC_MITCHELL) return -1;
    orc_src2d src = {tex, W, H, C, fmt};
    return orc_moments_src2d(&src, uv, n, filter, mean, var, nthreads);
}

int orc_dct_moments2d(const uint32_t* blocks, int W, int H, int C, const float* uv, int64_t n, int filter,
                      double* mean, double* var, int nthreads)
{
    if (W <= 0 || H <= 0 || W % 8 || H % 8 || C <= 0 || C > 16 || n < 0 || filter < ORC_LINEAR || filter > ORC_MITCHELL)
        return -1;
    orc_src2d src = {blocks, W, H, C, ORC_FMT_DCT};
    return orc_moments_src2d(&src, uv, n, filter, mean, var, nthreads);
}

/* ------------------------------------------------------------------------ */
/* Gaussian texture filtering (sections "Filter Importance Sampling" and     */
/* "Results", magnification; supplement, "Real-time discrete and filter      */
/* importance sampling").  Four modes, 2D, standard deviation sigma texels:  */
/*   ORC_G_FIS: the position is offset by sigma times a standard normal pair */
/*     from the Box-Muller transform of two uniforms (hash indices 0 and 1:  */
/*     r = sqrt(-2 ln(1 - u0)), angle 2 pi u1, x offset r cos, y offset      */
/*     r sin) and the nearest texel floor(x' + 1/2) is read (clamped);       */
/*   ORC_G_FIS_MEAN: what FIS estimates -- the Gaussian convolved with the   */
/*     nearest-texel box: tap k has weight Phi((k + 1/2 - x)/sigma) -        */
/*     Phi((k - 1/2 - x)/sigma) per axis, over |k - floor(x)| <= R with      */
/*     R = ceil(6 sigma) + 1 (the mass outside is below 2e-9);               */
/*   ORC_G_DISCRETE: one tap of the 4x4 window i-1..i+2 drawn with           */
/*     probability proportional to exp(-|d - t|^2 / (2 sigma^2)) (separable: */
/*     per axis, hash index a, cumulative rule on the four weights);         */
/*   ORC_G_DISCRETE_MEAN: the normalised weighted sum over that window.      */
/* Binary64 throughout (the decisions of ORC_G_FIS and ORC_G_DISCRETE go     */
/* through transcendental functions, so a device evaluating them with other  */
/* rounding can differ only where a sample lies within rounding distance of  */
/* a decision boundary).                                                     */
/* ------------------------------------------------------------------------ */
enum { ORC_G_FIS = 0, ORC_G_FIS_MEAN = 1, ORC_G_DISCRETE = 2, ORC_G_DISCRETE_MEAN = 3 };
#define ORC_GAUSS_PI 3.14159265358979323846

static double orc_phi(double z) { return 0.5 * erfc(-z / sqrt(2.0)); }

int orc_gauss_radius(double sigma) { return (int)ceil(6.0 * sigma) + 1; }

/* The FIS sample position of query qid (binary64). */
void orc_gauss_fis_position(double x, double y, double sigma, uint64_t seed, uint32_t qid, double* xs, double* ys)
{
    double u0 = (double)orc_uniform(seed, qid, 0), u1 = (double)orc_uniform(seed, qid, 1);
    double r = sqrt(-2.0 * log(1.0 - u0));
    *xs = x + sigma * (r * cos(2.0 * ORC_GAUSS_PI * u1));
    *ys = y + sigma * (r * sin(2.0 * ORC_GAUSS_PI * u1));
}

/* Discrete per-axis weights exp(-(d - t)^2 / (2 sigma^2)), d = -1..2. */
static void orc_gauss_discrete_weights(double t, double sigma, double w[4])
{
    for (int k = 0; k < 4; ++k) {
        double d = (double)(k - 1) - t;
        w[k] = exp(-d * d / (2.0 * sigma * sigma));
    }
}

static int orc_choice64(const double* m, int k, double u)
{
    double total = 0.0, c = 0.0;
    int last = 0, j = 0;
    for (int i = 0; i < k; ++i) {
        total += m[i];
        if (m[i] > 0.0) last = i;
    }
    double T = u * total;
    for (int i = 0; i < k - 1; ++i) {
        c += m[i];
        j += (T >= c);
    }
    return j > last ? last : j;
}

static void orc_gauss_query(const orc_src2d* src, const float* uv, double sigma, int gmode, uint64_t seed,
                            uint32_t qid, double* out, int32_t* idx)
{
    const int W = src->W, H = src->H, C = src->C;
    float x, y, tx, ty;
    int ix, iy;
    orc_raster2d(uv, W, H, &x, &y);
    if (!orc_cell(x, &ix, &tx) || !orc_cell(y, &iy, &ty)) { orc_nan_out(out, C, idx, 2); return; }
    double xe = (double)x, ye = (double)y;
    double fx = xe - floor(xe), fy = ye - floor(ye);   /* exact offsets */
    if (gmode == ORC_G_FIS) {
        double xs, ys;
        orc_gauss_fis_position(xe, ye, sigma, seed, qid, &xs, &ys);
        int sx = orc_clampi((int)fmax(fmin(floor(xs + 0.5), 2e9), -2e9), 0, W - 1);
        int sy = orc_clampi((int)fmax(fmin(floor(ys + 0.5), 2e9), -2e9), 0, H - 1);
        for (int c = 0; c < C; ++c) out[c] = orc_src_texel(src, sx, sy, c);
        if (idx) { idx[0] = sx; idx[1] = sy; }
        return;
    }
    if (gmode == ORC_G_DISCRETE) {
        double wx[4], wy[4];
        orc_gauss_discrete_weights(fx, sigma, wx);
        orc_gauss_discrete_weights(fy, sigma, wy);
        int sx = orc_clampi(ix - 1 + orc_choice64(wx, 4, (double)orc_uniform(seed, qid, 0)), 0, W - 1);
        int sy = orc_clampi(iy - 1 + orc_choice64(wy, 4, (double)orc_uniform(seed, qid, 1)), 0, H - 1);
        for (int c = 0; c < C; ++c) out[c] = orc_src_texel(src, sx, sy, c);
        if (idx) { idx[0] = sx; idx[1] = sy; }
        return;
    }
    if (gmode == ORC_G_DISCRETE_MEAN) {
        double wx[4], wy[4], sx = 0.0, sy = 0.0;
        orc_gauss_discrete_weights(fx, sigma, wx);
        orc_gauss_discrete_weights(fy, sigma, wy);
        for (int k = 0; k < 4; ++k) { sx += wx[k]; sy += wy[k]; }
        for (int c = 0; c < C; ++c) {
            double acc = 0.0;
            for (int b = 0; b < 4; ++b)
                for (int a = 0; a < 4; ++a) acc += wx[a] * wy[b] * orc_src_texel(src, ix - 1 + a, iy - 1 + b, c);
            out[c] = acc / (sx * sy);
        }
        return;
    }
    /* ORC_G_FIS_MEAN */
    int R = orc_gauss_radius(sigma), nt = 2 * R + 2;
    double* wx = (double*)malloc(sizeof(double) * (size_t)nt * 2);
    double* wy = wx + nt;
    for (int k = 0; k < nt; ++k) {
        double dx = (double)(ix - R + k) - xe, dy = (double)(iy - R + k) - ye;
        wx[k] = orc_phi((dx + 0.5) / sigma) - orc_phi((dx - 0.5) / sigma);
        wy[k] = orc_phi((dy + 0.5) / sigma) - orc_phi((dy - 0.5) / sigma);
    }
    for (int c = 0; c < C; ++c) {
        double acc = 0.0;
        for (int b = 0; b < nt; ++b) {
            double row = 0.0;
            for (int a = 0; a < nt; ++a) row += wx[a] * orc_src_texel(src, ix - R + a, iy - R + b, c);
            acc += wy[b] * row;
        }
        out[c] = acc;
    }
    free(wx);
}

static int orc_gauss_src2d(const orc_src2d* src, const float* uv, const int64_t* qids, int64_t n, double sigma,
                           int gmode, uint64_t seed, double* out, int32_t* idx, int nthreads)
{
    if (!(sigma > 0.0 && sigma <= 16.0) || gmode < ORC_G_FIS || gmode > ORC_G_DISCRETE_MEAN || n < 0) return -1;
    int nt = orc_threads(nthreads), C = src->C;
    (void)nt;
#pragma omp parallel for schedule(static) num_threads(nt)
    for (int64_t k = 0; k < n; ++k) {
        int64_t q = qids ? qids[k] : k;
        orc_gauss_query(src, uv + 2 * q, sigma, gmode, seed, (uint32_t)q, out + k * C, idx ? idx + 2 * k : NULL);
    }
    return 0;
}

int orc_gauss_filter2d(const void* tex, int W, int H, int C, int fmt, const float* uv, int64_t n, double sigma,
                       int gmode, uint64_t seed, double* out, int32_t* idx, int nthreads)
{
    if (W <= 0 || H <= 0 || C <= 0 || C > 16) return -1;
    orc_src2d src = {tex, W, H, C, fmt};
    return orc_gauss_src2d(&src, uv, NULL, n, sigma, gmode, seed, out, idx, nthreads);
}

int orc_dct_gauss_filter2d(const uint32_t* blocks, int W, int H, int C, const float* uv, int64_t n, double sigma,
                           int gmode, uint64_t seed, double* out, int32_t* idx, int nthreads)
{
    if (W <= 0 || H <= 0 || W % 8 || H % 8 || C <= 0 || C > 16) return -1;
    orc_src2d src = {blocks, W, H, C, ORC_FMT_DCT};
    return orc_gauss_src2d(&src, uv, NULL, n, sigma, gmode, seed, out, idx, nthreads);
}

int orc_dct_gauss_filter2d_at(const uint32_t* blocks, int W, int H, int C, const float* uv, const int64_t* qids,
                              int64_t m, double sigma, int gmode, uint64_t seed, double* out, int32_t* idx,
                              int nthreads)
{
    if (W <= 0 || H <= 0 || W % 8 || H % 8 || C <= 0 || C > 16) return -1;
    orc_src2d src = {blocks, W, H, C, ORC_FMT_DCT};
    return orc_gauss_src2d(&src, uv, qids, m, sigma, gmode, seed, out, idx, nthreads);
}

int orc_material_gauss_filter2d_at(const uint8_t* tex, int W, int H, const float* uv, const int64_t* qids, int64_t m,
                                   double sigma, int gmode, uint64_t seed, double* out, int32_t* idx, int nthreads)
{
    if (W <= 0 || H <= 0) return -1;
    orc_src2d src = {tex, W, H, 6, ORC_FMT_MATERIAL};
    return orc_gauss_src2d(&src, uv, qids, m, sigma, gmode, seed, out, idx, nthreads);
}

/* FIS sample positions (binary64) of a batch (or of its queries qids[k]),
 * for boundary-distance checks. */
int orc_gauss_fis_positions_at(int W, int H, const float* uv, const int64_t* qids, int64_t m, double sigma,
                               uint64_t seed, double* pos)
{
    for (int64_t k = 0; k < m; ++k) {
        int64_t q = qids ? qids[k] : k;
        float x, y;
        orc_raster2d(uv + 2 * q, W, H, &x, &y);
        orc_gauss_fis_position((double)x, (double)y, sigma, seed, (uint32_t)q, &pos[2 * k], &pos[2 * k + 1]);
    }
    return 0;
}

int orc_gauss_fis_positions(int W, int H, const float* uv, int64_t n, double sigma, uint64_t seed, double* pos)
{
    return orc_gauss_fis_positions_at(W, H, uv, NULL, n, sigma, seed, pos);
}

/* ------------------------------------------------------------------------ */
/* Elliptically weighted average filtering, deterministic and stochastic     */
/* (section "B-Spline and Anisotropic Filters": after a stochastic choice of */
/* MIP level from the ellipse's extent, one tap is drawn in proportion to    */
/* the EWA weights; supplement, "Stochastic sampling of the EWA kernel",     */
/* which follows pbrt's EWA lookup).                                         */
/* A query is (s, t, ds/dx, dt/dx, ds/dy, dt/dy) in [0,1] texture units.     */
/*   Axes: the longer of the two derivative vectors is the major axis; if    */
/*   shorter * max_aniso < longer (and shorter > 0) the shorter vector is    */
/*   scaled by longer / (shorter * max_aniso).  Binary32, each operation      */
/*   rounded once (lengths sqrt(x*x + y*y)).  shorter == 0: bilinear on      */
/*   level 0 (stochastic: the pinned linear draw with hash indices 2, 3).    */
/*   A record with a non-finite entry, an entry of magnitude >= 65536, or a  */
/*   level-0 raster position (s W0 - 0.5, t H0 - 0.5) of magnitude >= 2^24   */
/*   (the bound of every 2D filter) yields NaN.                              */
/*   Level of detail lod = max(0, (levels - 1) + log2(shorter)) in binary64; */
/*   deterministic: lerp(lod - floor(lod), EWA(floor), EWA(floor + 1));       */
/*   stochastic: level floor(lod) + [u0 < lod - floor(lod)] (hash index 0).  */
/*   The pyramid ends at a single texel (level sizes max(1, W >> l)), and a  */
/*   level at or past that last one yields that texel (pbrt's rule), so no   */
/*   footprint, however large, makes the scan over a bounding box unbounded. */
/*   EWA on level l (resolution W x H, binary32 as pbrt): st = (s W - 0.5,    */
/*   t H - 0.5), d0 = dst0 (W, H), d1 = dst1 (W, H);                          */
/*     A = (d0y^2 + d1y^2) + 1, B = -2 (d0x d0y + d1x d1y), C = (d0x^2 + d1x^2) + 1, */
/*     invF = 1 / (A C - B^2 * 0.25), A, B, C scaled by invF,                */
/*     det = -B^2 + 4 A C, invDet = 1/det, us = sqrt(det C), vs = sqrt(A det), */
/*     s0 = ceil(st.x - 2 invDet us), s1 = floor(st.x + 2 invDet us), same   */
/*     for t with vs; over t0..t1 (outer) and s0..s1 (inner): ss = s - st.x, */
/*     tt = t - st.y, r2 = ((A (ss ss)) + ((B ss) tt)) + (C (tt tt)); taps   */
/*     with r2 < 1 get weight LUT[min((int)(r2 * 128), 127)], LUT[i] =        */
/*     fl32(exp(-2 i/127) - exp(-2)) (a truncated Gaussian), taps clamped.   */
/*   Deterministic: sum w t / sum w.  Stochastic: a row of the box by        */
/*   weighted reservoir sampling over the row sums R_k (binary32 sums in     */
/*   scan order; row k replaces the choice iff u_(16+k) * S < R_k with S the */
/*   running sum of R), then a tap of that row: T = u1 R, the first tap whose */
/*   running sum exceeds T (the last tap with weight if none does).  One     */
/*   pass over the box and one over a row; the value is that texel.          */
/*   This draw is not the supplement's listing, which takes single taps by   */
/*   reservoir sampling with one re-scaled uniform (orc_ewa_listing_draws    */
/*   below); both draw tap (x, y) with probability w(x, y) / sum w, the row  */
/*   rule with fresh uniforms and no divisions, so its outcome is unique.    */
/* Values in binary64; the weights are the binary32 LUT values.              */
/* ------------------------------------------------------------------------ */
static float orc_ewa_lut[128];
static int orc_ewa_lut_ready = 0;

static void orc_ewa_init(void)
{
    if (orc_ewa_lut_ready) return;
    for (int i = 0; i < 128; ++i) orc_ewa_lut[i] = (float)(exp(-2.0 * i / 127.0) - exp(-2.0));
    orc_ewa_lut_ready = 1;
}

float orc_ewa_lut_value(int i)
{
    orc_ewa_init();
    return (i >= 0 && i < 128) ? orc_ewa_lut[i] : NAN;
}

typedef struct orc_ewa_tex {
    const void* const* lv;
    const int* W;
    const int* H;
    int levels, C, fmt;
} orc_ewa_tex;

static double orc_ewa_texel(const orc_ewa_tex* T, int l, int x, int y, int c)
{
    orc_src2d s = {T->lv[l], T->W[l], T->H[l], T->C, T->fmt};
    return orc_src_texel(&s, x, y, c);
}

/* The ellipse of one level in texel units (pbrt's construction, each
 * binary32 operation rounded once in the order written) and its bounding box. */
typedef struct orc_ellipse {
    float stx, sty, A, B, C;
    int s0, s1, t0, t1;
} orc_ellipse;

static orc_ellipse orc_ewa_ellipse(int W, int H, float s, float t, const float d0in[2], const float d1in[2])
{
    orc_ellipse e;
    e.stx = s * (float)W - 0.5f;
    e.sty = t * (float)H - 0.5f;
    float d0x = d0in[0] * (float)W, d0y = d0in[1] * (float)H;
    float d1x = d1in[0] * (float)W, d1y = d1in[1] * (float)H;
    float A = (d0y * d0y + d1y * d1y) + 1.0f;
    float B = -2.0f * (d0x * d0y + d1x * d1y);
    float Cc = (d0x * d0x + d1x * d1x) + 1.0f;
    float invF = 1.0f / (A * Cc - (B * B) * 0.25f);
    A *= invF;
    B *= invF;
    Cc *= invF;
    float det = -(B * B) + 4.0f * A * Cc;
    float invDet = 1.0f / det;
    float us = sqrtf(fmaxf(det * Cc, 0.0f)), vs = sqrtf(fmaxf(A * det, 0.0f));
    e.s0 = (int)ceilf(e.stx - 2.0f * invDet * us);
    e.s1 = (int)floorf(e.stx + 2.0f * invDet * us);
    e.t0 = (int)ceilf(e.sty - 2.0f * invDet * vs);
    e.t1 = (int)floorf(e.sty + 2.0f * invDet * vs);
    e.A = A;
    e.B = B;
    e.C = Cc;
    return e;
}

/* The LUT weight of tap (is, it): 0 outside the ellipse (r2 >= 1). */
static float orc_ewa_weight(const orc_ellipse* e, int is, int it)
{
    float ss = (float)is - e->stx, tt = (float)it - e->sty;
    float r2 = (e->A * (ss * ss) + (e->B * ss) * tt) + e->C * (tt * tt);
    if (!(r2 < 1.0f)) return 0.0f;
    int idx = (int)(r2 * 128.0f);
    if (idx > 127) idx = 127;
    return orc_ewa_lut[idx];
}

/* The taps of positive weight of the ellipse on a W x H level, in scan order
 * (rows t0..t1, each s0..s1; coordinates not clamped).  Writes at most cap
 * taps (x, y pairs in xy, weights in w) and returns how many there are. */
int64_t orc_ewa_weights(int W, int H, float s, float t, const float* d0, const float* d1, int64_t cap, int32_t* xy,
                        float* w)
{
    orc_ewa_init();
    orc_ellipse e = orc_ewa_ellipse(W, H, s, t, d0, d1);
    int64_t n = 0;
    for (int it = e.t0; it <= e.t1; ++it)
        for (int is = e.s0; is <= e.s1; ++is) {
            float wt = orc_ewa_weight(&e, is, it);
            if (!(wt > 0.0f)) continue;
            if (n < cap) {
                xy[2 * n] = is;
                xy[2 * n + 1] = it;
                w[n] = wt;
            }
            ++n;
        }
    return n;
}

/* The supplement's own sampler ("Stochastic sampling of the EWA kernel"),
 * for distribution tests only: one pass over the box in scan order with
 * weighted reservoir sampling of single taps driven by one uniform u, which
 * is re-scaled after every decision (u/p when the tap is taken, (u-p)/(1-p)
 * otherwise, p = w / running sum, binary32), kept below 1 as in the
 * reuse sampler above.  Draws K taps for one query, draw k with the
 * uniform of query k, hash index 1.  Returns the number of taps in the box. */
int64_t orc_ewa_listing_draws(int W, int H, float s, float t, const float* d0, const float* d1, uint64_t seed,
                              int64_t K, int32_t* xy)
{
    orc_ewa_init();
    orc_ellipse e = orc_ewa_ellipse(W, H, s, t, d0, d1);
    int64_t taps = 0;
    for (int64_t k = 0; k < K; ++k) {
        float u = orc_uniform(seed, (uint32_t)k, 1), sum = 0.0f;
        int cx = e.s0, cy = e.t0;
        taps = 0;
        for (int it = e.t0; it <= e.t1; ++it)
            for (int is = e.s0; is <= e.s1; ++is) {
                float wt = orc_ewa_weight(&e, is, it);
                if (!(wt > 0.0f)) continue;
                ++taps;
                sum += wt;
                float p = wt / sum;
                if (u < p) {
                    cx = is;
                    cy = it;
                    u = u / p;
                } else {
                    u = (u - p) / (1.0f - p);
                }
                if (!(u < 1.0f)) u = 0x1.fffffep-1f;
                if (!(u >= 0.0f)) u = 0.0f;
            }
        xy[2 * k] = cx;
        xy[2 * k + 1] = cy;
    }
    return taps;
}

/* EWA on one level: the deterministic value (per channel) and/or the drawn
 * tap.  The last level of a full pyramid is a single texel, which is the
 * value (and the tap) whatever the ellipse: pbrt reads it directly, so the
 * work stays bounded for footprints larger than the texture. */
static void orc_ewa_level(const orc_ewa_tex* T, int l, float s, float t, const float d0in[2], const float d1in[2],
                          int stochastic, float u, uint64_t seed, uint32_t qid, double* out, int* tx, int* ty)
{
    if (l == T->levels - 1) {
        if (stochastic) {
            *tx = 0;
            *ty = 0;
        } else {
            for (int c = 0; c < T->C; ++c) out[c] = orc_ewa_texel(T, l, 0, 0, c);
        }
        return;
    }
    const orc_ellipse e = orc_ewa_ellipse(T->W[l], T->H[l], s, t, d0in, d1in);
    if (!stochastic) {
        double acc[16] = {0};
        double wsum = 0.0;
        for (int it = e.t0; it <= e.t1; ++it)
            for (int is = e.s0; is <= e.s1; ++is) {
                float w = orc_ewa_weight(&e, is, it);
                if (!(w > 0.0f)) continue;
                wsum += (double)w;
                for (int c = 0; c < T->C; ++c) acc[c] += (double)w * orc_ewa_texel(T, l, is, it, c);
            }
        for (int c = 0; c < T->C; ++c) out[c] = acc[c] / wsum;
        return;
    }
    /* stochastic: a row by weighted reservoir sampling over the row sums
     * (row k of the box replaces the choice iff u_(16+k) * S < R_k, S the
     * running sum of row sums), then a tap of that row by the cumulative rule
     * (T = u1 * R, the first tap whose running sum exceeds T) */
    float S = 0.0f, Rsel = 0.0f;
    int rsel = e.t0, found = 0;
    for (int it = e.t0; it <= e.t1; ++it) {
        float R = 0.0f;
        for (int is = e.s0; is <= e.s1; ++is) {
            float w = orc_ewa_weight(&e, is, it);
            if (w > 0.0f) R += w;
        }
        if (!(R > 0.0f)) continue;
        S += R;
        if (orc_uniform(seed, qid, 16u + (uint32_t)(it - e.t0)) * S < R) { rsel = it; Rsel = R; found = 1; }
    }
    *tx = e.s0;
    *ty = rsel;
    if (!found) return;
    float Tq = u * Rsel, run = 0.0f;
    for (int is = e.s0; is <= e.s1; ++is) {
        float w = orc_ewa_weight(&e, is, rsel);
        if (!(w > 0.0f)) continue;
        run += w;
        *tx = is;   /* the last tap with weight, if the running sum never exceeds T */
        if (Tq < run) return;
    }
}

/* Level of detail and the two axes (binary32, then log2 in binary64). */
static double orc_ewa_axes(const float q[6], int levels, float max_aniso, float d0[2], float d1[2], float* shorter)
{
    d0[0] = q[2]; d0[1] = q[3];
    d1[0] = q[4]; d1[1] = q[5];
    if (d0[0] * d0[0] + d0[1] * d0[1] < d1[0] * d1[0] + d1[1] * d1[1]) {
        float a = d0[0], b = d0[1];
        d0[0] = d1[0]; d0[1] = d1[1];
        d1[0] = a; d1[1] = b;
    }
    float longer = sqrtf(d0[0] * d0[0] + d0[1] * d0[1]);
    float sh = sqrtf(d1[0] * d1[0] + d1[1] * d1[1]);
    if (sh * max_aniso < longer && sh > 0.0f) {
        float scale = longer / (sh * max_aniso);
        d1[0] *= scale;
        d1[1] *= scale;
        sh *= scale;
    }
    *shorter = sh;
    if (!(sh > 0.0f)) return 0.0;
    double lod = (double)(levels - 1) + log2((double)sh);
    return lod < 0.0 ? 0.0 : lod;
}

/* The binary64 level of detail of each query (for boundary checks). */
int orc_ewa_lods(const float* q, int64_t n, int levels, float max_aniso, double* lod)
{
    for (int64_t k = 0; k < n; ++k) {
        float d0[2], d1[2], sh;
        lod[k] = orc_ewa_axes(q + 6 * k, levels, max_aniso, d0, d1, &sh);
    }
    return 0;
}

int orc_ewa_filter2d_at(const void* const* level_texels, const int* W, const int* H, int levels, int C, int fmt,
                        const float* q, const int64_t* qids, int64_t n, float max_aniso, int mode, uint64_t seed,
                        double* out, int32_t* idx, int nthreads)
{
    if (!level_texels || levels < 1 || C < 1 || C > 16 || n < 0 || !(max_aniso >= 1.0f) ||
        (mode != ORC_DET && mode != ORC_STOCH))
        return -1;
    if (W[levels - 1] != 1 || H[levels - 1] != 1) return -1;   /* the pyramid must end at one texel */
    orc_ewa_init();
    orc_ewa_tex T = {level_texels, W, H, levels, C, fmt};
    int nt = orc_threads(nthreads);
    (void)nt;
#pragma omp parallel for schedule(dynamic, 256) num_threads(nt)
    for (int64_t k = 0; k < n; ++k) {
        const int64_t qi = qids ? qids[k] : k;
        const float* qk = q + 6 * qi;
        double* o = out + k * C;
        int32_t* ix = idx ? idx + 3 * k : NULL;
        int ok = 1;
        for (int j = 0; j < 6; ++j) ok &= isfinite(qk[j]) && fabsf(qk[j]) < 65536.0f;
        if (ok) {   /* the raster bound of every 2D filter, on level 0 (the coarser levels' positions are no larger) */
            float x0, y0;
            orc_raster2d(qk, W[0], H[0], &x0, &y0);
            ok = fabsf(x0) < 16777216.0f && fabsf(y0) < 16777216.0f;
        }
        if (!ok) { orc_nan_out(o, C, ix, 3); continue; }
        float d0[2], d1[2], sh;
        double lod = orc_ewa_axes(qk, levels, max_aniso, d0, d1, &sh);
        uint32_t qid = (uint32_t)qi;
        if (!(sh > 0.0f)) {   /* degenerate footprint: bilinear on level 0 */
            orc_src2d s0 = {level_texels[0], W[0], H[0], C, fmt};
            float uv[2] = {qk[0], qk[1]};
            if (mode == ORC_DET) {
                orc_query2d(&s0, uv, ORC_LINEAR, ORC_DET, seed, qid, o, NULL);
            } else {
                float x, y, tx, ty;
                int cx, cy;
                orc_raster2d(uv, W[0], H[0], &x, &y);
                if (!orc_cell(x, &cx, &tx) || !orc_cell(y, &cy, &ty)) { orc_nan_out(o, C, ix, 3); continue; }
                int sx = orc_clampi(cx + orc_select(ORC_LINEAR, tx, orc_uniform(seed, qid, 2)), 0, W[0] - 1);
                int sy = orc_clampi(cy + orc_select(ORC_LINEAR, ty, orc_uniform(seed, qid, 3)), 0, H[0] - 1);
                for (int c = 0; c < C; ++c) o[c] = orc_src_texel(&s0, sx, sy, c);
                if (ix) { ix[0] = sx; ix[1] = sy; ix[2] = 0; }
            }
            continue;
        }
        int il = (int)floor(lod);
        double frac = lod - (double)il;
        if (mode == ORC_DET) {
            double a[16], b[16];
            int l0 = il < levels ? il : levels - 1, l1 = il + 1 < levels ? il + 1 : levels - 1;
            orc_ewa_level(&T, l0, qk[0], qk[1], d0, d1, 0, 0.0f, seed, qid, a, NULL, NULL);
            orc_ewa_level(&T, l1, qk[0], qk[1], d0, d1, 0, 0.0f, seed, qid, b, NULL, NULL);
            for (int c = 0; c < C; ++c) o[c] = (1.0 - frac) * a[c] + frac * b[c];
        } else {
            int l = il + ((double)orc_uniform(seed, qid, 0) < frac ? 1 : 0);
            if (l > levels - 1) l = levels - 1;
            int tx, ty;
            orc_ewa_level(&T, l, qk[0], qk[1], d0, d1, 1, orc_uniform(seed, qid, 1), seed, qid, NULL, &tx, &ty);
            int sx = orc_clampi(tx, 0, W[l] - 1), sy = orc_clampi(ty, 0, H[l] - 1);
            for (int c = 0; c < C; ++c) o[c] = orc_ewa_texel(&T, l, sx, sy, c);
            if (ix) { ix[0] = sx; ix[1] = sy; ix[2] = l; }
        }
    }
    return 0;
}

int orc_ewa_filter2d(const void* const* level_texels, const int* W, const int* H, int levels, int C, int fmt,
                     const float* q, int64_t n, float max_aniso, int mode, uint64_t seed, double* out, int32_t* idx,
                     int nthreads)
{
    return orc_ewa_filter2d_at(level_texels, W, H, levels, C, fmt, q, NULL, n, max_aniso, mode, seed, out, idx,
                               nthreads);
}
