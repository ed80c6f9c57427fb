// device_common.h -- device-side building blocks of the filtering kernels:
// the counter-based uniform of each query axis, the per-axis cell and tap
// choice, the per-axis weights, and exact texel decoding.
//
// Every file that includes this header is compiled with -ffp-contract=off, so
// each binary32 expression below rounds after every operation exactly as
// written; fused multiply-adds appear only where __builtin_fmaf is spelled out
// (deterministic accumulation, which carries a stated tolerance instead of
// bit-exactness, and a few conversions whose results are exact).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace stf {

enum Fmt : int { F32 = 0, F16 = 1, BF16 = 2, FP8_E4M3 = 3, U8 = 4 };

// Bytes per stored value.
__host__ __device__ constexpr int fmt_bytes(int fmt)
{
    return fmt == F32 ? 4 : (fmt == F16 || fmt == BF16) ? 2 : 1;
}

// Where voxel (x, y, z) of a leaf (each 0..7) lies among the leaf's 512
// stored values: the leaf is kept in bricks of one 128-byte line -- 4x4x2
// voxels of binary32, 8x4x2 of 16-bit values, 8x8x2 of 8-bit values --
// x fastest within a brick, the bricks x, then y, then z.  A lookup whose
// neighbours step along any axis then finds them in the same line more often
// than in x-fastest rows.  The offset is the sum of one term per axis;
// x-runs of 4 binary32 or 8 narrower values stay contiguous and 16- (8-)
// byte aligned, so a row of taps is still read as whole chunks.
__host__ __device__ constexpr uint32_t leaf_ox(int fmt, uint32_t x)
{
    return fmt == F32 ? (x >> 2) * 32u + (x & 3u) : x;
}
__host__ __device__ constexpr uint32_t leaf_oy(int fmt, uint32_t y)
{
    return fmt == F32 ? (y >> 2) * 64u + (y & 3u) * 4u : (fmt == F16 || fmt == BF16) ? (y >> 2) * 64u + (y & 3u) * 8u
                                                                                      : y * 8u;
}
__host__ __device__ constexpr uint32_t leaf_oz(int fmt, uint32_t z)
{
    return fmt == F32 ? (z >> 1) * 128u + (z & 1u) * 16u
                      : (fmt == F16 || fmt == BF16) ? (z >> 1) * 128u + (z & 1u) * 32u : z * 64u;
}
__host__ __device__ constexpr uint32_t leaf_offset(int fmt, uint32_t x, uint32_t y, uint32_t z)
{
    return leaf_ox(fmt, x) + leaf_oy(fmt, y) + leaf_oz(fmt, z);
}

// One-round PCG hash (Jarzynski & Olano, JCGT 2020).  Integer arithmetic
// mod 2^32.
__host__ __device__ __forceinline__ uint32_t pcg(uint32_t x)
{
    uint32_t state = x * 747796405u + 2891336453u;
    uint32_t word = ((state >> ((state >> 28u) + 4u)) ^ state) * 277803737u;
    return (word >> 22u) ^ word;
}

// Per-call key of a 64-bit seed.
__host__ __device__ __forceinline__ uint32_t seed_key(uint64_t seed)
{
    return pcg((uint32_t)seed ^ pcg((uint32_t)(seed >> 32)));
}

// Uniforms in [0, 1 - 2^-24] on the 2^-24 grid.  Query q has the base hash
// b = pcg(key ^ q); its hash index a (a = 0, 1, 2 for the axes x, y, z; other
// indices for further draws) uses h_a = pcg(b + a).  The kernels work with
// m = u * 2^24 = h >> 8, an integer held exactly in binary32, and compare it
// with breakpoints scaled by 2^24; scaling by a power of two is exact, so
// every comparison has the same outcome as u against the unscaled breakpoint.
__device__ __forceinline__ float hash_m(uint32_t h)
{
    return (float)(h >> 8);
}

__device__ __forceinline__ float hash_uniform(uint32_t h)
{
    return hash_m(h) * 0x1p-24f;
}

__device__ __forceinline__ float axis_uniform(uint32_t b, uint32_t a)
{
    return hash_uniform(pcg(b + a));
}

// The hash of index a from base = b * M + C (the state of pcg(b)):
// (b + a) * M + C = base + a * M (mod 2^32), so the indices of one query
// share the first multiply.
__device__ __forceinline__ uint32_t pcg_from_base(uint32_t base, uint32_t a)
{
    const uint32_t state = base + a * 747796405u;
    const uint32_t word = ((state >> ((state >> 28u) + 4u)) ^ state) * 277803737u;
    return (word >> 22u) ^ word;
}

__device__ __forceinline__ uint32_t pcg_base(uint32_t b)
{
    return b * 747796405u + 2891336453u;
}

// pcg(b), pcg(b + 1), pcg(b + 2) with one shared multiply.
__device__ __forceinline__ void pcg_axes3(uint32_t b, uint32_t& h0, uint32_t& h1, uint32_t& h2)
{
    const uint32_t base = pcg_base(b);
    h0 = pcg_from_base(base, 0u);
    h1 = pcg_from_base(base, 1u);
    h2 = pcg_from_base(base, 2u);
}

// Cell of one binary32 coordinate: i = floor(x), t = x - floor(x).  Returns
// false for NaN, infinities and |x| >= 2^24 (no representable cell).
__device__ __forceinline__ bool cell_of(float x, int& i, float& t)
{
    if (!(__builtin_fabsf(x) < 16777216.0f)) return false;
    float f = __builtin_floorf(x);
    i = (int)f;
    t = x - f;
    return true;
}

constexpr float K6 = 0x1.555556p-3f;   // (float)(1/6)

// Six times the four cubic B-spline weights of the taps i-1..i+2 for the
// fractional offset t (Eq. cubic-bspline at distances t+1, t, 1-t, 2-t),
// written so every term is non-negative:
//   6 w0 = s^3, 6 w1 = 1 + 3s(1 + st), 6 w2 = 1 + 3t(1 + st), 6 w3 = t^3,
// with s = 1 - t.  They sum to 6.
struct Cubic6 {
    float a0, a1, a2, a3;
};

__device__ __forceinline__ Cubic6 cubic6(float t)
{
    float s = 1.0f - t;
    float st = s * t;
    Cubic6 w;
    w.a0 = (s * s) * s;
    w.a1 = 1.0f + (3.0f * s) * (1.0f + st);
    w.a2 = 1.0f + (3.0f * t) * (1.0f + st);
    w.a3 = (t * t) * t;
    return w;
}

constexpr float TWO24 = 16777216.0f;

// Tap offset from cell i chosen by the uniform on one axis ("sampling
// arrays": the first tap whose cumulative weight exceeds u).  m = u * 2^24.
//   linear: +1 iff u < t (strict comparison), else 0;
//   cubic:  -1 + [u >= c1] + [u >= c2] + [u >= c3] at the cumulative
//           B-spline weights c1 = w0 = ((s*s)*s)*K6, c2 = c1 + w1 with
//           w1 = (4 + (3*(t*t))*(t - 2))*K6, and c3 = 1 - w3 =
//           1 - ((t*t)*t)*K6 (s = 1 - t), each operation one binary32
//           rounding.  Since c1 <= c2 <= c3 for every binary32 t in [0, 1),
//           the sum equals (u >= c2 ? 1 : -1) + [u >= c_side] with c_side =
//           c3 above c2 and c1 below it.
__device__ __forceinline__ int choose_linear_m(float t, float m)
{
    return (m < t * TWO24) ? 1 : 0;
}

__device__ __forceinline__ int choose_cubic_m(float t, float m)
{
    constexpr float K6S = K6 * TWO24;
    const float s = 1.0f - t;
    const float c1 = ((s * s) * s) * K6S;
    const float c2 = c1 + (4.0f + (3.0f * (t * t)) * (t - 2.0f)) * K6S;
    const bool hi = m >= c2;
    const float side = hi ? TWO24 - ((t * t) * t) * K6S : c1;
    return (hi ? 1 : -1) + (int)(m >= side);
}

__device__ __forceinline__ int choose_linear(float t, float u)
{
    return choose_linear_m(t, u * TWO24);
}

__device__ __forceinline__ int choose_cubic(float t, float u)
{
    return choose_cubic_m(t, u * TWO24);
}

// ---------------------------------------------------------------------------
// exact decoding of stored values to binary32
// ---------------------------------------------------------------------------
__device__ __forceinline__ float dec_f16(uint16_t h)
{
    return (float)__builtin_bit_cast(_Float16, h);
}

__device__ __forceinline__ float dec_bf16(uint16_t h)
{
    return __builtin_bit_cast(float, (uint32_t)h << 16);
}

// OCP E4M3 "FN": bias 7, subnormals m * 2^-9, no infinity, S.1111.111 NaN.
// gfx950's conversion instruction implements exactly this format: for all 256
// codes it returns the same binary32 bits as the definition (sign, exponent
// e - 7 + 127 for e >= 1, m * 2^-9 for e = 0) and a NaN for the two NaN codes.
// `sel` picks the byte of q (a constant 0..3).
template <int sel = 0>
__device__ __forceinline__ float dec_e4m3_byte(uint32_t q)
{
    return __builtin_amdgcn_cvt_f32_fp8((int)q, sel);
}

__device__ __forceinline__ float dec_e4m3(uint32_t q)
{
    return dec_e4m3_byte<0>(q);
}

// v / 255 correctly rounded, for v = 0..255: the product with fl(1/255) and
// one residual correction, e = v - q 255 and q + e fl(1/255) (each an FMA,
// so rounded once), reaches the correctly rounded quotient for every one of
// the 256 codes (checked in exact rational arithmetic), without a division
// sequence.
__device__ __forceinline__ float dec_u8(uint32_t v)
{
    constexpr float R = 0x1.010102p-8f;   // fl(1/255)
    const float x = (float)v;             // exact
    const float q = x * R;
    const float e = __builtin_fmaf(-q, 255.0f, x);
    return __builtin_fmaf(e, R, q);
}

template <int FMT>
__device__ __forceinline__ float load_texel(const void* __restrict__ base, int64_t i)
{
    if constexpr (FMT == F32) return reinterpret_cast<const float*>(base)[i];
    if constexpr (FMT == F16) return dec_f16(reinterpret_cast<const uint16_t*>(base)[i]);
    if constexpr (FMT == BF16) return dec_bf16(reinterpret_cast<const uint16_t*>(base)[i]);
    if constexpr (FMT == FP8_E4M3) return dec_e4m3(reinterpret_cast<const uint8_t*>(base)[i]);
    if constexpr (FMT == U8) return dec_u8(reinterpret_cast<const uint8_t*>(base)[i]);
    return 0.0f;
}

constexpr int32_t BAD_INDEX = (int32_t)0x80000000;

}  // namespace stf
