// dct_decode.h -- single-texel decoding of DCT-compressed textures (section
// "Results", texture compression: 8x8 blocks, six lowest-frequency DCT
// coefficients per channel in one 32-bit word, 7-bit DC and 5-bit AC).
//
// Word layout: bits 0..6 DC code d; then five 5-bit AC codes (bits 7..11,
// 12..16, 17..21, 22..26, 27..31) for the zigzag coefficients (v, u) =
// (0,1), (1,0), (2,0), (1,1), (0,2), each stored as q + 16 with q in
// -15..15.  Dequantised values: d * 8/127 and q * 2/15.  The texel at (x, y)
// of its block is the orthonormal inverse DCT of these six coefficients:
//   f = a0^2 d 8/127 + sum_k q_k (2/15) a(u_k) a(v_k) cos((2x+1) u_k pi/16) cos((2y+1) v_k pi/16)
// with a(0) = sqrt(1/8), a(k > 0) = 1/2.  So f = d/127 + K (q1 c1(x) +
// q2 c1(y) + q3 c2(y) + q5 c2(x)) + K11 q4 c1(x) c1(y), where c1(i) =
// cos((2i+1) pi/16), c2(i) = cos((2i+1) pi/8), K = (2/15)/(4 sqrt 2) and
// K11 = (2/15)/4.
//
// Device layout: blocks row-major, CAP words per block (channels padded with
// zero words to a multiple of 4, so a block's channels load as 16-byte
// vectors).
#pragma once

#include "device_common.h"

namespace stf {

constexpr float DCT_DC = 0x1.020408p-7f;           // fl32(1/127)
constexpr float DCT_K = 0x1.822cb2p-6f;            // fl32((2/15) / (4 sqrt 2)) = 0.0235702...
constexpr float DCT_K11 = 0x1.111112p-5f;          // fl32((2/15) / 4) = 0.0333333...
// |cos(k pi/16)| for k = 1, 3, 5, 7 and |cos(k pi/8)| for k = 1, 3
constexpr float DCT_C1 = 0x1.f6297cp-1f, DCT_C3 = 0x1.a9b662p-1f, DCT_C5 = 0x1.1c73b4p-1f, DCT_C7 = 0x1.8f8b84p-3f;
constexpr float DCT_D1 = 0x1.d906bcp-1f, DCT_D3 = 0x1.87de2ap-2f;

// c1(i) = cos((2i+1) pi/16): +C1 +C3 +C5 +C7 -C7 -C5 -C3 -C1 for i = 0..7.
__device__ __forceinline__ float dct_c1(int i)
{
    int j = i < 4 ? i : 7 - i;
    float m = j == 0 ? DCT_C1 : (j == 1 ? DCT_C3 : (j == 2 ? DCT_C5 : DCT_C7));
    return i < 4 ? m : -m;
}

// c2(i) = cos((2i+1) pi/8): +D1 +D3 -D3 -D1 -D1 -D3 +D3 +D1 for i = 0..7.
__device__ __forceinline__ float dct_c2(int i)
{
    float m = (i == 0 || i == 3 || i == 4 || i == 7) ? DCT_D1 : DCT_D3;
    return (i >= 2 && i <= 5) ? -m : m;
}

// The five AC basis values of texel (xi, yi) of a block, scaled by the
// dequantisation step: B[k-1] for zigzag coefficient k = 1..5.
struct DctBasis {
    float b[5];
};

__device__ __forceinline__ DctBasis dct_basis(int xi, int yi)
{
    const float c1x = dct_c1(xi), c1y = dct_c1(yi), c2x = dct_c2(xi), c2y = dct_c2(yi);
    DctBasis B;
    B.b[0] = DCT_K * c1x;           // (v, u) = (0, 1)
    B.b[1] = DCT_K * c1y;           // (1, 0)
    B.b[2] = DCT_K * c2y;           // (2, 0)
    B.b[3] = (DCT_K11 * c1x) * c1y; // (1, 1)
    B.b[4] = DCT_K * c2x;           // (0, 2)
    return B;
}

// Decode one channel word at a texel with basis B.  The AC codes become
// 5-bit two's complement q by flipping bit 4 of every field (q + 16 xor 16 =
// q mod 32), and are sign-extended by a signed bit-field extract.
__device__ __forceinline__ float dct_decode_word(uint32_t word, const DctBasis& B)
{
    const uint32_t w = word ^ 0x84210800u;   // bit 4 of each AC field (bits 11, 16, 21, 26, 31)
    float f = (float)(word & 127u) * DCT_DC;
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        const int q = __builtin_amdgcn_sbfe((int)w, 7 + 5 * k, 5);
        f = __builtin_fmaf((float)q, B.b[k], f);
    }
    return f;
}

}  // namespace stf
