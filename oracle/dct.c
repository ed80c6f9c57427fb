/*
 * dct.c -- DCT-compressed textures for the oracle (section "Results",
 * real-time rendering, paragraph on texture compression): 8x8 texel blocks,
 * per channel the six lowest-frequency coefficients of the 2D DCT in 32 bits
 * (7 bits for the DC coefficient, 5 bits for each of the other five), 16x
 * smaller than 8-bit texels.  A lookup decodes single texels.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.c): nothing in the product library
 * calls, links or includes this file.
 *
 * The paper gives the budget but not the transform's scaling, the
 * coefficient order or the quantiser; this file pins them:
 *   - texel value f = v / 255 (8-bit UNORM input);
 *   - orthonormal 8x8 DCT-II,
 *       F(u, v) = a(u) a(v) sum_{x,y} f(x, y) cos((2x+1) u pi/16) cos((2y+1) v pi/16),
 *     a(0) = sqrt(1/8), a(k > 0) = 1/2, u horizontal and v vertical frequency;
 *   - kept coefficients in zigzag order (v, u) = (0,0), (0,1), (1,0), (2,0),
 *     (1,1), (0,2);
 *   - DC code d = clamp(round(F(0,0) * 127/8), 0, 127), value d * 8/127
 *     (F(0,0) = 8 * mean lies in [0, 8]);
 *   - AC code q = clamp(round(F * 15/2), -15, 15), value q * 2/15, stored as
 *     q + 16 (range +-2; larger coefficients saturate);
 *   - round() is to nearest with halves away from zero;
 *   - word layout: bits 0..6 DC, then 5 bits per AC coefficient in zigzag
 *     order (bits 7..11, 12..16, 17..21, 22..26, 27..31);
 *   - decoded texel = the inverse DCT of the six dequantised coefficients
 *     (the others zero), not clamped;
 *   - blocks row-major over the texture, C words per block (channel order).
 */
#include <math.h>
#include <stdint.h>

#define ORC_PI 3.14159265358979323846

static const int ORC_ZZ_V[6] = {0, 0, 1, 2, 1, 0};   /* vertical frequency of coefficient k */
static const int ORC_ZZ_U[6] = {0, 1, 0, 0, 1, 2};   /* horizontal frequency */

static double orc_dct_a(int k) { return k == 0 ? sqrt(1.0 / 8.0) : 0.5; }

static double orc_dct_cos(int i, int k) { return cos((2.0 * i + 1.0) * k * ORC_PI / 16.0); }

/* The orthonormal DCT-II coefficient F(u, v) of one 8x8 block (f[y][x]). */
double orc_dct_coefficient(const double f[8][8], int u, int v)
{
    double s = 0.0;
    for (int y = 0; y < 8; ++y)
        for (int x = 0; x < 8; ++x) s += f[y][x] * orc_dct_cos(x, u) * orc_dct_cos(y, v);
    return orc_dct_a(u) * orc_dct_a(v) * s;
}

static int orc_clamp_code(double r, int lo, int hi) { return r < lo ? lo : (r > hi ? hi : (int)r); }

/* Dequantised value of coefficient k (0 = DC) of a word. */
double orc_dct_dequant(uint32_t word, int k)
{
    if (k == 0) return (double)(word & 127u) * 8.0 / 127.0;
    int q = (int)((word >> (7 + 5 * (k - 1))) & 31u) - 16;
    return (double)q * 2.0 / 15.0;
}

/* Encode W x H x C 8-bit texels (row-major, channels interleaved; W and H
 * multiples of 8) into (W/8)(H/8) C words. */
int orc_dct_encode(const uint8_t* texels, int W, int H, int C, uint32_t* blocks)
{
    if (W <= 0 || H <= 0 || W % 8 || H % 8 || C <= 0 || C > 16) return -1;
    int BW = W / 8, BH = H / 8;
    for (int by = 0; by < BH; ++by)
        for (int bx = 0; bx < BW; ++bx)
            for (int c = 0; c < C; ++c) {
                double f[8][8];
                for (int y = 0; y < 8; ++y)
                    for (int x = 0; x < 8; ++x)
                        f[y][x] = texels[((int64_t)(by * 8 + y) * W + (bx * 8 + x)) * C + c] / 255.0;
                uint32_t word = 0;
                for (int k = 0; k < 6; ++k) {
                    double F = orc_dct_coefficient(f, ORC_ZZ_U[k], ORC_ZZ_V[k]);
                    if (k == 0) {
                        word |= (uint32_t)orc_clamp_code(round(F * 127.0 / 8.0), 0, 127);
                    } else {
                        int q = orc_clamp_code(round(F * 15.0 / 2.0), -15, 15);
                        word |= (uint32_t)(q + 16) << (7 + 5 * (k - 1));
                    }
                }
                blocks[((int64_t)by * BW + bx) * C + c] = word;
            }
    return 0;
}

/* Decoded value of channel c of texel (x, y): the inverse DCT of the kept
 * coefficients at that texel. */
double orc_dct_texel(const uint32_t* blocks, int W, int C, int x, int y, int c)
{
    int BW = W / 8;
    uint32_t word = blocks[((int64_t)(y / 8) * BW + (x / 8)) * C + c];
    int xi = x % 8, yi = y % 8;
    double f = 0.0;
    for (int k = 0; k < 6; ++k) {
        int u = ORC_ZZ_U[k], v = ORC_ZZ_V[k];
        f += orc_dct_a(u) * orc_dct_a(v) * orc_dct_dequant(word, k) * orc_dct_cos(xi, u) * orc_dct_cos(yi, v);
    }
    return f;
}
