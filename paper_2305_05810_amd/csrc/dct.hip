// dct.hip -- DCT-compressed 2D textures (section "Results", texture
// compression): the host-side encoder and texture creation.  Decoding and
// filtering run in the 2D kernels (filter2d.hip, dct_decode.h).
//
// Encoding of one channel of an 8x8 block of 8-bit texels f = v/255: the
// orthonormal 2D DCT-II evaluated separably in binary64 (rows, then
// columns), the six zigzag coefficients (v, u) = (0,0), (0,1), (1,0), (2,0),
// (1,1), (0,2) quantised to a 7-bit DC code round(F * 127/8) in 0..127 and
// 5-bit AC codes round(F * 15/2) in -15..15 stored + 16; round half away
// from zero.  Word: bits 0..6 DC, then 5 bits per AC code in zigzag order.
#include <cmath>
#include <new>
#include <vector>

#include "stf_internal.h"

namespace {

constexpr double kPi = 3.14159265358979323846;

struct DctTables {
    double t[3][8];   // t[k][i] = a(k) cos((2i + 1) k pi / 16), k = 0..2
    DctTables()
    {
        for (int k = 0; k < 3; ++k)
            for (int i = 0; i < 8; ++i)
                t[k][i] = (k == 0 ? std::sqrt(0.125) : 0.5) * std::cos((2 * i + 1) * k * kPi / 16.0);
    }
};

const DctTables& tables()
{
    static const DctTables tb;
    return tb;
}

uint32_t encode_block(const uint8_t* texels, int64_t row_stride, int channels)
{
    const DctTables& tb = tables();
    // r[k][y] = sum_x t[k][x] f(x, y): horizontal frequencies 0..2 per row
    double r[3][8];
    for (int y = 0; y < 8; ++y)
        for (int k = 0; k < 3; ++k) {
            double s = 0.0;
            for (int x = 0; x < 8; ++x) s += tb.t[k][x] * (texels[y * row_stride + (int64_t)x * channels] / 255.0);
            r[k][y] = s;
        }
    static const int zz_v[6] = {0, 0, 1, 2, 1, 0}, zz_u[6] = {0, 1, 0, 0, 1, 2};
    uint32_t word = 0;
    for (int k = 0; k < 6; ++k) {
        double F = 0.0;
        for (int y = 0; y < 8; ++y) F += tb.t[zz_v[k]][y] * r[zz_u[k]][y];
        if (k == 0) {
            double c = std::round(F * 127.0 / 8.0);
            word |= (uint32_t)(c < 0.0 ? 0.0 : (c > 127.0 ? 127.0 : c));
        } else {
            double c = std::round(F * 15.0 / 2.0);
            int q = (int)(c < -15.0 ? -15.0 : (c > 15.0 ? 15.0 : c));
            word |= (uint32_t)(q + 16) << (7 + 5 * (k - 1));
        }
    }
    return word;
}

stf_status check_dct_size(int32_t width, int32_t height, int32_t channels)
{
    if (width <= 0 || height <= 0 || width > 65536 || height > 65536 || width % 8 || height % 8)
        return stf_fail(STF_E_INVALID, "DCT texture size %dx%d: multiples of 8 up to 65536 required", width, height);
    if (channels < 1 || channels > 16) return stf_fail(STF_E_INVALID, "channels = %d out of range (1..16)", channels);
    return STF_OK;
}

}  // namespace

extern "C" {

stf_status stf_dct_encode(int32_t width, int32_t height, int32_t channels, const uint8_t* texels_host,
                          uint32_t* blocks_host)
{
    stf_clear_error();
    stf_status s = check_dct_size(width, height, channels);
    if (s != STF_OK) return s;
    if (!texels_host || !blocks_host) return stf_fail(STF_E_INVALID, "texels_host or blocks_host is NULL");
    const int bw = width / 8, bh = height / 8;
    const int64_t row = (int64_t)width * channels;
    for (int by = 0; by < bh; ++by)
        for (int bx = 0; bx < bw; ++bx)
            for (int c = 0; c < channels; ++c)
                blocks_host[((int64_t)by * bw + bx) * channels + c] =
                    encode_block(texels_host + (int64_t)by * 8 * row + (int64_t)bx * 8 * channels + c, row, channels);
    return STF_OK;
}

stf_status stf_create_dct_texture2d(int32_t width, int32_t height, int32_t channels, const uint32_t* blocks_host,
                                    stf_texture** out)
{
    stf_clear_error();
    if (!out) return stf_fail(STF_E_INVALID, "out is NULL");
    *out = nullptr;
    stf_status s = check_dct_size(width, height, channels);
    if (s != STF_OK) return s;
    if (!blocks_host) return stf_fail(STF_E_INVALID, "blocks_host is NULL");
    const int64_t nblocks = (int64_t)(width / 8) * (height / 8);
    const int wpb = (channels + 3) / 4 * 4;
    std::vector<uint32_t> padded;
    try {
        padded.assign((size_t)(nblocks * wpb), 0u);
    } catch (const std::bad_alloc&) {
        return stf_fail(STF_E_OOM, "host allocation failed");
    }
    for (int64_t b = 0; b < nblocks; ++b)
        for (int c = 0; c < channels; ++c) padded[(size_t)(b * wpb + c)] = blocks_host[b * channels + c];
    stf_texture* t = new (std::nothrow) stf_texture();
    if (!t) return stf_fail(STF_E_OOM, "host allocation failed");
    t->kind = STF_KIND_DCT2D;
    t->fmt = -1;
    t->channels = channels;
    t->levels = 1;
    t->dct_wpb = wpb;
    (void)hipGetDevice(&t->device);
    const size_t bytes = padded.size() * 4;
    void* d = nullptr;
    hipError_t e = hipMalloc(&d, bytes);
    if (e == hipSuccess) e = hipMemcpy(d, padded.data(), bytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        if (d) (void)hipFree(d);
        delete t;
        return stf_fail(STF_E_OOM, "DCT block upload of %zu bytes failed: %s", bytes, hipGetErrorString(e));
    }
    t->level_alloc[0] = d;
    t->level[0].texels = d;
    t->level[0].w = width;
    t->level[0].h = height;
    t->bytes = (int64_t)bytes;
    *out = t;
    return STF_OK;
}

}  // extern "C"
