// shade.hip -- filtering with shading, section "Effect of Texture Filtering
// on Rendering" (Eqs. traditional-lighting-integral and
// our-lighting-integral): the texture filter applied to the material before
// the BSDF (shade after filter), to the shaded results of every tap (filter
// after shade), or sampled so that only one tap is shaded (stochastic; the
// filter factor f/p is 1).
//
// Shading is f^ = BSDF * cos(theta_i) for one incident direction: a GGX
// microfacet lobe (Trowbridge-Reitz D, height-correlated Smith G2, Schlick F
// with F0 = 0.04) plus a Lambertian albedo term, evaluated in binary32.
#include <math.h>

#include "device_common.h"
#include "stf_internal.h"

using namespace stf;

namespace {

constexpr int BLOCK = 256;
constexpr float INV_PI = 0.318309886183790672f;

struct Material {
    float albedo[3];
    float rough;
    float nx, ny;
};

__device__ __forceinline__ Material decode_material(uint2 t)
{
    Material m;
    m.albedo[0] = dec_u8(t.x & 0xffu);
    m.albedo[1] = dec_u8((t.x >> 8) & 0xffu);
    m.albedo[2] = dec_u8((t.x >> 16) & 0xffu);
    m.rough = dec_u8(t.x >> 24);
    m.nx = dec_f16((uint16_t)(t.y & 0xffffu));
    m.ny = dec_f16((uint16_t)(t.y >> 16));
    return m;
}

struct V3 {
    float x, y, z;
};

__device__ __forceinline__ float dot(V3 a, V3 b)
{
    return a.x * b.x + a.y * b.y + a.z * b.z;
}

__device__ __forceinline__ float cross_norm2(V3 a, V3 b)
{
    float cx = a.y * b.z - a.z * b.y;
    float cy = a.z * b.x - a.x * b.z;
    float cz = a.x * b.y - a.y * b.x;
    return cx * cx + cy * cy + cz * cz;
}

// The shading arithmetic uses the hardware's reciprocal, square root and
// reciprocal square root (about one ulp each) instead of correctly rounded
// division and square root sequences: the shaded value is already sensitive
// to the binary32 rounding of the half vector at the 1e-5 level, and no
// decision of the filter depends on it.
__device__ __forceinline__ float frcp(float x)
{
    return __builtin_amdgcn_rcpf(x);
}

__device__ __forceinline__ float fsqrt(float x)
{
    return __builtin_amdgcn_sqrtf(x);
}

// Smith Lambda of GGX: (-1 + sqrt(1 + alpha^2 tan^2)) / 2.
__device__ __forceinline__ float lambda_ggx(V3 n, V3 w, float nw, float a2)
{
    float tan2 = cross_norm2(n, w) * frcp(nw * nw);
    return 0.5f * (-1.0f + fsqrt(1.0f + a2 * tan2));
}

// f^ for one material, directions in the tangent frame.
__device__ __forceinline__ void shade(const Material& m, V3 wo, V3 wi, float (&f)[3])
{
    V3 n = {m.nx, m.ny, fsqrt(fmaxf(0.0f, 1.0f - m.nx * m.nx - m.ny * m.ny))};
    float alpha = fmaxf(m.rough * m.rough, 1e-3f), a2 = alpha * alpha;
    float no = dot(n, wo), ni = dot(n, wi);
    if (!(no > 0.0f) || !(ni > 0.0f)) {
        f[0] = f[1] = f[2] = 0.0f;
        return;
    }
    V3 h = {wo.x + wi.x, wo.y + wi.y, wo.z + wi.z};
    float il = __builtin_amdgcn_rsqf(dot(h, h));
    h.x *= il;
    h.y *= il;
    h.z *= il;
    float nh = dot(n, h);
    float den = nh * nh * a2 + cross_norm2(n, h);
    float D = a2 * INV_PI * frcp(den * den);
    float G2 = frcp(1.0f + lambda_ggx(n, wo, no, a2) + lambda_ggx(n, wi, ni, a2));
    float x = 1.0f - dot(wi, h), x2 = x * x;
    float F = 0.04f + 0.96f * (x2 * x2 * x);
    float spec = D * G2 * F * frcp(4.0f * no * ni);
#pragma unroll
    for (int c = 0; c < 3; ++c) f[c] = (m.albedo[c] * INV_PI + spec) * ni;
}

__device__ __forceinline__ int clampi(int v, int hi)
{
    return v < 0 ? 0 : (v > hi ? hi : v);
}

struct Levels {
    TexLevel lv[3];
    int32_t n;
};

template <bool CUBIC, int MODE>
__global__ __launch_bounds__(BLOCK) void k_shade(Levels L, const float* __restrict__ q, int32_t n, uint32_t key,
                                                 float* __restrict__ out, int32_t* __restrict__ idx)
{
    int32_t i = blockIdx.x * BLOCK + threadIdx.x;
    if (i >= n) return;
    const float* e = q + 9 * (int64_t)i;
    float r[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) r[k] = __builtin_nontemporal_load(e + k);   // streamed in
    float u = r[0], v = r[1], s = r[2];
    V3 wo = {r[3], r[4], r[5]}, wi = {r[6], r[7], r[8]};
    int l = (int)(s >= 1.41421354f) + (int)(s >= 2.82842708f);
    l = l < L.n - 1 ? l : L.n - 1;
    TexLevel T = l == 0 ? L.lv[0] : (l == 1 ? L.lv[1] : L.lv[2]);
    const uint2* tex = reinterpret_cast<const uint2*>(T.texels);
    float x = u * (float)T.w - 0.5f, y = v * (float)T.h - 0.5f;
    int cx = 0, cy = 0;
    float tx = 0.0f, ty = 0.0f;
    bool ok = cell_of(x, cx, tx) & cell_of(y, cy, ty);
    float f[3] = {__builtin_nanf(""), __builtin_nanf(""), __builtin_nanf("")};
    if (ok) {
        if constexpr (MODE == STF_SHADE_STOCHASTIC) {
            const uint32_t b = pcg(key ^ (uint32_t)i);
            const uint32_t base = pcg_base(b);
            const float mx = hash_m(pcg_from_base(base, 0u)), my = hash_m(pcg_from_base(base, 1u));
            int sx, sy;
            if constexpr (CUBIC) {
                sx = cx + choose_cubic_m(tx, mx);
                sy = cy + choose_cubic_m(ty, my);
            } else {
                sx = cx + choose_linear_m(tx, mx);
                sy = cy + choose_linear_m(ty, my);
            }
            sx = clampi(sx, T.w - 1);
            sy = clampi(sy, T.h - 1);
            shade(decode_material(tex[material_index(sx, sy, T.w)]), wo, wi, f);
            if (idx) {
                idx[3 * (int64_t)i] = sx;
                idx[3 * (int64_t)i + 1] = sy;
                idx[3 * (int64_t)i + 2] = l;
            }
        } else {
            constexpr int NT = CUBIC ? 4 : 2;
            float wx[NT], wy[NT];
            if constexpr (CUBIC) {
                Cubic6 a = cubic6(tx), b = cubic6(ty);
                wx[0] = a.a0 * K6; wx[1] = a.a1 * K6; wx[2] = a.a2 * K6; wx[3] = a.a3 * K6;
                wy[0] = b.a0 * K6; wy[1] = b.a1 * K6; wy[2] = b.a2 * K6; wy[3] = b.a3 * K6;
                cx -= 1;
                cy -= 1;
            } else {
                wx[0] = 1.0f - tx; wx[1] = tx;
                wy[0] = 1.0f - ty; wy[1] = ty;
            }
            // all taps' texels first: their loads are then in flight together
            // instead of one latency per tap between shading evaluations
            uint2 texel[NT][NT];
#pragma unroll
            for (int b = 0; b < NT; ++b) {
                const int yy = clampi(cy + b, T.h - 1);
#pragma unroll
                for (int a = 0; a < NT; ++a) texel[b][a] = tex[material_index(clampi(cx + a, T.w - 1), yy, T.w)];
            }
            float acc[6] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int b = 0; b < NT; ++b) {
#pragma unroll
                for (int a = 0; a < NT; ++a) {
                    Material m = decode_material(texel[b][a]);
                    float w = wx[a] * wy[b];
                    if constexpr (MODE == STF_SHADE_AFTER_FILTER) {
                        acc[0] = __builtin_fmaf(w, m.albedo[0], acc[0]);
                        acc[1] = __builtin_fmaf(w, m.albedo[1], acc[1]);
                        acc[2] = __builtin_fmaf(w, m.albedo[2], acc[2]);
                        acc[3] = __builtin_fmaf(w, m.rough, acc[3]);
                        acc[4] = __builtin_fmaf(w, m.nx, acc[4]);
                        acc[5] = __builtin_fmaf(w, m.ny, acc[5]);
                    } else {
                        float g[3];
                        shade(m, wo, wi, g);
                        acc[0] = __builtin_fmaf(w, g[0], acc[0]);
                        acc[1] = __builtin_fmaf(w, g[1], acc[1]);
                        acc[2] = __builtin_fmaf(w, g[2], acc[2]);
                    }
                }
            }
            if constexpr (MODE == STF_SHADE_AFTER_FILTER) {
                Material m;
                m.albedo[0] = acc[0]; m.albedo[1] = acc[1]; m.albedo[2] = acc[2];
                m.rough = acc[3]; m.nx = acc[4]; m.ny = acc[5];
                shade(m, wo, wi, f);
            } else {
                f[0] = acc[0]; f[1] = acc[1]; f[2] = acc[2];
            }
        }
    } else if (idx && MODE == STF_SHADE_STOCHASTIC) {
        idx[3 * (int64_t)i] = BAD_INDEX;
        idx[3 * (int64_t)i + 1] = BAD_INDEX;
        idx[3 * (int64_t)i + 2] = BAD_INDEX;
    }
    // results are streamed out (nontemporal stores)
    __builtin_nontemporal_store(f[0], out + 3 * (int64_t)i);
    __builtin_nontemporal_store(f[1], out + 3 * (int64_t)i + 1);
    __builtin_nontemporal_store(f[2], out + 3 * (int64_t)i + 2);
}

template <bool CUBIC>
hipError_t launch_shade_f(const Levels& L, const float* q, int32_t n, int mode, uint32_t key, float* out,
                          int32_t* idx, hipStream_t s)
{
    dim3 grid((n + BLOCK - 1) / BLOCK), block(BLOCK);
    switch (mode) {
    case STF_SHADE_AFTER_FILTER:
        hipLaunchKernelGGL((k_shade<CUBIC, STF_SHADE_AFTER_FILTER>), grid, block, 0, s, L, q, n, key, out, idx);
        break;
    case STF_FILTER_AFTER_SHADE:
        hipLaunchKernelGGL((k_shade<CUBIC, STF_FILTER_AFTER_SHADE>), grid, block, 0, s, L, q, n, key, out, idx);
        break;
    default:
        hipLaunchKernelGGL((k_shade<CUBIC, STF_SHADE_STOCHASTIC>), grid, block, 0, s, L, q, n, key, out, idx);
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_shade(const stf_texture* mat, const float* q, int32_t n, int filter, int mode, uint32_t key,
                        float* out, int32_t* idx, hipStream_t s)
{
    Levels L;
    L.n = mat->levels < 3 ? mat->levels : 3;
    for (int l = 0; l < 3; ++l) L.lv[l] = mat->level[l < L.n ? l : L.n - 1];
    return filter == STF_CUBIC_BSPLINE ? launch_shade_f<true>(L, q, n, mode, key, out, idx, s)
                                       : launch_shade_f<false>(L, q, n, mode, key, out, idx, s);
}
