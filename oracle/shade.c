/*
 * shade.c -- oracle for filtering with shading (test infrastructure only).
 *
 * Section "Effect of Texture Filtering on Rendering" of Fajardo et al. writes
 * outgoing radiance with the texture filter either inside the BSDF's
 * arguments (Eq. traditional-lighting-integral: filter the material, then
 * shade) or outside the lighting integral (Eq. our-lighting-integral: shade
 * every texel, then filter the shaded results); sampling the filter makes the
 * second one a single shading evaluation per lookup (the closing paragraph of
 * that section: f/p = 1).  Here the lighting integral is a single incident
 * direction, so the quantity filtered is f^ = BSDF * cos(theta_i) itself.
 *
 * The BSDF is a GGX microfacet model (Trowbridge-Reitz normal distribution,
 * height-correlated Smith masking-shadowing, Schlick Fresnel with F0 = 0.04)
 * plus a Lambertian term; all arithmetic is binary64.  Tap choice and level
 * choice are the pinned binary32 rules of oracle.c.
 *
 * Material texel (8 bytes): albedo RGB UNORM8, roughness UNORM8, tangent
 * normal x and y binary16.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* from oracle.c */
float orc_uniform(uint64_t seed, uint32_t qid, uint32_t axis);
int orc_select(int filter, float t, float u);
void orc_axis_weights(int filter, double t, double w[4]);

enum { SH_AFTER_FILTER = 0, SH_FILTER_AFTER = 1, SH_STOCH = 2 };

#define ORC_PI 3.14159265358979323846

static double orc_h2d(uint16_t h)
{
    int sign = (h >> 15) & 1, e = (h >> 10) & 31, m = h & 1023;
    double v = (e == 0) ? ldexp((double)m, -24) : (e == 31 ? (m ? NAN : INFINITY) : ldexp((double)(1024 + m), e - 25));
    return sign ? -v : v;
}

void orc_material_decode(const uint8_t* texel, double out[6])
{
    uint16_t hx, hy;
    memcpy(&hx, texel + 4, 2);
    memcpy(&hy, texel + 6, 2);
    out[0] = texel[0] / 255.0;
    out[1] = texel[1] / 255.0;
    out[2] = texel[2] / 255.0;
    out[3] = texel[3] / 255.0;
    out[4] = orc_h2d(hx);
    out[5] = orc_h2d(hy);
}

static double dot3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

static void cross3(const double* a, const double* b, double* c)
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

/* Smith Lambda of the GGX distribution for direction w:
 * (-1 + sqrt(1 + alpha^2 tan^2 theta)) / 2, tan^2 = |n x w|^2 / (n.w)^2. */
static double orc_lambda(const double* n, const double* w, double a2)
{
    double c[3];
    cross3(n, w, c);
    double nw = dot3(n, w);
    double tan2 = dot3(c, c) / (nw * nw);
    return 0.5 * (-1.0 + sqrt(1.0 + a2 * tan2));
}

/* GGX normal distribution D(h) = alpha^2 / (pi ((n.h)^2 alpha^2 + |n x h|^2)^2)
 * for unit n, h. */
double orc_ggx_D(const double* n, const double* h, double alpha)
{
    double c[3];
    cross3(n, h, c);
    double nh = dot3(n, h), a2 = alpha * alpha;
    double den = nh * nh * a2 + dot3(c, c);
    return a2 / (ORC_PI * den * den);
}

/* The terms of the GGX specular lobe at unit normal n and unit directions
 * wo, wi (both above the surface): out = {D(h), Lambda(wo), Lambda(wi), G2,
 * F} with h = normalize(wo + wi), the height-correlated Smith
 * masking-shadowing G2 = 1 / (1 + Lambda(wo) + Lambda(wi)) (Heitz, "Understanding
 * the Masking-Shadowing Function", JCGT 2014) and Schlick's Fresnel
 * F = F0 + (1 - F0)(1 - wi.h)^5 with F0 = 0.04. */
void orc_ggx_terms(const double* n, const double* wo, const double* wi, double alpha, double out[5])
{
    double a2 = alpha * alpha;
    double h[3] = {wo[0] + wi[0], wo[1] + wi[1], wo[2] + wi[2]};
    double hl = sqrt(dot3(h, h));
    h[0] /= hl; h[1] /= hl; h[2] /= hl;
    out[0] = orc_ggx_D(n, h, alpha);
    out[1] = orc_lambda(n, wo, a2);
    out[2] = orc_lambda(n, wi, a2);
    out[3] = 1.0 / (1.0 + out[1] + out[2]);
    out[4] = 0.04 + 0.96 * pow(1.0 - dot3(wi, h), 5.0);
}

/* f^ = (albedo/pi + D G2 F / (4 (n.wo)(n.wi))) (n.wi) for one material. */
void orc_shade_eval(const double mat[6], const float* wo_f, const float* wi_f, double out[3])
{
    double wo[3] = {wo_f[0], wo_f[1], wo_f[2]}, wi[3] = {wi_f[0], wi_f[1], wi_f[2]};
    double nx = mat[4], ny = mat[5];
    double n[3] = {nx, ny, sqrt(fmax(0.0, 1.0 - nx * nx - ny * ny))};
    double r = mat[3];
    double alpha = fmax(r * r, 1e-3);
    double no = dot3(n, wo), ni = dot3(n, wi);
    if (!(no > 0.0) || !(ni > 0.0)) {
        out[0] = out[1] = out[2] = 0.0;
        return;
    }
    double g[5];
    orc_ggx_terms(n, wo, wi, alpha, g);
    double spec = g[0] * g[3] * g[4] / (4.0 * no * ni);
    for (int c = 0; c < 3; ++c) out[c] = (mat[c] / ORC_PI + spec) * ni;
}

/* Level choice from the footprint s: l = [s >= sqrt 2] + [s >= 2 sqrt 2]
 * (binary32 comparisons), capped at the last level. */
int orc_shade_level(float s, int levels)
{
    int l = (s >= 1.41421354f) + (s >= 2.82842708f);
    return l < levels - 1 ? l : levels - 1;
}

static int clampi(int v, int hi) { return v < 0 ? 0 : (v > hi ? hi : v); }

/* One shading query: record = uv(2), s, wo(3), wi(3). */
static void orc_shade_query(const uint8_t* const* lv, const int* W, const int* H, int levels, const float* rec,
                            int filter, int mode, uint64_t seed, uint32_t qid, double* out, int32_t* idx)
{
    int l = orc_shade_level(rec[2], levels);
    const uint8_t* tex = lv[l];
    int w = W[l], h = H[l];
    float x = rec[0] * (float)w - 0.5f, y = rec[1] * (float)h - 0.5f;
    const float* wo = rec + 3;
    const float* wi = rec + 6;
    if (!(fabsf(x) < 16777216.0f) || !(fabsf(y) < 16777216.0f)) {
        out[0] = out[1] = out[2] = NAN;
        if (idx) idx[0] = idx[1] = idx[2] = (int32_t)0x80000000;
        return;
    }
    float fx = floorf(x), fy = floorf(y);
    int ix = (int)fx, iy = (int)fy;
    int base = filter ? -1 : 0, nt = filter ? 4 : 2;
    double mat[6];
    if (mode == SH_STOCH) {
        int sx = clampi(ix + orc_select(filter, x - fx, orc_uniform(seed, qid, 0)), w - 1);
        int sy = clampi(iy + orc_select(filter, y - fy, orc_uniform(seed, qid, 1)), h - 1);
        orc_material_decode(tex + 8 * ((int64_t)sy * w + sx), mat);
        orc_shade_eval(mat, wo, wi, out);
        if (idx) { idx[0] = sx; idx[1] = sy; idx[2] = l; }
        return;
    }
    double wx[4], wy[4];
    orc_axis_weights(filter, (double)x - floor((double)x), wx);
    orc_axis_weights(filter, (double)y - floor((double)y), wy);
    double acc[6] = {0, 0, 0, 0, 0, 0};
    out[0] = out[1] = out[2] = 0.0;
    for (int b = 0; b < nt; ++b)
        for (int a = 0; a < nt; ++a) {
            int tx = clampi(ix + base + a, w - 1), ty = clampi(iy + base + b, h - 1);
            double wt = wx[a] * wy[b];
            orc_material_decode(tex + 8 * ((int64_t)ty * w + tx), mat);
            if (mode == SH_AFTER_FILTER) {
                for (int c = 0; c < 6; ++c) acc[c] += wt * mat[c];
            } else {
                double f[3];
                orc_shade_eval(mat, wo, wi, f);
                for (int c = 0; c < 3; ++c) out[c] += wt * f[c];
            }
        }
    if (mode == SH_AFTER_FILTER) orc_shade_eval(acc, wo, wi, out);
}

int orc_shade(const uint8_t* const* levels_px, const int* W, const int* H, int levels, const float* recs,
                     int64_t n, int filter, int mode, uint64_t seed, double* out, int32_t* idx, int nthreads)
{
    if (levels < 1 || n < 0) return -1;
#ifdef _OPENMP
    int nt = nthreads > 0 ? nthreads : omp_get_max_threads();
#endif
#pragma omp parallel for schedule(static) num_threads(nt)
    for (int64_t q = 0; q < n; ++q)
        orc_shade_query(levels_px, W, H, levels, recs + 9 * q, filter, mode, seed, (uint32_t)q, out + 3 * q,
                        idx ? idx + 3 * q : NULL);
    return 0;
}

/* Shading queries recs[qids[k]] evaluated as members of the whole batch (the
 * draw of a query depends on its index). */
int orc_shade_at(const uint8_t* const* levels_px, const int* W, const int* H, int levels, const float* recs,
                 const int64_t* qids, int64_t m, int filter, int mode, uint64_t seed, double* out, int32_t* idx,
                 int nthreads)
{
    if (levels < 1 || m < 0) return -1;
#ifdef _OPENMP
    int nt = nthreads > 0 ? nthreads : omp_get_max_threads();
#endif
#pragma omp parallel for schedule(static) num_threads(nt)
    for (int64_t k = 0; k < m; ++k)
        orc_shade_query(levels_px, W, H, levels, recs + 9 * qids[k], filter, mode, seed, (uint32_t)qids[k],
                        out + 3 * k, idx ? idx + 3 * k : NULL);
    return 0;
}

/* Exact mean and variance (per colour channel) of the stochastic shading
 * estimator: the taps are drawn with probability equal to their weights, so
 * the mean is the filter-after-shade value and the variance is
 * sum w f^2 - mean^2. */
int orc_shade_moments(const uint8_t* const* levels_px, const int* W, const int* H, int levels, const float* recs,
                      int64_t n, int filter, double* mean, double* var)
{
    for (int64_t q = 0; q < n; ++q) {
        const float* rec = recs + 9 * q;
        int l = orc_shade_level(rec[2], levels);
        int w = W[l], h = H[l];
        float x = rec[0] * (float)w - 0.5f, y = rec[1] * (float)h - 0.5f;
        int ix = (int)floorf(x), iy = (int)floorf(y);
        int base = filter ? -1 : 0, nt = filter ? 4 : 2;
        double wx[4], wy[4], m1[3] = {0, 0, 0}, m2[3] = {0, 0, 0};
        orc_axis_weights(filter, (double)x - floor((double)x), wx);
        orc_axis_weights(filter, (double)y - floor((double)y), wy);
        for (int b = 0; b < nt; ++b)
            for (int a = 0; a < nt; ++a) {
                int tx = clampi(ix + base + a, w - 1), ty = clampi(iy + base + b, h - 1);
                double mat[6], f[3];
                orc_material_decode(levels_px[l] + 8 * ((int64_t)ty * w + tx), mat);
                orc_shade_eval(mat, rec + 3, rec + 6, f);
                for (int c = 0; c < 3; ++c) {
                    m1[c] += wx[a] * wy[b] * f[c];
                    m2[c] += wx[a] * wy[b] * f[c] * f[c];
                }
            }
        for (int c = 0; c < 3; ++c) {
            mean[3 * q + c] = m1[c];
            var[3 * q + c] = m2[c] - m1[c] * m1[c];
        }
    }
    return 0;
}
