/*
 * neural.c -- oracle for the neural texture (test infrastructure only).
 *
 * The paper cites neural texture representations (section Introduction and
 * Background: neural and compressed encodings cost extra memory accesses and
 * computation for each texel lookup) and argues that stochastic filtering
 * decodes a single texel per lookup instead of one per filter tap.  Here the
 * decoded texel (i, j) of a W x H texture is
 *     y = W3 relu(W2 relu(W1 z + b1) + b2) + b3,
 * with z the bilinear interpolation of a LW x LH grid of 8-vectors at the
 * texel's centre, X = (i + 1/2) LW / W - 1/2 (clamped corners), and the
 * filters of oracle.c applied to decoded texels: the deterministic filter
 * decodes every tap, the stochastic one decodes the one sampled tap.
 *
 * Values are binary64.  With `emulate` set, values are rounded to bfloat16
 * (round to nearest even) where the inference kernel rounds them: the
 * interpolated latent z, every weight matrix, and each hidden activation
 * after its ReLU (biases and sums stay wide).
 *
 * MLP parameter vector (5256 values): W1[64][8], b1[64], W2[64][64], b2[64],
 * W3[8][64], b3[8] (row = output feature).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

float orc_uniform(uint64_t seed, uint32_t qid, uint32_t axis);
int orc_select(int filter, float t, float u);
void orc_axis_weights(int filter, double t, double w[4]);

#define NL 8    /* latent channels */
#define NH 64   /* hidden width */
#define NO 8    /* output channels */
#define OFF_W1 0
#define OFF_B1 (OFF_W1 + NH * NL)
#define OFF_W2 (OFF_B1 + NH)
#define OFF_B2 (OFF_W2 + NH * NH)
#define OFF_W3 (OFF_B2 + NH)
#define OFF_B3 (OFF_W3 + NO * NH)
#define NPARAM (OFF_B3 + NO)

int orc_ntex_nparams(void) { return NPARAM; }

/* binary64 -> nearest bfloat16 value (ties to even), as binary64 */
double orc_round_bf16(double x)
{
    if (x == 0.0 || !isfinite(x)) return x;
    int e;
    frexp(x, &e);                       /* x = m 2^e, 0.5 <= |m| < 1 */
    double q = ldexp(1.0, e - 8);       /* spacing of 8 significant bits */
    return nearbyint(x / q) * q;
}

static int clampi(int v, int hi) { return v < 0 ? 0 : (v > hi ? hi : v); }

/* bilinear latent of texel (i, j) */
static void orc_ntex_latent(const double* lat, int LW, int LH, int W, int H, int i, int j, double z[NL])
{
    double X = (i + 0.5) * LW / W - 0.5, Y = (j + 0.5) * LH / H - 0.5;
    double fx0 = floor(X), fy0 = floor(Y);
    double fx = X - fx0, fy = Y - fy0;
    int x0 = (int)fx0, y0 = (int)fy0;
    int xa = clampi(x0, LW - 1), xb = clampi(x0 + 1, LW - 1);
    int ya = clampi(y0, LH - 1), yb = clampi(y0 + 1, LH - 1);
    const double* c00 = lat + ((int64_t)ya * LW + xa) * NL;
    const double* c10 = lat + ((int64_t)ya * LW + xb) * NL;
    const double* c01 = lat + ((int64_t)yb * LW + xa) * NL;
    const double* c11 = lat + ((int64_t)yb * LW + xb) * NL;
    for (int k = 0; k < NL; ++k)
        z[k] = (1 - fy) * ((1 - fx) * c00[k] + fx * c10[k]) + fy * ((1 - fx) * c01[k] + fx * c11[k]);
}

static double rw(const double* p, int emulate) { return emulate ? orc_round_bf16(*p) : *p; }

/* MLP forward; keeps the activations for the backward pass */
static void orc_mlp(const double* mlp, const double z_in[NL], int emulate, double z[NL], double h1[NH],
                    double h2[NH], double y[NO])
{
    for (int k = 0; k < NL; ++k) z[k] = emulate ? orc_round_bf16(z_in[k]) : z_in[k];
    for (int a = 0; a < NH; ++a) {
        double s = mlp[OFF_B1 + a];
        for (int k = 0; k < NL; ++k) s += rw(mlp + OFF_W1 + a * NL + k, emulate) * z[k];
        s = s > 0 ? s : 0;
        h1[a] = emulate ? orc_round_bf16(s) : s;
    }
    for (int a = 0; a < NH; ++a) {
        double s = mlp[OFF_B2 + a];
        for (int b = 0; b < NH; ++b) s += rw(mlp + OFF_W2 + a * NH + b, emulate) * h1[b];
        s = s > 0 ? s : 0;
        h2[a] = emulate ? orc_round_bf16(s) : s;
    }
    for (int c = 0; c < NO; ++c) {
        double s = mlp[OFF_B3 + c];
        for (int a = 0; a < NH; ++a) s += rw(mlp + OFF_W3 + c * NH + a, emulate) * h2[a];
        y[c] = s;
    }
}

void orc_ntex_decode(const double* lat, int LW, int LH, int W, int H, const double* mlp, int i, int j, int emulate,
                     double out[NO])
{
    double z0[NL], z[NL], h1[NH], h2[NH];
    orc_ntex_latent(lat, LW, LH, W, H, i, j, z0);
    orc_mlp(mlp, z0, emulate, z, h1, h2, out);
}

/* Filtering of decoded texels: uv queries, raster x = fl32(fl32(uv W) - 0.5),
 * clamped taps, deterministic (every tap decoded) or stochastic (the sampled
 * tap decoded), the rules of oracle.c. */
static void orc_ntex_query(const double* lat, int LW, int LH, int W, int H, const double* mlp, const float* uv,
                           int filter, int mode, uint64_t seed, uint32_t qid, int emulate, double* out, int32_t* idx)
{
    float x = uv[0] * (float)W - 0.5f, y = uv[1] * (float)H - 0.5f;
    if (!(fabsf(x) < 16777216.0f) || !(fabsf(y) < 16777216.0f)) {
        for (int c = 0; c < NO; ++c) out[c] = NAN;
        if (idx) idx[0] = idx[1] = (int32_t)0x80000000;
        return;
    }
    float fx = floorf(x), fy = floorf(y);
    int ix = (int)fx, iy = (int)fy;
    double d[NO];
    if (mode != 0) {
        int sx = clampi(ix + orc_select(filter, x - fx, orc_uniform(seed, qid, 0)), W - 1);
        int sy = clampi(iy + orc_select(filter, y - fy, orc_uniform(seed, qid, 1)), H - 1);
        orc_ntex_decode(lat, LW, LH, W, H, mlp, sx, sy, emulate, out);
        if (idx) { idx[0] = sx; idx[1] = sy; }
        return;
    }
    double wx[4], wy[4];
    orc_axis_weights(filter, (double)x - floor((double)x), wx);
    orc_axis_weights(filter, (double)y - floor((double)y), wy);
    int base = filter ? -1 : 0, nt = filter ? 4 : 2;
    for (int c = 0; c < NO; ++c) out[c] = 0.0;
    for (int b = 0; b < nt; ++b)
        for (int a = 0; a < nt; ++a) {
            orc_ntex_decode(lat, LW, LH, W, H, mlp, clampi(ix + base + a, W - 1), clampi(iy + base + b, H - 1),
                            emulate, d);
            for (int c = 0; c < NO; ++c) out[c] += wx[a] * wy[b] * d[c];
        }
}

int orc_ntex_filter(const double* lat, int LW, int LH, int W, int H, const double* mlp, const float* uv,
                    const int64_t* qids, int64_t m, int filter, int mode, uint64_t seed, int emulate, double* out,
                    int32_t* idx, int nthreads)
{
#ifdef _OPENMP
    int nt = nthreads > 0 ? nthreads : omp_get_max_threads();
#endif
#pragma omp parallel for schedule(dynamic, 64) num_threads(nt)
    for (int64_t k = 0; k < m; ++k) {
        int64_t q = qids ? qids[k] : k;
        orc_ntex_query(lat, LW, LH, W, H, mlp, uv + 2 * q, filter, mode, seed, (uint32_t)q, emulate, out + NO * k,
                       idx ? idx + 2 * k : NULL);
    }
    return 0;
}

/* Mean squared error over a batch of texel positions (pos: B pairs (i, j))
 * against target texels (W x H x 8, binary32), and its exact gradient with
 * respect to every latent value and MLP parameter (back-propagation through
 * the MLP and the bilinear interpolation).  loss = (1/(8B)) sum (y - t)^2. */
double orc_ntex_loss_grad(const double* lat, int LW, int LH, int W, int H, const double* mlp, const float* target,
                          const int32_t* pos, int64_t B, double* g_lat, double* g_mlp)
{
    double loss = 0.0;
    if (g_lat) memset(g_lat, 0, sizeof(double) * (size_t)LW * LH * NL);
    if (g_mlp) memset(g_mlp, 0, sizeof(double) * NPARAM);
    const double scale = 1.0 / (8.0 * (double)B);
    for (int64_t s = 0; s < B; ++s) {
        int i = pos[2 * s], j = pos[2 * s + 1];
        double z0[NL], z[NL], h1[NH], h2[NH], y[NO];
        orc_ntex_latent(lat, LW, LH, W, H, i, j, z0);
        orc_mlp(mlp, z0, 0, z, h1, h2, y);
        const float* t = target + ((int64_t)j * W + i) * NO;
        double dy[NO], dh2[NH], dh1[NH], dz[NL];
        for (int c = 0; c < NO; ++c) {
            double e = y[c] - (double)t[c];
            loss += e * e;
            dy[c] = 2.0 * e * scale;
        }
        if (!g_mlp && !g_lat) continue;
        for (int a = 0; a < NH; ++a) {
            double s2 = 0.0;
            for (int c = 0; c < NO; ++c) s2 += mlp[OFF_W3 + c * NH + a] * dy[c];
            dh2[a] = h2[a] > 0 ? s2 : 0.0;
        }
        for (int b = 0; b < NH; ++b) {
            double s1 = 0.0;
            for (int a = 0; a < NH; ++a) s1 += mlp[OFF_W2 + a * NH + b] * dh2[a];
            dh1[b] = h1[b] > 0 ? s1 : 0.0;
        }
        for (int k = 0; k < NL; ++k) {
            double s0 = 0.0;
            for (int b = 0; b < NH; ++b) s0 += mlp[OFF_W1 + b * NL + k] * dh1[b];
            dz[k] = s0;
        }
        if (g_mlp) {
            for (int c = 0; c < NO; ++c) {
                g_mlp[OFF_B3 + c] += dy[c];
                for (int a = 0; a < NH; ++a) g_mlp[OFF_W3 + c * NH + a] += dy[c] * h2[a];
            }
            for (int a = 0; a < NH; ++a) {
                g_mlp[OFF_B2 + a] += dh2[a];
                for (int b = 0; b < NH; ++b) g_mlp[OFF_W2 + a * NH + b] += dh2[a] * h1[b];
            }
            for (int b = 0; b < NH; ++b) {
                g_mlp[OFF_B1 + b] += dh1[b];
                for (int k = 0; k < NL; ++k) g_mlp[OFF_W1 + b * NL + k] += dh1[b] * z[k];
            }
        }
        if (g_lat) {
            double X = (i + 0.5) * LW / W - 0.5, Y = (j + 0.5) * LH / H - 0.5;
            double fx0 = floor(X), fy0 = floor(Y);
            double fx = X - fx0, fy = Y - fy0;
            int x0 = (int)fx0, y0 = (int)fy0;
            int xs[2] = {clampi(x0, LW - 1), clampi(x0 + 1, LW - 1)};
            int ys[2] = {clampi(y0, LH - 1), clampi(y0 + 1, LH - 1)};
            double wxs[2] = {1 - fx, fx}, wys[2] = {1 - fy, fy};
            for (int b = 0; b < 2; ++b)
                for (int a = 0; a < 2; ++a) {
                    double* gl = g_lat + ((int64_t)ys[b] * LW + xs[a]) * NL;
                    for (int k = 0; k < NL; ++k) gl[k] += wxs[a] * wys[b] * dz[k];
                }
        }
    }
    return loss * scale;
}
