// neural.hip -- a neural texture (latent grid + MLP) trained on the GPU and
// filtered with BF16 MFMA inference.
//
// The paper argues that stochastic filtering makes expensive texel encodings
// viable because a lookup decodes one texel instead of one per filter tap
// (sections Introduction and Background, neural and compressed
// representations).  Here a W x H x 8 texture is represented by an
// LW x LH x 8 latent grid and an MLP 8 -> 64 -> 64 -> 8 (ReLU after the two
// hidden layers): texel (i, j) decodes to MLP(bilerp of the latent grid at
// X = (i + 1/2) LW/W - 1/2, clamped corners).  Filtering decodes every tap
// (deterministic) or the one sampled tap (stochastic), with the tap rules of
// the 2D filters.
//
// Training (binary32): per step a batch of texel positions, forward and
// backward through the MLP and the bilinear interpolation, mean squared
// error against the target texels, Adam.  One kernel processes tiles of 32
// samples with the weights in LDS and accumulates weight gradients per block;
// a second kernel reduces the blocks in a fixed order; latent gradients are
// scattered with atomics.
//
// Inference: latents rounded to binary16, weights to bfloat16, biases kept in
// binary32.  Each wave decodes 32 texels per MFMA batch with
// v_mfma_f32_32x32x16_bf16 in the transposed form out^T = W in^T, so each
// layer's accumulator registers are already the next layer's B operand once
// the hidden units are stored in the order the accumulator layout produces.
// A wave runs two batches at a time: each of its 64 lanes does the tap
// choice, latent gather and interpolation of one of the 64 decodes, and a
// lane-half swap forms both batches' first B operands.
#include <math.h>
#include <string.h>

#include <vector>

#include "device_common.h"
#include "stf_internal.h"

using namespace stf;

namespace {

constexpr int NL = 8, NH = 64, NO = 8;
constexpr int OFF_W1 = 0, OFF_B1 = OFF_W1 + NH * NL, OFF_W2 = OFF_B1 + NH, OFF_B2 = OFF_W2 + NH * NH,
              OFF_W3 = OFF_B2 + NH, OFF_B3 = OFF_W3 + NO * NH, NPARAM = OFF_B3 + NO;
constexpr int PSTRIDE = NPARAM + 1;   // per-block partial gradients + loss
constexpr int TS = 32;                 // samples per training tile
constexpr int TBLOCK = 256;
// Weight-gradient ownership (each in registers across all tiles of a
// block): thread t holds the W2 entries of rows 16 (t / 64) + r (r < 16),
// column t % 64; threads 0..63 also hold row t of W1 and b1[t], threads
// 64..127 column t - 64 of W3 and b2[t - 64], threads 128..135 b3[t - 128].
constexpr int OWN2 = NH * NH / TBLOCK;                        // 16
static_assert(NL == 8 && NO == 8 && NH == 64 && TBLOCK == 256, "the ownership above");

struct TrainArgs {
    const float* lat;
    const float* mlp;
    const float* target;
    const int32_t* pos;   // nullable: positions drawn from the counter hash
    int32_t B, W, H, LW, LH;
    float rx, ry;         // LW / W, LH / H (powers of two)
    uint32_t kstep;
    float dscale;         // 2 / (8 B)
    float* g_lat;
    float* partial;
};

__device__ __forceinline__ int clampi(int v, int hi)
{
    return v < 0 ? 0 : (v > hi ? hi : v);
}

__global__ __launch_bounds__(TBLOCK) void k_ntex_train(TrainArgs a)
{
    // Operands of the products are read four values at a time (16-byte LDS
    // reads), each read serving several FMAs; every sum keeps its order.
    // Rows of NH + 4 floats stay 16-byte aligned and spread the 16 lanes of a
    // read phase over all banks.  80 KiB per block: two blocks per CU.
    constexpr int R4 = NH + 4;
    __shared__ __align__(16) float sW2[NH][R4], sW2T[NH][R4], sW3[NO][R4], sW1T[NL][R4];
    __shared__ __align__(16) float sH1[TS][R4], sH2[TS][R4], sD2[TS][R4], sD1[TS][R4];
    __shared__ __align__(16) float sZ[TS][NL], sDY[TS][NO];
    __shared__ float sB1[NH], sB2[NH], sB3[NO], sT[TS][NO + 1];
    __shared__ int32_t sCI[TS][4];
    __shared__ float sCW[TS][4];
    __shared__ int32_t sTex[TS];
    static_assert(TS * (NO + 1) >= TBLOCK, "the loss reduction reuses sT");
    const int t = threadIdx.x;
    for (int p = t; p < NPARAM; p += TBLOCK) {
        float v = a.mlp[p];
        if (p < OFF_B1) sW1T[p % NL][p / NL] = v;
        else if (p < OFF_W2) sB1[p - OFF_B1] = v;
        else if (p < OFF_B2) {
            sW2[(p - OFF_W2) / NH][(p - OFF_W2) % NH] = v;
            sW2T[(p - OFF_W2) % NH][(p - OFF_W2) / NH] = v;
        }
        else if (p < OFF_W3) sB2[p - OFF_B2] = v;
        else if (p < OFF_B3) sW3[(p - OFF_W3) / NH][(p - OFF_W3) % NH] = v;
        else sB3[p - OFF_B3] = v;
    }
    // gradients owned by this thread (see the ownership note above)
    float acc2[OWN2], accw[NL], accb = 0.0f;
#pragma unroll
    for (int r = 0; r < OWN2; ++r) acc2[r] = 0.0f;
#pragma unroll
    for (int r = 0; r < NL; ++r) accw[r] = 0.0f;
    float lacc = 0.0f;
    const int s = t / 8, k = t % 8;       // (sample, channel) for the gather/scatter and output phases
    const int ha = t % NH, hs = t / NH;   // (hidden unit, first sample) for the 32 x 64 phases
    for (int tile = blockIdx.x; tile * TS < a.B; tile += gridDim.x) {
        const int gs = tile * TS + s;
        const bool live = gs < a.B;
        __syncthreads();   // previous tile's LDS reads are done
        if (k == 0) {
            int i = 0, j = 0;
            if (live) {
                if (a.pos) {   // caller-supplied positions are clamped into the texture
                    i = clampi(a.pos[2 * (int64_t)gs], a.W - 1);
                    j = clampi(a.pos[2 * (int64_t)gs + 1], a.H - 1);
                } else {
                    uint32_t h = pcg(a.kstep ^ (uint32_t)gs);
                    i = (int)(h % (uint32_t)a.W);
                    j = (int)(pcg(h + 1u) % (uint32_t)a.H);
                }
            }
            float X = ((float)i + 0.5f) * a.rx - 0.5f, Y = ((float)j + 0.5f) * a.ry - 0.5f;
            float fx0 = floorf(X), fy0 = floorf(Y);
            float fx = X - fx0, fy = Y - fy0;
            int x0 = (int)fx0, y0 = (int)fy0;
            int xa = clampi(x0, a.LW - 1), xb = clampi(x0 + 1, a.LW - 1);
            int ya = clampi(y0, a.LH - 1), yb = clampi(y0 + 1, a.LH - 1);
            sCI[s][0] = ya * a.LW + xa;
            sCI[s][1] = ya * a.LW + xb;
            sCI[s][2] = yb * a.LW + xa;
            sCI[s][3] = yb * a.LW + xb;
            sCW[s][0] = (1.0f - fx) * (1.0f - fy);
            sCW[s][1] = fx * (1.0f - fy);
            sCW[s][2] = (1.0f - fx) * fy;
            sCW[s][3] = fx * fy;
            sTex[s] = j * a.W + i;
        }
        __syncthreads();
        {
            float z = 0.0f;
#pragma unroll
            for (int c = 0; c < 4; ++c) z = __builtin_fmaf(sCW[s][c], a.lat[(int64_t)sCI[s][c] * NL + k], z);
            sZ[s][k] = live ? z : 0.0f;
            sT[s][k] = live ? a.target[(int64_t)sTex[s] * NO + k] : 0.0f;
        }
        __syncthreads();
        {   // H1 = relu(W1 Z + b1): the thread's W1 row once, two reads per sample
            float w[NL];
#pragma unroll
            for (int kk = 0; kk < NL; ++kk) w[kk] = sW1T[kk][ha];
#pragma unroll
            for (int r = 0; r < TS / 4; ++r) {
                const int s2 = hs + 4 * r;
                const float4 z0 = *reinterpret_cast<const float4*>(&sZ[s2][0]);
                const float4 z1 = *reinterpret_cast<const float4*>(&sZ[s2][4]);
                float v = sB1[ha];
                v = __builtin_fmaf(w[0], z0.x, v);
                v = __builtin_fmaf(w[1], z0.y, v);
                v = __builtin_fmaf(w[2], z0.z, v);
                v = __builtin_fmaf(w[3], z0.w, v);
                v = __builtin_fmaf(w[4], z1.x, v);
                v = __builtin_fmaf(w[5], z1.y, v);
                v = __builtin_fmaf(w[6], z1.z, v);
                v = __builtin_fmaf(w[7], z1.w, v);
                sH1[s2][ha] = fmaxf(v, 0.0f);
            }
        }
        __syncthreads();
        {   // H2 = relu(W2 H1 + b2): each W2 row read serves the thread's 8 samples
            float v[TS / 4];
#pragma unroll
            for (int r = 0; r < TS / 4; ++r) v[r] = sB2[ha];
#pragma unroll 4
            for (int b = 0; b < NH; b += 4) {
                const float4 w = *reinterpret_cast<const float4*>(&sW2[ha][b]);
#pragma unroll
                for (int r = 0; r < TS / 4; ++r) {
                    const float4 x = *reinterpret_cast<const float4*>(&sH1[hs + 4 * r][b]);
                    v[r] = __builtin_fmaf(w.x, x.x, v[r]);
                    v[r] = __builtin_fmaf(w.y, x.y, v[r]);
                    v[r] = __builtin_fmaf(w.z, x.z, v[r]);
                    v[r] = __builtin_fmaf(w.w, x.w, v[r]);
                }
            }
#pragma unroll
            for (int r = 0; r < TS / 4; ++r) sH2[hs + 4 * r][ha] = fmaxf(v[r], 0.0f);
        }
        __syncthreads();
        {   // Y = W3 H2 + b3 and the loss: thread (s, k)
            float y = sB3[k];
#pragma unroll 4
            for (int b = 0; b < NH; b += 4) {
                const float4 w = *reinterpret_cast<const float4*>(&sW3[k][b]);
                const float4 x = *reinterpret_cast<const float4*>(&sH2[s][b]);
                y = __builtin_fmaf(w.x, x.x, y);
                y = __builtin_fmaf(w.y, x.y, y);
                y = __builtin_fmaf(w.z, x.z, y);
                y = __builtin_fmaf(w.w, x.w, y);
            }
            float e = y - sT[s][k];
            if (live) lacc = __builtin_fmaf(e, e, lacc);
            sDY[s][k] = live ? e * a.dscale : 0.0f;
        }
        __syncthreads();
        {   // D2 = (W3^T dY) * [H2 > 0]: the thread's W3 column once
            float w[NO];
#pragma unroll
            for (int c = 0; c < NO; ++c) w[c] = sW3[c][ha];
#pragma unroll
            for (int r = 0; r < TS / 4; ++r) {
                const int s2 = hs + 4 * r;
                const float4 d0 = *reinterpret_cast<const float4*>(&sDY[s2][0]);
                const float4 d1 = *reinterpret_cast<const float4*>(&sDY[s2][4]);
                float v = 0.0f;
                v = __builtin_fmaf(w[0], d0.x, v);
                v = __builtin_fmaf(w[1], d0.y, v);
                v = __builtin_fmaf(w[2], d0.z, v);
                v = __builtin_fmaf(w[3], d0.w, v);
                v = __builtin_fmaf(w[4], d1.x, v);
                v = __builtin_fmaf(w[5], d1.y, v);
                v = __builtin_fmaf(w[6], d1.z, v);
                v = __builtin_fmaf(w[7], d1.w, v);
                sD2[s2][ha] = sH2[s2][ha] > 0.0f ? v : 0.0f;
            }
        }
        __syncthreads();
        {   // D1 = (W2^T D2) * [H1 > 0]
            float v[TS / 4];
#pragma unroll
            for (int r = 0; r < TS / 4; ++r) v[r] = 0.0f;
#pragma unroll 4
            for (int b = 0; b < NH; b += 4) {
                const float4 w = *reinterpret_cast<const float4*>(&sW2T[ha][b]);   // W2[b..b+3][ha]
#pragma unroll
                for (int r = 0; r < TS / 4; ++r) {
                    const float4 d = *reinterpret_cast<const float4*>(&sD2[hs + 4 * r][b]);
                    v[r] = __builtin_fmaf(w.x, d.x, v[r]);
                    v[r] = __builtin_fmaf(w.y, d.y, v[r]);
                    v[r] = __builtin_fmaf(w.z, d.z, v[r]);
                    v[r] = __builtin_fmaf(w.w, d.w, v[r]);
                }
            }
#pragma unroll
            for (int r = 0; r < TS / 4; ++r) sD1[hs + 4 * r][ha] = sH1[hs + 4 * r][ha] > 0.0f ? v[r] : 0.0f;
        }
        __syncthreads();
        {   // dZ = W1^T D1, scattered to the four latent corners
            float dz = 0.0f;
#pragma unroll 4
            for (int b = 0; b < NH; b += 4) {
                const float4 w = *reinterpret_cast<const float4*>(&sW1T[k][b]);   // W1[b..b+3][k]
                const float4 d = *reinterpret_cast<const float4*>(&sD1[s][b]);
                dz = __builtin_fmaf(w.x, d.x, dz);
                dz = __builtin_fmaf(w.y, d.y, dz);
                dz = __builtin_fmaf(w.z, d.z, dz);
                dz = __builtin_fmaf(w.w, d.w, dz);
            }
            if (live) {
#pragma unroll
                for (int c = 0; c < 4; ++c) atomicAdd(a.g_lat + (int64_t)sCI[s][c] * NL + k, sCW[s][c] * dz);
            }
        }
        {   // dW2[ua][ub] = sum_q D2[q][ua] H1[q][ub], ua = 16 (t/64) + r, ub = t%64:
            // per sample one H1 value and four 16-byte reads of D2
            float g[OWN2];
#pragma unroll
            for (int r = 0; r < OWN2; ++r) g[r] = 0.0f;
            const int u0 = OWN2 * (t / NH), ub = t % NH;
#pragma unroll 4
            for (int q = 0; q < TS; ++q) {
                const float h = sH1[q][ub];
#pragma unroll
                for (int r4 = 0; r4 < OWN2; r4 += 4) {
                    const float4 d = *reinterpret_cast<const float4*>(&sD2[q][u0 + r4]);
                    g[r4] = __builtin_fmaf(d.x, h, g[r4]);
                    g[r4 + 1] = __builtin_fmaf(d.y, h, g[r4 + 1]);
                    g[r4 + 2] = __builtin_fmaf(d.z, h, g[r4 + 2]);
                    g[r4 + 3] = __builtin_fmaf(d.w, h, g[r4 + 3]);
                }
            }
#pragma unroll
            for (int r = 0; r < OWN2; ++r) acc2[r] += g[r];
        }
        if (t < 2 * NH) {   // dW1 row t and b1[t] / dW3 column t - 64 and b2[t - 64]
            const int ua = t % NH;
            const bool first = t < NH;
            const float(*D)[R4] = first ? sD1 : sD2;
            const float(*X)[NL] = first ? sZ : sDY;
            const float(*Hq)[R4] = first ? sD1 : sH2;
            float g[NL], gb = 0.0f;
#pragma unroll
            for (int r = 0; r < NL; ++r) g[r] = 0.0f;
#pragma unroll 4
            for (int q = 0; q < TS; ++q) {
                const float hq = Hq[q][ua];   // D1[q][ua] (dW1) or H2[q][ua] (dW3)
                const float4 x0 = *reinterpret_cast<const float4*>(&X[q][0]);   // Z[q][.] or dY[q][.]
                const float4 x1 = *reinterpret_cast<const float4*>(&X[q][4]);
                g[0] = __builtin_fmaf(first ? hq : x0.x, first ? x0.x : hq, g[0]);
                g[1] = __builtin_fmaf(first ? hq : x0.y, first ? x0.y : hq, g[1]);
                g[2] = __builtin_fmaf(first ? hq : x0.z, first ? x0.z : hq, g[2]);
                g[3] = __builtin_fmaf(first ? hq : x0.w, first ? x0.w : hq, g[3]);
                g[4] = __builtin_fmaf(first ? hq : x1.x, first ? x1.x : hq, g[4]);
                g[5] = __builtin_fmaf(first ? hq : x1.y, first ? x1.y : hq, g[5]);
                g[6] = __builtin_fmaf(first ? hq : x1.z, first ? x1.z : hq, g[6]);
                g[7] = __builtin_fmaf(first ? hq : x1.w, first ? x1.w : hq, g[7]);
                gb += D[q][ua];   // b1 from D1, b2 from D2
            }
#pragma unroll
            for (int r = 0; r < NL; ++r) accw[r] += g[r];
            accb += gb;
        } else if (t < 2 * NH + NO) {   // b3
            float gb = 0.0f;
            for (int q = 0; q < TS; ++q) gb += sDY[q][t - 2 * NH];
            accb += gb;
        }
    }
    float* out = a.partial + (int64_t)blockIdx.x * PSTRIDE;
#pragma unroll
    for (int r = 0; r < OWN2; ++r) out[OFF_W2 + (OWN2 * (t / NH) + r) * NH + t % NH] = acc2[r];
    if (t < NH) {
#pragma unroll
        for (int r = 0; r < NL; ++r) out[OFF_W1 + t * NL + r] = accw[r];
        out[OFF_B1 + t] = accb;
    } else if (t < 2 * NH) {
#pragma unroll
        for (int r = 0; r < NO; ++r) out[OFF_W3 + r * NH + (t - NH)] = accw[r];
        out[OFF_B2 + t - NH] = accb;
    } else if (t < 2 * NH + NO) {
        out[OFF_B3 + t - 2 * NH] = accb;
    }
    float* sRed = &sT[0][0];
    __syncthreads();   // the last tile's reads of sT are done
    sRed[t] = lacc;
    __syncthreads();
    for (int st = TBLOCK / 2; st > 0; st >>= 1) {
        if (t < st) sRed[t] += sRed[t + st];
        __syncthreads();
    }
    if (t == 0) out[NPARAM] = sRed[0];
}

// Sum of the per-block partials in a fixed order (reproducible): stage 1
// sums consecutive groups of RGROUP blocks, stage 2 sums the group totals.
constexpr int RGROUP = 32;

__global__ void k_ntex_reduce1(const float* __restrict__ partial, int nblocks, float* __restrict__ group_sums)
{
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    int g = blockIdx.y;
    if (p >= PSTRIDE) return;
    float s = 0.0f;
    int b1 = min(nblocks, (g + 1) * RGROUP);
    for (int b = g * RGROUP; b < b1; ++b) s += partial[(int64_t)b * PSTRIDE + p];
    group_sums[(int64_t)g * PSTRIDE + p] = s;
}

__global__ void k_ntex_reduce2(const float* __restrict__ group_sums, int ngroups, float* __restrict__ g_mlp,
                               float* __restrict__ loss, float loss_scale)
{
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= PSTRIDE) return;
    float s = 0.0f;
    for (int g = 0; g < ngroups; ++g) s += group_sums[(int64_t)g * PSTRIDE + p];
    if (p < NPARAM) g_mlp[p] = s;
    else if (loss) *loss = s * loss_scale;
}

// Adam (beta1 = 0.9, beta2 = 0.999, eps = 1e-8, bias-corrected); clears the
// gradient it consumed.
__global__ void k_adam(float* __restrict__ param, float* __restrict__ grad, float* __restrict__ m,
                       float* __restrict__ v, int64_t n, float lr, float c1, float c2)
{
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    float g = grad[e];
    float mm = 0.9f * m[e] + 0.1f * g;
    float vv = 0.999f * v[e] + 0.001f * g * g;
    m[e] = mm;
    v[e] = vv;
    param[e] -= lr * (mm * c1) / (sqrtf(vv * c2) + 1e-8f);
    grad[e] = 0.0f;
}

__global__ void k_fill(float* __restrict__ p, int64_t n, float v)
{
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) p[e] = v;
}

// Corner quads for inference: entry (y0 + 1, x0 + 1) for every cell
// x0 = -1 .. LW - 1, y0 = -1 .. LH - 1 holds the binary16 latents of its
// clamped corners (x0, y0), (x0 + 1, y0), (x0, y0 + 1), (x0 + 1, y0 + 1), so a
// decode reads one 64-byte quad instead of two rows of the grid.
__global__ void k_to_quads(const float* __restrict__ lat, uint16_t* __restrict__ quad, int32_t LW, int32_t LH)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)(LW + 1) * (LH + 1)) return;
    const int x0 = (int)(e % (LW + 1)) - 1, y0 = (int)(e / (LW + 1)) - 1;
    const int xs[2] = {clampi(x0, LW - 1), clampi(x0 + 1, LW - 1)};
    const int ys[2] = {clampi(y0, LH - 1), clampi(y0 + 1, LH - 1)};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const float* src = lat + ((int64_t)ys[k / 2] * LW + xs[k % 2]) * NL;
        uint16_t h[NL];
#pragma unroll
        for (int c = 0; c < NL; ++c) h[c] = __builtin_bit_cast(uint16_t, (_Float16)src[c]);
        reinterpret_cast<uint4*>(quad)[4 * e + k] = __builtin_bit_cast(uint4, h);
    }
}

// ---------------------------------------------------------------------------
// inference
// ---------------------------------------------------------------------------
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// Operand images: one 8-value A slot per lane for every MFMA.  Biases enter
// the products themselves: every bias is split exactly into three bf16 terms
// held in k-slots 8..10 of an A operand, which meet ones in the same slots of
// the B operand.  Layer 1 uses its padding slots for this; layers 2 and 3
// start their accumulation with one bias-only MFMA.
struct Packed {
    bf16x8 a1[2][64];      // layer 1, M-blocks of 32 hidden units; k 0..7 latent, 8..10 bias terms
    bf16x8 a2[2][4][64];   // layer 2, M-blocks x K-blocks of 16
    bf16x8 a3[4][64];      // layer 3, rows 0..7 real, 8..31 zero
    bf16x8 ab2[2][64];     // layer 2 bias terms per M-block
    bf16x8 ab3[64];        // layer 3 bias terms
};

// Hidden unit held by k-slot kappa = 16 kb + 8 h + j of the B operand when
// the previous layer's accumulator registers are used in place.
__host__ __device__ constexpr int hidden_of_slot(int kb, int h, int j)
{
    return 16 * kb + 8 * (j / 4) + 4 * h + (j % 4);
}

// Hidden/output unit held by accumulator register r of lane half h in M-block mb.
__host__ __device__ constexpr int row_of_acc(int mb, int h, int r)
{
    return 32 * mb + 8 * (r / 4) + 4 * h + (r % 4);
}
static_assert(row_of_acc(0, 0, 0) == 0 && row_of_acc(0, 1, 3) == 7,
              "registers 0..3 of lane half h hold output channels 4h..4h+3");

struct InferArgs {
    const Packed* pk;
    const uint16_t* quad16;   // (LH + 1) x (LW + 1) corner quads, 4 x 8 binary16 each
    const float* q;          // n x 2 uv
    int32_t n, W, H, LW, LH;
    float rx, ry;
    uint32_t key;
    float* out;              // n x 8
    int32_t* idx;            // n x 2 (stochastic) or null
};

typedef short i16x8 __attribute__((ext_vector_type(8)));
typedef short i16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

// ReLU after rounding to bf16, done on the bit patterns: a bf16 whose sign
// bit is set reads as a negative int16, so a signed 16-bit max with zero maps
// it (and -0) to +0 and leaves every other value as it is.  Rounding keeps
// the sign, so this equals rounding the ReLU of the fp32 value.
__device__ __forceinline__ bf16x8 relu_bf16(const f32x16& d, int base)
{
    i16x8 v;
#pragma unroll
    for (int j = 0; j < 8; j += 2) {
        i16x2 p = __builtin_bit_cast(i16x2, __builtin_convertvector((f32x2){d[base + j], d[base + j + 1]}, bf16x2));
        p = __builtin_elementwise_max(p, (i16x2)0);
        v[j] = p[0];
        v[j + 1] = p[1];
    }
    return __builtin_bit_cast(bf16x8, v);
}

// One lane's decode: the tap it stands for, the texel it decodes and the
// tap's filter weight.
struct Decode {
    int sx, sy;
    float w;
    bool fin;
};

template <bool CUBIC, bool STOCH>
__device__ __forceinline__ Decode locate(const InferArgs& a, uint32_t qi, int tap, float2 uv)
{
    Decode d;
    float x = uv.x * (float)a.W - 0.5f, y = uv.y * (float)a.H - 0.5f;
    int cx = 0, cy = 0;
    float tx = 0.0f, ty = 0.0f;
    d.fin = cell_of(x, cx, tx) & cell_of(y, cy, ty);
    d.w = 1.0f;
    if constexpr (STOCH) {
        const uint32_t base = pcg_base(pcg(a.key ^ qi));
        const float mx = hash_m(pcg_from_base(base, 0u)), my = hash_m(pcg_from_base(base, 1u));
        if constexpr (CUBIC) {
            d.sx = cx + choose_cubic_m(tx, mx);
            d.sy = cy + choose_cubic_m(ty, my);
        } else {
            d.sx = cx + choose_linear_m(tx, mx);
            d.sy = cy + choose_linear_m(ty, my);
        }
    } else if constexpr (CUBIC) {
        int ta = tap % 4, tb = tap / 4;
        Cubic6 wa = cubic6(tx), wb = cubic6(ty);
        float fa = ta == 0 ? wa.a0 : ta == 1 ? wa.a1 : ta == 2 ? wa.a2 : wa.a3;
        float fb = tb == 0 ? wb.a0 : tb == 1 ? wb.a1 : tb == 2 ? wb.a2 : wb.a3;
        d.w = (fa * K6) * (fb * K6);
        d.sx = cx - 1 + ta;
        d.sy = cy - 1 + tb;
    } else {
        int ta = tap % 2, tb = tap / 2;
        d.w = (ta ? tx : 1.0f - tx) * (tb ? ty : 1.0f - ty);
        d.sx = cx + ta;
        d.sy = cy + tb;
    }
    d.sx = clampi(d.sx, a.W - 1);
    d.sy = clampi(d.sy, a.H - 1);
    return d;
}

// The corner quad of a decode's texel (its four clamped latent corners,
// 64 contiguous bytes: one cache line) and their bilinear weights.  With
// LW <= W the cell x0 = floor(X) lies in -1 .. LW - 1 (likewise y0).
__device__ __forceinline__ uint32_t latent_quad(const InferArgs& a, const Decode& d, float (&w)[4])
{
    float X = ((float)d.sx + 0.5f) * a.rx - 0.5f, Y = ((float)d.sy + 0.5f) * a.ry - 0.5f;
    float fx0 = floorf(X), fy0 = floorf(Y);
    float fx = X - fx0, fy = Y - fy0;
    const int x0 = min(max((int)fx0, -1), a.LW - 1), y0 = min(max((int)fy0, -1), a.LH - 1);
    w[0] = (1.0f - fx) * (1.0f - fy);
    w[1] = fx * (1.0f - fy);
    w[2] = (1.0f - fx) * fy;
    w[3] = fx * fy;
    return (uint32_t)((y0 + 1) * (a.LW + 1) + (x0 + 1));   // below 2^27 quads
}

// The decoder MLP on one 32-decode batch: B1 holds the bf16 latents of the
// batch's decodes in k-slots 0..7 (lanes 0..31) and ones in the bias slots
// 8..10 (lanes 32..63).  Returns layer 3's accumulator.
__device__ __forceinline__ f32x16 mlp_batch(const bf16x8& B1, const bf16x8 (&A1)[2], const bf16x8 (&A2)[2][4],
                                            const bf16x8 (&A3)[4], const bf16x8 (&AB2)[2], const bf16x8& AB3,
                                            const bf16x8& ONES)
{
    const f32x16 Z = {};
    // A wave in its matrix chain runs at raised issue priority, so the
    // SIMD's other waves fill the gaps with their VALU work (latent
    // interpolation, ReLU conversions, tap sums) instead of contending with
    // it; the chain itself is one dependent sequence per layer.
    __builtin_amdgcn_s_setprio(1);
    // layer 1: 64 x 16 by 16 x 32 (k 0..7 latents, 8..10 bias terms)
    f32x16 D1[2];
#pragma unroll
    for (int mb = 0; mb < 2; ++mb) D1[mb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A1[mb], B1, Z, 0, 0, 0);
    bf16x8 B2[4];
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) B2[kb] = relu_bf16(D1[kb / 2], 8 * (kb % 2));
    // layer 2: bias, then 64 x 64 by 64 x 32
    f32x16 D2[2];
#pragma unroll
    for (int mb = 0; mb < 2; ++mb) {
        D2[mb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(AB2[mb], ONES, Z, 0, 0, 0);
#pragma unroll
        for (int kb = 0; kb < 4; ++kb)
            D2[mb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A2[mb][kb], B2[kb], D2[mb], 0, 0, 0);
    }
    bf16x8 B3[4];
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) B3[kb] = relu_bf16(D2[kb / 2], 8 * (kb % 2));
    // layer 3: bias, then 8 (of 32) x 64 by 64 x 32
    f32x16 D3 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(AB3, ONES, Z, 0, 0, 0);
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) D3 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A3[kb], B3[kb], D3, 0, 0, 0);
    __builtin_amdgcn_s_setprio(0);
    return D3;
}

// Sum of v over each group of TAPS consecutive lanes (TAPS = 1, 4 or 16),
// left in every lane of the group, by data-parallel-primitive moves within a
// row of 16 lanes: swapping neighbours, then pairs, gives each quad its sum;
// mirroring within 8 lanes adds the neighbouring quad, mirroring within 16
// lanes the other half-row.
template <int TAPS>
__device__ __forceinline__ float tap_sum(float v)
{
    static_assert(TAPS == 1 || TAPS == 4 || TAPS == 16, "taps per query");
    auto dpp = [](float x, int ctrl) {
        switch (ctrl) {   // the control word must be a constant
        case 0:  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, x), 0xB1, 0xF, 0xF, true));
        case 1:  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, x), 0x4E, 0xF, 0xF, true));
        case 2:  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, x), 0x141, 0xF, 0xF, true));
        default: return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, x), 0x140, 0xF, 0xF, true));
        }
    };
    if constexpr (TAPS >= 4) {
        v += dpp(v, 0);   // quad_perm [1,0,3,2]
        v += dpp(v, 1);   // quad_perm [2,3,0,1]
    }
    if constexpr (TAPS >= 16) {
        v += dpp(v, 2);   // row_half_mirror
        v += dpp(v, 3);   // row_mirror
    }
    return v;
}

// Registers 0..3 of layer 3's accumulator hold channels 4h..4h+3 of decode
// jd; weight them, sum the taps of each query and store.  A non-finite query
// carries a NaN weight, so every channel it stores is NaN.
template <int TAPS>
__device__ __forceinline__ void emit(const InferArgs& a, const f32x16& D3, float w, uint32_t qi, int tap, int h)
{
    float o[4] = {D3[0] * w, D3[1] * w, D3[2] * w, D3[3] * w};
#pragma unroll
    for (int c = 0; c < 4; ++c) o[c] = tap_sum<TAPS>(o[c]);
    typedef float f32x4_nt __attribute__((ext_vector_type(4)));   // results are streamed out
    if (qi < (uint32_t)a.n && tap == 0)
        __builtin_nontemporal_store((f32x4_nt){o[0], o[1], o[2], o[3]},
                                    reinterpret_cast<f32x4_nt*>(a.out) + (2 * (size_t)qi + h));
}

// Persistent waves; each handles pairs of 32-decode batches p = wave,
// wave + nwaves, ...  Lane l does the per-decode work (tap choice, latent
// gather and interpolation) for decode l of the pair, so no lane repeats
// another's; one cross-half swap then lays the two batches' latents out as
// MFMA B operands, each with the bias ones in its upper half.  The loop is
// software-pipelined: while pair i runs its MFMAs, the latents of pair i + 1
// and the queries of pair i + 2 are in flight.
template <bool CUBIC, bool STOCH>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void k_ntex_infer(InferArgs a)
{
    constexpr int TAPS = STOCH ? 1 : (CUBIC ? 16 : 4);
    constexpr int QPB = 32 / TAPS;   // queries per 32-decode batch
    constexpr int QPP = 2 * QPB;     // queries per pair of batches
    const int lane = threadIdx.x % 64, h = lane / 32, jd = lane % 32;
    const int wave = (blockIdx.x * blockDim.x + threadIdx.x) / 64;
    const int nwaves = gridDim.x * blockDim.x / 64;
    const Packed* __restrict__ pk = a.pk;
    bf16x8 A1[2], A2[2][4], A3[4], AB2[2], AB3, ONES;
#pragma unroll
    for (int mb = 0; mb < 2; ++mb) {
        A1[mb] = pk->a1[mb][lane];
        AB2[mb] = pk->ab2[mb][lane];
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) A2[mb][kb] = pk->a2[mb][kb][lane];
    }
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) A3[kb] = pk->a3[kb][lane];
    AB3 = pk->ab3[lane];
#pragma unroll
    for (int j = 0; j < 8; ++j) ONES[j] = (__bf16)((h == 1 && j < 3) ? 1.0f : 0.0f);   // k-slots 8..10
    // The bias ones as every lane's slots j = 0..2 hold them in the upper
    // half: (1, 1, 1, 0, 0, 0, 0, 0) in bf16, as four 32-bit words.
    const uint32_t ONE_WORDS[4] = {0x3F803F80u, 0x00003F80u, 0u, 0u};

    const int32_t npair = (int32_t)(((int64_t)a.n + QPP - 1) / QPP);
    const uint32_t nq = (uint32_t)a.n;
    const int tap = lane % TAPS;
    const uint4* L = reinterpret_cast<const uint4*>(a.quad16);
    auto load_uv = [&](int32_t p) {
        const uint32_t qi = (uint32_t)p * QPP + lane / TAPS;
        return (p < npair && qi < nq) ? reinterpret_cast<const float2*>(a.q)[qi] : make_float2(0.5f, 0.5f);
    };
    // Every lane loads: the quad index is in the table for any query
    // (padding lanes carry uv = (0.5, 0.5)).
    auto load_lat = [&](const Decode& d, uint4 (&v)[4], float (&w)[4]) {
        const uint32_t e = latent_quad(a, d, w);
#pragma unroll
        for (int k = 0; k < 4; ++k) v[k] = L[4 * (size_t)e + k];
    };

    int32_t p = wave;
    float2 uv_next = load_uv(p + nwaves);
    Decode cur = locate<CUBIC, STOCH>(a, (uint32_t)p * QPP + lane / TAPS, tap, load_uv(p));
    uint4 lat_cur[4];
    float wl_cur[4];
    load_lat(cur, lat_cur, wl_cur);
    for (; p < npair; p += nwaves) {
        // ---- stage the next two pairs
        const float2 uv_after = load_uv(p + 2 * nwaves);
        const Decode nxt = locate<CUBIC, STOCH>(a, (uint32_t)(p + nwaves) * QPP + lane / TAPS, tap, uv_next);
        uint4 lat_nxt[4];
        float wl_nxt[4];
        load_lat(nxt, lat_nxt, wl_nxt);
        // ---- latent interpolation of this lane's decode, rounded to bf16
        uint32_t X[4];
#pragma unroll
        for (int wsel = 0; wsel < 4; ++wsel) {
            float v[2];
#pragma unroll
            for (int half = 0; half < 2; ++half) {
                const int sh = 16 * half;
                const uint32_t* p0 = reinterpret_cast<const uint32_t*>(&lat_cur[0]);
                const uint32_t* p1 = reinterpret_cast<const uint32_t*>(&lat_cur[1]);
                const uint32_t* p2 = reinterpret_cast<const uint32_t*>(&lat_cur[2]);
                const uint32_t* p3 = reinterpret_cast<const uint32_t*>(&lat_cur[3]);
                float s = wl_cur[0] * dec_f16((uint16_t)(p0[wsel] >> sh));
                s = __builtin_fmaf(wl_cur[1], dec_f16((uint16_t)(p1[wsel] >> sh)), s);
                s = __builtin_fmaf(wl_cur[2], dec_f16((uint16_t)(p2[wsel] >> sh)), s);
                s = __builtin_fmaf(wl_cur[3], dec_f16((uint16_t)(p3[wsel] >> sh)), s);
                v[half] = s;
            }
            X[wsel] = __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2){v[0], v[1]}, bf16x2));
        }
        // ---- batch 0 = decodes 0..31, batch 1 = decodes 32..63.  Swapping
        // the upper half of X with the lower half of the ones gives batch 0's
        // B operand in the first result and batch 1's in the second.
        uint32_t B1w[2][4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            auto r = __builtin_amdgcn_permlane32_swap(X[k], ONE_WORDS[k], false, false);
            B1w[0][k] = r[0];
            B1w[1][k] = r[1];
        }
        // decode weights in the same way: lane l of batch b needs decode 32 b + l % 32's
        const float wd = cur.fin ? cur.w : __builtin_nanf("");
        const uint32_t wb = __builtin_bit_cast(uint32_t, wd);
        const auto rw = __builtin_amdgcn_permlane32_swap(wb, wb, false, false);
        const uint32_t q0 = (uint32_t)p * QPP + jd / TAPS;
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const bf16x8 B1 = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(B1w[b]));
            const f32x16 D3 = mlp_batch(B1, A1, A2, A3, AB2, AB3, ONES);
            emit<TAPS>(a, D3, __builtin_bit_cast(float, (uint32_t)rw[b]), q0 + b * QPB, tap, h);
        }
        // selected texel of this lane's own decode (stochastic: one decode per query)
        if (STOCH && a.idx) {
            const uint32_t qi = (uint32_t)p * QPP + lane;
            if (qi < nq) {
                a.idx[2 * (size_t)qi] = cur.fin ? cur.sx : BAD_INDEX;
                a.idx[2 * (size_t)qi + 1] = cur.fin ? cur.sy : BAD_INDEX;
            }
        }
        cur = nxt;
        uv_next = uv_after;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            lat_cur[k] = lat_nxt[k];
            wl_cur[k] = wl_nxt[k];
        }
    }
}

uint16_t f2bf16_host(float f)
{
    // round to nearest even (finite inputs)
    uint32_t b;
    memcpy(&b, &f, 4);
    b += 0x7fffu + ((b >> 16) & 1u);
    return (uint16_t)(b >> 16);
}

// Exact split of an fp32 value into three bf16 terms: each term takes the
// leading 8 significant bits of what the previous ones left, and 24 bits of
// significand are used up after three.
void split3_bf16(float v, uint16_t (&t)[3])
{
    float rest = v;
    for (int i = 0; i < 3; ++i) {
        t[i] = f2bf16_host(rest);
        uint32_t b = (uint32_t)t[i] << 16;
        float f;
        memcpy(&f, &b, 4);
        rest -= f;
    }
}

void pack_weights(const float* mlp, Packed* pk)
{
    memset(pk, 0, sizeof(Packed));
    auto put = [](bf16x8& dst, int j, float v) {
        uint16_t u = f2bf16_host(v);
        memcpy(reinterpret_cast<char*>(&dst) + 2 * j, &u, 2);
    };
    auto put_bias = [](bf16x8& dst, float v) {   // k-slots 8..10: lanes 32..63, j = 0..2
        uint16_t t[3];
        split3_bf16(v, t);
        memcpy(&dst, t, sizeof t);
    };
    for (int lane = 0; lane < 64; ++lane) {
        int h = lane / 32, m = lane % 32;
        for (int mb = 0; mb < 2; ++mb) {
            if (h == 0)
                for (int j = 0; j < 8; ++j) put(pk->a1[mb][lane], j, mlp[OFF_W1 + (32 * mb + m) * NL + j]);
            else {
                put_bias(pk->a1[mb][lane], mlp[OFF_B1 + 32 * mb + m]);
                put_bias(pk->ab2[mb][lane], mlp[OFF_B2 + 32 * mb + m]);
            }
            for (int kb = 0; kb < 4; ++kb)
                for (int j = 0; j < 8; ++j)
                    put(pk->a2[mb][kb][lane], j, mlp[OFF_W2 + (32 * mb + m) * NH + hidden_of_slot(kb, h, j)]);
        }
        for (int kb = 0; kb < 4; ++kb)
            for (int j = 0; j < 8; ++j)
                put(pk->a3[kb][lane], j, m < NO ? mlp[OFF_W3 + m * NH + hidden_of_slot(kb, h, j)] : 0.0f);
        if (h == 1 && m < NO) put_bias(pk->ab3[lane], mlp[OFF_B3 + m]);
    }
}

bool pow2_ratio(int big, int small)
{
    if (small <= 0 || big < small || big % small) return false;
    int r = big / small;
    return (r & (r - 1)) == 0;
}

}  // namespace

struct stf_neural {
    int32_t W, H, LW, LH;
    int device;
    float* lat;
    float* mlp;
    float* m_lat;
    float* v_lat;
    float* m_mlp;
    float* v_mlp;
    float* g_lat;
    float* g_mlp;
    float* partial;
    int32_t partial_blocks;
    int64_t step;
    uint16_t* quad16;
    Packed* packed;
    bool ready;
};

namespace {

int64_t nlat(const stf_neural* nt)
{
    return (int64_t)nt->LW * nt->LH * NL;
}

void free_neural(stf_neural* nt)
{
    if (!nt) return;
    void* ptrs[] = {nt->lat, nt->mlp, nt->m_lat, nt->v_lat, nt->m_mlp, nt->v_mlp,
                    nt->g_lat, nt->g_mlp, nt->partial, nt->quad16, nt->packed};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    delete nt;
}

stf_status dalloc(void** p, size_t bytes, const char* what)
{
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        return stf_fail(STF_E_OOM, "hipMalloc of %zu bytes for %s failed", bytes, what);
    }
    return STF_OK;
}

hipError_t fill(float* p, int64_t n, float v, hipStream_t s)
{
    hipLaunchKernelGGL(k_fill, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

constexpr int TRAIN_BLOCKS = 512;   // one resident set: two 80 KiB blocks per CU

stf_status ensure_partial(stf_neural* nt, int32_t blocks)
{
    if (nt->partial && nt->partial_blocks >= blocks) return STF_OK;
    if (nt->partial) {
        (void)hipDeviceSynchronize();
        (void)hipFree(nt->partial);
        nt->partial = nullptr;
    }
    size_t groups = ((size_t)blocks + RGROUP - 1) / RGROUP;
    stf_status s = dalloc((void**)&nt->partial, ((size_t)blocks + groups) * PSTRIDE * 4, "gradient partials");
    nt->partial_blocks = s == STF_OK ? blocks : 0;
    return s;
}

// One forward/backward pass over a batch; leaves the MLP gradient in g_mlp,
// the latent gradient accumulated in g_lat and the loss in *loss.
hipError_t run_fwd_bwd(stf_neural* nt, const float* target, const int32_t* pos, int32_t B, uint32_t kstep,
                       float* loss, hipStream_t s)
{
    int32_t blocks = (B + TS - 1) / TS;
    if (blocks > nt->partial_blocks) blocks = nt->partial_blocks;
    TrainArgs a;
    a.lat = nt->lat;
    a.mlp = nt->mlp;
    a.target = target;
    a.pos = pos;
    a.B = B;
    a.W = nt->W;
    a.H = nt->H;
    a.LW = nt->LW;
    a.LH = nt->LH;
    a.rx = (float)nt->LW / (float)nt->W;
    a.ry = (float)nt->LH / (float)nt->H;
    a.kstep = kstep;
    a.dscale = 2.0f / (8.0f * (float)B);
    a.g_lat = nt->g_lat;
    a.partial = nt->partial;
    hipLaunchKernelGGL(k_ntex_train, dim3(blocks), dim3(TBLOCK), 0, s, a);
    int ngroups = (blocks + RGROUP - 1) / RGROUP;
    float* group_sums = nt->partial + (int64_t)nt->partial_blocks * PSTRIDE;
    hipLaunchKernelGGL(k_ntex_reduce1, dim3((PSTRIDE + 255) / 256, ngroups), dim3(256), 0, s, nt->partial, blocks,
                       group_sums);
    hipLaunchKernelGGL(k_ntex_reduce2, dim3((PSTRIDE + 255) / 256), dim3(256), 0, s, group_sums, ngroups, nt->g_mlp,
                       loss, 1.0f / (8.0f * (float)B));
    return hipGetLastError();
}

stf_status check_neural(const stf_neural* nt)
{
    if (!nt) return stf_fail(STF_E_INVALID, "neural texture is NULL");
    return STF_OK;
}

stf_status check_dev(const void* p, const char* what, size_t align)
{
    if (!p) return stf_fail(STF_E_INVALID, "%s is NULL", what);
    if ((uintptr_t)p % align) return stf_fail(STF_E_INVALID, "%s is not %zu-byte aligned", what, align);
    hipPointerAttribute_t attr;
    hipError_t e = hipPointerGetAttributes(&attr, p);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return stf_fail(STF_E_INVALID, "%s is not a device pointer", what);
    }
    if (attr.type != hipMemoryTypeDevice && attr.type != hipMemoryTypeManaged)
        return stf_fail(STF_E_INVALID, "%s is not device memory", what);
    return STF_OK;
}

}  // namespace

extern "C" {

int32_t stf_ntex_param_count(void)
{
    return NPARAM;
}

stf_status stf_ntex_create(int32_t tex_w, int32_t tex_h, int32_t lat_w, int32_t lat_h, const float* latents_host,
                           const float* mlp_host, stf_neural** out)
{
    stf_clear_error();
    if (!out) return stf_fail(STF_E_INVALID, "out is NULL");
    *out = nullptr;
    if (tex_w < 1 || tex_h < 1 || tex_w > 65536 || tex_h > 65536 || lat_w < 1 || lat_h < 1)
        return stf_fail(STF_E_INVALID, "sizes out of range");
    if (!pow2_ratio(tex_w, lat_w) || !pow2_ratio(tex_h, lat_h))
        return stf_fail(STF_E_UNSUPPORTED, "texture/latent size ratios must be powers of two");
    if ((int64_t)lat_w * lat_h * NL * 2 >= ((int64_t)1 << 31))
        return stf_fail(STF_E_UNSUPPORTED, "latent grid too large");
    if (!latents_host || !mlp_host) return stf_fail(STF_E_INVALID, "initial parameters are NULL");
    stf_neural* nt = new (std::nothrow) stf_neural();
    if (!nt) return stf_fail(STF_E_OOM, "host allocation failed");
    nt->W = tex_w;
    nt->H = tex_h;
    nt->LW = lat_w;
    nt->LH = lat_h;
    (void)hipGetDevice(&nt->device);
    size_t lb = (size_t)nlat(nt) * 4;
    stf_status s = STF_OK;
    float** bufs[] = {&nt->lat, &nt->m_lat, &nt->v_lat, &nt->g_lat};
    for (float** b : bufs)
        if (s == STF_OK) s = dalloc((void**)b, lb, "latents");
    float** mbufs[] = {&nt->mlp, &nt->m_mlp, &nt->v_mlp, &nt->g_mlp};
    for (float** b : mbufs)
        if (s == STF_OK) s = dalloc((void**)b, NPARAM * 4, "MLP parameters");
    if (s == STF_OK)
        s = dalloc((void**)&nt->quad16, (size_t)(lat_w + 1) * (lat_h + 1) * 4 * NL * 2, "binary16 corner quads");
    if (s == STF_OK) s = dalloc((void**)&nt->packed, sizeof(Packed), "packed weights");
    if (s == STF_OK) s = ensure_partial(nt, TRAIN_BLOCKS);
    if (s == STF_OK) {
        hipError_t e = hipMemcpy(nt->lat, latents_host, lb, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(nt->mlp, mlp_host, NPARAM * 4, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = fill(nt->m_lat, nlat(nt), 0.0f, 0);
        if (e == hipSuccess) e = fill(nt->v_lat, nlat(nt), 0.0f, 0);
        if (e == hipSuccess) e = fill(nt->g_lat, nlat(nt), 0.0f, 0);
        if (e == hipSuccess) e = fill(nt->m_mlp, NPARAM, 0.0f, 0);
        if (e == hipSuccess) e = fill(nt->v_mlp, NPARAM, 0.0f, 0);
        if (e == hipSuccess) e = hipDeviceSynchronize();
        if (e != hipSuccess) s = stf_fail(STF_E_DEVICE, "initialising the neural texture failed: %s", hipGetErrorString(e));
    }
    if (s != STF_OK) {
        free_neural(nt);
        return s;
    }
    *out = nt;
    return STF_OK;
}

void stf_ntex_destroy(stf_neural* nt)
{
    free_neural(nt);
}

stf_status stf_ntex_train(stf_neural* nt, const float* target_dev, int32_t steps, int32_t batch, float lr_latent,
                          float lr_mlp, uint64_t seed, float* loss_dev, void* hip_stream)
{
    stf_clear_error();
    stf_status s = check_neural(nt);
    if (s != STF_OK) return s;
    if (steps < 0 || batch < 1) return stf_fail(STF_E_INVALID, "steps = %d, batch = %d", steps, batch);
    if (!(lr_latent >= 0.0f) || !(lr_mlp >= 0.0f)) return stf_fail(STF_E_INVALID, "learning rates must be >= 0");
    if (steps == 0) return STF_OK;
    s = check_dev(target_dev, "target_dev", 16);
    if (s == STF_OK && loss_dev) s = check_dev(loss_dev, "loss_dev", 4);
    if (s != STF_OK) return s;
    hipStream_t st = (hipStream_t)hip_stream;
    uint32_t key = seed_key(seed);
    for (int32_t k = 0; k < steps; ++k) {
        nt->step += 1;
        double c1 = 1.0 / (1.0 - pow(0.9, (double)nt->step)), c2 = 1.0 / (1.0 - pow(0.999, (double)nt->step));
        hipError_t e = run_fwd_bwd(nt, target_dev, nullptr, batch, pcg(key ^ (uint32_t)nt->step),
                                   loss_dev ? loss_dev + k : nullptr, st);
        if (e == hipSuccess) {
            hipLaunchKernelGGL(k_adam, dim3((NPARAM + 255) / 256), dim3(256), 0, st, nt->mlp, nt->g_mlp, nt->m_mlp,
                               nt->v_mlp, (int64_t)NPARAM, lr_mlp, (float)c1, (float)c2);
            hipLaunchKernelGGL(k_adam, dim3((unsigned)((nlat(nt) + 255) / 256)), dim3(256), 0, st, nt->lat,
                               nt->g_lat, nt->m_lat, nt->v_lat, nlat(nt), lr_latent, (float)c1, (float)c2);
            e = hipGetLastError();
        }
        if (e != hipSuccess) return stf_fail(STF_E_DEVICE, "training launch failed: %s", hipGetErrorString(e));
    }
    nt->ready = false;
    return STF_OK;
}

stf_status stf_ntex_gradients(stf_neural* nt, const float* target_dev, const int32_t* positions_dev, int32_t batch,
                              float* grad_latents_dev, float* grad_mlp_dev, float* loss_dev, void* hip_stream)
{
    stf_clear_error();
    stf_status s = check_neural(nt);
    if (s != STF_OK) return s;
    if (batch < 1) return stf_fail(STF_E_INVALID, "batch = %d", batch);
    s = check_dev(target_dev, "target_dev", 16);
    if (s == STF_OK) s = check_dev(positions_dev, "positions_dev", 4);
    if (s == STF_OK) s = check_dev(grad_latents_dev, "grad_latents_dev", 4);
    if (s == STF_OK) s = check_dev(grad_mlp_dev, "grad_mlp_dev", 4);
    if (s == STF_OK && loss_dev) s = check_dev(loss_dev, "loss_dev", 4);
    if (s != STF_OK) return s;
    hipStream_t st = (hipStream_t)hip_stream;
    hipError_t e = fill(nt->g_lat, nlat(nt), 0.0f, st);
    if (e == hipSuccess) e = run_fwd_bwd(nt, target_dev, positions_dev, batch, 0u, loss_dev, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(grad_latents_dev, nt->g_lat, (size_t)nlat(nt) * 4, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(grad_mlp_dev, nt->g_mlp, NPARAM * 4, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess) e = fill(nt->g_lat, nlat(nt), 0.0f, st);
    if (e != hipSuccess) return stf_fail(STF_E_DEVICE, "gradient launch failed: %s", hipGetErrorString(e));
    return STF_OK;
}

stf_status stf_ntex_get_params(const stf_neural* nt, float* latents_host, float* mlp_host)
{
    stf_clear_error();
    stf_status s = check_neural(nt);
    if (s != STF_OK) return s;
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess && latents_host) e = hipMemcpy(latents_host, nt->lat, (size_t)nlat(nt) * 4, hipMemcpyDeviceToHost);
    if (e == hipSuccess && mlp_host) e = hipMemcpy(mlp_host, nt->mlp, NPARAM * 4, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return stf_fail(STF_E_DEVICE, "copying parameters failed: %s", hipGetErrorString(e));
    return STF_OK;
}

stf_status stf_ntex_prepare_inference(stf_neural* nt, void* hip_stream)
{
    stf_clear_error();
    stf_status s = check_neural(nt);
    if (s != STF_OK) return s;
    std::vector<float> mlp(NPARAM);
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipMemcpy(mlp.data(), nt->mlp, NPARAM * 4, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return stf_fail(STF_E_DEVICE, "reading the MLP failed: %s", hipGetErrorString(e));
    Packed* pk = new (std::nothrow) Packed;
    if (!pk) return stf_fail(STF_E_OOM, "host allocation failed");
    pack_weights(mlp.data(), pk);
    e = hipMemcpy(nt->packed, pk, sizeof(Packed), hipMemcpyHostToDevice);
    delete pk;
    hipStream_t st = (hipStream_t)hip_stream;
    if (e == hipSuccess) {
        const int64_t nq = (int64_t)(nt->LW + 1) * (nt->LH + 1);
        hipLaunchKernelGGL(k_to_quads, dim3((unsigned)((nq + 255) / 256)), dim3(256), 0, st, nt->lat, nt->quad16, nt->LW,
                           nt->LH);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return stf_fail(STF_E_DEVICE, "preparing inference failed: %s", hipGetErrorString(e));
    nt->ready = true;
    return STF_OK;
}

stf_status stf_ntex_filter(const stf_neural* nt, const float* queries_dev, int64_t n, stf_filter_kind filter,
                           stf_mode mode, uint64_t seed, float* out_dev, int32_t* out_index_dev, void* hip_stream)
{
    stf_clear_error();
    stf_status s = check_neural(nt);
    if (s != STF_OK) return s;
    if (!nt->ready) return stf_fail(STF_E_INVALID, "call stf_ntex_prepare_inference after training");
    if (n < 0 || n > 0x7fffffff) return stf_fail(STF_E_INVALID, "n = %lld out of range", (long long)n);
    if (!valid_filter(filter)) return stf_fail(STF_E_INVALID, "unknown filter");
    if (filter != STF_LINEAR && filter != STF_CUBIC_BSPLINE)
        return stf_fail(STF_E_UNSUPPORTED, "neural textures support the linear and B-spline filters only");
    if (mode != STF_DETERMINISTIC && mode != STF_STOCHASTIC) return stf_fail(STF_E_INVALID, "unknown mode");
    if (mode == STF_DETERMINISTIC && out_index_dev)
        return stf_fail(STF_E_INVALID, "out_index_dev must be NULL in deterministic mode");
    if (n == 0) return STF_OK;
    s = check_dev(queries_dev, "queries_dev", 8);
    if (s == STF_OK) s = check_dev(out_dev, "out_dev", 16);
    if (s == STF_OK && out_index_dev) s = check_dev(out_index_dev, "out_index_dev", 4);
    if (s != STF_OK) return s;
    InferArgs a;
    a.pk = nt->packed;
    a.quad16 = nt->quad16;
    a.q = queries_dev;
    a.n = (int32_t)n;
    a.W = nt->W;
    a.H = nt->H;
    a.LW = nt->LW;
    a.LH = nt->LH;
    a.rx = (float)nt->LW / (float)nt->W;
    a.ry = (float)nt->LH / (float)nt->H;
    a.key = seed_key(seed);
    a.out = out_dev;
    a.idx = out_index_dev;
    int taps = mode == STF_STOCHASTIC ? 1 : (filter == STF_CUBIC_BSPLINE ? 16 : 4);
    int64_t pairs = (n * taps + 63) / 64;   // pairs of 32-decode batches
    // Persistent waves, one resident set (3 per SIMD on 256 CUs): the weights
    // load once per wave.
    int64_t waves = pairs < 3072 ? pairs : 3072;
    dim3 grid((unsigned)((waves + 3) / 4)), block(256);
    hipStream_t st = (hipStream_t)hip_stream;
    bool cubic = filter == STF_CUBIC_BSPLINE;
    if (mode == STF_STOCHASTIC) {
        if (cubic) hipLaunchKernelGGL((k_ntex_infer<true, true>), grid, block, 0, st, a);
        else hipLaunchKernelGGL((k_ntex_infer<false, true>), grid, block, 0, st, a);
    } else {
        if (cubic) hipLaunchKernelGGL((k_ntex_infer<true, false>), grid, block, 0, st, a);
        else hipLaunchKernelGGL((k_ntex_infer<false, false>), grid, block, 0, st, a);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return stf_fail(STF_E_DEVICE, "kernel launch failed: %s", hipGetErrorString(e));
    return STF_OK;
}

}  // extern "C"
