/*
 * stf.h -- C ABI of libstf, stochastic texture filtering on AMD Instinct
 * MI355X (gfx950).
 *
 * The library implements the filtered texture lookup of Fajardo, Wronski,
 * Salvi and Pharr, "Stochastic Texture Filtering" (2023): a filter is a
 * weighted sum of texels (Eq. filtered-texture); the stochastic estimator
 * draws one texel with probability equal to its normalised weight and returns
 * it unweighted (Eq. stochastic-sum).  Both are provided for the linear
 * (tent, Eq. stochastic-lerp / stochastic-bilerp) and cubic B-spline
 * (Eq. cubic-bspline, Eq. bicubic-bspline-texfilt) filters, on dense 2D
 * textures and on sparse 3D voxel grids, plus the filter-after-shading
 * variant of section "Effect of Texture Filtering on Rendering"
 * (Eqs. traditional-lighting-integral and our-lighting-integral).
 *
 * General rules
 *   - Every entry point returns stf_status.  On failure nothing is launched
 *     and stf_last_error() describes the problem.
 *   - Query and output buffers are device memory owned by the caller.  The
 *     library reads/writes them only from work enqueued on the caller's HIP
 *     stream (`hip_stream`, a hipStream_t; NULL = the null stream) and keeps
 *     no reference after the call returns.  Calls return after enqueueing;
 *     the caller synchronises.
 *   - Host arrays passed to create functions are copied before the call
 *     returns and may be freed afterwards.
 *   - Textures are owned by the library from create until stf_destroy.
 *     Destroying a texture while work that reads it is still in flight on a
 *     stream is a caller error.
 *   - n == 0 is a valid no-op.  n must be < 2^31 per call.
 *   - Random numbers: the uniform of hash index a of query q (its index
 *     within the call) is a pure function of (seed, q, a):
 *        pcg(x): state = x*747796405 + 2891336453;
 *                word  = ((state >> ((state >> 28) + 4)) ^ state) * 277803737;
 *                return (word >> 22) ^ word          (all arithmetic mod 2^32)
 *        s = pcg(lo32(seed) ^ pcg(hi32(seed)));  b = pcg(s ^ q);
 *        h_a = pcg(b + a) for every a >= 0;  u_a = (h_a >> 8) * 2^-24
 *     (a = 0, 1, 2 for the axes x, y, z; other indices as each call states),
 *     so results do not depend on launch shape, ordering or other work.
 *     (Known answers: pcg(0) = 0x07bb2fe2, s = 0x30be035e for seed 0, and
 *     u_0 = 0.551548481 for seed 0, q = 0.)
 *   - Tap choice (stochastic mode), per axis, with i = floor(x), t = x - i in
 *     binary32:  linear: upper tap i+1 iff u < t, else i.  Cubic: with
 *     s = 1-t and K6 = 0x1.555556p-3f (binary32 1/6):
 *     c1 = ((s*s)*s)*K6, c2 = c1 + (4 + (3*(t*t))*(t - 2))*K6,
 *     c3 = 1 - ((t*t)*t)*K6, tap = i - 1 + [u >= c1] + [u >= c2] +
 *     [u >= c3] -- the cumulative B-spline weights w0, w0 + w1, 1 - w3.
 *     Every operation is a single binary32 rounding (no fused multiply-add),
 *     so the chosen tap is reproducible bit for bit.  ("Sampling arrays",
 *     section "Sampling Techniques", applied per axis as in section
 *     "B-Spline and Anisotropic Filters".)
 *   - A query coordinate that is NaN, infinite, or of magnitude >= 2^24 after
 *     the raster transform yields NaN in every output channel and INT32_MIN
 *     in every index component.  It is not an error.
 */
#ifndef STF_H
#define STF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct stf_texture stf_texture;   /* opaque, library-owned */

typedef enum {
    STF_OK = 0,
    STF_E_INVALID = -1,      /* bad argument; nothing launched */
    STF_E_OOM = -2,          /* device or host allocation failed */
    STF_E_UNSUPPORTED = -3,  /* valid request this build does not implement */
    STF_E_DEVICE = -4,       /* a HIP runtime call failed */
    STF_E_BUSY = -5,         /* serving: no admission possible right now */
    STF_E_CANCELLED = -6     /* serving: request was cancelled */
} stf_status;

/* Texel storage formats.  Texels are decoded exactly to binary32 before any
 * arithmetic (U8 is UNORM: v / 255.0f correctly rounded).  Weights and
 * accumulation are binary32 on the device. */
typedef enum {
    STF_FMT_F32 = 0,
    STF_FMT_F16 = 1,       /* IEEE binary16 */
    STF_FMT_BF16 = 2,      /* bfloat16 */
    STF_FMT_FP8_E4M3 = 3,  /* OCP E4M3 "FN": bias 7, no infinity, 0x7f/0xff NaN */
    STF_FMT_U8 = 4         /* UNORM8 */
} stf_format;

/* Filters.  The B-spline and linear filters have non-negative weights and
 * their stochastic mode reads one tap.  The interpolating cubics have
 * negative lobes; their stochastic mode is positivization (section
 * "Sampling Techniques", positivization; supplement, "The interpolating
 * (negative lobe) bicubic filter"): one tap j+ drawn in proportion to the
 * positive weights and one tap j- in proportion to the magnitudes of the
 * negative ones, result S+ t(j+) - S- t(j-) with S+/S- the two weight
 * masses (the second term only when S- > 0).  Taps i-1..i+2 of cell i. */
typedef enum {
    STF_LINEAR = 0,          /* bilinear (2D, 4 taps) / trilinear (3D, 8 taps) */
    STF_CUBIC_BSPLINE = 1,   /* bicubic (16 taps) / tricubic (64 taps) B-spline */
    STF_CUBIC_KEYS = 2,      /* the cubic polynomial kernel K_3 with a = -1/2 (supplement, "Filter
                                Kernels"; Catmull-Rom, interpolating); stochastic: 2 taps */
    STF_CUBIC_MITCHELL = 3   /* Mitchell-Netravali cubic, B = C = 1/3; stochastic: 2 taps */
} stf_filter_kind;

typedef enum {
    STF_DETERMINISTIC = 0,   /* weighted sum over all taps (Eq. filtered-texture) */
    STF_STOCHASTIC = 1,      /* one tap drawn with probability = weight (Eq. stochastic-sum) */
    STF_STOCHASTIC_FIS = 2   /* linear / B-spline only: filter importance sampling (section "Filter
                                Importance Sampling") -- the position jittered by a draw of the
                                B-spline one degree lower (u - 1/2 for the tent; u_a + u_b + u_c - 3/2,
                                a quadratic B-spline, for the cubic) and the nearest texel
                                floor(x' + 1/2) read; the same tap distribution as STF_STOCHASTIC,
                                no weights evaluated.  The tap is floor((x + s) + 1/2) evaluated in
                                binary64 in that order: exact for |x| >= 2^-29, where the kernels
                                form it in binary32 and integers with the same result. */
} stf_mode;

typedef enum {
    STF_SHADE_AFTER_FILTER = 0,   /* filter the material, shade once (Eq. traditional-lighting-integral) */
    STF_FILTER_AFTER_SHADE = 1,   /* shade every tap, filter the results (Eq. our-lighting-integral) */
    STF_SHADE_STOCHASTIC = 2      /* shade the one sampled tap (Eq. our-lighting-integral, sampled) */
} stf_shade_mode;

/* ---------------------------------------------------------------------- */
/* Texture creation                                                        */
/* ---------------------------------------------------------------------- */

/* Dense 2D texture with `levels` >= 1 levels.  Level l has size
 * max(1, width >> l) x max(1, height >> l); level_texels_host[l] points to
 * its texels, row-major (x fastest), `channels` (1..4) interleaved values
 * per texel in format `fmt`.  Queries are normalised uv in texture space;
 * raster position x = uv.x * W - 0.5 (binary32, two roundings), so texel
 * centres lie at half-integers of uv * W.  Taps are clamped to the level
 * (clamp addressing). */
stf_status stf_create_texture2d(int32_t width, int32_t height, int32_t channels, stf_format fmt,
                                int32_t levels, const void* const* level_texels_host,
                                stf_texture** out);

/* Material texture for stf_shade_filter: 8-byte texels, bytes 0..2 albedo
 * RGB (UNORM8, linear), byte 3 roughness (UNORM8), bytes 4..5 and 6..7 the
 * tangent-space normal x and y as binary16.  Levels as for
 * stf_create_texture2d; level l must be supplied by the caller.
 * stf_filter, stf_sort_queries, stf_filter_gaussian and the server also read
 * level 0 of a material as a 2D texture of six channels (albedo R, G, B,
 * roughness, normal x, normal y; each decoded exactly: v / 255 and binary16
 * widened), so a material is filtered before shading (Eq.
 * traditional-lighting-integral) with every filter and mode of stf_filter.
 * The caller passes row-major levels; the library stores each level in
 * tiles of 4x4 texels (one 128-byte line per tile), padded to whole tiles,
 * which stf_texture_bytes counts. */
stf_status stf_create_material2d(int32_t width, int32_t height, int32_t levels,
                                 const void* const* level_texels_host, stf_texture** out);

/* Sparse 3D voxel grid over the domain [0,dim_x) x [0,dim_y) x [0,dim_z)
 * (each dim in 1..32768).  The grid is a set of dense 8^3 leaves; leaf k has
 * its corner at leaf_origins_host[3k..3k+2] = (x, y, z), each a multiple of 8
 * inside the domain, no two leaves alike, and its 512 values at
 * leaf_values_host + 512*k*sizeof(texel), x fastest, then y, then z.
 * Voxels not covered by a leaf, and positions outside the domain, read as
 * `background`.  Queries are positions in voxel index space (voxel (i,j,k)
 * centred at (i,j,k)), 3 binary32 per query. */
stf_status stf_create_sparse_grid3d(int32_t dim_x, int32_t dim_y, int32_t dim_z, stf_format fmt,
                                    int64_t n_leaves, const int32_t* leaf_origins_host,
                                    const void* leaf_values_host, float background,
                                    stf_texture** out);

void stf_destroy(stf_texture* tex);

/* Device bytes held by a texture (texels + index structures). */
stf_status stf_texture_bytes(const stf_texture* tex, int64_t* bytes);

/* ---------------------------------------------------------------------- */
/* Filtering                                                               */
/* ---------------------------------------------------------------------- */

/* Filter n queries.
 *   queries_dev:   n x 2 binary32 uv (2D textures, level 0) or n x 3 binary32
 *                  index-space positions (3D grids); 4-byte aligned.
 *   out_dev:       n x channels binary32 results (channels = 1 for grids,
 *                  6 for materials).
 *   out_index_dev: NULL, or (stochastic mode only) n x dims int32: the texel
 *                  that was read -- clamped (x, y) for 2D, (x, y, z) for 3D
 *                  (may lie outside the domain, which reads as background).
 *                  For STF_CUBIC_KEYS / STF_CUBIC_MITCHELL: n x 2*dims, the
 *                  positive tap then the negative tap (INT32_MIN entries
 *                  when there is no negative weight).
 *   flags:         0.
 * Deterministic results carry binary32 weight and accumulation error only;
 * stochastic results are the decoded texel exactly. */
stf_status stf_filter(const stf_texture* tex, const float* queries_dev, int64_t n,
                      stf_filter_kind filter, stf_mode mode, uint64_t seed,
                      float* out_dev, int32_t* out_index_dev, uint32_t flags, void* hip_stream);

/* ---------------------------------------------------------------------- */
/* Gaussian filters                                                        */
/* ---------------------------------------------------------------------- */
/* Gaussian filtering of 2D (and DCT) textures with standard deviation sigma
 * texels (sections "Filter Importance Sampling" and "Results",
 * magnification; supplement, "Real-time discrete and filter importance
 * sampling"):
 *   STF_GAUSS_FIS: the position offset by sigma * (r cos 2 pi u1,
 *     r sin 2 pi u1), r = sqrt(-2 ln(1 - u0)) (Box-Muller), and the nearest
 *     texel floor(x' + 1/2) read -- an infinite-support filter, one texel;
 *   STF_GAUSS_FIS_MEAN: what FIS estimates, the Gaussian convolved with the
 *     nearest-texel box: per-axis weights Phi((k + 1/2 - x)/sigma) -
 *     Phi((k - 1/2 - x)/sigma) over |k - floor(x)| <= ceil(6 sigma) + 1
 *     (sigma <= 4 for this mode);
 *   STF_GAUSS_DISCRETE: one tap of the 4x4 window i-1..i+2 with probability
 *     proportional to exp(-|d - t|^2 / (2 sigma^2));
 *   STF_GAUSS_DISCRETE_MEAN: the normalised weighted sum over that window.
 * 0 < sigma <= 16.  Weights and decisions in binary64 (transcendental
 * functions), accumulation in binary32.  out_index_dev: NULL or, for the two
 * stochastic modes, n x 2 int32 (clamped texel). */
typedef enum {
    STF_GAUSS_FIS = 0,
    STF_GAUSS_FIS_MEAN = 1,
    STF_GAUSS_DISCRETE = 2,
    STF_GAUSS_DISCRETE_MEAN = 3
} stf_gauss_mode;

stf_status stf_filter_gaussian(const stf_texture* tex, const float* queries_dev, int64_t n, float sigma,
                               stf_gauss_mode mode, uint64_t seed, float* out_dev, int32_t* out_index_dev,
                               void* hip_stream);

/* ---------------------------------------------------------------------- */
/* Elliptically weighted average filtering                                 */
/* ---------------------------------------------------------------------- */
/* EWA filtering of a 2D texture's MIP levels (section "B-Spline and
 * Anisotropic Filters"; supplement, "Stochastic sampling of the EWA kernel",
 * after pbrt's EWA lookup).  Each query is 6 binary32: (s, t) in [0, 1] and
 * the texture-space derivatives (ds/dx, dt/dx, ds/dy, dt/dy).
 *   - The texture must hold the full pyramid: its last level is 1x1
 *     (STF_E_INVALID otherwise).
 *   - The longer derivative vector is the major axis; the shorter one is
 *     raised to longer / max_anisotropy if needed (binary32).
 *   - lod = max(0, (levels - 1) + log2(shorter)) (binary64).
 *   - EWA on a level = over the texels of the ellipse's bounding box with
 *     r2 = A ss^2 + B ss tt + C tt^2 < 1 (pbrt's ellipse coefficients in
 *     texels), weights w = LUT[min(floor(128 r2), 127)], LUT[i] =
 *     exp(-2 i/127) - exp(-2).  On the last level (one texel) it is that
 *     texel, read directly (pbrt's rule), so a footprint larger than the
 *     texture costs one read.
 *   - Deterministic: lerp(lod - floor(lod), EWA(floor(lod)), EWA(floor(lod)
 *     + 1)) with EWA = sum w t / sum w (levels clamped to the last).
 *   - Stochastic: level l = floor(lod) + [u_0 < lod - floor(lod)] (clamped
 *     to the last), then one texel drawn with probability w / sum w: a row
 *     k of the box by weighted reservoir sampling over the binary32 row sums
 *     R_k in scan order (row k replaces the choice iff u_(16+k) S < R_k, S
 *     the running sum), then within that row the first texel whose running
 *     binary32 sum exceeds u_1 R (the last texel of positive weight if none
 *     does).  u_a is hash index a of the query.  One texel read per lookup.
 *   - A zero footprint reads bilinearly from level 0 (stochastic: the linear
 *     draw with hash indices 2, 3); taps are clamped.
 * Work per query is bounded: the ellipse is scanned only where its minor
 * axis spans fewer than 4 texels, so its box holds O(max_anisotropy) taps.
 * Queries with a non-finite or |value| >= 65536 entry give NaN, and so do
 * queries whose raster position on level 0, s W0 - 1/2 or t H0 - 1/2 in
 * binary32, is not below 2^24 in magnitude (as for every 2D filter; indices
 * INT32_MIN).
 * max_anisotropy in [1, 64] (the real-time implementation's maximum).
 * out_index_dev: NULL or (stochastic) n x 3 int32 (x, y, level).  Binary32
 * accumulation. */
stf_status stf_filter_ewa(const stf_texture* tex, const float* queries_dev, int64_t n, float max_anisotropy,
                          stf_mode mode, uint64_t seed, float* out_dev, int32_t* out_index_dev, void* hip_stream);

/* ---------------------------------------------------------------------- */
/* DCT-compressed textures                                                 */
/* ---------------------------------------------------------------------- */
/* A texture of 8x8 texel blocks, each channel of a block stored as one
 * 32-bit word: the six lowest-frequency coefficients of its orthonormal 2D
 * DCT (section "Results", texture compression), 16x smaller than 8-bit
 * texels.  A lookup decodes single texels, so stochastic filtering decodes
 * one texel per lookup where deterministic bilinear / bicubic decode 4 / 16.
 *
 * Word layout: bits 0..6 DC code d (value d * 8/127), then five 5-bit AC
 * codes (bits 7..11, 12..16, 17..21, 22..26, 27..31) for the coefficients
 * (v, u) = (0,1), (1,0), (2,0), (1,1), (0,2) (v vertical, u horizontal
 * frequency), each q + 16 with q in -15..15 (value q * 2/15).  A decoded
 * texel is the inverse DCT of these six coefficients (not clamped); the
 * device decodes in binary32. */

/* Encodes width x height x channels 8-bit texels (row-major, channels
 * interleaved, value v/255) into (height/8)(width/8) channels words (blocks
 * row-major, channel words consecutive) on the host: DCT in binary64, codes
 * rounded to nearest (halves away from zero) and saturated.  width and
 * height: multiples of 8 up to 65536; channels 1..16. */
stf_status stf_dct_encode(int32_t width, int32_t height, int32_t channels, const uint8_t* texels_host,
                          uint32_t* blocks_host);

/* Creates a DCT texture from words laid out as stf_dct_encode writes them
 * (copied; may be freed on return).  Filter it with stf_filter /
 * stf_filter_ordered / stf_filter_moments and uv queries (raster rules and
 * clamping of stf_create_texture2d); results are channels binary32 per
 * query.  Not usable with shading, neural or serving calls. */
stf_status stf_create_dct_texture2d(int32_t width, int32_t height, int32_t channels, const uint32_t* blocks_host,
                                    stf_texture** out);

/* ---------------------------------------------------------------------- */
/* Morton-ordered query streams                                            */
/* ---------------------------------------------------------------------- */
/* Device workspace (bytes) that stf_sort_queries needs for n queries. */
stf_status stf_sort_workspace_bytes(int64_t n, size_t* bytes);

/* Orders n queries of `tex` by the Morton code of their cell, so that
 * queries touching the same region run next to each other: the cell is the
 * 8^3 leaf of a 3D grid (cells of 8 * 2^s voxels when a grid has more than
 * 1024 leaves along an axis) or the 4x4 texel tile of level 0 of a 2D
 * texture, cell coordinates clamped to the texture's cells (queries outside
 * go with the border cells), b bits per axis where 2^b cells cover the
 * longest axis.  Queries with a non-finite coordinate go last.  The sort is
 * stable: equal keys keep their input order.  Writes order_dev[k] = the
 * index in queries_dev of the k-th query in that order (a permutation) and
 * sorted_queries_dev[k] = queries_dev[order_dev[k]].  workspace_dev: at
 * least stf_sort_workspace_bytes(n) bytes of device memory, 256-byte
 * aligned, used only during the call's stream work. */
stf_status stf_sort_queries(const stf_texture* tex, const float* queries_dev, int64_t n,
                            float* sorted_queries_dev, int32_t* order_dev, void* workspace_dev,
                            size_t workspace_bytes, void* hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * sort as stf_sort_queries, with the same results bit for bit, whose
 * workspace is a fixed device array inside the library instead of a
 * caller-provided buffer.  The call allocates nothing (no hipMalloc, no
 * allocating library routine); the caller still provides the queries and
 * the two outputs.
 *   - n <= STF_SORT_NOALLOC_MAX_QUERIES (2^20); larger n gives STF_E_INVALID.
 *   - The array takes 16.3 MB of device memory on each device the call runs
 *     on, from the library's load until the process ends.
 *   - Every call on a device uses that device's single array: calls that
 *     overlap on one device (concurrent streams or host threads) race and
 *     must be serialized by the caller.  The array keeps the last call's
 *     contents; the sort needs no part of it cleared. */
#define STF_SORT_NOALLOC_MAX_QUERIES (1 << 20)
stf_status stf_sort_queries_noalloc(const stf_texture* tex, const float* queries_dev, int64_t n,
                                    float* sorted_queries_dev, int32_t* order_dev, void* hip_stream);

#define STF_ORDER_SCATTER 1u   /* results at out[order[k]] (the caller's order) */

/* stf_filter on a sorted stream: query k of sorted_queries_dev is query
 * order_dev[k] of the caller's batch and draws its random numbers as that
 * query.  Results go to out[k] (sorted order), or to out[order_dev[k]] with
 * STF_ORDER_SCATTER, where they equal stf_filter's on the unsorted batch
 * bit for bit.  Deterministic bicubic / tricubic filtering of a sorted
 * stream of a 3D grid or a DCT texture reads the texels its neighbouring
 * queries share once per block (staged in LDS) where that pays. */
stf_status stf_filter_ordered(const stf_texture* tex, const float* sorted_queries_dev,
                              const int32_t* order_dev, int64_t n, stf_filter_kind filter,
                              stf_mode mode, uint64_t seed, float* out_dev, int32_t* out_index_dev,
                              uint32_t flags, void* hip_stream);

/* Per-query first and second moments of the stochastic estimator over
 * n_seeds draws (seeds seed_base .. seed_base + n_seeds - 1), accumulated in
 * binary64 on the device: sum_dev[q] = sum_k v_k, sumsq_dev[q] = sum_k v_k^2,
 * where v_k is exactly what stf_filter(..., STF_STOCHASTIC, seed_base + k)
 * returns for query q (channel 0 of 2D textures).  This is the statistic of
 * the unbiasedness claim of Eq. stochastic-sum (and, for the interpolating
 * cubics, of the positivized estimate). */
stf_status stf_filter_moments(const stf_texture* tex, const float* queries_dev, int64_t n,
                              stf_filter_kind filter, uint64_t seed_base, int32_t n_seeds,
                              double* sum_dev, double* sumsq_dev, void* hip_stream);

/* Shading with a filtered material (section "Effect of Texture Filtering on
 * Rendering").  Each query is 9 binary32: uv (2), footprint scale s in
 * texels (1), outgoing direction wo (3), incident direction wi (3), both
 * unit vectors in the tangent frame (z = geometric normal).  The level is
 * l = [s >= 1.41421354f] + [s >= 2.82842708f], capped at levels-1.  The
 * filter is the B-spline (`filter` = STF_CUBIC_BSPLINE) or linear one on
 * that level (the interpolating cubics give STF_E_UNSUPPORTED).  Shading
 * f^ = BSDF * cos is a GGX microfacet model:
 *   albedo = rgb/255, alpha = max(r^2, 1e-3) with r = roughness/255,
 *   n = normalize-free (x, y, sqrt(max(0, 1 - x^2 - y^2))),
 *   h = normalize(wo + wi), D = alpha^2 / (pi (c^2 alpha^2 + |n x h|^2)^2)
 *   with c = n.h, G2 = 1/(1 + L(wo) + L(wi)),
 *   L(w) = (-1 + sqrt(1 + alpha^2 tan^2)) / 2 with tan^2 = |n x w|^2/(n.w)^2,
 *   F = 0.04 + 0.96 (1 - wi.h)^5,
 *   f^ = (albedo/pi + D G2 F / (4 (n.wo)(n.wi))) (n.wi), 0 if n.wo <= 0
 *   or n.wi <= 0.
 * Only levels 0..2 are reachable by the level rule; further levels are
 * stored but unused.  out_rgb_dev: n x 3 binary32.  out_index_dev: NULL or,
 * in stochastic mode, n x 3 int32 (x, y, level).  Results are binary32
 * evaluations of the formulas above, reciprocals and square roots by the
 * hardware's approximations (about one ulp each); no bit-exactness is
 * promised for the shaded values (they agree with a binary64 evaluation to
 * 1e-4 relative + 1e-6 absolute), the sampled tap is exact. */
stf_status stf_shade_filter(const stf_texture* material, const float* shade_queries_dev, int64_t n,
                            stf_filter_kind filter, stf_shade_mode mode, uint64_t seed,
                            float* out_rgb_dev, int32_t* out_index_dev, void* hip_stream);

/* ---------------------------------------------------------------------- */
/* Neural texture                                                          */
/* ---------------------------------------------------------------------- */
/* A tex_w x tex_h texture of 8 channels represented by a lat_w x lat_h grid
 * of 8-vectors and an MLP 8 -> 64 -> 64 -> 8 with ReLU after both hidden
 * layers: texel (i, j) decodes to MLP(z), z the bilinear interpolation of
 * the latent grid at X = (i + 1/2) lat_w/tex_w - 1/2 (likewise Y), corners
 * clamped.  The paper's case for stochastic filtering of such encodings: a
 * lookup decodes one texel instead of one per tap (sections Introduction
 * and Background on neural and compressed representations).
 *
 * MLP parameter vector (stf_ntex_param_count() = 5256 binary32 values):
 * W1[64][8], b1[64], W2[64][64], b2[64], W3[8][64], b3[8], row = output
 * feature.  Latents: lat_h x lat_w x 8 binary32, channels interleaved. */
typedef struct stf_neural stf_neural;   /* opaque, library-owned */

int32_t stf_ntex_param_count(void);

/* tex_w / lat_w and tex_h / lat_h must be powers of two (else
 * STF_E_UNSUPPORTED).  Initial parameters are copied from host memory. */
stf_status stf_ntex_create(int32_t tex_w, int32_t tex_h, int32_t lat_w, int32_t lat_h,
                           const float* latents_host, const float* mlp_host, stf_neural** out);
void stf_ntex_destroy(stf_neural* nt);

/* `steps` Adam steps (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected) on
 * the mean squared error (1/(8B)) sum (decoded - target)^2 over batches of
 * `batch` texel positions drawn from the counter hash of (seed, step).
 * target_dev: tex_h x tex_w x 8 binary32 on the device (16-byte aligned).
 * loss_dev: NULL or `steps` binary32, the loss of each step.  Training runs
 * in binary32 with the library's own kernels; the latent gradient is
 * accumulated with atomics, so it is not bitwise reproducible. */
stf_status stf_ntex_train(stf_neural* nt, const float* target_dev, int32_t steps, int32_t batch,
                          float lr_latent, float lr_mlp, uint64_t seed, float* loss_dev, void* hip_stream);

/* The gradient of the same loss over an explicit batch: positions_dev is
 * batch x 2 int32 texel coordinates (i, j).  Writes lat_h*lat_w*8 latent
 * gradients, 5256 MLP gradients and the loss (nullable), all device memory.
 * Positions outside the texture are clamped to it.
 * The parameters are not changed. */
stf_status stf_ntex_gradients(stf_neural* nt, const float* target_dev, const int32_t* positions_dev,
                              int32_t batch, float* grad_latents_dev, float* grad_mlp_dev,
                              float* loss_dev, void* hip_stream);

/* Copies the current binary32 parameters to host memory (synchronises the
 * device).  Either pointer may be NULL. */
stf_status stf_ntex_get_params(const stf_neural* nt, float* latents_host, float* mlp_host);

/* Freezes the current parameters for inference: latents rounded to binary16,
 * weights to bfloat16 (round to nearest even), biases kept in binary32.
 * Must be called after training and before stf_ntex_filter.  The inference
 * copy of the latents holds, per latent cell, the four corners a bilinear
 * lookup reads (64 (lat_w + 1)(lat_h + 1) bytes, allocated at creation). */
stf_status stf_ntex_prepare_inference(stf_neural* nt, void* hip_stream);

/* Filters decoded texels at n uv queries (n x 2 binary32, raster rules of
 * stf_create_texture2d, clamped taps), bilinear or bicubic B-spline;
 * deterministic decodes every tap (4 or 16 decodes per query), stochastic
 * decodes the one sampled tap.  Decoding runs on BF16 matrix cores with
 * binary32 accumulation: the interpolated latent and each hidden activation
 * (after ReLU) are rounded to bfloat16.  out_dev: n x 8 binary32 (16-byte
 * aligned); out_index_dev: NULL or (stochastic) n x 2 int32 texel (x, y).
 * The interpolating cubics give STF_E_UNSUPPORTED. */
stf_status stf_ntex_filter(const stf_neural* nt, const float* queries_dev, int64_t n,
                           stf_filter_kind filter, stf_mode mode, uint64_t seed, float* out_dev,
                           int32_t* out_index_dev, void* hip_stream);

/* ---------------------------------------------------------------------- */
/* Serving                                                                 */
/* ---------------------------------------------------------------------- */
/* A server batches stochastic lookup requests of any size against resident
 * textures (2D textures, materials and 3D grids) as they arrive.  A worker thread
 * admits requests in arrival order while fewer than max_resident are
 * resident and their staged state fits in a memory_budget_bytes arena
 * (queries unless STF_SERVE_QUERIES_ON_DEVICE; results and indices unless
 * STF_SERVE_RESULTS_ON_DEVICE, in which case the kernels write them straight
 * into the caller's out / out_index), serves the next chunk (<= chunk_queries)
 * of every resident request in each round with one launch per (texture,
 * filter), copies finished host results to the caller's buffer, and records
 * each request's latency from its arrival to the moment its results are in
 * place.  Requests arriving while others run
 * join the next round.  The random draw of a query depends only on (seed,
 * index within the request), so each request's results are bit-identical to
 * stf_filter(tex, queries, n, filter, STF_STOCHASTIC, seed, ...) alone.
 * Buffers passed to a request must stay valid until it has completed. */
typedef struct stf_server stf_server;   /* opaque, library-owned */

typedef struct {
    int64_t memory_budget_bytes;   /* device arena for request state (>= 4096) */
    int32_t max_resident;          /* requests resident at once (1..65536) */
    int32_t chunk_queries;         /* queries of one request per round (>= 1) */
} stf_server_config;

typedef struct {
    int64_t completed, cancelled, queries, launches, rounds;
    int64_t peak_resident, peak_arena_bytes, pending, resident;
    double p50_ms, p99_ms, max_ms, mean_ms;   /* latency, arrival -> results in place */
    double lookups_per_s;                     /* completed queries / (last completion - first arrival) */
    double span_s;
} stf_serve_stats;

/* With a flag set, the buffers it names must be device memory of the
 * request's size; submission rejects (STF_E_INVALID) a buffer that is not
 * device memory or does not fit in the device allocation holding it (a
 * buffer carved from a larger allocation is checked against that
 * allocation only).
 * Device results are written chunk by chunk in place, so a cancelled request
 * may leave some of them written; host results are copied only on
 * completion. */
#define STF_SERVE_QUERIES_ON_DEVICE 1u   /* queries are device memory (else host) */
#define STF_SERVE_RESULTS_ON_DEVICE 2u   /* out/out_index are device memory (else host) */

stf_status stf_server_create(const stf_server_config* cfg, stf_server** out);
/* Cancels pending requests, lets resident ones finish, frees everything. */
void stf_server_destroy(stf_server* s);

/* Queue a request of n queries (2 or 3 binary32 each, per the texture).
 * out: n x channels binary32; out_index: NULL or n x dims int32.  flags:
 * STF_SERVE_* bits.  A request whose state can never fit the arena is
 * rejected with STF_E_OOM; the interpolating cubics give
 * STF_E_UNSUPPORTED.  *ticket identifies it. */
stf_status stf_server_submit(stf_server* s, const stf_texture* tex, const float* queries, int64_t n,
                             stf_filter_kind filter, uint64_t seed, float* out, int32_t* out_index,
                             uint32_t flags, uint64_t* ticket);
/* *done = 1 once results are in place (STF_E_CANCELLED / STF_E_DEVICE if
 * the request was cancelled / failed). */
stf_status stf_server_poll(stf_server* s, uint64_t ticket, int32_t* done);
/* Blocks until done or timeout (STF_E_BUSY on timeout); timeout_s >= 0,
 * values above 1e6 (or HUGE_VAL) wait without a deadline. */
stf_status stf_server_wait(stf_server* s, uint64_t ticket, double timeout_s);
/* A pending request is dropped at once; a resident one gets no further
 * chunks and is retired once none of its copies or launches is in flight
 * (the staging copy of host queries included), so its buffers may be freed
 * as soon as poll or wait reports it cancelled. */
stf_status stf_server_cancel(stf_server* s, uint64_t ticket);
/* Forget a finished request (its ticket becomes unknown). */
stf_status stf_server_release(stf_server* s, uint64_t ticket);
stf_status stf_server_stats(stf_server* s, stf_serve_stats* st);
stf_status stf_server_reset_stats(stf_server* s);

/* Open-loop replay: submits reqs[k] at arrival_s seconds after the call
 * starts (arrivals non-decreasing), latency counted from that scheduled
 * time, waits for all (at most timeout_s) and releases them.  If a submit
 * fails or the time-out passes, the requests still outstanding are
 * cancelled and the call returns (with the error) only once none of them
 * can write to its out / out_index buffers any more. */
typedef struct {
    const stf_texture* tex;
    const float* queries;
    int64_t n;
    stf_filter_kind filter;
    uint64_t seed;
    float* out;
    int32_t* out_index;
    double arrival_s;
} stf_serve_request;

stf_status stf_server_replay(stf_server* s, const stf_serve_request* reqs, int64_t count, uint32_t flags,
                             double timeout_s);

/* Staging counters, for tests and tuning.  The deterministic bicubic /
 * tricubic kernels of sorted streams (stf_filter_ordered on a 3D grid) and
 * of DCT textures decide per block of 256 queries whether to stage the
 * texels of the block's tap box in LDS (when the box is small enough and
 * each staged texel serves at least 4 taps) or to read taps from global
 * memory.  stf_stage_counting(1) zeroes two device counters of the current
 * device and makes those kernels count {blocks that staged, blocks} from
 * then on; stf_stage_counting(0) stops counting (the default: nothing is
 * counted).  stf_stage_counts synchronizes the device and reads them.  The
 * counters are shared by every stream and thread using the device. */
stf_status stf_stage_counting(int32_t on);
stf_status stf_stage_counts(uint64_t* staged_blocks, uint64_t* blocks);

/* Message for the last failing call on this thread ("" if none). */
const char* stf_last_error(void);

/* Library version string. */
const char* stf_version(void);

#ifdef __cplusplus
}
#endif

#endif /* STF_H */
