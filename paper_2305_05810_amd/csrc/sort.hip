// sort.hip -- Morton ordering of query streams.
//
// Queries that land in the same region of a texture should run next to each
// other: neighbouring lanes then share leaves, tree nodes and cache lines.
// stf_sort_queries computes a Morton key per query -- the interleaved bits of
// its cell coordinates, a cell being an 8^3 leaf of a 3D grid or a 4x4 texel
// tile of a 2D texture -- sorts the queries by key with a stable LSD radix
// sort written for this purpose, and writes the permutation and the queries
// in that order.  stf_filter_ordered then filters the sorted stream with each
// query's draw keyed by its original id, so its results are exactly those of
// stf_filter on the unsorted batch.
//
// The key has b bits per axis, b the smallest count with 2^b cells covering
// the longest axis (at most 10 in 3D: larger grids use cells of 8 * 2^s
// voxels), coordinates clamped to the texture's cells, plus one bit above
// them that is set for a query with a non-finite coordinate (those go last).
// The 512^3 grid has 64 leaves per axis: 18 + 1 = 19 key bits, three passes
// of 7-bit digits (passes of at most 8 bits: 10-bit digits need one pass
// fewer, but their tiles hold 4 keys per digit on average, and the scatter
// of such short runs measured 0.64 against 0.58 ms for the 16M stream).
//
// One pass of the radix sort, for digit bits [shift, shift + D) with R = 2^D:
//   1. histogram: each tile of 4096 keys counts its digits (ballot-matched
//      lanes of equal digit add once) into row t of a tile-major table
//      H[t][R]; the first pass computes the keys from the queries here;
//   2. offsets: a four-kernel scan turns H into the global position of the
//      first key of digit d of tile t (per-chunk digit sums, a scan over the
//      chunks of each digit, a scan over the digits, then each chunk's
//      running sums written in place);
//   3. scatter: each tile ranks its keys stably (a wave takes 1024 contiguous
//      keys in rounds of 64; lanes of equal digit find each other with D
//      ballots and count in the wave's LDS counters), places them in LDS in
//      sorted order, and writes them out so that consecutive lanes write
//      consecutive positions of a digit's run.  The last pass writes the
//      permutation and gathers the queries instead of (key, id) pairs.
#include <algorithm>
#include <mutex>

#include "device_common.h"
#include "stf_internal.h"

using namespace stf;

namespace {

constexpr int BLOCK = 256;
constexpr int WAVES = BLOCK / 64;
constexpr int ITEMS = 16;                  // keys per thread
constexpr int TILE = BLOCK * ITEMS;        // keys per tile: 4096
constexpr int WAVE_KEYS = TILE / WAVES;    // contiguous keys per wave: 1024
#ifndef STF_SORT_DIGIT_BITS
#define STF_SORT_DIGIT_BITS 8
#endif
constexpr int MAX_DIGIT = STF_SORT_DIGIT_BITS;   // widest digit of one pass
constexpr int MAX_R = 1 << MAX_DIGIT;
constexpr int CHUNK = 16;                  // tiles per chunk of the offset scan
constexpr uint32_t MAX_CELL_BITS_3D = 10;

struct KeySpec {
    int dims;           // 2 or 3
    int cell_shift;     // log2 of the cell edge in texels / voxels
    int bits;           // Morton bits per axis
    int cells[3];       // cells per axis
    float w, h;         // 2D: level-0 size (raster x = uv * w - 1/2)
};

__device__ __forceinline__ uint32_t spread3(uint32_t v)   // 10 bits -> every third bit
{
    v &= 0x3ffu;
    v = (v | (v << 16)) & 0x030000ffu;
    v = (v | (v << 8)) & 0x0300f00fu;
    v = (v | (v << 4)) & 0x030c30c3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}

__device__ __forceinline__ uint32_t spread2(uint32_t v)   // 15 bits -> every other bit
{
    v &= 0x7fffu;
    v = (v | (v << 8)) & 0x00ff00ffu;
    v = (v | (v << 4)) & 0x0f0f0f0fu;
    v = (v | (v << 2)) & 0x33333333u;
    v = (v | (v << 1)) & 0x55555555u;
    return v;
}

// Cell of a finite coordinate: floor(x) >> shift clamped to [0, cells - 1].
__device__ __forceinline__ uint32_t cell_of_coord(float x, int shift, int cells)
{
    const float f = __builtin_floorf(fminf(fmaxf(x, -1.0f), 16777215.0f));
    const int c = (int)f >> shift;   // arithmetic: -1 >> s = -1
    return c < 0 ? 0u : (c >= cells ? (uint32_t)(cells - 1) : (uint32_t)c);
}

__device__ __forceinline__ uint32_t query_key(const KeySpec& s, const float* __restrict__ q, int64_t i)
{
    if (s.dims == 3) {
        const float x = q[3 * i], y = q[3 * i + 1], z = q[3 * i + 2];
        if (!(__builtin_isfinite(x) && __builtin_isfinite(y) && __builtin_isfinite(z))) return 1u << (3 * s.bits);
        return spread3(cell_of_coord(x, s.cell_shift, s.cells[0])) |
               (spread3(cell_of_coord(y, s.cell_shift, s.cells[1])) << 1) |
               (spread3(cell_of_coord(z, s.cell_shift, s.cells[2])) << 2);
    }
    const float2 uv = reinterpret_cast<const float2*>(q)[i];
    if (!(__builtin_isfinite(uv.x) && __builtin_isfinite(uv.y))) return 1u << (2 * s.bits);
    const float x = uv.x * s.w - 0.5f, y = uv.y * s.h - 0.5f;
    return spread2(cell_of_coord(x, s.cell_shift, s.cells[0])) |
           (spread2(cell_of_coord(y, s.cell_shift, s.cells[1])) << 1);
}

// Lanes of the wave whose digit equals this lane's, among the lanes in
// `live` (D ballots: a lane keeps the lanes that agree with it on every bit).
__device__ __forceinline__ uint64_t match_digit(uint32_t d, int dbits, uint64_t live)
{
    uint64_t m = live;
    for (int b = 0; b < dbits; ++b) {
        const bool bit = (d >> b) & 1u;
        const uint64_t on = __ballot(bit);
        m &= bit ? on : ~on;
    }
    return m;
}

__device__ __forceinline__ uint32_t lanes_below(uint64_t m, int lane)
{
    return (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
}

// Histogram of one tile's digits into H[t][0..R).  FIRST: the keys are
// computed from the queries and stored.
template <bool FIRST>
__global__ __launch_bounds__(BLOCK) void k_hist(KeySpec spec, const float* __restrict__ q,
                                                uint32_t* __restrict__ keys, int32_t n, int shift, int dbits,
                                                uint32_t* __restrict__ H)
{
    __shared__ uint32_t hist[MAX_R];
    const int R = 1 << dbits;
    for (int d = threadIdx.x; d < R; d += BLOCK) hist[d] = 0;
    __syncthreads();
    const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
    const int64_t w0 = (int64_t)blockIdx.x * TILE + wave * WAVE_KEYS;
    uint32_t key[ITEMS];
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {   // all loads first, so they are in flight together
        const int64_t i = w0 + r * 64 + lane;
        key[r] = 0;
        if (i < n) {
            if constexpr (FIRST)
                key[r] = query_key(spec, q, i);
            else
                key[r] = keys[i];
        }
    }
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
        const int64_t i = w0 + r * 64 + lane;
        const bool live = i < n;
        if constexpr (FIRST)
            if (live) keys[i] = key[r];
        const uint32_t d = (key[r] >> shift) & (uint32_t)(R - 1);
        const uint64_t m = match_digit(d, dbits, __ballot(live));
        if (live && lanes_below(m, lane) == 0) atomicAdd(&hist[d], (uint32_t)__popcll(m));
    }
    __syncthreads();
    for (int d = threadIdx.x; d < R; d += BLOCK) H[(int64_t)blockIdx.x * R + d] = hist[d];
}

// Offsets, step 1 (grid: chunks x digit groups of BLOCK, a thread per
// digit): S[c][d] = sum of H[t][d] over the CHUNK tiles t of chunk c.
__global__ __launch_bounds__(BLOCK) void k_chunk_sums(const uint32_t* __restrict__ H, int ntiles, int R,
                                                      uint32_t* __restrict__ S)
{
    const int d = blockIdx.y * BLOCK + threadIdx.x;
    if (d >= R) return;
    const int t0 = blockIdx.x * CHUNK;
    uint32_t v[CHUNK];
#pragma unroll
    for (int k = 0; k < CHUNK; ++k) v[k] = t0 + k < ntiles ? H[(int64_t)(t0 + k) * R + d] : 0u;
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < CHUNK; ++k) s += v[k];
    S[(int64_t)blockIdx.x * R + d] = s;
}

// Exclusive scan across a block of BLOCK threads of one value per thread;
// returns this thread's exclusive prefix and (in *total) the block's sum.
__device__ __forceinline__ uint32_t block_scan_excl(uint32_t x, uint32_t* wsum, uint32_t* total)
{
    const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
    uint32_t incl = x;
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t v = __shfl_up(incl, off, 64);
        if (lane >= off) incl += v;
    }
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    uint32_t before = 0, all = 0;
#pragma unroll
    for (int k = 0; k < WAVES; ++k) {
        before += k < wave ? wsum[k] : 0u;
        all += wsum[k];
    }
    __syncthreads();
    *total = all;
    return before + incl - x;
}

// Offsets, step 2 (a block per digit d): S[c][d] becomes the count of digit
// d in the chunks before c, and T[d] the count of digit d in all tiles.  A
// thread takes `per` consecutive chunks.
__global__ __launch_bounds__(BLOCK) void k_spine(uint32_t* __restrict__ S, int nchunks, int R,
                                                 uint32_t* __restrict__ T)
{
    __shared__ uint32_t wsum[WAVES];
    const int d = blockIdx.x;
    const int per = (nchunks + BLOCK - 1) / BLOCK, c0 = threadIdx.x * per;
    uint32_t s = 0;
    for (int k = 0; k < per; ++k)
        if (c0 + k < nchunks) s += S[(int64_t)(c0 + k) * R + d];
    uint32_t total;
    uint32_t run = block_scan_excl(s, wsum, &total);
    for (int k = 0; k < per; ++k)
        if (c0 + k < nchunks) {
            const uint32_t v = S[(int64_t)(c0 + k) * R + d];
            S[(int64_t)(c0 + k) * R + d] = run;
            run += v;
        }
    if (threadIdx.x == 0) T[d] = total;
}

// Offsets, step 3 (one block of MAX_R threads): base[d] = the count of all
// digits below d.
__global__ __launch_bounds__(MAX_R) void k_digit_base(const uint32_t* __restrict__ T, int R,
                                                      uint32_t* __restrict__ base)
{
    __shared__ uint32_t wsum[MAX_R / 64];
    const int d = threadIdx.x;
    const uint32_t total = d < R ? T[d] : 0u;
    const int lane = d % 64, wave = d / 64;
    uint32_t incl = total;
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t v = __shfl_up(incl, off, 64);
        if (lane >= off) incl += v;
    }
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    uint32_t before = 0;
    for (int k = 0; k < wave; ++k) before += wsum[k];
    if (d < R) base[d] = before + incl - total;
}

// Offsets, step 4 (grid as step 1): H[t][d] becomes the global position of
// tile t's first key of digit d.
__global__ __launch_bounds__(BLOCK) void k_chunk_offsets(uint32_t* __restrict__ H, int ntiles, int R,
                                                         const uint32_t* __restrict__ S,
                                                         const uint32_t* __restrict__ base)
{
    const int d = blockIdx.y * BLOCK + threadIdx.x;
    if (d >= R) return;
    const int t0 = blockIdx.x * CHUNK;
    uint32_t v[CHUNK];
#pragma unroll
    for (int k = 0; k < CHUNK; ++k) v[k] = t0 + k < ntiles ? H[(int64_t)(t0 + k) * R + d] : 0u;
    uint32_t run = S[(int64_t)blockIdx.x * R + d] + base[d];
#pragma unroll
    for (int k = 0; k < CHUNK; ++k)
        if (t0 + k < ntiles) {
            H[(int64_t)(t0 + k) * R + d] = run;
            run += v[k];
        }
}

// Exclusive scan of v[0..R) in place, by the whole block (R <= MAX_R).
__device__ void block_exclusive_scan(uint32_t* v, int R, uint32_t* wsum)
{
    const int per = (R + BLOCK - 1) / BLOCK;   // consecutive entries per thread
    const int d0 = threadIdx.x * per;
    uint32_t s = 0;
    for (int k = 0; k < per; ++k)
        if (d0 + k < R) s += v[d0 + k];
    const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
    uint32_t incl = s;
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t x = __shfl_up(incl, off, 64);
        if (lane >= off) incl += x;
    }
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    uint32_t run = incl - s;
    for (int k = 0; k < wave; ++k) run += wsum[k];
    for (int k = 0; k < per; ++k)
        if (d0 + k < R) {
            const uint32_t x = v[d0 + k];
            v[d0 + k] = run;
            run += x;
        }
    __syncthreads();
}

// One scatter pass.  FIRST: the ids are the keys' indices.  LAST: writes
// order[pos] = id and the query itself instead of (key, id).
template <bool FIRST, bool LAST, int DIMS>
__global__ __launch_bounds__(BLOCK) void k_scatter(const uint32_t* __restrict__ keys_in,
                                                   const int32_t* __restrict__ ids_in, int32_t n, int shift,
                                                   int dbits, const uint32_t* __restrict__ H,
                                                   uint32_t* __restrict__ keys_out, int32_t* __restrict__ ids_out,
                                                   const float* __restrict__ q, float* __restrict__ sorted,
                                                   int32_t* __restrict__ order)
{
    __shared__ uint32_t cnt[WAVES][MAX_R];   // per-wave digit counts, then the wave's start within the digit
    __shared__ uint32_t lstart[MAX_R];       // first position of digit d within the tile
    __shared__ uint32_t gstart[MAX_R];       // first global position of digit d for this tile
    __shared__ uint32_t skey[TILE];
    __shared__ int32_t sid[TILE];
    __shared__ uint32_t wsum[WAVES];
    const int R = 1 << dbits;
    for (int k = threadIdx.x; k < WAVES * MAX_R; k += BLOCK) (&cnt[0][0])[k] = 0;
    __syncthreads();
    const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
    const int64_t tile0 = (int64_t)blockIdx.x * TILE;
    const int64_t w0 = tile0 + wave * WAVE_KEYS;
    uint32_t key[ITEMS], rank[ITEMS];
    int32_t id[ITEMS];
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {   // all loads first, so they are in flight together
        const int64_t i = w0 + r * 64 + lane;
        const bool live = i < n;
        key[r] = live ? keys_in[i] : 0u;
        id[r] = FIRST ? (int32_t)i : (live ? ids_in[i] : 0);
    }
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
        const int64_t i = w0 + r * 64 + lane;
        const bool live = i < n;
        const uint32_t d = (key[r] >> shift) & (uint32_t)(R - 1);
        const uint64_t m = match_digit(d, dbits, __ballot(live));
        const int leader = m ? __ffsll((unsigned long long)m) - 1 : lane;
        uint32_t b = 0;
        if (live && leader == lane) {
            b = cnt[wave][d];
            cnt[wave][d] = b + (uint32_t)__popcll(m);
        }
        b = __shfl(b, leader, 64);
        rank[r] = b + lanes_below(m, lane);   // stable: earlier rounds, then lower lanes
    }
    __syncthreads();
    // per digit: the tile's count, each wave's start within the digit
    for (int d = threadIdx.x; d < R; d += BLOCK) {
        uint32_t run = 0;
#pragma unroll
        for (int w = 0; w < WAVES; ++w) {
            const uint32_t c = cnt[w][d];
            cnt[w][d] = run;
            run += c;
        }
        lstart[d] = run;
        gstart[d] = H[(int64_t)blockIdx.x * R + d];
    }
    __syncthreads();
    block_exclusive_scan(lstart, R, wsum);
    // place the tile in LDS in sorted order
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
        const int64_t i = w0 + r * 64 + lane;
        if (i < n) {
            const uint32_t d = (key[r] >> shift) & (uint32_t)(R - 1);
            const uint32_t p = lstart[d] + cnt[wave][d] + rank[r];
            if (p < (uint32_t)TILE) {   // always true; keeps a ranking fault inside the tile
                skey[p] = key[r];
                sid[p] = id[r];
            }
        }
    }
    __syncthreads();
    // write out: consecutive lanes take consecutive positions of a digit's
    // run; a thread handles entries threadIdx.x + r BLOCK, all read first
    const int count = (int)min((int64_t)TILE, (int64_t)n - tile0);
    uint32_t pos[ITEMS];
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
        const int e = (int)threadIdx.x + r * BLOCK;
        pos[r] = 0xffffffffu;
        if (e < count) {
            const uint32_t k = skey[e];
            const uint32_t d = (k >> shift) & (uint32_t)(R - 1);
            const uint32_t ps = gstart[d] + ((uint32_t)e - lstart[d]);
            const int32_t v = sid[e];
            if (ps < (uint32_t)n && (uint32_t)v < (uint32_t)n) {   // always true; guards the buffers
                pos[r] = ps;
                key[r] = k;
                id[r] = v;
            }
        }
    }
    if constexpr (LAST) {
        float g[ITEMS][DIMS];
#pragma unroll
        for (int r = 0; r < ITEMS; ++r)   // the gathers of the thread's queries, in flight together
#pragma unroll
            for (int a = 0; a < DIMS; ++a)
                g[r][a] = pos[r] != 0xffffffffu ? q[(int64_t)DIMS * id[r] + a] : 0.0f;
#pragma unroll
        for (int r = 0; r < ITEMS; ++r) {
            if (pos[r] == 0xffffffffu) continue;
            order[pos[r]] = id[r];
#pragma unroll
            for (int a = 0; a < DIMS; ++a) sorted[(int64_t)DIMS * pos[r] + a] = g[r][a];
        }
    } else {
#pragma unroll
        for (int r = 0; r < ITEMS; ++r) {
            if (pos[r] == 0xffffffffu) continue;
            keys_out[pos[r]] = key[r];
            ids_out[pos[r]] = id[r];
        }
    }
}

size_t align256(size_t b)
{
    return (b + 255) & ~(size_t)255;
}

int ntiles_of(int64_t n)
{
    return (int)((n + TILE - 1) / TILE);
}

int nchunks_of(int64_t n)
{
    return (ntiles_of(n) + CHUNK - 1) / CHUNK;
}

// Workspace layout: keys[2][n], ids[2][n], H[ntiles][MAX_R], S[nchunks][MAX_R], T[MAX_R], base[MAX_R].
struct SortWork {
    uint32_t* keys[2];
    int32_t* ids[2];
    uint32_t *H, *S, *T, *base;
};

size_t work_bytes(int64_t n)
{
    return 4 * align256((size_t)n * 4) + align256((size_t)ntiles_of(n) * MAX_R * 4) +
           align256((size_t)nchunks_of(n) * MAX_R * 4) + 2 * align256(MAX_R * 4);
}

SortWork carve(void* ws, int64_t n)
{
    char* p = (char*)ws;
    SortWork w;
    for (int k = 0; k < 2; ++k) {
        w.keys[k] = (uint32_t*)p;
        p += align256((size_t)n * 4);
    }
    for (int k = 0; k < 2; ++k) {
        w.ids[k] = (int32_t*)p;
        p += align256((size_t)n * 4);
    }
    w.H = (uint32_t*)p;
    p += align256((size_t)ntiles_of(n) * MAX_R * 4);
    w.S = (uint32_t*)p;
    p += align256((size_t)nchunks_of(n) * MAX_R * 4);
    w.T = (uint32_t*)p;
    p += align256(MAX_R * 4);
    w.base = (uint32_t*)p;
    return w;
}

int bits_for(int cells)   // smallest b with 2^b >= cells
{
    int b = 0;
    while ((1 << b) < cells) ++b;
    return b;
}

KeySpec key_spec(const stf_texture* tex)
{
    KeySpec s{};
    if (tex->kind == STF_KIND_GRID3D) {
        const int dims[3] = {tex->grid.dx, tex->grid.dy, tex->grid.dz};
        s.dims = 3;
        int widest = 1;
        for (int a = 0; a < 3; ++a) widest = std::max(widest, (dims[a] + 7) >> 3);
        const int b = bits_for(widest);
        const int extra = b > (int)MAX_CELL_BITS_3D ? b - (int)MAX_CELL_BITS_3D : 0;
        s.cell_shift = 3 + extra;
        s.bits = b - extra;
        for (int a = 0; a < 3; ++a) s.cells[a] = (dims[a] + (1 << s.cell_shift) - 1) >> s.cell_shift;
    } else {
        const TexLevel& L = tex->level[0];
        const int w = L.w, h = L.h;   // level 0 in texels (DCT textures too)
        s.dims = 2;
        s.cell_shift = 2;
        s.cells[0] = (w + 3) >> 2;
        s.cells[1] = (h + 3) >> 2;
        s.cells[2] = 1;
        s.bits = bits_for(std::max(s.cells[0], s.cells[1]));
        s.w = (float)w;
        s.h = (float)h;
    }
    return s;
}

stf_status check_ptr(const void* p, const char* what, size_t align)
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

template <int DIMS>
void launch_scatter(bool first, bool last, const SortWork& w, int src, int32_t n, int shift, int dbits,
                    const float* q, float* sorted, int32_t* order, hipStream_t st)
{
    const dim3 grid((unsigned)ntiles_of(n)), block(BLOCK);
    const uint32_t* kin = w.keys[src];
    const int32_t* iin = w.ids[src];
    uint32_t* kout = w.keys[1 - src];
    int32_t* iout = w.ids[1 - src];
    if (first && last)
        hipLaunchKernelGGL((k_scatter<true, true, DIMS>), grid, block, 0, st, kin, iin, n, shift, dbits, w.H, kout,
                           iout, q, sorted, order);
    else if (first)
        hipLaunchKernelGGL((k_scatter<true, false, DIMS>), grid, block, 0, st, kin, iin, n, shift, dbits, w.H, kout,
                           iout, q, sorted, order);
    else if (last)
        hipLaunchKernelGGL((k_scatter<false, true, DIMS>), grid, block, 0, st, kin, iin, n, shift, dbits, w.H, kout,
                           iout, q, sorted, order);
    else
        hipLaunchKernelGGL((k_scatter<false, false, DIMS>), grid, block, 0, st, kin, iin, n, shift, dbits, w.H, kout,
                           iout, q, sorted, order);
}

// The whole sort on stream st with the workspace w.
hipError_t run_sort(const stf_texture* tex, const float* q, int32_t n, float* sorted, int32_t* order,
                    const SortWork& w, hipStream_t st)
{
    const KeySpec spec = key_spec(tex);
    const int key_bits = spec.dims * spec.bits + 1;
    const int passes = (key_bits + MAX_DIGIT - 1) / MAX_DIGIT;
    const int dbits = (key_bits + passes - 1) / passes;
    const int R = 1 << dbits;
    const int ntiles = ntiles_of(n), nchunks = nchunks_of(n);
    const dim3 tiles((unsigned)ntiles), chunks((unsigned)nchunks, (unsigned)((R + BLOCK - 1) / BLOCK)), block(BLOCK);
    int src = 0;
    for (int p = 0; p < passes; ++p) {
        const int shift = p * dbits;
        if (p == 0)
            hipLaunchKernelGGL((k_hist<true>), tiles, block, 0, st, spec, q, w.keys[0], n, shift, dbits, w.H);
        else
            hipLaunchKernelGGL((k_hist<false>), tiles, block, 0, st, spec, q, w.keys[src], n, shift, dbits, w.H);
        hipLaunchKernelGGL(k_chunk_sums, chunks, block, 0, st, w.H, ntiles, R, w.S);
        hipLaunchKernelGGL(k_spine, dim3((unsigned)R), block, 0, st, w.S, nchunks, R, w.T);
        hipLaunchKernelGGL(k_digit_base, dim3(1), dim3(MAX_R), 0, st, w.T, R, w.base);
        hipLaunchKernelGGL(k_chunk_offsets, chunks, block, 0, st, w.H, ntiles, R, w.S, w.base);
        const bool last = p == passes - 1;
        if (spec.dims == 3)
            launch_scatter<3>(p == 0, last, w, src, n, shift, dbits, q, sorted, order, st);
        else
            launch_scatter<2>(p == 0, last, w, src, n, shift, dbits, q, sorted, order, st);
        src = 1 - src;
    }
    return hipGetLastError();
}

stf_status check_sort_args(const stf_texture* tex, const float* queries_dev, int64_t n, const float* sorted_dev,
                           const int32_t* order_dev)
{
    if (!tex) return stf_fail(STF_E_INVALID, "texture is NULL");
    if (tex->kind != STF_KIND_GRID3D && tex->kind != STF_KIND_MATERIAL && !is_2d_filterable(tex))
        return stf_fail(STF_E_INVALID, "sorting needs a 3D grid, a 2D texture or a material");
    if (n < 0 || n > 0x7fffffff) return stf_fail(STF_E_INVALID, "n = %lld out of range", (long long)n);
    if (n == 0) return STF_OK;
    const bool is3d = tex->kind == STF_KIND_GRID3D;
    stf_status s = check_ptr(queries_dev, "queries_dev", is3d ? 4 : 8);
    if (s == STF_OK) s = check_ptr(sorted_dev, "sorted_queries_dev", is3d ? 4 : 8);
    if (s == STF_OK) s = check_ptr(order_dev, "order_dev", 4);
    if (s != STF_OK) return s;
    if (sorted_dev == queries_dev) return stf_fail(STF_E_INVALID, "the sorted copy must not alias the queries");
    return STF_OK;
}

// The allocation-free variant's workspace: a file-scope device array of a
// fixed size, one copy per device, held until the process ends.  Host code
// never passes the array's name to a kernel (on the host it only stands for
// the symbol); it uses the device address that hipGetSymbolAddress returns on
// each device, looked up on the first call there.
constexpr int64_t NOALLOC_MAX_QUERIES = STF_SORT_NOALLOC_MAX_QUERIES;   // from stf.h
constexpr size_t NOALLOC_BYTES = (size_t)NOALLOC_MAX_QUERIES * 16 + ((size_t)NOALLOC_MAX_QUERIES / TILE) * MAX_R * 4 +
                                 ((size_t)NOALLOC_MAX_QUERIES / TILE / CHUNK + 1) * MAX_R * 4 + 2 * MAX_R * 4 +
                                 8 * 256;
static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

constexpr int MAX_DEVICES = 64;
static void* g_scratch_ptr[MAX_DEVICES];
static std::mutex g_scratch_mu;

// The device address of `scratch` on the current device (nullptr on failure).
void* scratch_address(int* dev_out)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) return nullptr;
    *dev_out = dev;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        g_scratch_ptr[dev] = p;
    }
    return g_scratch_ptr[dev];
}

}  // namespace

extern "C" {

stf_status stf_sort_queries_noalloc(const stf_texture* tex, const float* queries_dev, int64_t n,
                                    float* sorted_queries_dev, int32_t* order_dev, void* hip_stream)
{
    stf_clear_error();
    if (n > NOALLOC_MAX_QUERIES)
        return stf_fail(STF_E_INVALID, "n = %lld exceeds the %lld queries of the allocation-free sort's workspace",
                        (long long)n, (long long)NOALLOC_MAX_QUERIES);
    stf_status s = check_sort_args(tex, queries_dev, n, sorted_queries_dev, order_dev);
    if (s != STF_OK || n == 0) return s;
    if (work_bytes(n) > NOALLOC_BYTES) return stf_fail(STF_E_INVALID, "workspace layout exceeds the static array");
    int dev = 0;
    void* ws = scratch_address(&dev);
    if (!ws) return stf_fail(STF_E_DEVICE, "hipGetSymbolAddress of the sort workspace failed");
    hipError_t e = run_sort(tex, queries_dev, (int32_t)n, sorted_queries_dev, order_dev, carve(ws, n),
                            (hipStream_t)hip_stream);
    if (e != hipSuccess) return stf_fail(STF_E_DEVICE, "sorting failed: %s", hipGetErrorString(e));
    return STF_OK;
}

stf_status stf_sort_workspace_bytes(int64_t n, size_t* bytes)
{
    stf_clear_error();
    if (!bytes) return stf_fail(STF_E_INVALID, "bytes is NULL");
    if (n < 0 || n > 0x7fffffff) return stf_fail(STF_E_INVALID, "n = %lld out of range", (long long)n);
    *bytes = work_bytes(n);
    return STF_OK;
}

stf_status stf_sort_queries(const stf_texture* tex, const float* queries_dev, int64_t n, float* sorted_queries_dev,
                            int32_t* order_dev, void* workspace_dev, size_t workspace_bytes, void* hip_stream)
{
    stf_clear_error();
    stf_status s = check_sort_args(tex, queries_dev, n, sorted_queries_dev, order_dev);
    if (s != STF_OK || n == 0) return s;
    const size_t need = work_bytes(n);
    if (workspace_bytes < need) return stf_fail(STF_E_INVALID, "workspace of %zu bytes < %zu needed", workspace_bytes, need);
    s = check_ptr(workspace_dev, "workspace_dev", 256);
    if (s != STF_OK) return s;
    hipError_t e = run_sort(tex, queries_dev, (int32_t)n, sorted_queries_dev, order_dev, carve(workspace_dev, n),
                            (hipStream_t)hip_stream);
    if (e != hipSuccess) return stf_fail(STF_E_DEVICE, "sorting failed: %s", hipGetErrorString(e));
    return STF_OK;
}

stf_status stf_filter_ordered(const stf_texture* tex, const float* sorted_queries_dev, const int32_t* order_dev,
                              int64_t n, stf_filter_kind filter, stf_mode mode, uint64_t seed, float* out_dev,
                              int32_t* out_index_dev, uint32_t flags, void* hip_stream)
{
    stf_clear_error();
    if (!tex) return stf_fail(STF_E_INVALID, "texture is NULL");
    if (!is_2d_filterable(tex) && tex->kind != STF_KIND_GRID3D)
        return stf_fail(STF_E_INVALID, "stf_filter_ordered needs a 2D texture or a 3D grid");
    if (n < 0 || n > 0x7fffffff) return stf_fail(STF_E_INVALID, "n = %lld out of range", (long long)n);
    if (!valid_filter(filter)) return stf_fail(STF_E_INVALID, "unknown filter %d", (int)filter);
    if (!valid_mode(filter, mode)) return stf_fail(STF_E_INVALID, "mode %d is not available for filter %d", (int)mode, (int)filter);
    if (flags & ~(uint32_t)STF_ORDER_SCATTER) return stf_fail(STF_E_INVALID, "unknown flags 0x%x", flags);
    if (mode == STF_DETERMINISTIC && out_index_dev)
        return stf_fail(STF_E_INVALID, "out_index_dev must be NULL in deterministic mode");
    if (n == 0) return STF_OK;
    bool is2d = is_2d_filterable(tex);
    stf_status s = check_ptr(sorted_queries_dev, "sorted_queries_dev", is2d ? 8 : 4);
    if (s == STF_OK) s = check_ptr(order_dev, "order_dev", 4);
    if (s == STF_OK) s = check_ptr(out_dev, "out_dev", 4);
    if (s == STF_OK && out_index_dev) s = check_ptr(out_index_dev, "out_index_dev", 4);
    if (s != STF_OK) return s;
    int scatter = (flags & STF_ORDER_SCATTER) ? 1 : 0;
    uint32_t key = seed_key(seed);
    hipStream_t st = (hipStream_t)hip_stream;
    hipError_t e = is2d ? launch_filter2d(tex, sorted_queries_dev, (int32_t)n, filter, mode, key, out_dev,
                                          out_index_dev, order_dev, scatter, st)
                        : launch_filter3d(tex, sorted_queries_dev, (int32_t)n, filter, mode, key, out_dev,
                                          out_index_dev, order_dev, scatter, st);
    if (e != hipSuccess) return stf_fail(STF_E_DEVICE, "kernel launch failed: %s", hipGetErrorString(e));
    return STF_OK;
}

}  // extern "C"
