// stf_internal.h -- library-private declarations shared by the C ABI layer
// and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/stf.h"

enum stf_kind : int { STF_KIND_TEX2D = 1, STF_KIND_MATERIAL = 2, STF_KIND_GRID3D = 3, STF_KIND_DCT2D = 4 };

constexpr int STF_MAX_LEVELS = 16;

// Device view of one 2D level.
struct TexLevel {
    const void* texels;   // row-major, channels interleaved (materials: 4x4 tiles, see material_index)
    int32_t w, h;
};

// Materials are stored in tiles of 4x4 texels (8 bytes each: one 128-byte
// line per tile), tiles row-major over ceil(w/4) x ceil(h/4), texels
// row-major within a tile: a 4x4 filter footprint touches 1-4 lines
// (3.1 on average) instead of 4-8 rows of a row-major level.
__host__ __device__ inline int64_t material_index(int x, int y, int w)
{
    const int tiles_w = (w + 3) >> 2;
    return (((int64_t)(y >> 2) * tiles_w + (x >> 2)) << 4) + ((y & 3) << 2) + (x & 3);
}

// Device view of a sparse grid: root table -> internal nodes of 16^3 children
// -> dense 8^3 leaves.  A root slot covers 128^3 voxels, a node child slot
// 8^3 voxels.  -1 marks an empty slot.
struct GridView {
    const int32_t* root;   // rx * ry * rz node ids
    const int32_t* nodes;  // n_nodes * 4096 leaf ids, child (cx, cy, cz) at (cz*16 + cy)*16 + cx
    const void* leaves;    // n_leaves * 512 values, x fastest
    int32_t dx, dy, dz;    // domain
    int32_t rx, ry;        // root extents in x and y
    float background;
};

struct stf_texture {
    int kind;
    int fmt;
    int channels;
    int device;
    int64_t bytes;
    // 2D textures and materials (DCT textures: level 0 holds the blocks)
    int levels;
    TexLevel level[STF_MAX_LEVELS];
    void* level_alloc[STF_MAX_LEVELS];
    int32_t dct_wpb;   // DCT textures: words per block on the device (channels padded to a multiple of 4)
    // 3D grids
    GridView grid;
    int32_t rz;
    int64_t n_leaves;
    int32_t n_nodes;
    void* grid_alloc[3];
};

// One serving chunk: queries [0, count) of a request's slice, drawn with ids
// qid0 + index under the request's key, served by blocks [block0, next
// chunk's block0).
struct ServeChunk {
    const float* q;
    float* out;
    int32_t* idx;
    int32_t count;
    uint32_t qid0;
    uint32_t key;
    int32_t block0;
};

// Error reporting (thread-local message).
stf_status stf_fail(stf_status code, const char* fmt, ...);

// Textures that stf_filter reads with 2D (uv) queries.
inline bool is_2d_filterable(const stf_texture* t)
{
    return t->kind == STF_KIND_TEX2D || t->kind == STF_KIND_DCT2D || t->kind == STF_KIND_MATERIAL;
}

// Modes of stf_filter for a filter (filter importance sampling covers the
// B-spline family only).
inline bool valid_mode(int filter, int mode)
{
    if (mode == STF_DETERMINISTIC || mode == STF_STOCHASTIC) return true;
    return mode == STF_STOCHASTIC_FIS && (filter == STF_LINEAR || filter == STF_CUBIC_BSPLINE);
}

// Filters of stf_filter / stf_filter_ordered / stf_filter_moments.
inline bool valid_filter(int f)
{
    return f == STF_LINEAR || f == STF_CUBIC_BSPLINE || f == STF_CUBIC_KEYS || f == STF_CUBIC_MITCHELL;
}
void stf_clear_error();

// Device address of the staging counters {staged blocks, blocks} of the
// current device while counting is on (stf_stage_counting), else nullptr.
// The staged deterministic kernels take it as an argument.
unsigned long long* stage_counters();

// Kernel launchers; each returns hipSuccess or the launch error.
// order: NULL, or the caller-batch index of each (sorted) query, which keys
// its random draw; scatter: results go to out[order[i]] instead of out[i].
hipError_t launch_filter2d(const stf_texture* tex, const float* q, int32_t n, int filter, int mode,
                           uint32_t skey, float* out, int32_t* idx, const int32_t* order, int scatter,
                           hipStream_t stream);
hipError_t launch_filter3d(const stf_texture* tex, const float* q, int32_t n, int filter, int mode,
                           uint32_t skey, float* out, int32_t* idx, const int32_t* order, int scatter,
                           hipStream_t stream);
hipError_t launch_gauss2d(const stf_texture* t, const float* q, int32_t n, float sigma, int gmode, uint32_t key,
                          float* out, int32_t* idx, hipStream_t s);
hipError_t launch_moments2d(const stf_texture* tex, const float* q, int32_t n, int filter,
                            uint64_t seed_base, int32_t n_seeds, double* sum, double* sumsq,
                            hipStream_t stream);
hipError_t launch_moments3d(const stf_texture* tex, const float* q, int32_t n, int filter,
                            uint64_t seed_base, int32_t n_seeds, double* sum, double* sumsq,
                            hipStream_t stream);
hipError_t launch_shade(const stf_texture* mat, const float* q, int32_t n, int filter, int mode,
                        uint32_t skey, float* out, int32_t* idx, hipStream_t stream);

int32_t serve3d_queries_per_block();
int32_t serve2d_queries_per_block();
hipError_t launch_serve3d(const stf_texture* tex, int filter, const ServeChunk* chunks, int32_t nchunks,
                          int32_t nblocks, hipStream_t stream);
hipError_t launch_serve2d(const stf_texture* tex, int filter, const ServeChunk* chunks, int32_t nchunks,
                          int32_t nblocks, hipStream_t stream);
