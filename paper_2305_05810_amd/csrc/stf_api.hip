// stf_api.hip -- the C ABI of libstf: argument validation, texture creation
// and destruction, and dispatch to the kernel launchers.  Nothing is launched
// when validation fails.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <string>
#include <unordered_set>
#include <vector>

#include "device_common.h"
#include "stf_internal.h"

namespace {

thread_local std::string g_last_error;

constexpr int64_t MAX_QUERIES = 0x7fffffff;   // queries are indexed by a 32-bit id

bool valid_format(int fmt)
{
    return fmt >= STF_FMT_F32 && fmt <= STF_FMT_U8;
}

// A device pointer the caller passed for the kernels to read or write.
stf_status check_device_ptr(const void* p, const char* what, size_t align)
{
    if (!p) return stf_fail(STF_E_INVALID, "%s is NULL", what);
    if ((uintptr_t)p % align) return stf_fail(STF_E_INVALID, "%s is not %zu-byte aligned", what, align);
    hipPointerAttribute_t attr;
    hipError_t e = hipPointerGetAttributes(&attr, p);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return stf_fail(STF_E_INVALID, "%s is not a device pointer (%s)", what, hipGetErrorString(e));
    }
    if (attr.type != hipMemoryTypeDevice && attr.type != hipMemoryTypeManaged)
        return stf_fail(STF_E_INVALID, "%s is not device memory", what);
    return STF_OK;
}

stf_status upload(void** dst, const void* src, size_t bytes, const char* what)
{
    *dst = nullptr;
    if (bytes == 0) bytes = 4;   // keep a valid pointer for empty tables
    hipError_t e = hipMalloc(dst, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *dst = nullptr;
        return stf_fail(STF_E_OOM, "hipMalloc of %zu bytes for %s failed: %s", bytes, what, hipGetErrorString(e));
    }
    if (src) {
        e = hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            (void)hipFree(*dst);
            *dst = nullptr;
            return stf_fail(STF_E_DEVICE, "copy of %s to the device failed: %s", what, hipGetErrorString(e));
        }
    }
    return STF_OK;
}

void free_texture(stf_texture* t)
{
    if (!t) return;
    for (int l = 0; l < STF_MAX_LEVELS; ++l)
        if (t->level_alloc[l]) (void)hipFree(t->level_alloc[l]);
    for (int k = 0; k < 3; ++k)
        if (t->grid_alloc[k]) (void)hipFree(t->grid_alloc[k]);
    delete t;
}

stf_status create_levels(stf_texture* t, int32_t width, int32_t height, int32_t levels,
                         const void* const* level_texels_host, size_t texel_bytes)
{
    if (width <= 0 || height <= 0 || width > 65536 || height > 65536)
        return stf_fail(STF_E_INVALID, "texture size %dx%d out of range (1..65536)", width, height);
    if (levels < 1 || levels > STF_MAX_LEVELS)
        return stf_fail(STF_E_INVALID, "levels = %d out of range (1..%d)", levels, STF_MAX_LEVELS);
    if (!level_texels_host) return stf_fail(STF_E_INVALID, "level_texels_host is NULL");
    t->levels = levels;
    t->bytes = 0;
    for (int l = 0; l < levels; ++l) {
        int32_t w = width >> l, h = height >> l;
        if (w < 1) w = 1;
        if (h < 1) h = 1;
        if (!level_texels_host[l]) return stf_fail(STF_E_INVALID, "level %d texels are NULL", l);
        size_t bytes = (size_t)w * (size_t)h * texel_bytes;
        stf_status s = upload(&t->level_alloc[l], level_texels_host[l], bytes, "texture level");
        if (s != STF_OK) return s;
        t->level[l].texels = t->level_alloc[l];
        t->level[l].w = w;
        t->level[l].h = h;
        t->bytes += (int64_t)bytes;
    }
    return STF_OK;
}

}  // namespace

stf_status stf_fail(stf_status code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

void stf_clear_error()
{
    g_last_error.clear();
}

// Staging counters {blocks that staged their taps in LDS, blocks} of the
// staged deterministic kernels.  Each device holds its own copy of the array;
// host code uses the address hipGetSymbolAddress returns on that device.
static __device__ unsigned long long g_stage_count[2];
static unsigned long long* g_stage_ptr[64];   // per device, while counting is on
static std::mutex g_stage_mu;

unsigned long long* stage_counters()
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
    std::lock_guard<std::mutex> lk(g_stage_mu);
    return g_stage_ptr[dev];
}

extern "C" {

const char* stf_last_error(void)
{
    return g_last_error.c_str();
}

const char* stf_version(void)
{
    return "stf 0.1 (gfx950)";
}

stf_status stf_stage_counting(int32_t on)
{
    stf_clear_error();
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return stf_fail(STF_E_DEVICE, "no current device");
    std::lock_guard<std::mutex> lk(g_stage_mu);
    if (!on) {
        g_stage_ptr[dev] = nullptr;
        return STF_OK;
    }
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(g_stage_count));
    if (e == hipSuccess) e = hipMemset(p, 0, sizeof(g_stage_count));
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) return stf_fail(STF_E_DEVICE, "staging counters: %s", hipGetErrorString(e));
    g_stage_ptr[dev] = (unsigned long long*)p;
    return STF_OK;
}

stf_status stf_stage_counts(uint64_t* staged_blocks, uint64_t* blocks)
{
    stf_clear_error();
    if (!staged_blocks || !blocks) return stf_fail(STF_E_INVALID, "NULL argument");
    void* p = nullptr;
    unsigned long long h[2] = {0, 0};
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(g_stage_count));
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipMemcpy(h, p, sizeof h, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return stf_fail(STF_E_DEVICE, "staging counters: %s", hipGetErrorString(e));
    *staged_blocks = h[0];
    *blocks = h[1];
    return STF_OK;
}

stf_status stf_create_texture2d(int32_t width, int32_t height, int32_t channels, stf_format fmt, int32_t levels,
                                const void* const* level_texels_host, stf_texture** out)
{
    stf_clear_error();
    if (!out) return stf_fail(STF_E_INVALID, "out is NULL");
    *out = nullptr;
    if (channels < 1 || channels > 4) return stf_fail(STF_E_INVALID, "channels = %d out of range (1..4)", channels);
    if (!valid_format(fmt)) return stf_fail(STF_E_INVALID, "unknown format %d", (int)fmt);
    if (width <= 0 || height <= 0 || width > 65536 || height > 65536)
        return stf_fail(STF_E_INVALID, "texture size %dx%d out of range (1..65536)", width, height);
    if (levels < 1 || levels > STF_MAX_LEVELS)
        return stf_fail(STF_E_INVALID, "levels = %d out of range (1..%d)", levels, STF_MAX_LEVELS);
    if (!level_texels_host) return stf_fail(STF_E_INVALID, "level_texels_host is NULL");
    stf_texture* t = new (std::nothrow) stf_texture();
    if (!t) return stf_fail(STF_E_OOM, "host allocation failed");
    t->kind = STF_KIND_TEX2D;
    t->fmt = fmt;
    t->channels = channels;
    (void)hipGetDevice(&t->device);
    stf_status s = create_levels(t, width, height, levels, level_texels_host,
                                 (size_t)channels * stf::fmt_bytes(fmt));
    if (s != STF_OK) {
        free_texture(t);
        return s;
    }
    *out = t;
    return STF_OK;
}

stf_status stf_create_material2d(int32_t width, int32_t height, int32_t levels, const void* const* level_texels_host,
                                 stf_texture** out)
{
    stf_clear_error();
    if (!out) return stf_fail(STF_E_INVALID, "out is NULL");
    *out = nullptr;
    if (width <= 0 || height <= 0 || width > 65536 || height > 65536)
        return stf_fail(STF_E_INVALID, "texture size %dx%d out of range (1..65536)", width, height);
    if (levels < 1 || levels > STF_MAX_LEVELS)
        return stf_fail(STF_E_INVALID, "levels = %d out of range (1..%d)", levels, STF_MAX_LEVELS);
    if (!level_texels_host) return stf_fail(STF_E_INVALID, "level_texels_host is NULL");
    stf_texture* t = new (std::nothrow) stf_texture();
    if (!t) return stf_fail(STF_E_OOM, "host allocation failed");
    t->kind = STF_KIND_MATERIAL;
    t->fmt = -1;
    t->channels = 6;   // filtered as albedo RGB, roughness, normal x, y
    (void)hipGetDevice(&t->device);
    // each level re-laid out in 4x4-texel tiles (material_index), padded
    // with zero texels to whole tiles
    t->levels = levels;
    t->bytes = 0;
    for (int l = 0; l < levels; ++l) {
        const int32_t w = std::max(width >> l, 1), h = std::max(height >> l, 1);
        if (!level_texels_host[l]) {
            free_texture(t);
            return stf_fail(STF_E_INVALID, "level %d texels are NULL", l);
        }
        const size_t tiles = (size_t)((w + 3) / 4) * (size_t)((h + 3) / 4);
        std::vector<uint64_t> tiled;
        try {
            tiled.assign(tiles * 16, 0);
        } catch (const std::bad_alloc&) {
            free_texture(t);
            return stf_fail(STF_E_OOM, "host allocation of %zu bytes failed", tiles * 128);
        }
        const uint64_t* src = static_cast<const uint64_t*>(level_texels_host[l]);
        for (int32_t y = 0; y < h; ++y)
            for (int32_t x = 0; x < w; ++x) tiled[(size_t)material_index(x, y, w)] = src[(size_t)y * w + x];
        stf_status s = upload(&t->level_alloc[l], tiled.data(), tiles * 128, "material level");
        if (s != STF_OK) {
            free_texture(t);
            return s;
        }
        t->level[l].texels = t->level_alloc[l];
        t->level[l].w = w;
        t->level[l].h = h;
        t->bytes += (int64_t)(tiles * 128);
    }
    *out = t;
    return STF_OK;
}

stf_status stf_create_sparse_grid3d(int32_t dim_x, int32_t dim_y, int32_t dim_z, stf_format fmt, int64_t n_leaves,
                                    const int32_t* leaf_origins_host, const void* leaf_values_host, float background,
                                    stf_texture** out)
{
    stf_clear_error();
    if (!out) return stf_fail(STF_E_INVALID, "out is NULL");
    *out = nullptr;
    const int32_t dims[3] = {dim_x, dim_y, dim_z};
    for (int a = 0; a < 3; ++a)
        if (dims[a] < 1 || dims[a] > 32768)
            return stf_fail(STF_E_INVALID, "grid dimension %d = %d out of range (1..32768)", a, dims[a]);
    if (!valid_format(fmt)) return stf_fail(STF_E_INVALID, "unknown format %d", (int)fmt);
    if (n_leaves < 0 || n_leaves > 0x7fffffff) return stf_fail(STF_E_INVALID, "n_leaves = %lld", (long long)n_leaves);
    if (n_leaves > 0 && (!leaf_origins_host || !leaf_values_host))
        return stf_fail(STF_E_INVALID, "leaf arrays are NULL");

    // Host build of the index: root slots of 128^3 voxels, each pointing to an
    // internal node of 16^3 child slots of 8^3 voxels, each holding a leaf id.
    int32_t r[3];
    for (int a = 0; a < 3; ++a) r[a] = (dims[a] + 127) >> 7;
    std::vector<int32_t> root((size_t)r[0] * r[1] * r[2], -1);
    std::vector<int32_t> nodes;
    for (int64_t k = 0; k < n_leaves; ++k) {
        const int32_t* o = leaf_origins_host + 3 * k;
        for (int a = 0; a < 3; ++a)
            if (o[a] < 0 || o[a] >= dims[a] || (o[a] & 7))
                return stf_fail(STF_E_INVALID, "leaf %lld origin (%d,%d,%d) is not a multiple of 8 inside the domain",
                                (long long)k, o[0], o[1], o[2]);
        size_t rs = ((size_t)(o[2] >> 7) * r[1] + (o[1] >> 7)) * r[0] + (o[0] >> 7);
        if (root[rs] < 0) {
            root[rs] = (int32_t)(nodes.size() / 4096);
            nodes.resize(nodes.size() + 4096, -1);
        }
        size_t cs = (size_t)root[rs] * 4096 + (((o[2] >> 3) & 15) * 16 + ((o[1] >> 3) & 15)) * 16 + ((o[0] >> 3) & 15);
        if (nodes[cs] >= 0)
            return stf_fail(STF_E_INVALID, "leaf %lld duplicates leaf %d at (%d,%d,%d)", (long long)k, nodes[cs], o[0],
                            o[1], o[2]);
        nodes[cs] = (int32_t)k;
    }

    // the kernels address the node table and the leaf values with 32-bit byte offsets
    if (nodes.size() * 4 >= ((size_t)1 << 32))
        return stf_fail(STF_E_UNSUPPORTED, "grid needs %zu internal nodes; at most 262143 are supported",
                        nodes.size() / 4096);
    if ((size_t)n_leaves * 512 * stf::fmt_bytes(fmt) >= ((size_t)1 << 32))
        return stf_fail(STF_E_UNSUPPORTED, "leaf values exceed 4 GiB (%lld leaves)", (long long)n_leaves);
    stf_texture* t = new (std::nothrow) stf_texture();
    if (!t) return stf_fail(STF_E_OOM, "host allocation failed");
    t->kind = STF_KIND_GRID3D;
    t->fmt = fmt;
    t->channels = 1;
    (void)hipGetDevice(&t->device);
    size_t leaf_bytes = (size_t)n_leaves * 512 * stf::fmt_bytes(fmt);
    stf_status s = upload(&t->grid_alloc[0], root.data(), root.size() * 4, "grid root");
    if (s == STF_OK) s = upload(&t->grid_alloc[1], nodes.empty() ? nullptr : nodes.data(), nodes.size() * 4, "grid nodes");
    if (s == STF_OK && n_leaves) {
        // each leaf's values from x-fastest order into its bricks (leaf_offset)
        const int tb = stf::fmt_bytes(fmt);
        std::vector<uint8_t> bricked;
        try {
            bricked.resize(leaf_bytes);
        } catch (const std::bad_alloc&) {
            free_texture(t);
            return stf_fail(STF_E_OOM, "host allocation of %zu bytes failed", leaf_bytes);
        }
        uint32_t where[512];
        for (uint32_t v = 0; v < 512; ++v) where[v] = stf::leaf_offset(fmt, v & 7u, (v >> 3) & 7u, v >> 6);
        const uint8_t* src = static_cast<const uint8_t*>(leaf_values_host);
        for (int64_t k = 0; k < n_leaves; ++k) {
            const uint8_t* ls = src + (size_t)k * 512 * tb;
            uint8_t* ld = bricked.data() + (size_t)k * 512 * tb;
            for (uint32_t v = 0; v < 512; ++v) memcpy(ld + (size_t)where[v] * tb, ls + (size_t)v * tb, tb);
        }
        s = upload(&t->grid_alloc[2], bricked.data(), leaf_bytes, "grid leaves");
    } else if (s == STF_OK) {
        s = upload(&t->grid_alloc[2], nullptr, 0, "grid leaves");
    }
    if (s != STF_OK) {
        free_texture(t);
        return s;
    }
    t->grid.root = (const int32_t*)t->grid_alloc[0];
    t->grid.nodes = (const int32_t*)t->grid_alloc[1];
    t->grid.leaves = t->grid_alloc[2];
    t->grid.dx = dim_x;
    t->grid.dy = dim_y;
    t->grid.dz = dim_z;
    t->grid.rx = r[0];
    t->grid.ry = r[1];
    t->grid.background = background;
    t->rz = r[2];
    t->n_leaves = n_leaves;
    t->n_nodes = (int32_t)(nodes.size() / 4096);
    t->bytes = (int64_t)(root.size() * 4 + nodes.size() * 4 + leaf_bytes);
    *out = t;
    return STF_OK;
}

void stf_destroy(stf_texture* tex)
{
    free_texture(tex);
}

stf_status stf_texture_bytes(const stf_texture* tex, int64_t* bytes)
{
    stf_clear_error();
    if (!tex || !bytes) return stf_fail(STF_E_INVALID, "NULL argument");
    *bytes = tex->bytes;
    return STF_OK;
}

stf_status stf_filter(const stf_texture* tex, const float* queries_dev, int64_t n, stf_filter_kind filter,
                      stf_mode mode, uint64_t seed, float* out_dev, int32_t* out_index_dev, uint32_t flags,
                      void* hip_stream)
{
    stf_clear_error();
    if (!tex) return stf_fail(STF_E_INVALID, "texture is NULL");
    if (!is_2d_filterable(tex) && tex->kind != STF_KIND_GRID3D)
        return stf_fail(STF_E_INVALID, "stf_filter needs a 2D texture or a 3D grid");
    if (n < 0 || n > MAX_QUERIES) return stf_fail(STF_E_INVALID, "n = %lld out of range (0..2^31-1)", (long long)n);
    if (!valid_filter(filter)) return stf_fail(STF_E_INVALID, "unknown filter %d", (int)filter);
    if (!valid_mode(filter, mode)) return stf_fail(STF_E_INVALID, "mode %d is not available for filter %d", (int)mode, (int)filter);
    if (flags != 0) return stf_fail(STF_E_INVALID, "unknown flags 0x%x", flags);
    if (mode == STF_DETERMINISTIC && out_index_dev)
        return stf_fail(STF_E_INVALID, "out_index_dev must be NULL in deterministic mode");
    if (n == 0) return STF_OK;
    bool is2d = is_2d_filterable(tex);
    stf_status s = check_device_ptr(queries_dev, "queries_dev", is2d ? 8 : 4);
    if (s == STF_OK) s = check_device_ptr(out_dev, "out_dev", 4);
    if (s == STF_OK && out_index_dev) s = check_device_ptr(out_index_dev, "out_index_dev", 4);
    if (s != STF_OK) return s;
    uint32_t key = stf::seed_key(seed);
    hipStream_t st = (hipStream_t)hip_stream;
    hipError_t e = is2d ? launch_filter2d(tex, queries_dev, (int32_t)n, filter, mode, key, out_dev, out_index_dev,
                                          nullptr, 0, st)
                        : launch_filter3d(tex, queries_dev, (int32_t)n, filter, mode, key, out_dev, out_index_dev,
                                          nullptr, 0, st);
    if (e != hipSuccess) return stf_fail(STF_E_DEVICE, "kernel launch failed: %s", hipGetErrorString(e));
    return STF_OK;
}

stf_status stf_filter_gaussian(const stf_texture* tex, const float* queries_dev, int64_t n, float sigma,
                               stf_gauss_mode mode, uint64_t seed, float* out_dev, int32_t* out_index_dev,
                               void* hip_stream)
{
    stf_clear_error();
    if (!tex) return stf_fail(STF_E_INVALID, "texture is NULL");
    if (!is_2d_filterable(tex)) return stf_fail(STF_E_INVALID, "stf_filter_gaussian needs a 2D texture");
    if (n < 0 || n > MAX_QUERIES) return stf_fail(STF_E_INVALID, "n = %lld out of range", (long long)n);
    if (!(sigma > 0.0f && sigma <= 16.0f)) return stf_fail(STF_E_INVALID, "sigma = %g out of range (0, 16]", (double)sigma);
    if (mode < STF_GAUSS_FIS || mode > STF_GAUSS_DISCRETE_MEAN) return stf_fail(STF_E_INVALID, "unknown mode %d", (int)mode);
    if (mode == STF_GAUSS_FIS_MEAN && sigma > 4.0f)
        return stf_fail(STF_E_UNSUPPORTED, "STF_GAUSS_FIS_MEAN supports sigma <= 4 (window of 52 taps per axis)");
    if (out_index_dev && (mode == STF_GAUSS_FIS_MEAN || mode == STF_GAUSS_DISCRETE_MEAN))
        return stf_fail(STF_E_INVALID, "out_index_dev must be NULL in the deterministic modes");
    if (n == 0) return STF_OK;
    stf_status s = check_device_ptr(queries_dev, "queries_dev", 8);
    if (s == STF_OK) s = check_device_ptr(out_dev, "out_dev", 4);
    if (s == STF_OK && out_index_dev) s = check_device_ptr(out_index_dev, "out_index_dev", 4);
    if (s != STF_OK) return s;
    hipError_t e = launch_gauss2d(tex, queries_dev, (int32_t)n, sigma, (int)mode, stf::seed_key(seed), out_dev,
                                  out_index_dev, (hipStream_t)hip_stream);
    if (e != hipSuccess) return stf_fail(STF_E_DEVICE, "kernel launch failed: %s", hipGetErrorString(e));
    return STF_OK;
}

stf_status stf_filter_moments(const stf_texture* tex, const float* queries_dev, int64_t n, stf_filter_kind filter,
                              uint64_t seed_base, int32_t n_seeds, double* sum_dev, double* sumsq_dev,
                              void* hip_stream)
{
    stf_clear_error();
    if (!tex) return stf_fail(STF_E_INVALID, "texture is NULL");
    if (!is_2d_filterable(tex) && tex->kind != STF_KIND_GRID3D)
        return stf_fail(STF_E_INVALID, "stf_filter_moments needs a 2D texture or a 3D grid");
    if (n < 0 || n > MAX_QUERIES) return stf_fail(STF_E_INVALID, "n = %lld out of range", (long long)n);
    if (n_seeds < 1) return stf_fail(STF_E_INVALID, "n_seeds = %d must be >= 1", n_seeds);
    if (!valid_filter(filter)) return stf_fail(STF_E_INVALID, "unknown filter %d", (int)filter);
    if (n == 0) return STF_OK;
    bool is2d = is_2d_filterable(tex);
    stf_status s = check_device_ptr(queries_dev, "queries_dev", is2d ? 8 : 4);
    if (s == STF_OK) s = check_device_ptr(sum_dev, "sum_dev", 8);
    if (s == STF_OK) s = check_device_ptr(sumsq_dev, "sumsq_dev", 8);
    if (s != STF_OK) return s;
    hipStream_t st = (hipStream_t)hip_stream;
    hipError_t e = is2d ? launch_moments2d(tex, queries_dev, (int32_t)n, filter, seed_base, n_seeds, sum_dev, sumsq_dev, st)
                        : launch_moments3d(tex, queries_dev, (int32_t)n, filter, seed_base, n_seeds, sum_dev, sumsq_dev, st);
    if (e != hipSuccess) return stf_fail(STF_E_DEVICE, "kernel launch failed: %s", hipGetErrorString(e));
    return STF_OK;
}

stf_status stf_shade_filter(const stf_texture* material, const float* shade_queries_dev, int64_t n,
                            stf_filter_kind filter, stf_shade_mode mode, uint64_t seed, float* out_rgb_dev,
                            int32_t* out_index_dev, void* hip_stream)
{
    stf_clear_error();
    if (!material || material->kind != STF_KIND_MATERIAL)
        return stf_fail(STF_E_INVALID, "stf_shade_filter needs a material texture");
    if (n < 0 || n > MAX_QUERIES) return stf_fail(STF_E_INVALID, "n = %lld out of range", (long long)n);
    if (!valid_filter(filter)) return stf_fail(STF_E_INVALID, "unknown filter %d", (int)filter);
    if (filter != STF_LINEAR && filter != STF_CUBIC_BSPLINE)
        return stf_fail(STF_E_UNSUPPORTED, "shading supports the linear and B-spline filters only");
    if (mode != STF_SHADE_AFTER_FILTER && mode != STF_FILTER_AFTER_SHADE && mode != STF_SHADE_STOCHASTIC)
        return stf_fail(STF_E_INVALID, "unknown shade mode %d", (int)mode);
    if (mode != STF_SHADE_STOCHASTIC && out_index_dev)
        return stf_fail(STF_E_INVALID, "out_index_dev must be NULL unless the mode is stochastic");
    if (n == 0) return STF_OK;
    stf_status s = check_device_ptr(shade_queries_dev, "shade_queries_dev", 4);
    if (s == STF_OK) s = check_device_ptr(out_rgb_dev, "out_rgb_dev", 4);
    if (s == STF_OK && out_index_dev) s = check_device_ptr(out_index_dev, "out_index_dev", 4);
    if (s != STF_OK) return s;
    hipError_t e = launch_shade(material, shade_queries_dev, (int32_t)n, filter, mode, stf::seed_key(seed), out_rgb_dev,
                                out_index_dev, (hipStream_t)hip_stream);
    if (e != hipSuccess) return stf_fail(STF_E_DEVICE, "kernel launch failed: %s", hipGetErrorString(e));
    return STF_OK;
}

}  // extern "C"
