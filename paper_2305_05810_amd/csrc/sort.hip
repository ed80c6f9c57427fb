// sort.hip -- Morton ordering of query streams.
//
// Queries that land in the same region of a texture should run next to each
// other: neighbouring lanes then share leaves, tree nodes and cache lines.
// stf_sort_queries computes a Morton key per query -- the interleaved bits of
// its 8^3 leaf coordinates (3D grids) or 4x4 texel tile coordinates (2D
// textures and materials) -- radix-sorts (key, query id) pairs (rocPRIM),
// and gathers the queries in that order.  stf_filter_ordered then filters
// the sorted stream with each query's draw keyed by its original id, so its
// results are exactly those of stf_filter on the unsorted batch.
#include <rocprim/device/device_radix_sort.hpp>

#include "device_common.h"
#include "stf_internal.h"

using namespace stf;

namespace {

constexpr int BLOCK = 256;

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

__device__ __forceinline__ uint32_t clamp_cell(float x, int shift, uint32_t hi)
{
    float f = __builtin_floorf(fminf(fmaxf(x, -1.0f), 16777215.0f));
    int c = (int)f >> shift;
    return c < 0 ? 0u : ((uint32_t)c > hi ? hi : (uint32_t)c);
}

__global__ __launch_bounds__(BLOCK) void k_morton3d(const float* __restrict__ q, int32_t n, uint32_t* __restrict__ keys,
                                                    int32_t* __restrict__ ids)
{
    int32_t i = blockIdx.x * BLOCK + threadIdx.x;
    if (i >= n) return;
    float x = q[3 * (int64_t)i], y = q[3 * (int64_t)i + 1], z = q[3 * (int64_t)i + 2];
    uint32_t key = 0xffffffffu;   // non-finite queries go last
    if (x == x && y == y && z == z)
        key = spread3(clamp_cell(x, 3, 1023)) | (spread3(clamp_cell(y, 3, 1023)) << 1) |
              (spread3(clamp_cell(z, 3, 1023)) << 2);
    keys[i] = key;
    ids[i] = i;
}

__global__ __launch_bounds__(BLOCK) void k_morton2d(const float* __restrict__ q, int32_t n, float w, float h,
                                                    uint32_t* __restrict__ keys, int32_t* __restrict__ ids)
{
    int32_t i = blockIdx.x * BLOCK + threadIdx.x;
    if (i >= n) return;
    float2 uv = reinterpret_cast<const float2*>(q)[i];
    uint32_t key = 0xffffffffu;
    if (uv.x == uv.x && uv.y == uv.y)
        key = spread2(clamp_cell(uv.x * w - 0.5f, 2, 32767)) | (spread2(clamp_cell(uv.y * h - 0.5f, 2, 32767)) << 1);
    keys[i] = key;
    ids[i] = i;
}

template <int D>
__global__ __launch_bounds__(BLOCK) void k_gather(const float* __restrict__ q, const int32_t* __restrict__ order,
                                                  int32_t n, float* __restrict__ sorted)
{
    int32_t i = blockIdx.x * BLOCK + threadIdx.x;
    if (i >= n) return;
    int64_t src = order[i];
#pragma unroll
    for (int d = 0; d < D; ++d) sorted[(int64_t)D * i + d] = q[D * src + d];
}

size_t align256(size_t b)
{
    return (b + 255) & ~(size_t)255;
}

size_t rocprim_bytes(int64_t n)
{
    size_t b = 0;
    (void)rocprim::radix_sort_pairs(nullptr, b, (uint32_t*)nullptr, (uint32_t*)nullptr, (int32_t*)nullptr,
                                    (int32_t*)nullptr, (size_t)n, 0, 32);
    return b;
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

}  // namespace

extern "C" {

stf_status stf_sort_workspace_bytes(int64_t n, size_t* bytes)
{
    stf_clear_error();
    if (!bytes) return stf_fail(STF_E_INVALID, "bytes is NULL");
    if (n < 0 || n > 0x7fffffff) return stf_fail(STF_E_INVALID, "n = %lld out of range", (long long)n);
    *bytes = 3 * align256((size_t)n * 4) + align256(rocprim_bytes(n));
    return STF_OK;
}

stf_status stf_sort_queries(const stf_texture* tex, const float* queries_dev, int64_t n, float* sorted_queries_dev,
                            int32_t* order_dev, void* workspace_dev, size_t workspace_bytes, void* hip_stream)
{
    stf_clear_error();
    if (!tex) return stf_fail(STF_E_INVALID, "texture is NULL");
    if (n < 0 || n > 0x7fffffff) return stf_fail(STF_E_INVALID, "n = %lld out of range", (long long)n);
    if (n == 0) return STF_OK;
    size_t need;
    stf_sort_workspace_bytes(n, &need);
    if (workspace_bytes < need) return stf_fail(STF_E_INVALID, "workspace of %zu bytes < %zu needed", workspace_bytes, need);
    bool is3d = tex->kind == STF_KIND_GRID3D;
    int dims = is3d ? 3 : 2;
    stf_status s = check_ptr(queries_dev, "queries_dev", is3d ? 4 : 8);
    if (s == STF_OK) s = check_ptr(sorted_queries_dev, "sorted_queries_dev", is3d ? 4 : 8);
    if (s == STF_OK) s = check_ptr(order_dev, "order_dev", 4);
    if (s == STF_OK) s = check_ptr(workspace_dev, "workspace_dev", 256);
    if (s != STF_OK) return s;
    if (sorted_queries_dev == queries_dev) return stf_fail(STF_E_INVALID, "the sorted copy must not alias the queries");
    hipStream_t st = (hipStream_t)hip_stream;
    char* ws = (char*)workspace_dev;
    uint32_t* keys_in = (uint32_t*)ws;
    uint32_t* keys_out = (uint32_t*)(ws + align256((size_t)n * 4));
    int32_t* ids_in = (int32_t*)(ws + 2 * align256((size_t)n * 4));
    void* temp = ws + 3 * align256((size_t)n * 4);
    size_t temp_bytes = workspace_bytes - 3 * align256((size_t)n * 4);
    dim3 grid((unsigned)((n + BLOCK - 1) / BLOCK)), block(BLOCK);
    if (is3d) {
        hipLaunchKernelGGL(k_morton3d, grid, block, 0, st, queries_dev, (int32_t)n, keys_in, ids_in);
    } else {
        const TexLevel& L = tex->level[0];
        hipLaunchKernelGGL(k_morton2d, grid, block, 0, st, queries_dev, (int32_t)n, (float)L.w, (float)L.h, keys_in,
                           ids_in);
    }
    hipError_t e = hipGetLastError();
    if (e == hipSuccess)
        e = rocprim::radix_sort_pairs(temp, temp_bytes, keys_in, keys_out, ids_in, order_dev, (size_t)n, 0, 32, st);
    if (e == hipSuccess) {
        if (dims == 3)
            hipLaunchKernelGGL(k_gather<3>, grid, block, 0, st, queries_dev, order_dev, (int32_t)n, sorted_queries_dev);
        else
            hipLaunchKernelGGL(k_gather<2>, grid, block, 0, st, queries_dev, order_dev, (int32_t)n, sorted_queries_dev);
        e = hipGetLastError();
    }
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
