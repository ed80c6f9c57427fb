// Exhaustive error bounds of the hardware transcendental instructions the
// kernels take binary32 decisions with, each followed by a binary64 fallback
// inside a margin that these bounds must fit (checked by
// tests/test_gpu_hw_bounds.py):
//   - Gaussian filter importance sampling (Box-Muller): r = sqrt(-2 ln(1 - u))
//     by v_log_f32 and v_sqrt_f32, and sin, cos(2 pi u) by v_sin_f32 and
//     v_cos_f32 (angle in turns), over every uniform u = k 2^-24 the counter
//     hash can give;
//   - discrete 4x4 Gaussian sampling: 2^y by v_exp_f32, relative, over every
//     binary32 y in [-64, 0];
//   - the EWA level draw: log2 x by v_log_f32, absolute, over every binary32
//     x in [2^-32, 2^32].
// Each maximum is taken against the binary64 function and printed as
// "name value".  Test infrastructure only: the library does not use it.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

namespace {

__device__ void max_into(unsigned int* slot, double err)
{
    atomicMax(slot, __float_as_uint((float)fabs(err)));   // non-negative floats order as their bits
}

__global__ void k_box_muller(unsigned int* res)
{
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= (1u << 24)) return;
    const float u = (float)k * 0x1p-24f;
    const float r_hw = __builtin_amdgcn_sqrtf(-1.38629436112f * __builtin_amdgcn_logf(1.0f - u));
    const double r = sqrt(-2.0 * log(1.0 - (double)u));
    double s, c;
    sincos(6.283185307179586476925286766559 * (double)u, &s, &c);
    max_into(res + 0, (double)r_hw - r);
    max_into(res + 1, (double)__builtin_amdgcn_sinf(u) - s);
    max_into(res + 2, (double)__builtin_amdgcn_cosf(u) - c);
}

__global__ void k_exp2(unsigned int* res, uint32_t count)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const float y = __uint_as_float(0x80000000u + i);   // -0 .. -64
    const double ref = exp2((double)y);
    max_into(res + 3, ((double)__builtin_amdgcn_exp2f(y) - ref) / ref);
}

__global__ void k_log2(unsigned int* res, uint32_t first, uint32_t count)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const float x = __uint_as_float(first + i);   // 2^-32 .. 2^32
    max_into(res + 4, (double)__builtin_amdgcn_logf(x) - log2((double)x));
}

bool ok(hipError_t e, const char* what)
{
    if (e == hipSuccess) return true;
    fprintf(stderr, "%s: %s\n", what, hipGetErrorString(e));
    return false;
}

}  // namespace

int main()
{
    unsigned int* d = nullptr;
    if (!ok(hipMalloc(&d, 8 * sizeof(unsigned int)), "hipMalloc")) return 1;
    if (!ok(hipMemset(d, 0, 8 * sizeof(unsigned int)), "hipMemset")) return 1;
    hipLaunchKernelGGL(k_box_muller, dim3((1u << 24) / 256), dim3(256), 0, 0, d);
    const uint32_t n_exp = 0x42800000u + 1u;                 // bit patterns 0x80000000 .. 0xC2800000
    hipLaunchKernelGGL(k_exp2, dim3((n_exp + 255u) / 256u), dim3(256), 0, 0, d, n_exp);
    const uint32_t lo = 0x2F800000u, hi = 0x4F800000u;       // 2^-32 .. 2^32
    hipLaunchKernelGGL(k_log2, dim3((hi - lo + 1u + 255u) / 256u), dim3(256), 0, 0, d, lo, hi - lo + 1u);
    if (!ok(hipGetLastError(), "launch") || !ok(hipDeviceSynchronize(), "kernels")) return 1;
    unsigned int h[8];
    if (!ok(hipMemcpy(h, d, sizeof h, hipMemcpyDeviceToHost), "hipMemcpy")) return 1;
    const char* names[5] = {"box_muller_radius_abs", "sin_turns_abs", "cos_turns_abs", "exp2_rel_neg64_0",
                            "log2_abs_2m32_2p32"};
    for (int i = 0; i < 5; ++i) {
        float f;
        memcpy(&f, &h[i], sizeof f);
        printf("%s %.6e\n", names[i], (double)f);
    }
    (void)hipFree(d);
    return 0;
}
