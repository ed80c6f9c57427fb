// shade.hip -- filter-after-shading kernels (placeholder until implemented).
#include "device_common.h"
#include "stf_internal.h"

hipError_t launch_shade(const stf_texture*, const float*, int32_t, int, int, uint32_t, float*, int32_t*, hipStream_t)
{
    return hipErrorNotSupported;
}
