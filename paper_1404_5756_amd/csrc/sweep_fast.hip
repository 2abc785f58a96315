// Tiled FP32 sweep kernels (placeholder until the tiled kernels land).
#include "rf3_internal.h"
#include "sweeps.h"

namespace rf {
hipError_t fast_rf3_f32(const float *, float *, const float4 *, const float4 *, const uint8_t *,
                        const LineGeom &, int, bool, hipStream_t)
{
    return hipErrorNotSupported;
}
}  // namespace rf
