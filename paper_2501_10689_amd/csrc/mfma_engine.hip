// MFMA engine (complex64, 16 right-hand sides per workgroup).
#include <hip/hip_runtime.h>

#include "device_common.h"
#include "kernels.h"

int vrk_mfma_supported(int32_t, int32_t) { return 0; }
size_t vrk_mfma_lds_bytes(int32_t, int32_t) { return 0; }
hipError_t vrk_launch_mfma_solve(const VrkSolveArgs &, const VrkWork *, int32_t, int32_t, int32_t,
                                 size_t, hipStream_t)
{
    return hipErrorNotSupported;
}
