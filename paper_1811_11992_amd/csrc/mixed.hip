// Precision form, set-up: FP32 copy of the decoupled matrix and its block
// ILU(0) factor (computed in FP64 arithmetic from the FP32 blocks, stored in
// FP32).  The FP64 flexible GMRES that uses them is in krylov.hip.
#include "common.h"

hipError_t isc_launch_bilu0_factor32(isc_ctx*, const float*, float*, int32_t*);

namespace isc {
__global__ void __launch_bounds__(256) to_f32(int64_t len, const double* __restrict__ a, float* __restrict__ b) {
    for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < len; t += (int64_t)gridDim.x * 256)
        b[t] = (float)a[t];
}
}  // namespace isc

// Launches only (no host synchronisation); a singular pivot block is reported
// through bad_dev like the FP64 factor.
isc_status isc_prepare_mixed_dev(isc_ctx* ctx, const double* A, int32_t* bad_dev) {
    if (!ctx->J32) {
        ctx->err = "mixed precision needs a context created with max inner_iters >= 1";
        return ISC_ERR_ARG;
    }
    const int64_t len = (int64_t)ctx->nnzb * isc::BS;
    hipLaunchKernelGGL(isc::to_f32, dim3(2048), dim3(256), 0, ctx->stream, len, A, ctx->J32);
    ISC_HIP(isc_launch_bilu0_factor32(ctx, ctx->J32, ctx->Dinv32, bad_dev));
    return ISC_OK;
}
