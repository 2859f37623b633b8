// Precision form, set-up: the block ILU(0) factor of the decoupled matrix
// rounded to FP32 (computed in FP64 arithmetic from the FP32-rounded blocks,
// stored in FP32, with the sweeps' FP32 packs).  The FP32 copy of the matrix
// itself is made only for the per-hyperplane schedule, whose sweeps read it.
// The FP64 flexible GMRES that uses them is in krylov.hip.
#include "common.h"

hipError_t isc_launch_bilu0_factor32_from64(isc_ctx*, const double*, float*, float*, int32_t*);

// Launches only (no host synchronisation); a singular pivot block is reported
// through bad_dev like the FP64 factor.
isc_status isc_prepare_mixed_dev(isc_ctx* ctx, const double* A, int32_t* bad_dev) {
    if (!ctx->J32) {
        ctx->err = "mixed precision needs a context created with max inner_iters >= 1";
        return ISC_ERR_ARG;
    }
    ISC_HIP(isc_launch_bilu0_factor32_from64(ctx, A, ctx->J32, ctx->Dinv32, bad_dev));
    return ISC_OK;
}
