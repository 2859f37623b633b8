// Precision form: FP32 preconditioner and inner SpMV inside FP64 FGMRES.
#include "common.h"

isc_status isc_prepare_mixed(isc_ctx* ctx, const double*) {
    ctx->err = "mixed precision solve not available in this build";
    return ISC_ERR_ARG;
}
isc_status isc_solve_mixed(isc_ctx* ctx, const double*, const double*, double*, const isc_solve_opts*,
                           isc_solve_info*) {
    ctx->err = "mixed precision solve not available in this build";
    return ISC_ERR_ARG;
}
