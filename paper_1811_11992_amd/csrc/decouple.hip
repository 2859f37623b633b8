// Gauss-Jordan decoupling (Section 3.2).  For every block row the augmented
// matrix [J_ii | J_i,neighbours | F_i] (8 x (8 nb + 1), nb <= 7 blocks) is
// reduced by Gauss-Jordan elimination with partial pivoting to
// [I | J_ii^-1 J_i,neighbours | J_ii^-1 F_i], i.e. C_L J and C_L F with
// C_L = blockdiag(J_ii^-1), without forming J_ii^-1.  Row exchanges are the
// paper's dynamic equation alignment.
//
// Mapping: one wavefront per block row; lane c holds augmented column c
// (8 values), so a row exchange is a register swap inside each lane and the
// pivot column is read from lane k into scalar registers.
#include "common.h"

namespace isc {

__global__ void __launch_bounds__(256) decouple_kernel(int32_t n, const int32_t* __restrict__ row_ptr,
                                                       const int32_t* __restrict__ diag_pos,
                                                       double* __restrict__ J, double* __restrict__ F,
                                                       int32_t* __restrict__ bad) {
    const int32_t i = (int32_t)(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    if (i >= n) return;
    const int32_t b0 = row_ptr[i];
    const int32_t nb = row_ptr[i + 1] - b0;
    const int32_t dp = diag_pos[i];
    const int ncolb = 8 * nb;
    const int slot = lane >> 3, cc = lane & 7;
    const bool is_blk = lane < ncolb;
    const bool is_rhs = lane == ncolb;
    int32_t blk = -1;
    if (is_blk) {
        if (slot == 0) {
            blk = dp;
        } else {
            const int32_t k = b0 + slot - 1;      // off-diagonal blocks in column order
            blk = k >= dp ? k + 1 : k;
        }
    }
    double a[8];
#pragma unroll
    for (int r = 0; r < 8; ++r)
        a[r] = is_blk ? J[(size_t)blk * BS + r * 8 + cc] : (is_rhs ? F[(size_t)i * NU + r] : 0.0);
    double cmax = 0.0;   // lanes 0..7: column maxima of J_ii
#pragma unroll
    for (int r = 0; r < 8; ++r) cmax = fmax(cmax, fabs(a[r]));
    bool singular = false;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        double col[8];
#pragma unroll
        for (int r = 0; r < 8; ++r) col[r] = read_lane(a[r], k);
        const double cm = read_lane(cmax, k);
        int piv = k;
        double best = fabs(col[k]);
#pragma unroll
        for (int r = k + 1; r < 8; ++r) {
            const double t = fabs(col[r]);
            if (t > best) { best = t; piv = r; }
        }
#pragma unroll
        for (int r = k + 1; r < 8; ++r) {
            if (r == piv) {
                const double t = a[k]; a[k] = a[r]; a[r] = t;
                const double tc = col[k]; col[k] = col[r]; col[r] = tc;
            }
        }
        const double pv = col[k];
        if (!(fabs(pv) > 1e-14 * cm) || !isfinite(pv)) { singular = true; break; }
        a[k] = a[k] / pv;
#pragma unroll
        for (int r = 0; r < 8; ++r)
            if (r != k) a[r] -= col[r] * a[k];
    }
    if (singular) {
        if (lane == 0) atomicMin(bad, i);
        return;
    }
    if (is_blk) {
#pragma unroll
        for (int r = 0; r < 8; ++r)
            J[(size_t)blk * BS + r * 8 + cc] = (slot == 0) ? (r == cc ? 1.0 : 0.0) : a[r];
    } else if (is_rhs) {
#pragma unroll
        for (int r = 0; r < 8; ++r) F[(size_t)i * NU + r] = a[r];
    }
}

__global__ void fill_i32_kernel(int32_t* p, int32_t v, int32_t cnt) {
    const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < cnt) p[t] = v;
}

}  // namespace isc

hipError_t isc_launch_decouple(isc_ctx* ctx, double* J, double* F, int32_t* bad_dev) {
    hipLaunchKernelGGL(isc::fill_i32_kernel, dim3(1), dim3(64), 0, ctx->stream, bad_dev, INT32_MAX, 1);
    const int blocks = (ctx->n + 3) / 4;
    hipLaunchKernelGGL(isc::decouple_kernel, dim3(blocks), dim3(256), 0, ctx->stream, ctx->n,
                       ctx->row_ptr, ctx->diag_pos, J, F, bad_dev);
    return hipGetLastError();
}
