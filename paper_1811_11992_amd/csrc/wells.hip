// Controlled wells in Newton's system: the rows of the bottom-hole pressure
// unknowns (well-modelling subsection of Section 2.2; the last row of the
// table of unknowns and equations) and their elimination.
//
// Newton's system with the well rows is bordered,
//     [J  B] [du  ]     [F]
//     [C  D] [dbhp] = - [R],
// with one row per controlled well: R = bhp - held BHP (D = 1, C = 0) under
// BHP control or at the limit, else R = q - target with q the rate it holds
// (D = dq/dbhp, C = dq/du at its perforated cells).  B has one column per
// well, nonzero in the rows of its perforated cells.  The wells are few and
// D is diagonal, so they are eliminated:
//     (J - B D^-1 C) du = -(F - B D^-1 R),   dbhp = -D^-1 (R + C du).
// After the decoupling (rows scaled by J_ii^-1) the reduced operator is
// J~ x - Bt D^-1 (C x), Bt = J_ii^-1 B: the sweeps and the sparse product
// work on J~ as before and one small launch per product adds the well term
// (one workgroup per well: a dot product over its perforations and an
// update of those rows).  The preconditioners see J~ alone.
#include "common.h"

namespace isc {

// sum over the 256 threads of a workgroup (every thread gets it)
__device__ __forceinline__ double wg_sum(double v, double* red) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    return (red[0] + red[1]) + (red[2] + red[3]);
}

// Each well's row: R and D, and the largest scaled |R| into *wres (rate
// rows by V phi rho_ref,W / dt of the first perforated cell, BHP rows by the
// pressure held, at least 1 Pa).  One workgroup of 256 for all wells.
__global__ void __launch_bounds__(256) well_reduce_kernel(int32_t ncw, CWell* cw, const double* __restrict__ cwp,
                                                         double dt, double* wres) {
    __shared__ double red[4];
    double mx = 0.0;
    for (int32_t w = 0; w < ncw; ++w) {
        CWell& W = cw[w];
        double R, D, scale;
        if (W.control == ISC_CTRL_BHP || W.on_limit) {
            const double held = W.control == ISC_CTRL_BHP ? W.target : W.limit;
            R = W.bhp - held;
            D = 1.0;
            scale = fmax(fabs(held), 1.0);
        } else {
            double q = 0.0, dq = 0.0;
            for (int k = threadIdx.x; k < W.np; k += 256) {
                q += cwp[(size_t)(W.c0 + k) * CWP_W + CWP_Q];
                dq += cwp[(size_t)(W.c0 + k) * CWP_W + CWP_DQ];
            }
            q = wg_sum(q, red);
            dq = wg_sum(dq, red);
            R = q - W.target;
            D = dq;
            scale = W.rscale / dt;
        }
        if (threadIdx.x == 0) {
            W.R = R;
            W.D = D;
            const double v = fabs(R) / scale;
            if (!(v <= mx)) mx = v;   // NaN propagates
        }
    }
    if (threadIdx.x == 0) *wres = mx;
}

// rhs += Bt R / D at the perforated cells (rhs = -F~ on entry)
__global__ void __launch_bounds__(256) well_rhs_kernel(int32_t ncp, const int32_t* __restrict__ pcell,
                                                      const int32_t* __restrict__ pwell,
                                                      const CWell* __restrict__ cw, const double* __restrict__ cwp,
                                                      double* __restrict__ rhs) {
    const int32_t t = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
    const int32_t p = t >> 3, e = t & 7;
    if (p >= ncp) return;
    const CWell& W = cw[pwell[p]];
    rhs[(size_t)pcell[p] * 8 + e] += cwp[(size_t)p * CWP_W + CWP_BT + e] * (W.R / W.D);
}

// w -= Bt D^-1 (C x) for the wells on a rate (one workgroup per well)
__global__ void __launch_bounds__(256) well_apply_kernel(const CWell* __restrict__ cw,
                                                        const int32_t* __restrict__ pcell,
                                                        const double* __restrict__ cwp, const double* __restrict__ x,
                                                        double* __restrict__ w) {
    __shared__ double red[4];
    const CWell& W = cw[blockIdx.x];
    if (W.control == ISC_CTRL_BHP || W.on_limit) return;
    const int32_t len = W.np * 8;
    double s = 0.0;
    for (int32_t t = threadIdx.x; t < len; t += 256) {
        const int32_t k = t >> 3, v = t & 7;
        s += cwp[(size_t)(W.c0 + k) * CWP_W + CWP_C + v] * x[(size_t)pcell[W.c0 + k] * 8 + v];
    }
    s = wg_sum(s, red) / W.D;
    for (int32_t t = threadIdx.x; t < len; t += 256) {
        const int32_t k = t >> 3, e = t & 7;
        w[(size_t)pcell[W.c0 + k] * 8 + e] -= cwp[(size_t)(W.c0 + k) * CWP_W + CWP_BT + e] * s;
    }
}

// bhp += dbhp = -(R + C du) / D (one workgroup of 256 for all wells)
__global__ void __launch_bounds__(256) well_update_kernel(int32_t ncw, CWell* cw, const int32_t* __restrict__ pcell,
                                                         const double* __restrict__ cwp,
                                                         const double* __restrict__ du, int32_t* nonfinite) {
    __shared__ double red[4];
    for (int32_t w = 0; w < ncw; ++w) {
        CWell& W = cw[w];
        double s = 0.0;
        if (!(W.control == ISC_CTRL_BHP || W.on_limit)) {
            const int32_t len = W.np * 8;
            for (int32_t t = threadIdx.x; t < len; t += 256) {
                const int32_t k = t >> 3, v = t & 7;
                s += cwp[(size_t)(W.c0 + k) * CWP_W + CWP_C + v] * du[(size_t)pcell[W.c0 + k] * 8 + v];
            }
            s = wg_sum(s, red);
        }
        if (threadIdx.x == 0) {
            W.bhp -= (W.R + s) / W.D;
            if (!isfinite(W.bhp)) *nonfinite = 1;
        }
    }
}

}  // namespace isc

hipError_t isc_launch_well_reduce(isc_ctx* ctx, double dt) {
    if (ctx->ncw == 0) return hipSuccess;
    hipLaunchKernelGGL(isc::well_reduce_kernel, dim3(1), dim3(256), 0, ctx->stream, ctx->ncw, ctx->cw, ctx->cwp, dt,
                       ctx->wres);
    return hipGetLastError();
}

hipError_t isc_launch_well_rhs(isc_ctx* ctx, double* rhs) {
    if (ctx->ncp == 0) return hipSuccess;
    const int blocks = (int)(((int64_t)ctx->ncp * 8 + 255) / 256);
    hipLaunchKernelGGL(isc::well_rhs_kernel, dim3(blocks), dim3(256), 0, ctx->stream, ctx->ncp, ctx->cwp_cell,
                       ctx->cwp_well, ctx->cw, ctx->cwp, rhs);
    return hipGetLastError();
}

// The well term of the Krylov operator, while isc_newton_step has set the
// border; a no-op otherwise.
void isc_well_apply(isc_ctx* ctx, const double* x, double* w) {
    if (!ctx->border || ctx->ncw == 0) return;
    hipLaunchKernelGGL(isc::well_apply_kernel, dim3(ctx->ncw), dim3(256), 0, ctx->stream, ctx->cw, ctx->cwp_cell,
                       ctx->cwp, x, w);
}

hipError_t isc_launch_well_update(isc_ctx* ctx, const double* du, int32_t* nonfinite_dev) {
    if (ctx->ncw == 0) return hipSuccess;
    hipLaunchKernelGGL(isc::well_update_kernel, dim3(1), dim3(256), 0, ctx->stream, ctx->ncw, ctx->cw,
                       ctx->cwp_cell, ctx->cwp, du, nonfinite_dev);
    return hipGetLastError();
}
