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
// B D^-1 C couples every pair of one well's perforated cells.  The pairs
// that the 7-point pattern holds (a cell with itself and with its stencil
// neighbours along the well) are folded into J before the decoupling, so
// that the preconditioners see them; the rest stays matrix-free.  With J'
// the folded matrix and the rows scaled by J'_ii^-1, the reduced operator
// is J~ x - Bt D^-1 (C x)|off-pattern, Bt = J'_ii^-1 B: the sweeps and the
// sparse product work on J~ and one small launch per product adds the
// well term (one workgroup per well: the products C_l x_l of its
// perforations, their sum, and for each perforated row the sum less its
// in-pattern partners).
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

// J'_kl = J_kl - B_k C_l / D for the in-pattern pairs (k, l) of the wells on
// a rate (B D^-1 C vanishes for a well held at a BHP: C = 0).  One thread
// per entry of a pair's 8x8 block; each ordered pair owns its block.
__global__ void __launch_bounds__(256) well_fold_kernel(int32_t ncp, const int32_t* __restrict__ pwell,
                                                       const int32_t* __restrict__ nb, const CWell* __restrict__ cw,
                                                       const double* __restrict__ cwp, double* __restrict__ J) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int32_t p = (int32_t)(t / (CW_NB * 64));
    if (p >= ncp) return;
    const int32_t slot = (int32_t)((t >> 6) % CW_NB), e = (int32_t)((t >> 3) & 7), v = (int32_t)(t & 7);
    const int32_t l = nb[((size_t)p * CW_NB + slot) * 2], b = nb[((size_t)p * CW_NB + slot) * 2 + 1];
    const CWell& W = cw[pwell[p]];
    if (l < 0 || W.control == ISC_CTRL_BHP || W.on_limit) return;
    J[(size_t)b * 64 + e * 8 + v] -= cwp[(size_t)p * CWP_W + CWP_B + e] * cwp[(size_t)l * CWP_W + CWP_C + v] / W.D;
}

// Bt = J'_ii^-1 B per perforation, by Gauss-Jordan elimination with partial
// pivoting of [J'_ii | B] in LDS (eight lanes load a perforation's tile,
// one eliminates).  A singular block is left to the decoupling to report.
__global__ void __launch_bounds__(256) well_bt_kernel(int32_t ncp, const int32_t* __restrict__ pcell,
                                                     const int32_t* __restrict__ diag_pos,
                                                     const double* __restrict__ J, double* __restrict__ cwp) {
    __shared__ double tile[32][8][9];
    const int32_t p = (int32_t)((blockIdx.x * blockDim.x + threadIdx.x) >> 3);
    const int k = threadIdx.x & 7, gi = threadIdx.x >> 3;
    const bool live = p < ncp;
    if (live) {
        const double* Jd = J + (size_t)diag_pos[pcell[p]] * 64;
#pragma unroll
        for (int c = 0; c < 8; ++c) tile[gi][k][c] = Jd[k * 8 + c];
        tile[gi][k][8] = cwp[(size_t)p * CWP_W + CWP_B + k];
    }
    __syncthreads();
    if (!live || k != 0) return;
    double (*a)[9] = tile[gi];
    bool ok = true;
    for (int col = 0; col < 8 && ok; ++col) {
        int piv = col;
        for (int r = col + 1; r < 8; ++r)
            if (fabs(a[r][col]) > fabs(a[piv][col])) piv = r;
        if (!(fabs(a[piv][col]) > 0.0)) { ok = false; break; }
        if (piv != col)
            for (int c = 0; c < 9; ++c) { const double t = a[col][c]; a[col][c] = a[piv][c]; a[piv][c] = t; }
        const double d = a[col][col];
        for (int c = col; c < 9; ++c) a[col][c] /= d;
        for (int r = 0; r < 8; ++r) {
            if (r == col) continue;
            const double f = a[r][col];
            if (f == 0.0) continue;
            for (int c = col; c < 9; ++c) a[r][c] -= f * a[col][c];
        }
    }
    double* o = cwp + (size_t)p * CWP_W;
    for (int e = 0; e < 8; ++e) o[CWP_BT + e] = ok ? a[e][8] : 0.0;
}

// w -= Bt D^-1 (C x)|off-pattern for the wells on a rate (one workgroup per
// well; d holds C_l x_l per perforation, np doubles of dynamic LDS)
__global__ void __launch_bounds__(256) well_apply_kernel(const CWell* __restrict__ cw,
                                                        const int32_t* __restrict__ pcell,
                                                        const int32_t* __restrict__ nb,
                                                        const double* __restrict__ cwp, const double* __restrict__ x,
                                                        double* __restrict__ w) {
    extern __shared__ double d[];
    __shared__ double red[4];
    const CWell& W = cw[blockIdx.x];
    if (W.control == ISC_CTRL_BHP || W.on_limit) return;
    const int32_t len = W.np * 8;
    // eight lanes per perforation (len is a multiple of 8 and so is 256:
    // the eight lanes of a perforation enter and leave the loop together)
    for (int32_t t = threadIdx.x; t < len; t += 256) {
        const int32_t k = t >> 3, v = t & 7;
        double c = cwp[(size_t)(W.c0 + k) * CWP_W + CWP_C + v] * x[(size_t)pcell[W.c0 + k] * 8 + v];
        c += __shfl_xor(c, 1, 64);
        c += __shfl_xor(c, 2, 64);
        c += __shfl_xor(c, 4, 64);
        if (v == 0) d[k] = c;
    }
    __syncthreads();
    double s = 0.0;
    for (int32_t k = threadIdx.x; k < W.np; k += 256) s += d[k];
    s = wg_sum(s, red);
    for (int32_t t = threadIdx.x; t < len; t += 256) {
        const int32_t k = t >> 3, e = t & 7;
        const int32_t* nk = nb + (size_t)(W.c0 + k) * CW_NB * 2;
        double in = 0.0;
        for (int j = 0; j < CW_NB && nk[2 * j] >= 0; ++j) in += d[nk[2 * j] - W.c0];
        w[(size_t)pcell[W.c0 + k] * 8 + e] -= cwp[(size_t)(W.c0 + k) * CWP_W + CWP_BT + e] * ((s - in) / W.D);
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

// Fold the in-pattern couplings of B D^-1 C into J (before the decoupling)
// and form Bt from the folded diagonal blocks.
hipError_t isc_launch_well_fold(isc_ctx* ctx, double* J) {
    if (ctx->ncp == 0) return hipSuccess;
    const int64_t threads = (int64_t)ctx->ncp * isc::CW_NB * 64;
    hipLaunchKernelGGL(isc::well_fold_kernel, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, ctx->stream,
                       ctx->ncp, ctx->cwp_well, ctx->cwp_nb, ctx->cw, ctx->cwp, J);
    const int blocks = (int)(((int64_t)ctx->ncp * 8 + 255) / 256);
    hipLaunchKernelGGL(isc::well_bt_kernel, dim3(blocks), dim3(256), 0, ctx->stream, ctx->ncp, ctx->cwp_cell,
                       ctx->diag_pos, J, ctx->cwp);
    return hipGetLastError();
}

// The well term of the Krylov operator, while isc_newton_step has set the
// border; a no-op otherwise.
void isc_well_apply(isc_ctx* ctx, const double* x, double* w) {
    if (!ctx->border || ctx->ncw == 0) return;
    hipLaunchKernelGGL(isc::well_apply_kernel, dim3(ctx->ncw), dim3(256), (size_t)ctx->cw_maxnp * sizeof(double),
                       ctx->stream, ctx->cw, ctx->cwp_cell, ctx->cwp_nb, ctx->cwp, x, w);
}

hipError_t isc_launch_well_update(isc_ctx* ctx, const double* du, int32_t* nonfinite_dev) {
    if (ctx->ncw == 0) return hipSuccess;
    hipLaunchKernelGGL(isc::well_update_kernel, dim3(1), dim3(256), 0, ctx->stream, ctx->ncw, ctx->cw,
                       ctx->cwp_cell, ctx->cwp, du, nonfinite_dev);
    return hipGetLastError();
}
