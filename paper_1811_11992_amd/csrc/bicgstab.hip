// Right-preconditioned BiCGSTAB with block ILU(0) on the decoupled system:
// van der Vorst's stabilised bi-conjugate gradients, the Krylov method of the
// paper's experiments (Section 4, there with RAS or CPR-PF preconditioning).
// The host drives the iteration.  Each iteration applies A M^-1 twice through
// the fused sweep + SpMV of the GMRES path; the vector updates are fused with
// the inner products the next step needs, and every reduction runs in a
// fixed order (block partials, then one block per product).
#include <cmath>

#include "common.h"

hipError_t isc_launch_bilu0_apply_spmv(isc_ctx*, const double*, const double*, const double*, double*, double*);
hipError_t isc_launch_spmv(isc_ctx*, const double*, const double*, double*);
void isc_well_apply(isc_ctx*, const double* x, double* w);   // eliminated well rows (isc_newton_step only)
isc_status isc_bicgstab_run(isc_ctx*, const double* Jdec, const double* b, double* x, int32_t max_iters, double rtol,
                            isc_solve_info* info_h);

namespace isc {
namespace bcg {

constexpr int BCG_BLOCKS = 1024;   // blocks of the reducing kernels (at most NPART)
// |(r~, r)| <= BCG_BREAKDOWN ||r~|| ||r|| or |(r~, v)| <= BCG_BREAKDOWN ||r~|| ||v||
// is a breakdown; the solve restarts from its true residual at most
// BCG_MAX_BREAKDOWNS times
constexpr double BCG_BREAKDOWN = 1e-12;
constexpr int BCG_MAX_BREAKDOWNS = 8;
static_assert(BCG_BLOCKS <= NPART, "partial rows hold NPART entries");

__device__ __forceinline__ double bcg_wave_sum(double x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
    return x;
}

// Block sums of NQ per-thread values -> partial[q * BCG_BLOCKS + block].
template <int NQ>
__device__ __forceinline__ void bcg_store(const double (&a)[NQ], double* __restrict__ partial) {
    __shared__ double red[NQ][4];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const double s = bcg_wave_sum(a[q]);
        if (lane == 0) red[q][w] = s;
    }
    __syncthreads();
    if (threadIdx.x < NQ) {
        const int q = threadIdx.x;
        partial[(size_t)q * BCG_BLOCKS + blockIdx.x] = (red[q][0] + red[q][1]) + (red[q][2] + red[q][3]);
    }
}

#define BCG_LOOP(t) for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < len; t += (int64_t)gridDim.x * 256)

__global__ void __launch_bounds__(256) bcg_zero(int64_t len, double* __restrict__ x) {
    BCG_LOOP(t) x[t] = 0.0;
}

// (Re)start from the true residual: r = b - Ax, shadow r~ = r, p = v = 0; (r, r).
__global__ void __launch_bounds__(256) bcg_restart(int64_t len, const double* __restrict__ b,
                                                   const double* __restrict__ ax, double* __restrict__ r,
                                                   double* __restrict__ rs, double* __restrict__ p,
                                                   double* __restrict__ v, double* __restrict__ partial) {
    double a[1] = {0.0};
    BCG_LOOP(t) {
        const double rr = b[t] - ax[t];
        r[t] = rr;
        rs[t] = rr;
        p[t] = 0.0;
        v[t] = 0.0;
        a[0] += rr * rr;
    }
    bcg_store<1>(a, partial);
}

// p = r + beta (p - omega v)
__global__ void __launch_bounds__(256) bcg_p(int64_t len, const double* __restrict__ r, const double* __restrict__ v,
                                             double beta, double omega, double* __restrict__ p) {
    BCG_LOOP(t) p[t] = r[t] + beta * (p[t] - omega * v[t]);
}

// (a, b)
__global__ void __launch_bounds__(256) bcg_dot(int64_t len, const double* __restrict__ a_,
                                               const double* __restrict__ b_, double* __restrict__ partial) {
    double a[1] = {0.0};
    BCG_LOOP(t) a[0] += a_[t] * b_[t];
    bcg_store<1>(a, partial);
}

// (a, b) and (b, b)
__global__ void __launch_bounds__(256) bcg_dot2(int64_t len, const double* __restrict__ a_,
                                                const double* __restrict__ b_, double* __restrict__ partial) {
    double a[2] = {0.0, 0.0};
    BCG_LOOP(t) {
        const double bt = b_[t];
        a[0] += a_[t] * bt;
        a[1] += bt * bt;
    }
    bcg_store<2>(a, partial);
}

// s = r - alpha v, in place of r; (s, s)
__global__ void __launch_bounds__(256) bcg_s(int64_t len, double* __restrict__ rs_io, const double* __restrict__ v,
                                             double alpha, double* __restrict__ partial) {
    double a[1] = {0.0};
    BCG_LOOP(t) {
        const double s = rs_io[t] - alpha * v[t];
        rs_io[t] = s;
        a[0] += s * s;
    }
    bcg_store<1>(a, partial);
}

// x += alpha p^
__global__ void __launch_bounds__(256) bcg_x_half(int64_t len, double* __restrict__ x, const double* __restrict__ ph,
                                                  double alpha) {
    BCG_LOOP(t) x[t] += alpha * ph[t];
}

// (t, s) and (t, t)
__global__ void __launch_bounds__(256) bcg_ts(int64_t len, const double* __restrict__ tv, const double* __restrict__ s,
                                              double* __restrict__ partial) {
    double a[2] = {0.0, 0.0};
    BCG_LOOP(k) {
        const double tk = tv[k];
        a[0] += tk * s[k];
        a[1] += tk * tk;
    }
    bcg_store<2>(a, partial);
}

// x += alpha p^ + omega s^;  r = s - omega t, in place of s;  (r~, r) and (r, r)
__global__ void __launch_bounds__(256) bcg_xr(int64_t len, double* __restrict__ x, const double* __restrict__ ph,
                                              const double* __restrict__ sh, double alpha, double omega,
                                              double* __restrict__ sr_io, const double* __restrict__ tv,
                                              const double* __restrict__ rsh, double* __restrict__ partial) {
    double a[2] = {0.0, 0.0};
    BCG_LOOP(k) {
        x[k] += alpha * ph[k] + omega * sh[k];
        const double r = sr_io[k] - omega * tv[k];
        sr_io[k] = r;
        a[0] += rsh[k] * r;
        a[1] += r * r;
    }
    bcg_store<2>(a, partial);
}

// out[q] = sum of partial[q][0..nblk), in a fixed order; one block per q
__global__ void __launch_bounds__(256) bcg_reduce(const double* __restrict__ partial, int nblk,
                                                  double* __restrict__ out) {
    __shared__ double red[4];
    const int q = blockIdx.x;
    double s = 0.0;
    for (int b = threadIdx.x; b < nblk; b += 256) s += partial[(size_t)q * BCG_BLOCKS + b];
    s = bcg_wave_sum(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) out[q] = (red[0] + red[1]) + (red[2] + red[3]);
}

#undef BCG_LOOP

// Launch geometry and the host read of the reduced products.
struct Bcg {
    isc_ctx* ctx;
    int64_t len;
    int nb;
    double* partial;
    double* out;
    // reduce the first nq partial rows and copy them to h[0..nq)
    hipError_t read(int nq, double* h) {
        hipLaunchKernelGGL(bcg_reduce, dim3(nq), dim3(256), 0, ctx->stream, partial, nb, out);
        hipError_t e = hipGetLastError();   // this launch or an earlier one of the step
        if (e != hipSuccess) return e;
        e = hipMemcpyAsync(ctx->hscratch, out, (size_t)nq * sizeof(double), hipMemcpyDeviceToHost,
                                      ctx->stream);
        if (e != hipSuccess) return e;
        e = hipStreamSynchronize(ctx->stream);
        for (int q = 0; q < nq; ++q) h[q] = ctx->hscratch[q];
        return e;
    }
};

}  // namespace bcg
}  // namespace isc

isc_status isc_solve_bicgstab(isc_ctx* ctx, const double* Jdec, const double* b, double* x, int32_t max_iters,
                              double rtol, isc_solve_info* info_h) {
    if (!ctx) return ISC_ERR_ARG;
    if (!Jdec || !b || !x || x == b || max_iters < 1 || !(rtol > 0)) {
        ctx->err = "isc_solve_bicgstab: invalid argument (max_iters >= 1, rtol > 0, x distinct from b)";
        return ISC_ERR_ARG;
    }
    if (ctx->mmax < 6) {
        ctx->err = "isc_solve_bicgstab: uses seven of the context's Krylov vectors (max restart >= 6)";
        return ISC_ERR_ARG;
    }
    const isc_status fs = isc_bilu0(ctx, Jdec, ctx->Dinv);
    if (fs != ISC_OK) return fs;
    return isc_bicgstab_run(ctx, Jdec, b, x, max_iters, rtol, info_h);
}

// The iteration on a factor already in ctx->Dinv (isc_solve_bicgstab, and
// isc_newton_step with ISC_KRYLOV_BICGSTAB, where the operator also takes
// the eliminated well rows).
isc_status isc_bicgstab_run(isc_ctx* ctx, const double* Jdec, const double* b, double* x, int32_t max_iters,
                            double rtol, isc_solve_info* info_h) {
    using namespace isc;
    using namespace isc::bcg;
    const int64_t len = (int64_t)ctx->n * NU;
    const int64_t want = (len + 255) / 256;
    Bcg B{ctx, len, (int)(want < BCG_BLOCKS ? (want > 0 ? want : 1) : BCG_BLOCKS), ctx->partial, ctx->small + 3600};
    const dim3 grid(B.nb), blk(256);
    // r (also s), the shadow vector, p, v, t, p^, s^ in the context's Krylov basis
    double* r = ctx->V;
    double* rs = ctx->V + len;
    double* p = ctx->V + 2 * len;
    double* v = ctx->V + 3 * len;
    double* tv = ctx->V + 4 * len;
    double* ph = ctx->V + 5 * len;
    double* sh = ctx->V + 6 * len;

    isc_solve_info inf{};
    double h[2];
    hipLaunchKernelGGL(bcg_zero, grid, blk, 0, ctx->stream, len, x);
    hipLaunchKernelGGL(bcg_dot, grid, blk, 0, ctx->stream, len, b, b, B.partial);
    ISC_HIP(B.read(1, h));
    const double bnorm = std::sqrt(h[0]);
    if (bnorm == 0.0) {
        if (info_h) *info_h = inf;
        return ISC_OK;
    }
    if (!std::isfinite(bnorm)) {
        ctx->err = "isc_solve_bicgstab: right-hand side is not finite";
        return ISC_ERR_NONFINITE;
    }
    const double tol = rtol * bnorm;
    int32_t it = 0, starts = 0, breakdowns = 0;
    bool done = false;
    while (it < max_iters) {
        // (re)start from the true residual, the shadow vector r~ = r
        ISC_HIP(isc_launch_spmv(ctx, Jdec, x, tv));
        isc_well_apply(ctx, x, tv);
        hipLaunchKernelGGL(bcg_restart, grid, blk, 0, ctx->stream, len, b, tv, r, rs, p, v, B.partial);
        ISC_HIP(B.read(1, h));
        const double rn0 = std::sqrt(h[0]);
        inf.relres_true = rn0 / bnorm;
        if (rn0 <= tol) {
            done = true;
            break;
        }
        inf.restarts = starts++;
        double rho_old = 1.0, alpha = 1.0, omega = 1.0, rho = h[0];   // (r~, r) = (r, r) at a start
        double rn = rn0;                                                 // ||r||
        bool converged = false, breakdown = false;
        while (it < max_iters) {
            // breakdown: r~ (nearly) orthogonal to r, or to v below
            if (!(std::fabs(rho) > BCG_BREAKDOWN * rn0 * rn) || !std::isfinite(rho)) { breakdown = true; break; }
            const double beta = (rho / rho_old) * (alpha / omega);
            hipLaunchKernelGGL(bcg_p, grid, blk, 0, ctx->stream, len, r, v, beta, omega, p);
            int tk = isc_prof_begin(ctx, ISC_PROF_ILU_SPMV);
            ISC_HIP(isc_launch_bilu0_apply_spmv(ctx, Jdec, ctx->Dinv, p, ph, v));
            isc_prof_end(ctx, tk);
            isc_well_apply(ctx, ph, v);
            hipLaunchKernelGGL(bcg_dot2, grid, blk, 0, ctx->stream, len, rs, v, B.partial);
            ISC_HIP(B.read(2, h));
            const double rv = h[0];
            if (!(std::fabs(rv) > BCG_BREAKDOWN * rn0 * std::sqrt(h[1])) || !std::isfinite(rv)) {
                breakdown = true;
                break;
            }
            alpha = rho / rv;
            hipLaunchKernelGGL(bcg_s, grid, blk, 0, ctx->stream, len, r, v, alpha, B.partial);
            ISC_HIP(B.read(1, h));
            ++it;
            const double sn = std::sqrt(h[0]);
            inf.relres_est = sn / bnorm;
            if (sn <= tol) {
                hipLaunchKernelGGL(bcg_x_half, grid, blk, 0, ctx->stream, len, x, ph, alpha);
                converged = true;
                break;
            }
            tk = isc_prof_begin(ctx, ISC_PROF_ILU_SPMV);
            ISC_HIP(isc_launch_bilu0_apply_spmv(ctx, Jdec, ctx->Dinv, r, sh, tv));
            isc_prof_end(ctx, tk);
            isc_well_apply(ctx, sh, tv);
            hipLaunchKernelGGL(bcg_ts, grid, blk, 0, ctx->stream, len, tv, r, B.partial);
            ISC_HIP(B.read(2, h));
            const double tt = h[1];
            if (!(tt > 0.0) || !std::isfinite(tt)) {
                // s is the residual of x + alpha p^: keep that half step
                hipLaunchKernelGGL(bcg_x_half, grid, blk, 0, ctx->stream, len, x, ph, alpha);
                breakdown = true;
                break;
            }
            omega = h[0] / tt;
            hipLaunchKernelGGL(bcg_xr, grid, blk, 0, ctx->stream, len, x, ph, sh, alpha, omega, r, tv, rs,
                               B.partial);
            ISC_HIP(B.read(2, h));
            rn = std::sqrt(h[1]);
            inf.relres_est = rn / bnorm;
            if (rn <= tol) {
                converged = true;
                break;
            }
            if (omega == 0.0) { breakdown = true; break; }
            rho_old = rho;
            rho = h[0];
        }
        // a breakdown restarts from the true residual (a new shadow vector), a bounded number of times
        if (breakdown && ++breakdowns <= BCG_MAX_BREAKDOWNS) continue;
        if (!converged) break;
    }
    const isc_status sw = isc_check_sweeps(ctx);
    if (sw != ISC_OK) return sw;
    if (!done) {   // the true residual of the last iterate
        ISC_HIP(isc_launch_spmv(ctx, Jdec, x, tv));
        isc_well_apply(ctx, x, tv);
        hipLaunchKernelGGL(bcg_restart, grid, blk, 0, ctx->stream, len, b, tv, r, rs, p, v, B.partial);
        ISC_HIP(B.read(1, h));
        inf.relres_true = std::sqrt(h[0]) / bnorm;
        done = inf.relres_true <= rtol;
    }
    inf.iters = it;
    if (info_h) *info_h = inf;
    if (!done) {
        ctx->err = "isc_solve_bicgstab: no convergence (iterations exhausted or breakdown), relative residual " +
                   std::to_string(inf.relres_true);
        return ISC_ERR_LINEAR_NOCONV;
    }
    return ISC_OK;
}
