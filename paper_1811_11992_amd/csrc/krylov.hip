#include <cmath>
// Restarted GMRES with right preconditioning for the decoupled system.
//
// FP64 solver: classical Gram-Schmidt with one reorthogonalisation, the
// reorthogonalisation delayed by one iteration (DCGS2, after Swirydowicz,
// Langou, Ananthan, Yang and Thomas, "Low synchronization Gram-Schmidt and
// GMRES algorithms").  The Krylov vector of step j is formed from the lagged,
// once-projected vector u_j; the next iteration's single multi-dot pass gives
// both the reorthogonalisation coefficients of u_j and the projections of
// w = A M^-1 u_j, the Arnoldi relation corrects the Hessenberg column, and one
// fused pass writes q_j and u_{j+1}.  That is two passes over the basis per
// iteration instead of three, with CGS2's orthogonality.  The flexible outer
// solver of the precision form and its fixed-length FP32 inner solver use the
// same iteration.
// Reductions are two-stage with a fixed block count and a fixed order, so
// results are bitwise reproducible.  The Hessenberg matrix, the Givens
// rotations and the least-squares solution stay on the device; the host reads
// one scalar (the residual estimate) per iteration.
#include "common.h"

namespace isc {

constexpr int MAXV = 32;   // basis vectors handled by one multi-dot

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
    return x;
}

// block-level sum of nv per-thread values -> partial[k * nblk + block]
__device__ __forceinline__ void block_store(const double* acc, int nv, double* partial, int nblk) {
    __shared__ double red[4][MAXV];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int k = 0; k < MAXV; ++k) {
        if (k < nv) {
            const double s = wave_sum(acc[k]);
            if (lane == 0) red[w][k] = s;
        }
    }
    __syncthreads();
    if ((int)threadIdx.x < nv) {
        const int k = threadIdx.x;
        partial[(size_t)k * nblk + blockIdx.x] = (red[0][k] + red[1][k]) + (red[2][k] + red[3][k]);
    }
}

// partial[k] = <V_k, w>, k < nv
template <class TV>
__global__ void __launch_bounds__(256) multidot(int64_t len, const TV* __restrict__ V, int64_t ldv, int nv,
                                                const TV* __restrict__ w, double* __restrict__ partial) {
    double acc[MAXV];
#pragma unroll
    for (int k = 0; k < MAXV; ++k) acc[k] = 0.0;
    for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < len; t += (int64_t)gridDim.x * 256) {
        const double wv = (double)w[t];
#pragma unroll
        for (int k = 0; k < MAXV; ++k)
            if (k < nv) acc[k] += (double)V[(size_t)k * ldv + t] * wv;
    }
    block_store(acc, nv, partial, gridDim.x);
}

// out[k] = sum of partial[k][0..nblk), fixed order; one block per k
__global__ void __launch_bounds__(256) reduce_partials(const double* __restrict__ partial, int nblk,
                                                       double* __restrict__ out) {
    __shared__ double red[4];
    const int k = blockIdx.x;
    double s = 0.0;
    for (int b = threadIdx.x; b < nblk; b += 256) s += partial[(size_t)k * nblk + b];
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) out[k] = (red[0] + red[1]) + (red[2] + red[3]);
}

// out = sum_k y[k] V_k (+ out if accumulate)
template <class TV, class TO>
__global__ void __launch_bounds__(256) lincomb(int64_t len, const TV* __restrict__ V, int64_t ldv, int nv,
                                               const double* __restrict__ y, TO* __restrict__ out, int accumulate) {
    double yk[MAXV];
#pragma unroll
    for (int k = 0; k < MAXV; ++k) yk[k] = k < nv ? y[k] : 0.0;
    for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < len; t += (int64_t)gridDim.x * 256) {
        double s = accumulate ? (double)out[t] : 0.0;
#pragma unroll
        for (int k = 0; k < MAXV; ++k)
            if (k < nv) s += yk[k] * (double)V[(size_t)k * ldv + t];
        out[t] = (TO)s;
    }
}

// r = b - Ax (Ax given), partial[0] = ||r||^2
__global__ void __launch_bounds__(256) residual_norm(int64_t len, const double* __restrict__ b,
                                                     const double* __restrict__ Ax, double* __restrict__ r,
                                                     double* __restrict__ partial) {
    double acc[1] = {0.0};
    for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < len; t += (int64_t)gridDim.x * 256) {
        const double v = b[t] - Ax[t];
        r[t] = v;
        acc[0] += v * v;
    }
    block_store(acc, 1, partial, gridDim.x);
}

__global__ void __launch_bounds__(256) axpy_kernel(int64_t len, const double* __restrict__ x, double* __restrict__ y) {
    for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < len; t += (int64_t)gridDim.x * 256) y[t] += x[t];
}

__global__ void __launch_bounds__(256) zero_kernel(int64_t len, double* __restrict__ y) {
    for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < len; t += (int64_t)gridDim.x * 256) y[t] = 0.0;
}

// Small dense state of one GMRES cycle (device memory, updated by single-wavefront kernels):
//   H[(m+1) x m] column-major by iteration, cs[m], sn[m], g[m+1], y[m]
struct Hess {
    double* H; double* cs; double* sn; double* g; double* y; double* scal;
    int m;
};
// scal: [0] beta, [2] residual estimate of the current column count, [4] breakdown flag

// x = R^-1 rhs for the leading k x k upper triangle of R (column-major,
// leading dimension ld, k <= MAXV), on one wavefront: lane i owns row i,
// holding its rhs entry on entry and its x entry on return.  Column by
// column from the last: the lane of the column divides by the diagonal (a
// zero diagonal gives 0) and the entry, broadcast, is taken off the rows
// above.
__device__ __forceinline__ double upper_solve_wave(const double* __restrict__ R, int ld, int k, double rhs) {
    const int i = threadIdx.x;
    double r[MAXV];
#pragma unroll
    for (int l = 0; l < MAXV; ++l) r[l] = (i < k && l >= i && l < k) ? R[(size_t)l * ld + i] : 0.0;
    double s = i < k ? rhs : 0.0;
    double xi = 0.0;
#pragma unroll
    for (int c = MAXV - 1; c >= 0; --c) {
        if (c >= k) continue;
        if (i == c) xi = r[c] != 0.0 ? s / r[c] : 0.0;
        const double xc = __shfl(xi, c);
        if (i < c) s -= r[c] * xc;
    }
    return xi;
}

// ------------------------------------------------------------------ DCGS2
// Vectors are read as double2 (lengths are multiples of 8 doubles).
// Row layout of the dot results: r (r <= j) = <X_r, u>, MAXV + r = <X_r, w>,
// with X_r = Q_r for r < j and X_j = u.
// One pass: <Q_k, u>, <Q_k, w> (k < j), <u, u>, <u, w>; w may be null.
// Wavefront wv of a block accumulates the basis vectors k = wv, wv + 4, ...
// (at most 8 of them, so few registers) over the block's elements; the four
// wavefronts read the same u and w, which the cache serves after the first.
template <class V2>
__global__ void __launch_bounds__(256) dcgs2_dots(int64_t len2, const V2* __restrict__ Q, int64_t ldv2, int j,
                                                  const V2* __restrict__ u, const V2* __restrict__ w,
                                                  double* __restrict__ partial) {
    constexpr int PER = MAXV / 4;
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    double a1[PER], a2[PER];
#pragma unroll
    for (int m = 0; m < PER; ++m) { a1[m] = 0.0; a2[m] = 0.0; }
    double au = 0.0, aw = 0.0;
    const bool hw = w != nullptr;
    for (int64_t t = (int64_t)blockIdx.x * 64 + lane; t < len2; t += (int64_t)gridDim.x * 64) {
        const V2 uvr = u[t];
        const double ux = (double)uvr.x, uy = (double)uvr.y;
        double wxx = 0.0, wxy = 0.0;
        if (hw) {
            const V2 wr = w[t];
            wxx = (double)wr.x;
            wxy = (double)wr.y;
        }
#pragma unroll
        for (int m = 0; m < PER; ++m) {
            const int k = wv + 4 * m;
            if (k < j) {
                const V2 q = Q[(size_t)k * ldv2 + t];
                const double qx = (double)q.x, qy = (double)q.y;
                a1[m] += qx * ux + qy * uy;
                a2[m] += qx * wxx + qy * wxy;
            }
        }
        if (wv == 0) {
            au += ux * ux + uy * uy;
            aw += ux * wxx + uy * wxy;
        }
    }
    const int nblk = gridDim.x;
#pragma unroll
    for (int m = 0; m < PER; ++m) {
        const int k = wv + 4 * m;
        if (k < j) {
            const double s1 = wave_sum(a1[m]);
            const double s2 = wave_sum(a2[m]);
            if (lane == 0) {
                partial[(size_t)k * nblk + blockIdx.x] = s1;
                if (hw) partial[(size_t)(MAXV + k) * nblk + blockIdx.x] = s2;
            }
        }
    }
    if (wv == 0) {
        const double su = wave_sum(au), sw = wave_sum(aw);
        if (lane == 0) {
            partial[(size_t)j * nblk + blockIdx.x] = su;
            if (hw) partial[(size_t)(MAXV + j) * nblk + blockIdx.x] = sw;
        }
    }
}

// out[row] = sum over blocks of partial[row] (row layout above)
__global__ void __launch_bounds__(256) reduce_rows_dcgs(const double* __restrict__ partial, int nblk, int j,
                                                        double* __restrict__ out) {
    __shared__ double red[4];
    const int r = blockIdx.x;
    const int row = r <= j ? r : MAXV + (r - j - 1);
    double s = 0.0;
#pragma unroll 8
    for (int b = threadIdx.x; b < nblk; b += 256) s += partial[(size_t)row * nblk + b];
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) out[row] = (red[0] + red[1]) + (red[2] + red[3]);
}

// Device state of the delayed scheme: the unrotated Hessenberg matrix, the
// first-pass coefficients of the pending column and (omega, zeta).
struct Dcgs {
    double* Hraw;    // [(m+1) x m], column-major
    double* hprev;   // [m+1]
    double* omz;     // [0] omega_j, [1] zeta_j
    double* Rs;      // flexible variant only (else null): [m x (m+1)], column j = (s_j, omega_j)
};

// Iteration j, one wavefront: lane i owns row i of the columns below (the
// restart length is at most 31, so every row has a lane).  c holds the dots
// of this iteration.  Finishes the reorthogonalisation of u_j (s = Q_j^T u_j,
// omega = ||u_j - Q_j s|| by Pythagoras), completes Hessenberg column j-1 and
// its Givens rotation (residual estimate of a j-column solution in scal[2]),
// then forms the first-pass coefficients of A M^-1 q_j from those of
// w = A M^-1 u_j:
//   zeta = q_j^T w = (u_j^T w - s^T z) / omega,  z = Q_j^T w,
//   h    = ([z; zeta] - H_j s) / omega           (H_j: columns 0..j-1).
// scal[4] = 1 flags omega = 0 (u_j in the span of Q_j).
__global__ void __launch_bounds__(64) dcgs2_step(Hess hs, Dcgs d, int j, int last, const double* __restrict__ c) {
    __shared__ double sc[MAXV], scol[MAXV + 1], scs[MAXV], ssn[MAXV];
    const int l = threadIdx.x;
    const int m = hs.m;
    const int ld = m + 1;
    const double cl = l <= j ? c[l] : 0.0;
    const double czl = (!last && l <= j) ? c[MAXV + l] : 0.0;
    // H_j rows of this lane (columns lo..j-2 of the unrotated matrix), all loads in flight at once
    const int lo = l > 0 ? l - 1 : 0;
    double hr[MAXV];
#pragma unroll
    for (int k = 0; k < MAXV; ++k)
        hr[k] = (!last && l <= j && k >= lo && k < j - 1) ? d.Hraw[(size_t)k * ld + l] : 0.0;
    const double hp = (j > 0 && l < j) ? d.hprev[l] : 0.0;
    if (l < j - 1) {
        scs[l] = hs.cs[l];
        ssn[l] = hs.sn[l];
    }
    if (l < j) sc[l] = cl;
    const double om2 = __shfl(cl, j) - wave_sum(l < j ? cl * cl : 0.0);
    if (!isfinite(om2)) {
        if (l == 0) {
            hs.scal[2] = om2;
            hs.scal[4] = 1.0;
        }
        return;
    }
    const double om = om2 > 0.0 ? sqrt(om2) : 0.0;
    if (d.Rs && j < m) {   // u_j = omega_j q_j + Q_j s_j
        if (l < j) d.Rs[(size_t)j * ld + l] = cl;
        if (l == j) d.Rs[(size_t)j * ld + j] = om;
    }
    double rawl = 0.0;
    if (j == 0) {
        for (int k = l; k <= m; k += 64) hs.g[k] = k == 0 ? om : 0.0;
        if (l == 0) {
            hs.scal[0] = om;
            hs.scal[2] = om;
        }
    } else {
        rawl = l < j ? hp + cl : (l == j ? om : 0.0);
        if (l <= m) d.Hraw[(size_t)(j - 1) * ld + l] = rawl;
        if (l <= j) scol[l] = rawl;
        __syncthreads();
        if (l == 0) {   // the earlier rotations, then a new one for rows j-1, j
            double a = scol[0];
            for (int i = 0; i < j - 1; ++i) {
                const double b = scol[i + 1];
                scol[i] = scs[i] * a + ssn[i] * b;
                a = -ssn[i] * a + scs[i] * b;
            }
            const double b = scol[j];
            const double den = hypot(a, b);
            const double cn = den > 0.0 ? a / den : 1.0;
            const double sn = den > 0.0 ? b / den : 0.0;
            hs.cs[j - 1] = cn;
            hs.sn[j - 1] = sn;
            scol[j - 1] = den;
            scol[j] = 0.0;
            const double g = hs.g[j - 1];
            hs.g[j] = -sn * g;
            hs.g[j - 1] = cn * g;
            hs.scal[2] = fabs(sn * g);
        }
        __syncthreads();
        if (l <= j) hs.H[(size_t)(j - 1) * ld + l] = scol[l];
    }
    if (l == 0) hs.scal[4] = om > 0.0 ? 0.0 : 1.0;
    if (last) return;
    if (!(om > 0.0)) {   // u_j lies in the span of Q_j: q_j = u_{j+1} = 0 from here on
        if (l <= j) d.hprev[l] = 0.0;
        if (l == 0) {
            d.omz[0] = 0.0;
            d.omz[1] = 0.0;
        }
        return;
    }
    const double zeta = (__shfl(czl, j) - wave_sum(l < j ? cl * czl : 0.0)) / om;
    __syncthreads();
    if (l <= j) {
        double v = l < j ? czl : zeta;
#pragma unroll
        for (int k = 0; k < MAXV; ++k)
            if (k >= lo && k < j) v -= (k == j - 1 ? rawl : hr[k]) * sc[k];
        d.hprev[l] = v / om;
    }
    if (l == 0) {
        d.omz[0] = om;
        d.omz[1] = zeta;
    }
}

// Residual estimate a j-column solution would have, taking column j-1 as
// (hprev, ||u_j||): the reorthogonalisation coefficients s_j of u_j are left
// out (they are of the order of rounding), so no preconditioner application
// is needed to decide whether the cycle has converged.  State is not changed;
// the estimate goes to scal[5].
__global__ void dcgs2_probe(Hess hs, Dcgs d, int j, const double* __restrict__ nrm2) {
    double col[MAXV + 1];
    for (int i = 0; i < j; ++i) col[i] = d.hprev[i];
    col[j] = sqrt(fmax(nrm2[0], 0.0));
    for (int i = 0; i < j - 1; ++i) {
        const double a = col[i], b = col[i + 1];
        col[i] = hs.cs[i] * a + hs.sn[i] * b;
        col[i + 1] = -hs.sn[i] * a + hs.cs[i] * b;
    }
    const double den = hypot(col[j - 1], col[j]);
    const double sn = den > 0.0 ? col[j] / den : 0.0;
    hs.scal[5] = fabs(sn * hs.g[j - 1]);
}

// Coefficients of a cycle's solution, one wavefront.  y = R^-1 g for the
// leading k x k triangle of the rotated Hessenberg matrix; the stored vectors
// are zt_j = P(u_j) = omega_j z_j + Z_j s_j, i.e. Zt = Z Rs with Rs upper
// triangular, so the solution Z y becomes Zt (Rs^-1 y): hs.y = Rs^-1 R^-1 g.
__global__ void __launch_bounds__(64) cycle_coefficients(Hess hs, Dcgs d, int k) {
    const int ld = hs.m + 1;
    const int i = threadIdx.x;
    double t = upper_solve_wave(hs.H, ld, k, i < k ? hs.g[i] : 0.0);
    t = upper_solve_wave(d.Rs, ld, k, t);
    if (i < k) hs.y[i] = t;
}

// One pass: q_j = (u - Q_j s) / omega  and  u <- (w - Q_j z - zeta q_j) / omega
// (omega = 0, a breakdown, leaves q_j = u = 0).
template <class V2>
__global__ void __launch_bounds__(256) dcgs2_update(int64_t len2, V2* Q, int64_t ldv2, int j,
                                                    const double* __restrict__ c, const double* __restrict__ omz,
                                                    V2* u, const V2* __restrict__ w, double* __restrict__ nrm_partial) {
    double sk[MAXV], zk[MAXV];
#pragma unroll
    for (int k = 0; k < MAXV; ++k) {
        sk[k] = k < j ? c[k] : 0.0;
        zk[k] = k < j ? c[MAXV + k] : 0.0;
    }
    const double rom = omz[0] > 0.0 ? 1.0 / omz[0] : 0.0, zeta = omz[1];
    V2* qj = Q + (size_t)j * ldv2;
    double nacc[1] = {0.0};
    for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < len2; t += (int64_t)gridDim.x * 256) {
        const V2 uv = u[t];
        const V2 wv = w[t];
        double sx = 0.0, sy = 0.0, zx = 0.0, zy = 0.0;
#pragma unroll
        for (int k = 0; k < MAXV; ++k) {
            if (k < j) {
                const V2 q = Q[(size_t)k * ldv2 + t];
                sx += sk[k] * (double)q.x;
                sy += sk[k] * (double)q.y;
                zx += zk[k] * (double)q.x;
                zy += zk[k] * (double)q.y;
            }
        }
        const double qx = ((double)uv.x - sx) * rom, qy = ((double)uv.y - sy) * rom;
        V2 qo, uo;
        qo.x = qx;
        qo.y = qy;
        uo.x = ((double)wv.x - zx - zeta * qx) * rom;
        uo.y = ((double)wv.y - zy - zeta * qy) * rom;
        qj[t] = qo;
        u[t] = uo;
        nacc[0] += (double)uo.x * (double)uo.x + (double)uo.y * (double)uo.y;
    }
    if (nrm_partial) block_store(nacc, 1, nrm_partial, gridDim.x);   // ||u_{j+1}||^2 per block
}

}  // namespace isc

// ---------------------------------------------------------------- host side
hipError_t isc_launch_bilu0_apply(isc_ctx*, const double*, const double*, const double*, double*);
hipError_t isc_launch_spmv(isc_ctx*, const double*, const double*, double*);
hipError_t isc_launch_bilu0_apply_spmv(isc_ctx*, const double*, const double*, const double*, double*, double*);
hipError_t isc_launch_update_apply_spmv(isc_ctx*, const double*, const double*, const isc::LagUpdate&, double*,
                                        double*);
hipError_t isc_launch_bilu0_factor(isc_ctx*, const double*, double*, int32_t*);
void isc_well_apply(isc_ctx*, const double* x, double* w);   // eliminated well rows (isc_newton_step only)

namespace isc {

static int nblocks(int64_t len) {
    int64_t b = (len + 255) / 256;
    return (int)(b < NPART ? (b > 0 ? b : 1) : NPART);
}

// reductions: results land in ctx->small + RED_OFF
constexpr int RED_OFF = 0;          // [0, 2*MAXV): h1, h2 ; [2*MAXV]: norm^2
Hess hess_at(double* small, int m) {
    Hess h;
    double* base = small + 4 * MAXV;
    h.H = base;
    h.cs = h.H + (size_t)(m + 1) * m;
    h.sn = h.cs + m;
    h.g = h.sn + m;
    h.y = h.g + m + 1;
    h.scal = h.y + m;
    h.m = m;
    return h;
}
Hess hess_of(isc_ctx* ctx) { return hess_at(ctx->small, ctx->mmax); }

// ||v||^2 -> dst (device)
static void norm2_dev(isc_ctx* ctx, int64_t len, const double* v, double* dst) {
    const int nb = nblocks(len);
    hipLaunchKernelGGL(multidot<double>, dim3(nb), dim3(256), 0, ctx->stream, len, v, (int64_t)0, 1, v,
                       ctx->partial);
    hipLaunchKernelGGL(reduce_partials, dim3(1), dim3(256), 0, ctx->stream, ctx->partial, nb, dst);
}

static hipError_t read_scalar(isc_ctx* ctx, const double* dsrc, double* out) {
    hipError_t e = hipMemcpyAsync(ctx->hscratch, dsrc, sizeof(double), hipMemcpyDeviceToHost, ctx->stream);
    if (e != hipSuccess) return e;
    e = hipStreamSynchronize(ctx->stream);
    *out = ctx->hscratch[0];
    isc_prof_drain(ctx);
    return e;
}

}  // namespace isc

namespace isc {
// delayed-CGS2 state lives after the Hessenberg block of ctx->small
constexpr int DCGS_OFF = 1400;
constexpr int RS_OFF = 4096;     // Rs of the flexible solver: (m+1)^2 doubles past the first 4096
Dcgs dcgs_at(double* small, int m) {
    Dcgs d;
    d.Hraw = small + DCGS_OFF;
    d.hprev = d.Hraw + (size_t)(m + 1) * m;
    d.omz = d.hprev + (m + 1);
    d.Rs = nullptr;
    return d;
}
}  // namespace isc

// FP64 right-preconditioned GMRES(m) with BILU(0); Dinv must hold the factor.
// Iteration j applies A M^-1 to the lagged vector u_j (kept in basis slot m),
// reduces once, finishes column j-1 on the device and, while the host reads
// the residual estimate of the j-column solution, already runs the update
// pass that writes q_j and u_{j+1}.  A cycle that reaches m columns needs one
// more reduction (no product) to finish column m-1.
isc_status isc_gmres_fp64(isc_ctx* ctx, const double* A, const double* Dinv, const double* b, double* x,
                          const isc_solve_opts* o, isc_solve_info* info) {
    using namespace isc;
    const int64_t len = (int64_t)ctx->n * NU;
    const int64_t ldv = len;
    const int64_t len2 = len / 2, ldv2 = ldv / 2;
    const int m = o->restart;
    const int nb = nblocks(len);
    const int nb2 = nblocks(len2);
    Hess hs = hess_of(ctx);
    Dcgs dc = dcgs_at(ctx->small, ctx->mmax);
    dc.Rs = ctx->small + RS_OFF;   // u_j = Q_j s_j + omega_j q_j, kept to form the solution from Z
    double* red = ctx->small + RED_OFF;
    double2* Q2 = reinterpret_cast<double2*>(ctx->V);
    double* u = ctx->V + (size_t)m * ldv;
    double2* u2 = reinterpret_cast<double2*>(u);
    const double2* w2 = reinterpret_cast<const double2*>(ctx->w);
    isc_solve_info inf{};
    double bn2;
    norm2_dev(ctx, len, b, red + 2 * MAXV);
    ISC_HIP(read_scalar(ctx, red + 2 * MAXV, &bn2));
    const double bnorm = sqrt(bn2);
    hipLaunchKernelGGL(zero_kernel, dim3(nb), dim3(256), 0, ctx->stream, len, x);
    if (bnorm == 0.0) {
        if (info) *info = inf;
        return ISC_OK;
    }
    if (!std::isfinite(bnorm)) {
        ctx->err = "isc_solve: right-hand side is not finite";
        return ISC_ERR_NONFINITE;
    }
    isc_status st = ISC_ERR_LINEAR_NOCONV;
    hipEvent_t ev = ctx->ev[7];
    for (int cyc = 0; cyc < o->max_restarts; ++cyc) {
        // u_0 = r = b - A x  (x = 0 on the first cycle)
        if (cyc == 0) {
            ISC_HIP(hipMemcpyAsync(u, b, (size_t)len * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
        } else {
            isc_launch_spmv(ctx, A, x, ctx->tvec);
            isc_well_apply(ctx, x, ctx->tvec);
            hipLaunchKernelGGL(residual_norm, dim3(nb), dim3(256), 0, ctx->stream, len, b, ctx->tvec, u,
                               ctx->partial);
            hipLaunchKernelGGL(reduce_partials, dim3(1), dim3(256), 0, ctx->stream, ctx->partial, nb,
                               red + 2 * MAXV);
            double rn2;
            ISC_HIP(read_scalar(ctx, red + 2 * MAXV, &rn2));
            inf.relres_true = sqrt(rn2) / bnorm;
            if (sqrt(rn2) <= o->rtol * bnorm) { st = ISC_OK; break; }
            inf.restarts = cyc;
        }
        int k = m;
        // The Gram-Schmidt update of iteration j-1 (q_{j-1} and u_j) runs
        // inside iteration j's forward sweep where the sync-free sweeps allow
        // it (fold mode); otherwise as a pass of its own, launched while the
        // host reads iteration j-1's residual estimate.
        const bool fold_mode = ctx->syncfree && ctx->fold_update;
        for (int j = 0; j <= m; ++j) {
            const bool last = j == m;
            const bool fold = fold_mode && j > 0 && !last;
            if (fold_mode && j > 0 && !fold) {
                const int tk = isc_prof_begin(ctx, ISC_PROF_KRYLOV);
                hipLaunchKernelGGL(dcgs2_update<double2>, dim3(nb2), dim3(256), 0, ctx->stream, len2, Q2, ldv2, j - 1,
                                   red, dc.omz, u2, w2, (double*)nullptr);
                isc_prof_end(ctx, tk);
            }
            if (!last) {   // z_j = M^-1 u_j (kept in Z) and w = A z_j
                const int tk = isc_prof_begin(ctx, ISC_PROF_ILU_SPMV);
                double* Zj = ctx->Z + (size_t)j * ldv;
                if (fold) {
                    const LagUpdate lu{ctx->V, ldv, j - 1, red, red + MAXV, dc.omz, u, ctx->w};
                    isc_launch_update_apply_spmv(ctx, A, Dinv, lu, Zj, ctx->w);
                    isc_prof_vectors(ctx, ISC_PROF_ILU_SPMV, (double)(j + 2));
                } else {
                    isc_launch_bilu0_apply_spmv(ctx, A, Dinv, u, Zj, ctx->w);
                }
                isc_well_apply(ctx, Zj, ctx->w);
                isc_prof_end(ctx, tk);
            }
            const int tk = isc_prof_begin(ctx, ISC_PROF_KRYLOV);
            hipLaunchKernelGGL(dcgs2_dots<double2>, dim3(nb2), dim3(256), 0, ctx->stream, len2, Q2, ldv2, j, u2,
                               last ? nullptr : w2, ctx->partial);
            hipLaunchKernelGGL(reduce_rows_dcgs, dim3(last ? j + 1 : 2 * (j + 1)), dim3(256), 0, ctx->stream,
                               ctx->partial, nb2, j, red);
            hipLaunchKernelGGL(dcgs2_step, dim3(1), dim3(64), 0, ctx->stream, hs, dc, j, last ? 1 : 0, red);
            ISC_HIP(hipMemcpyAsync(ctx->hscratch, hs.scal, 8 * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
            ISC_HIP(hipEventRecord(ev, ctx->stream));
            if (!fold_mode && !last)   // speculative: unused if the estimate below ends the cycle
                hipLaunchKernelGGL(dcgs2_update<double2>, dim3(nb2), dim3(256), 0, ctx->stream, len2, Q2, ldv2, j,
                                   red, dc.omz, u2, w2, (double*)nullptr);
            isc_prof_end(ctx, tk);
            ISC_HIP(hipEventSynchronize(ev));
            const double est = ctx->hscratch[2];
            const bool breakdown = ctx->hscratch[4] != 0.0;
            if (!std::isfinite(est)) {
                (void)hipStreamSynchronize(ctx->stream);
                isc_prof_drain(ctx);
                if (isc_check_sweeps(ctx) != ISC_OK) return ISC_ERR_HIP;
                ctx->err = "isc_solve: GMRES breakdown (non-finite residual estimate)";
                return ISC_ERR_NONFINITE;
            }
            if (j == 0) {
                if (breakdown) {   // u_0 = r has zero norm: nothing to do
                    k = 0;
                    break;
                }
                continue;
            }
            inf.iters++;
            inf.relres_est = est / bnorm;
            if (est <= o->rtol * bnorm || breakdown || last) {
                k = j;
                break;
            }
        }
        // x += M^-1 Q_k y = Z_k (Rs^-1 y): the preconditioned lagged vectors are
        // at hand, so no further BILU(0) apply
        if (k > 0) {
            hipLaunchKernelGGL(cycle_coefficients, dim3(1), dim3(64), 0, ctx->stream, hs, dc, k);
            hipLaunchKernelGGL((lincomb<double, double>), dim3(nb), dim3(256), 0, ctx->stream, len, ctx->Z, ldv, k,
                               hs.y, x, 1);
        }
    }
    if (st != ISC_OK) {
        isc_launch_spmv(ctx, A, x, ctx->tvec);
        isc_well_apply(ctx, x, ctx->tvec);
        hipLaunchKernelGGL(residual_norm, dim3(nb), dim3(256), 0, ctx->stream, len, b, ctx->tvec, ctx->w,
                           ctx->partial);
        hipLaunchKernelGGL(reduce_partials, dim3(1), dim3(256), 0, ctx->stream, ctx->partial, nb, red + 2 * MAXV);
        double rn2;
        ISC_HIP(read_scalar(ctx, red + 2 * MAXV, &rn2));
        inf.relres_true = sqrt(rn2) / bnorm;
        if (sqrt(rn2) <= o->rtol * bnorm) st = ISC_OK;
        else ctx->err = "isc_solve: GMRES did not reach the tolerance";
    }
    if (info) *info = inf;
    ISC_HIP(hipGetLastError());
    {
        const isc_status sw = isc_check_sweeps(ctx);
        if (sw != ISC_OK) return sw;
    }
    return st;
}

// ---------------------------------------------------------------- precision form
hipError_t isc_launch_bilu0_apply_spmv32(isc_ctx*, const float*, const float*, const float*, float*, float*);
hipError_t isc_launch_bilu0_factor32_from64(isc_ctx*, const double*, float*, float*, int32_t*);

// Set-up of the precision form: the block ILU(0) factor of the decoupled
// matrix rounded to FP32 (computed in FP64 arithmetic from the FP32-rounded
// blocks, stored in FP32, with the sweeps' FP32 packs).  The FP32 copy of the
// matrix itself is made only for the per-hyperplane schedule, whose sweeps
// read it.  Launches only (no host synchronisation); a singular pivot block
// is reported through bad_dev like the FP64 factor.
isc_status isc_prepare_mixed_dev(isc_ctx* ctx, const double* A, int32_t* bad_dev) {
    if (!ctx->J32) {
        ctx->err = "mixed precision needs a context created with max inner_iters >= 1";
        return ISC_ERR_ARG;
    }
    ISC_HIP(isc_launch_bilu0_factor32_from64(ctx, A, ctx->J32, ctx->Dinv32, bad_dev));
    return ISC_OK;
}
hipError_t isc_launch_update_apply_spmv32(isc_ctx*, const float*, const float*, const isc::LagUpdateT<float>&, float*,
                                          float*);

namespace isc {

__global__ void __launch_bounds__(256) to_f64(int64_t len, const float* __restrict__ a, double* __restrict__ b) {
    for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < len; t += (int64_t)gridDim.x * 256)
        b[t] = (double)a[t];
}

__global__ void __launch_bounds__(256) narrow_f32(int64_t len, const double* __restrict__ a, float* __restrict__ b) {
    for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < len; t += (int64_t)gridDim.x * 256)
        b[t] = (float)a[t];
}

// z ~= A^-1 v by m_in iterations of FP32 right-preconditioned GMRES from 0
// (FP32 storage of the basis, the matrix and the ILU factor; FP64 reductions
// and small dense work), orthogonalised by the same delayed CGS2 as the FP64
// solver.  No host synchronisation: the iteration count is fixed, and a
// breakdown leaves zero vectors and zero Hessenberg columns, which the
// triangular solve skips.
static void inner_gmres32(isc_ctx* ctx, const float* A32, const float* D32, const double* v, double* z, int m_in) {
    const int64_t len = (int64_t)ctx->n * NU;
    const int64_t len2 = len / 2;
    const int nb = nblocks(len);
    const int nb2 = nblocks(len2);
    Hess hi = hess_at(ctx->small32, ctx->inner_max);
    Dcgs di = dcgs_at(ctx->small32, ctx->inner_max);
    di.Rs = ctx->small32 + RS_OFF;   // u_j = Q_j s_j + omega_j q_j, to form the result from Z32
    double* red = ctx->small32 + RED_OFF;
    float2* Q2 = reinterpret_cast<float2*>(ctx->V32);
    float* u = ctx->V32 + (size_t)m_in * len;
    float2* u2 = reinterpret_cast<float2*>(u);
    const float2* w2 = reinterpret_cast<const float2*>(ctx->w32);
    hipLaunchKernelGGL(narrow_f32, dim3(nb), dim3(256), 0, ctx->stream, len, v, u);
    for (int j = 0; j <= m_in; ++j) {
        const bool last = j == m_in;
        // iteration j-1's Gram-Schmidt update (q_{j-1}, u_j): in this iteration's
        // forward sweep where the sync-free sweeps run, else a pass of its own
        const bool fold = j > 0 && !last && ctx->syncfree;
        if (j > 0 && !fold) {
            const int tk = isc_prof_begin(ctx, ISC_PROF_KRYLOV);
            hipLaunchKernelGGL(dcgs2_update<float2>, dim3(nb2), dim3(256), 0, ctx->stream, len2, Q2, len2, j - 1,
                               red, di.omz, u2, w2, (double*)nullptr);
            isc_prof_end(ctx, tk);
        }
        if (!last) {   // w = A M^-1 u_j in FP32: forward sweep, backward sweep fused with the SpMV
            const int tk = isc_prof_begin(ctx, ISC_PROF_ILU_SPMV32);
            float* Zj = ctx->Z32 + (size_t)j * len;   // z_j = M^-1 u_j, kept
            if (fold) {
                const LagUpdateT<float> lu{ctx->V32, len, j - 1, red, red + MAXV, di.omz, u, ctx->w32};
                isc_launch_update_apply_spmv32(ctx, A32, D32, lu, Zj, ctx->w32);
                isc_prof_vectors(ctx, ISC_PROF_ILU_SPMV32, (double)(j + 2));
            } else {
                isc_launch_bilu0_apply_spmv32(ctx, A32, D32, u, Zj, ctx->w32);
            }
            isc_prof_end(ctx, tk);
        }
        const int tk = isc_prof_begin(ctx, ISC_PROF_KRYLOV);
        hipLaunchKernelGGL(dcgs2_dots<float2>, dim3(nb2), dim3(256), 0, ctx->stream, len2, Q2, len2, j, u2,
                           last ? nullptr : w2, ctx->partial);
        hipLaunchKernelGGL(reduce_rows_dcgs, dim3(last ? j + 1 : 2 * (j + 1)), dim3(256), 0, ctx->stream,
                           ctx->partial, nb2, j, red);
        hipLaunchKernelGGL(dcgs2_step, dim3(1), dim3(64), 0, ctx->stream, hi, di, j, last ? 1 : 0, red);
        isc_prof_end(ctx, tk);
    }
    // z = M^-1 Q y = Z32 (Rs^-1 y): no further BILU(0) apply
    hipLaunchKernelGGL(cycle_coefficients, dim3(1), dim3(64), 0, ctx->stream, hi, di, m_in);
    hipLaunchKernelGGL((lincomb<float, float>), dim3(nb), dim3(256), 0, ctx->stream, len, ctx->Z32, len, m_in, hi.y,
                       ctx->t32, 0);
    hipLaunchKernelGGL(to_f64, dim3(nb), dim3(256), 0, ctx->stream, len, ctx->t32, z);
}

// e = the CPR stage-1 pressure solve of rp (vectors of ctx->cpr_npad doubles,
// the entries past the cell count zero): k steps of FP64 GMRES from 0 on
// A_p e = rp, right-preconditioned by one V-cycle of the pressure multigrid,
// orthogonalised by the same delayed CGS2; no host synchronisation (k is
// fixed; a breakdown leaves zero vectors and zero Hessenberg columns, which
// the triangular solves skip).  k = 0: e = one V-cycle applied to rp.
static void pressure_gmres(isc_ctx* ctx, const double* rp, double* e, int k) {
    if (k == 0) {
        isc_cpr_vcycle(ctx, rp, e);
        return;
    }
    const int64_t len = ctx->cpr_npad;
    const int64_t len2 = len / 2;
    const int nb = nblocks(len);
    const int nb2 = nblocks(len2);
    Hess hp = hess_at(ctx->small_p, ctx->cpr_kmax);
    Dcgs dp = dcgs_at(ctx->small_p, ctx->cpr_kmax);
    dp.Rs = ctx->small_p + RS_OFF;   // u_j = Q_j s_j + omega_j q_j, to form the result from Z
    double* red = ctx->small_p + RED_OFF;
    double2* Q2 = reinterpret_cast<double2*>(ctx->cpr_V);
    double* u = ctx->cpr_V + (size_t)k * len;   // the lagged vector
    double2* u2 = reinterpret_cast<double2*>(u);
    const double2* w2 = reinterpret_cast<const double2*>(ctx->cpr_w);
    (void)hipMemcpyAsync(u, rp, (size_t)len * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream);
    for (int j = 0; j <= k; ++j) {
        const bool last = j == k;
        if (j > 0)   // q_{j-1} and u_j
            hipLaunchKernelGGL(dcgs2_update<double2>, dim3(nb2), dim3(256), 0, ctx->stream, len2, Q2, len2, j - 1,
                               red, dp.omz, u2, w2, (double*)nullptr);
        if (!last) {   // z_j = V-cycle(u_j) (kept), w = A_p z_j
            double* Zj = ctx->cpr_Z + (size_t)j * len;
            isc_cpr_vcycle(ctx, u, Zj);
            isc_cpr_pressure_apply(ctx, Zj, ctx->cpr_w);
        }
        hipLaunchKernelGGL(dcgs2_dots<double2>, dim3(nb2), dim3(256), 0, ctx->stream, len2, Q2, len2, j, u2,
                           last ? nullptr : w2, ctx->partial);
        hipLaunchKernelGGL(reduce_rows_dcgs, dim3(last ? j + 1 : 2 * (j + 1)), dim3(256), 0, ctx->stream,
                           ctx->partial, nb2, j, red);
        hipLaunchKernelGGL(dcgs2_step, dim3(1), dim3(64), 0, ctx->stream, hp, dp, j, last ? 1 : 0, red);
    }
    hipLaunchKernelGGL(cycle_coefficients, dim3(1), dim3(64), 0, ctx->stream, hp, dp, k);
    hipLaunchKernelGGL((lincomb<double, double>), dim3(nb), dim3(256), 0, ctx->stream, len, ctx->cpr_Z, len, k, hp.y,
                       e, 0);
}

// z = CPR(u) and w = A z (FP64): the pressure solve, the stage-1 correction
// (w1 = A E e_p, r2 = u - w1), block ILU(0) on r2 fused with the SpMV
// (z2, w2 = A z2), then z = z2 + E e_p and w = w2 + w1.  ctx->Dinv and the
// sweep packs must hold the factor of A, and the CPR set-up must be done.
static void cpr_apply_w(isc_ctx* ctx, const double* A, const double* u, double* z, double* w, int k) {
    int tk = isc_prof_begin(ctx, ISC_PROF_CPR_PRESSURE);
    isc_cpr_gather(ctx, u, ctx->cpr_rp);
    pressure_gmres(ctx, ctx->cpr_rp, ctx->cpr_ep, k);
    isc_cpr_stage1(ctx, ctx->cpr_ep, u, ctx->cpr_w1, ctx->cpr_r2);
    isc_prof_end(ctx, tk);
    tk = isc_prof_begin(ctx, ISC_PROF_ILU_SPMV);
    isc_launch_bilu0_apply_spmv(ctx, A, ctx->Dinv, ctx->cpr_r2, z, w);
    isc_prof_end(ctx, tk);
    tk = isc_prof_begin(ctx, ISC_PROF_CPR_PRESSURE);
    isc_cpr_combine(ctx, ctx->cpr_ep, z, w, ctx->cpr_w1);
    isc_prof_end(ctx, tk);
}

}  // namespace isc

void isc_cpr_pressure_gmres(isc_ctx* ctx, const double* rp, double* e, int k) { isc::pressure_gmres(ctx, rp, e, k); }

// z = M32^-1 r and w = A32 z with the FP32 factor and matrix data prepared by
// isc_prepare_mixed_dev (the inner iteration's product, without its folded
// Gram-Schmidt update); r, z, w FP64, rounded to and from FP32 storage.
void isc_apply_spmv32_from64(isc_ctx* ctx, const double* r, double* z, double* w) {
    using namespace isc;
    const int64_t len = (int64_t)ctx->n * NU;
    const int nb = nblocks(len);
    float* r32 = ctx->V32;
    float* z32 = ctx->Z32;
    hipLaunchKernelGGL(narrow_f32, dim3(nb), dim3(256), 0, ctx->stream, len, r, r32);
    isc_launch_bilu0_apply_spmv32(ctx, ctx->J32, ctx->Dinv32, r32, z32, ctx->w32);
    hipLaunchKernelGGL(to_f64, dim3(nb), dim3(256), 0, ctx->stream, len, (const float*)z32, z);
    hipLaunchKernelGGL(to_f64, dim3(nb), dim3(256), 0, ctx->stream, len, (const float*)ctx->w32, w);
}
void isc_cpr_apply_w(isc_ctx* ctx, const double* A, const double* u, double* z, double* w, int k) {
    isc::cpr_apply_w(ctx, A, u, z, w, k);
}

// FP64 flexible GMRES(m) whose preconditioner is either the FP32 inner GMRES
// above (ISC_MIXED) or the CPR preconditioner (ISC_PC_CPR),
// with the same delayed CGS2 as the FP64 solver.  Iteration j stores
// zt_j = P(u_j) for the lagged vector u_j; since u_j = omega_j q_j + Q_j s_j,
// zt_j = omega_j z_j + Z_j s_j for the vectors z_j that satisfy the flexible
// Arnoldi relation A Z = Q H, so the update x += Z y is done as
// x += Zt (Rs^-1 y) with the small triangular Rs of the (s_j, omega_j).
// ISC_MIXED: ctx->J32 / ctx->Dinv32 must hold the FP32 matrix and factor;
// ISC_PC_CPR: ctx->Dinv the FP64 factor and the CPR set-up done.
isc_status isc_fgmres(isc_ctx* ctx, const double* A, const double* b, double* x, const isc_solve_opts* o,
                      isc_solve_info* info) {
    using namespace isc;
    const bool cpr = o->precond == ISC_PC_CPR;
    const int64_t len = (int64_t)ctx->n * NU;
    const int64_t ldv = len;
    const int64_t len2 = len / 2, ldv2 = ldv / 2;
    const int m = o->restart;
    const int m_in = o->inner_iters;
    const int nb = nblocks(len);
    const int nb2 = nblocks(len2);
    const int nb2u = nb2;   // blocks of the update pass (its norm partials)
    Hess hs = hess_of(ctx);
    Dcgs dc = dcgs_at(ctx->small, ctx->mmax);
    dc.Rs = ctx->small + RS_OFF;
    double* red = ctx->small + RED_OFF;
    double2* Q2 = reinterpret_cast<double2*>(ctx->V);
    double* u = ctx->V + (size_t)m * ldv;
    double2* u2 = reinterpret_cast<double2*>(u);
    const double2* w2 = reinterpret_cast<const double2*>(ctx->w);
    isc_solve_info inf{};
    double bn2;
    norm2_dev(ctx, len, b, red + 2 * MAXV);
    ISC_HIP(read_scalar(ctx, red + 2 * MAXV, &bn2));
    const double bnorm = sqrt(bn2);
    hipLaunchKernelGGL(zero_kernel, dim3(nb), dim3(256), 0, ctx->stream, len, x);
    if (bnorm == 0.0) {
        if (info) *info = inf;
        return ISC_OK;
    }
    if (!std::isfinite(bnorm)) {
        ctx->err = "isc_solve: right-hand side is not finite";
        return ISC_ERR_NONFINITE;
    }
    isc_status st = ISC_ERR_LINEAR_NOCONV;
    hipEvent_t ev = ctx->ev[7];
    for (int cyc = 0; cyc < o->max_restarts; ++cyc) {
        // u_0 = r = b - A x  (x = 0 on the first cycle)
        if (cyc == 0) {
            ISC_HIP(hipMemcpyAsync(u, b, (size_t)len * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
        } else {
            isc_launch_spmv(ctx, A, x, ctx->tvec);
            isc_well_apply(ctx, x, ctx->tvec);
            hipLaunchKernelGGL(residual_norm, dim3(nb), dim3(256), 0, ctx->stream, len, b, ctx->tvec, u,
                               ctx->partial);
            hipLaunchKernelGGL(reduce_partials, dim3(1), dim3(256), 0, ctx->stream, ctx->partial, nb,
                               red + 2 * MAXV);
            double rn2;
            ISC_HIP(read_scalar(ctx, red + 2 * MAXV, &rn2));
            inf.relres_true = sqrt(rn2) / bnorm;
            if (sqrt(rn2) <= o->rtol * bnorm) { st = ISC_OK; break; }
            inf.restarts = cyc;
        }
        int k = m;
        for (int j = 0; j <= m; ++j) {
            bool last = j == m;
            if (!last && j > 0) {
                // probe: does the cycle converge with j columns?  (||u_j||^2 from the update pass)
                hipLaunchKernelGGL(reduce_partials, dim3(1), dim3(256), 0, ctx->stream, ctx->partial + (size_t)2 * MAXV * NPART,
                                   nb2u, red + 2 * MAXV + 1);
                hipLaunchKernelGGL(dcgs2_probe, dim3(1), dim3(1), 0, ctx->stream, hs, dc, j, red + 2 * MAXV + 1);
                double probe;
                ISC_HIP(read_scalar(ctx, hs.scal + 5, &probe));
                if (probe <= o->rtol * bnorm) last = true;   // finish the cycle without another P application
            }
            if (!last) {
                double* Zj = ctx->Z + (size_t)j * ldv;
                if (cpr) {
                    cpr_apply_w(ctx, A, u, Zj, ctx->w, o->p_iters);
                } else {
                    inner_gmres32(ctx, ctx->J32, ctx->Dinv32, u, Zj, m_in);
                    const int tk = isc_prof_begin(ctx, ISC_PROF_SPMV);
                    isc_launch_spmv(ctx, A, Zj, ctx->w);
                    isc_prof_end(ctx, tk);
                }
                isc_well_apply(ctx, Zj, ctx->w);
            }
            const int tk = isc_prof_begin(ctx, ISC_PROF_KRYLOV);
            hipLaunchKernelGGL(dcgs2_dots<double2>, dim3(nb2), dim3(256), 0, ctx->stream, len2, Q2, ldv2, j, u2,
                               last ? nullptr : w2, ctx->partial);
            hipLaunchKernelGGL(reduce_rows_dcgs, dim3(last ? j + 1 : 2 * (j + 1)), dim3(256), 0, ctx->stream,
                               ctx->partial, nb2, j, red);
            hipLaunchKernelGGL(dcgs2_step, dim3(1), dim3(64), 0, ctx->stream, hs, dc, j, last ? 1 : 0, red);
            ISC_HIP(hipMemcpyAsync(ctx->hscratch, hs.scal, 8 * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
            ISC_HIP(hipEventRecord(ev, ctx->stream));
            if (!last)   // speculative: unused if the estimate below ends the cycle
                hipLaunchKernelGGL(dcgs2_update<double2>, dim3(nb2), dim3(256), 0, ctx->stream, len2, Q2, ldv2, j,
                                   red, dc.omz, u2, w2, ctx->partial + (size_t)2 * MAXV * NPART);
            isc_prof_end(ctx, tk);
            ISC_HIP(hipEventSynchronize(ev));
            const double est = ctx->hscratch[2];
            const bool breakdown = ctx->hscratch[4] != 0.0;
            if (!std::isfinite(est)) {
                (void)hipStreamSynchronize(ctx->stream);
                isc_prof_drain(ctx);
                if (isc_check_sweeps(ctx) != ISC_OK) return ISC_ERR_HIP;
                ctx->err = "isc_solve: FGMRES breakdown (non-finite residual estimate)";
                return ISC_ERR_NONFINITE;
            }
            if (!last) inf.inner_iters_total += cpr ? o->p_iters : m_in;
            if (j == 0) {
                if (breakdown) {
                    k = 0;
                    break;
                }
                continue;
            }
            inf.iters++;
            inf.relres_est = est / bnorm;
            if (est <= o->rtol * bnorm || breakdown || last) {
                k = j;
                break;
            }
        }
        if (k > 0) {   // x += Zt (Rs^-1 R^-1 g)
            hipLaunchKernelGGL(cycle_coefficients, dim3(1), dim3(64), 0, ctx->stream, hs, dc, k);
            hipLaunchKernelGGL((lincomb<double, double>), dim3(nb), dim3(256), 0, ctx->stream, len, ctx->Z, ldv, k,
                               hs.y, x, 1);
        }
    }
    if (st != ISC_OK) {
        isc_launch_spmv(ctx, A, x, ctx->tvec);
        isc_well_apply(ctx, x, ctx->tvec);
        hipLaunchKernelGGL(residual_norm, dim3(nb), dim3(256), 0, ctx->stream, len, b, ctx->tvec, ctx->w,
                           ctx->partial);
        hipLaunchKernelGGL(reduce_partials, dim3(1), dim3(256), 0, ctx->stream, ctx->partial, nb, red + 2 * MAXV);
        double rn2;
        ISC_HIP(read_scalar(ctx, red + 2 * MAXV, &rn2));
        inf.relres_true = sqrt(rn2) / bnorm;
        if (sqrt(rn2) <= o->rtol * bnorm) st = ISC_OK;
        else ctx->err = "isc_solve: FGMRES did not reach the tolerance";
    }
    if (info) *info = inf;
    ISC_HIP(hipGetLastError());
    {
        const isc_status sw = isc_check_sweeps(ctx);
        if (sw != ISC_OK) return sw;
    }
    return st;
}
