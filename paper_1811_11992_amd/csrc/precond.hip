// Block ILU(0) preconditioner and block sparse matrix-vector product for the
// decoupled system A = C_L J (unit diagonal blocks).
//
// On the 7-point stencil two distinct neighbours of a cell are never
// neighbours of each other, so ILU(0) in natural cell order only modifies the
// diagonal blocks: M = (D + L) D^-1 (D + U) with L, U the strict lower and
// upper block parts of A and
//     D_i = I - sum_{k lower neighbour of i} A_ik D_k^-1 A_ki.
// The factor, forward and backward recurrences are scheduled by hyperplanes
// ix + iy + iz = s (all rows of a hyperplane are independent); the result is
// the natural-order factorisation exactly.
//
// Mappings: factor - one wavefront per row, lane (r, c) with LDS-staged 8x8
// products and a column-per-lane Gauss-Jordan inverse; apply and SpMV - eight
// lanes per block row, lane r owns output row r.
#include "common.h"

namespace isc {

// position in row k's block list of its upper neighbour i = k + stride
__device__ __forceinline__ int32_t upper_block(int32_t k, int dir, int32_t nx, int32_t ny, int32_t nz,
                                               const int32_t* __restrict__ diag_pos) {
    const int32_t ix = k % nx, iy = (k / nx) % ny;
    int32_t b = diag_pos[k] + 1;
    if (dir >= 1) b += (ix + 1 < nx);
    if (dir >= 2) b += (iy + 1 < ny);
    (void)nz;
    return b;
}

template <class T>
__global__ void __launch_bounds__(256) bilu0_factor_level(
    const int32_t* __restrict__ rows, int32_t cnt, int32_t nx, int32_t ny, int32_t nz,
    const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ diag_pos, const T* __restrict__ A,
    T* __restrict__ Dinv, int32_t* __restrict__ bad) {
    __shared__ double sm[4][4][64];
    const int w = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int32_t t = blockIdx.x * 4 + w;
    if (t >= cnt) return;
    const int32_t i = rows[t];
    const int r = lane >> 3, c = lane & 7;
    double* sA = sm[w][0];
    double* sK = sm[w][1];
    double* sB = sm[w][2];
    double* sP = sm[w][3];
    const int32_t nxy = nx * ny;
    const int32_t ix = i % nx, iy = (i / nx) % ny, iz = i / nxy;
    double D = (r == c) ? 1.0 : 0.0;
    int32_t blk = row_ptr[i];
    const int32_t lower[3] = {iz > 0 ? i - nxy : -1, iy > 0 ? i - nx : -1, ix > 0 ? i - 1 : -1};
    const int ldir[3] = {2, 1, 0};
    for (int q = 0; q < 3; ++q) {
        const int32_t k = lower[q];
        if (k < 0) continue;
        const int32_t bki = upper_block(k, ldir[q], nx, ny, nz, diag_pos);
        sA[lane] = (double)A[(size_t)blk * BS + lane];
        sK[lane] = (double)Dinv[(size_t)k * BS + lane];
        sB[lane] = (double)A[(size_t)bki * BS + lane];
        ++blk;
        __builtin_amdgcn_wave_barrier();
        double p = 0.0;
#pragma unroll
        for (int j = 0; j < 8; ++j) p += sA[r * 8 + j] * sK[j * 8 + c];
        sP[lane] = p;
        __builtin_amdgcn_wave_barrier();
        double q2 = 0.0;
#pragma unroll
        for (int j = 0; j < 8; ++j) q2 += sP[r * 8 + j] * sB[j * 8 + c];
        D -= q2;
        __builtin_amdgcn_wave_barrier();
    }
    // invert D: lanes 0..15 hold the columns of [D | I]
    sP[lane] = D;
    __builtin_amdgcn_wave_barrier();
    double a[8];
#pragma unroll
    for (int rr = 0; rr < 8; ++rr) a[rr] = lane < 8 ? sP[rr * 8 + lane] : ((lane - 8) == rr ? 1.0 : 0.0);
    bool singular = false;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        double col[8];
#pragma unroll
        for (int rr = 0; rr < 8; ++rr) col[rr] = __shfl(a[rr], k);
        int piv = k;
        double best = fabs(col[k]);
#pragma unroll
        for (int rr = k + 1; rr < 8; ++rr) {
            const double tt = fabs(col[rr]);
            if (tt > best) { best = tt; piv = rr; }
        }
#pragma unroll
        for (int rr = k + 1; rr < 8; ++rr)
            if (rr == piv) {
                const double x = a[k]; a[k] = a[rr]; a[rr] = x;
                const double y = col[k]; col[k] = col[rr]; col[rr] = y;
            }
        const double pv = col[k];
        if (!(fabs(pv) > 0.0) || !isfinite(pv)) { singular = true; break; }
        a[k] = a[k] / pv;
#pragma unroll
        for (int rr = 0; rr < 8; ++rr)
            if (rr != k) a[rr] -= col[rr] * a[k];
    }
    if (singular) {
        if (lane == 0) atomicMin(bad, i);
        return;
    }
    if (lane >= 8 && lane < 16) {
#pragma unroll
        for (int rr = 0; rr < 8; ++rr) Dinv[(size_t)i * BS + rr * 8 + (lane - 8)] = (T)a[rr];
    }
}

// Forward sweep of one level: v_i = D_i^-1 (r_i - sum_{k lower} A_ik v_k).
template <class T, class TV>
__global__ void __launch_bounds__(256) bilu0_fwd_level(
    const int32_t* __restrict__ rows, int32_t cnt, int32_t nx, int32_t ny, const int32_t* __restrict__ row_ptr,
    const T* __restrict__ A, const T* __restrict__ Dinv, const TV* rin, TV* v) {
    const int32_t t = (int32_t)((blockIdx.x * blockDim.x + threadIdx.x) >> 3);
    const int r = threadIdx.x & 7;
    const int gbase = threadIdx.x & 56;   // first lane of this row's group in the wavefront
    if (t >= cnt) return;
    const int32_t i = rows[t];
    const int32_t nxy = nx * ny;
    const int32_t ix = i % nx, iy = (i / nx) % ny, iz = i / nxy;
    double acc = (double)rin[(size_t)i * NU + r];
    int32_t blk = row_ptr[i];
    const int32_t lower[3] = {iz > 0 ? i - nxy : -1, iy > 0 ? i - nx : -1, ix > 0 ? i - 1 : -1};
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        const int32_t k = lower[q];
        if (k < 0) continue;
        const T* a = A + (size_t)blk * BS + r * 8;
        const TV* x = v + (size_t)k * NU;
#pragma unroll
        for (int c = 0; c < 8; ++c) acc -= (double)a[c] * (double)x[c];
        ++blk;
    }
    const T* d = Dinv + (size_t)i * BS + r * 8;
    double out = 0.0;
#pragma unroll
    for (int c = 0; c < 8; ++c) out += (double)d[c] * __shfl(acc, gbase + c);
    v[(size_t)i * NU + r] = (TV)out;
}

// Backward sweep of one level (in place over v): z_i = v_i - D_i^-1 sum_{j upper} A_ij z_j.
template <class T, class TV>
__global__ void __launch_bounds__(256) bilu0_bwd_level(
    const int32_t* __restrict__ rows, int32_t cnt, int32_t nx, int32_t ny, int32_t nz,
    const int32_t* __restrict__ diag_pos, const T* __restrict__ A, const T* __restrict__ Dinv,
    TV* z) {
    const int32_t t = (int32_t)((blockIdx.x * blockDim.x + threadIdx.x) >> 3);
    const int r = threadIdx.x & 7;
    const int gbase = threadIdx.x & 56;   // first lane of this row's group in the wavefront
    if (t >= cnt) return;
    const int32_t i = rows[t];
    const int32_t nxy = nx * ny;
    const int32_t ix = i % nx, iy = (i / nx) % ny, iz = i / nxy;
    double acc = 0.0;
    int32_t blk = diag_pos[i] + 1;
    const int32_t upper[3] = {ix + 1 < nx ? i + 1 : -1, iy + 1 < ny ? i + nx : -1,
                              iz + 1 < nz ? i + nxy : -1};
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        const int32_t j = upper[q];
        if (j < 0) continue;
        const T* a = A + (size_t)blk * BS + r * 8;
        const TV* x = z + (size_t)j * NU;
#pragma unroll
        for (int c = 0; c < 8; ++c) acc += (double)a[c] * (double)x[c];
        ++blk;
    }
    const T* d = Dinv + (size_t)i * BS + r * 8;
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < 8; ++c) s += (double)d[c] * __shfl(acc, gbase + c);
    z[(size_t)i * NU + r] = (TV)((double)z[(size_t)i * NU + r] - s);
}

// y = A x for the decoupled matrix (unit diagonal blocks are not read).
template <class T, class TV>
__global__ void __launch_bounds__(256) spmv_unitdiag(int32_t n, const int32_t* __restrict__ row_ptr,
                                                     const int32_t* __restrict__ col_idx,
                                                     const int32_t* __restrict__ diag_pos,
                                                     const T* __restrict__ A, const TV* __restrict__ x,
                                                     TV* __restrict__ y) {
    const int32_t i = (int32_t)((blockIdx.x * blockDim.x + threadIdx.x) >> 3);
    const int r = threadIdx.x & 7;
    if (i >= n) return;
    double acc = (double)x[(size_t)i * NU + r];
    const int32_t b0 = row_ptr[i], b1 = row_ptr[i + 1], dp = diag_pos[i];
    for (int32_t b = b0; b < b1; ++b) {
        if (b == dp) continue;
        const T* a = A + (size_t)b * BS + r * 8;
        const TV* xx = x + (size_t)col_idx[b] * NU;
#pragma unroll
        for (int c = 0; c < 8; ++c) acc += (double)a[c] * (double)xx[c];
    }
    y[(size_t)i * NU + r] = (TV)acc;
}

}  // namespace isc

// ------------------------------------------------------------------ launchers
template <class T>
hipError_t isc_launch_bilu0_factor_t(isc_ctx* ctx, const T* A, T* Dinv, int32_t* bad_dev) {
    for (int32_t s = 0; s < ctx->nlev; ++s) {
        const int32_t off = ctx->lvl_off_h[s], cnt = ctx->lvl_off_h[s + 1] - off;
        hipLaunchKernelGGL(isc::bilu0_factor_level<T>, dim3((cnt + 3) / 4), dim3(256), 0, ctx->stream,
                           ctx->lvl_rows + off, cnt, ctx->g.nx, ctx->g.ny, ctx->g.nz, ctx->row_ptr,
                           ctx->diag_pos, A, Dinv, bad_dev);
    }
    return hipGetLastError();
}

template <class T, class TV>
hipError_t isc_launch_bilu0_apply_t(isc_ctx* ctx, const T* A, const T* Dinv, const TV* r, TV* z) {
    for (int32_t s = 0; s < ctx->nlev; ++s) {
        const int32_t off = ctx->lvl_off_h[s], cnt = ctx->lvl_off_h[s + 1] - off;
        hipLaunchKernelGGL((isc::bilu0_fwd_level<T, TV>), dim3((cnt + 31) / 32), dim3(256), 0, ctx->stream,
                           ctx->lvl_rows + off, cnt, ctx->g.nx, ctx->g.ny, ctx->row_ptr, A, Dinv, r, z);
    }
    for (int32_t s = ctx->nlev - 1; s >= 0; --s) {
        const int32_t off = ctx->lvl_off_h[s], cnt = ctx->lvl_off_h[s + 1] - off;
        hipLaunchKernelGGL((isc::bilu0_bwd_level<T, TV>), dim3((cnt + 31) / 32), dim3(256), 0, ctx->stream,
                           ctx->lvl_rows + off, cnt, ctx->g.nx, ctx->g.ny, ctx->g.nz, ctx->diag_pos, A,
                           Dinv, z);
    }
    return hipGetLastError();
}

template <class T, class TV>
hipError_t isc_launch_spmv_t(isc_ctx* ctx, const T* A, const TV* x, TV* y) {
    const int blocks = (int)(((int64_t)ctx->n * 8 + 255) / 256);
    hipLaunchKernelGGL((isc::spmv_unitdiag<T, TV>), dim3(blocks), dim3(256), 0, ctx->stream, ctx->n,
                       ctx->row_ptr, ctx->col_idx, ctx->diag_pos, A, x, y);
    return hipGetLastError();
}

hipError_t isc_launch_bilu0_factor(isc_ctx* ctx, const double* A, double* Dinv, int32_t* bad) {
    return isc_launch_bilu0_factor_t<double>(ctx, A, Dinv, bad);
}
hipError_t isc_launch_bilu0_factor32(isc_ctx* ctx, const float* A, float* Dinv, int32_t* bad) {
    return isc_launch_bilu0_factor_t<float>(ctx, A, Dinv, bad);
}
hipError_t isc_launch_bilu0_apply(isc_ctx* ctx, const double* A, const double* Dinv, const double* r, double* z) {
    return isc_launch_bilu0_apply_t<double, double>(ctx, A, Dinv, r, z);
}
hipError_t isc_launch_bilu0_apply32(isc_ctx* ctx, const float* A, const float* Dinv, const float* r, float* z) {
    return isc_launch_bilu0_apply_t<float, float>(ctx, A, Dinv, r, z);
}
hipError_t isc_launch_spmv(isc_ctx* ctx, const double* A, const double* x, double* y) {
    return isc_launch_spmv_t<double, double>(ctx, A, x, y);
}
hipError_t isc_launch_spmv32(isc_ctx* ctx, const float* A, const float* x, float* y) {
    return isc_launch_spmv_t<float, float>(ctx, A, x, y);
}
