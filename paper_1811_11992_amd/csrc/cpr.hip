// CPR two-stage preconditioner (the CPR-PF preconditioner of the paper's
// scalability runs, Section 4.3, Example 2) for the decoupled system
// A = C_L J, whose diagonal blocks are the identity:
//   stage 1  e_p ~= A_p^-1 (E^T r): the pressure equation, A_p the scalar
//            matrix of the pressure-row, pressure-column entries (A_ij)[0][0],
//            E^T the pressure component of every cell;
//   stage 2  z = E e_p + M^-1 (r - A E e_p), M the block ILU(0) of A.
// The pressure solve is a few steps of GMRES (krylov.hip) preconditioned by
// one V-cycle of an aggregation multigrid on the structured grid: level l + 1
// lumps 2 x 2 x 2 boxes of level l (ragged at odd sizes), its matrix is the
// Galerkin product P^T A_l P for the piecewise-constant P, which is again a
// 7-point stencil; smoothing is red-black Gauss-Seidel, colour
// (ix + iy + iz) mod 2; the coarse correction is scaled by ISC_CPR_CF; the
// coarsest level (at most ISC_CPR_COARSEST cells) is solved with its inverse,
// formed at set-up.
//
// Storage: each level's stencil is structure-of-arrays, co[d * n + i] with
// d = 0 the diagonal and 1..6 the couplings to the -x, +x, -y, +y, -z, +z
// neighbours (0 outside the grid).  Sums over a row run in ascending
// neighbour order (-z, -y, -x, self, +x, +y, +z).  Stage 1 also keeps
// column 0 of every off-diagonal block (cpr_pc[nnzb][8]) so that A E e_p
// reads 64 bytes per block instead of 512.
#include "common.h"

namespace isc {

enum { ST_D = 0, ST_XM, ST_XP, ST_YM, ST_YP, ST_ZM, ST_ZP };

struct MgLev {
    const double* co;
    int32_t nx, ny, nz, n;
};

// Pressure stencil of level 0 and column 0 of the off-diagonal blocks; eight
// threads per cell, thread r reads row r of each block's column 0.
__global__ void __launch_bounds__(256) cpr_extract(int32_t n, int32_t nx, int32_t ny,
                                                   const int32_t* __restrict__ row_ptr,
                                                   const int32_t* __restrict__ col_idx,
                                                   const double* __restrict__ A, double* __restrict__ co,
                                                   double* __restrict__ pc) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int32_t i = (int32_t)(t >> 3);
    const int r = (int)(t & 7);
    if (i >= n) return;
    const int32_t nxy = nx * ny;
    const int32_t ix = i % nx, iy = (i / nx) % ny, iz = i / nxy;
    double c[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int32_t b = row_ptr[i]; b < row_ptr[i + 1]; ++b) {
        const int32_t j = col_idx[b];
        const double v = A[(size_t)b * BS + r * 8];
        int d = ST_D;
        if (j != i) {
            pc[(size_t)b * 8 + r] = v;
            const int32_t jx = j % nx, jy = (j / nx) % ny, jz = j / nxy;
            d = jx < ix ? ST_XM : jx > ix ? ST_XP : jy < iy ? ST_YM : jy > iy ? ST_YP : jz < iz ? ST_ZM : ST_ZP;
        }
#pragma unroll
        for (int k = 0; k < 7; ++k) c[k] = d == k ? v : c[k];
    }
    if (r == 0) {
#pragma unroll
        for (int k = 0; k < 7; ++k) co[(size_t)k * n + i] = c[k];
    }
}

// Galerkin product of one level: coarse cell I sums the entries of the fine
// rows in its box; a coupling to a cell of the same box goes to the
// diagonal, one to another box to the coarse coupling in that direction.
// Fine cells and each row's entries are taken in ascending order.
__global__ void __launch_bounds__(256) mg_galerkin(MgLev f, double* __restrict__ cco, int32_t cnx, int32_t cny,
                                                   int32_t cnz) {
    const int32_t I = (int32_t)(blockIdx.x * 256 + threadIdx.x);
    const int32_t nc = cnx * cny * cnz;
    if (I >= nc) return;
    const int32_t cx = I % cnx, cy = (I / cnx) % cny, cz = I / (cnx * cny);
    const int32_t n = f.n;
    double a[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int32_t z = 2 * cz; z < 2 * cz + 2 && z < f.nz; ++z)
        for (int32_t y = 2 * cy; y < 2 * cy + 2 && y < f.ny; ++y)
            for (int32_t x = 2 * cx; x < 2 * cx + 2 && x < f.nx; ++x) {
                const int32_t i = x + f.nx * (y + f.ny * z);
                const double* c = f.co + i;
                // -z, -y, -x: inside the box when the coordinate is odd
                if (z & 1) a[ST_D] += c[(size_t)ST_ZM * n]; else a[ST_ZM] += c[(size_t)ST_ZM * n];
                if (y & 1) a[ST_D] += c[(size_t)ST_YM * n]; else a[ST_YM] += c[(size_t)ST_YM * n];
                if (x & 1) a[ST_D] += c[(size_t)ST_XM * n]; else a[ST_XM] += c[(size_t)ST_XM * n];
                a[ST_D] += c[0];
                // +x, +y, +z: inside the box when the coordinate is even and the neighbour exists
                if (!(x & 1) && x + 1 < f.nx) a[ST_D] += c[(size_t)ST_XP * n]; else a[ST_XP] += c[(size_t)ST_XP * n];
                if (!(y & 1) && y + 1 < f.ny) a[ST_D] += c[(size_t)ST_YP * n]; else a[ST_YP] += c[(size_t)ST_YP * n];
                if (!(z & 1) && z + 1 < f.nz) a[ST_D] += c[(size_t)ST_ZP * n]; else a[ST_ZP] += c[(size_t)ST_ZP * n];
            }
#pragma unroll
    for (int k = 0; k < 7; ++k) cco[(size_t)k * nc + I] = a[k];
}

// sum over the off-diagonal entries of row i (cell (x, y, z)) of a_ij x_j,
// split around the diagonal so that callers can keep the ascending order
__device__ __forceinline__ double row_lower(const MgLev& A, int32_t i, int32_t x, int32_t y, int32_t z,
                                            const double* __restrict__ v, double s) {
    const int32_t n = A.n, nxy = A.nx * A.ny;
    if (z > 0) s -= A.co[(size_t)ST_ZM * n + i] * v[i - nxy];
    if (y > 0) s -= A.co[(size_t)ST_YM * n + i] * v[i - A.nx];
    if (x > 0) s -= A.co[(size_t)ST_XM * n + i] * v[i - 1];
    return s;
}
__device__ __forceinline__ double row_upper(const MgLev& A, int32_t i, int32_t x, int32_t y, int32_t z,
                                            const double* __restrict__ v, double s) {
    const int32_t n = A.n, nxy = A.nx * A.ny;
    if (x + 1 < A.nx) s -= A.co[(size_t)ST_XP * n + i] * v[i + 1];
    if (y + 1 < A.ny) s -= A.co[(size_t)ST_YP * n + i] * v[i + A.nx];
    if (z + 1 < A.nz) s -= A.co[(size_t)ST_ZP * n + i] * v[i + nxy];
    return s;
}

// (A v)_i, summed in ascending column order from 0
__device__ __forceinline__ double row_dot(const MgLev& A, int32_t i, int32_t x, int32_t y, int32_t z,
                                          const double* __restrict__ v) {
    const int32_t n = A.n, nxy = A.nx * A.ny;
    double s = 0.0;
    if (z > 0) s += A.co[(size_t)ST_ZM * n + i] * v[i - nxy];
    if (y > 0) s += A.co[(size_t)ST_YM * n + i] * v[i - A.nx];
    if (x > 0) s += A.co[(size_t)ST_XM * n + i] * v[i - 1];
    s += A.co[i] * v[i];
    if (x + 1 < A.nx) s += A.co[(size_t)ST_XP * n + i] * v[i + 1];
    if (y + 1 < A.ny) s += A.co[(size_t)ST_YP * n + i] * v[i + A.nx];
    if (z + 1 < A.nz) s += A.co[(size_t)ST_ZP * n + i] * v[i + nxy];
    return s;
}

// One colour of a red-black Gauss-Seidel sweep: the cells of that colour
// (about half) take x_i = (b_i - sum_{j != i} a_ij x_j) / a_ii.  Thread t
// takes the k-th cell of colour `colour` in grid row (y, z).
__global__ void __launch_bounds__(256) mg_smooth(MgLev A, const double* __restrict__ b, double* __restrict__ x,
                                                 int colour) {
    const int32_t hx = (A.nx + 1) >> 1;
    const int32_t t = (int32_t)(blockIdx.x * 256 + threadIdx.x);
    const int32_t row = t / hx, k = t - row * hx;
    if (row >= A.ny * A.nz) return;
    const int32_t y = row % A.ny, z = row / A.ny;
    const int32_t cx = 2 * k + ((colour + y + z) & 1);
    if (cx >= A.nx) return;
    const int32_t i = cx + A.nx * row;
    double s = row_lower(A, i, cx, y, z, x, b[i]);
    s = row_upper(A, i, cx, y, z, x, s);
    x[i] = s / A.co[i];
}

// Residual of level l restricted to level l + 1: bc_I = sum over the box's
// cells (ascending) of b_i - (A x)_i, (A x)_i summed in ascending order.
__global__ void __launch_bounds__(256) mg_restrict(MgLev A, const double* __restrict__ b,
                                                   const double* __restrict__ x, double* __restrict__ bc,
                                                   int32_t cnx, int32_t cny, int32_t cnz) {
    const int32_t I = (int32_t)(blockIdx.x * 256 + threadIdx.x);
    if (I >= cnx * cny * cnz) return;
    const int32_t cx = I % cnx, cy = (I / cnx) % cny, cz = I / (cnx * cny);
    double acc = 0.0;
    for (int32_t z = 2 * cz; z < 2 * cz + 2 && z < A.nz; ++z)
        for (int32_t y = 2 * cy; y < 2 * cy + 2 && y < A.ny; ++y)
            for (int32_t xx = 2 * cx; xx < 2 * cx + 2 && xx < A.nx; ++xx) {
                const int32_t i = xx + A.nx * (y + A.ny * z);
                acc += b[i] - row_dot(A, i, xx, y, z, x);
            }
    bc[I] = acc;
}

// x_i += cf x_c[agg(i)]
__global__ void __launch_bounds__(256) mg_prolong(int32_t nx, int32_t ny, int32_t nz, double* __restrict__ x,
                                                  const double* __restrict__ xc, int32_t cnx, int32_t cny, double cf) {
    const int32_t i = (int32_t)(blockIdx.x * 256 + threadIdx.x);
    if (i >= nx * ny * nz) return;
    const int32_t ix = i % nx, iy = (i / nx) % ny, iz = i / (nx * ny);
    x[i] += cf * xc[ix / 2 + cnx * (iy / 2 + cny * (iz / 2))];
}

// y = A x on one level (ascending order within each row)
__global__ void __launch_bounds__(256) mg_apply(MgLev A, const double* __restrict__ x, double* __restrict__ y) {
    const int32_t i = (int32_t)(blockIdx.x * 256 + threadIdx.x);
    if (i >= A.n) return;
    const int32_t xx = i % A.nx, yy = (i / A.nx) % A.ny, zz = i / (A.nx * A.ny);
    y[i] = row_dot(A, i, xx, yy, zz, x);
}

__global__ void __launch_bounds__(256) mg_zero(int32_t n, double* __restrict__ x) {
    const int32_t i = (int32_t)(blockIdx.x * 256 + threadIdx.x);
    if (i < n) x[i] = 0.0;
}

// Inverse of the coarsest matrix (n <= 64) by Gauss-Jordan elimination with
// partial pivoting on [A | I], one wavefront, lane t owning row t.  A zero
// pivot raises *bad.
__global__ void __launch_bounds__(64) mg_coarse_invert(MgLev A, double* __restrict__ cinv,
                                                       int32_t* __restrict__ bad) {
    __shared__ double a[ISC_CPR_COARSEST][2 * ISC_CPR_COARSEST];
    const int t = threadIdx.x;
    const int nc = A.n;
    const int w = 2 * nc;
    for (int r = 0; r < nc; ++r)
        for (int c = t; c < w; c += 64) a[r][c] = c == nc + r ? 1.0 : 0.0;
    __syncthreads();
    if (t < nc) {
        const int32_t x = t % A.nx, y = (t / A.nx) % A.ny, z = t / (A.nx * A.ny), nxy = A.nx * A.ny;
        a[t][t] = A.co[t];
        if (x > 0) a[t][t - 1] = A.co[(size_t)ST_XM * nc + t];
        if (x + 1 < A.nx) a[t][t + 1] = A.co[(size_t)ST_XP * nc + t];
        if (y > 0) a[t][t - A.nx] = A.co[(size_t)ST_YM * nc + t];
        if (y + 1 < A.ny) a[t][t + A.nx] = A.co[(size_t)ST_YP * nc + t];
        if (z > 0) a[t][t - nxy] = A.co[(size_t)ST_ZM * nc + t];
        if (z + 1 < A.nz) a[t][t + nxy] = A.co[(size_t)ST_ZP * nc + t];
    }
    __syncthreads();
    for (int k = 0; k < nc; ++k) {
        // pivot: largest |a[r][k]| over r >= k, lowest row on ties (a wave reduction)
        double v = (t >= k && t < nc) ? fabs(a[t][k]) : -1.0;
        int p = t;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const double ov = __shfl_xor(v, o);
            const int op = __shfl_xor(p, o);
            if (ov > v || (ov == v && op < p)) { v = ov; p = op; }
        }
        if (!(v > 0.0)) {
            if (t == 0) atomicMin(bad, 0);
            return;
        }
        for (int c = t; c < w; c += 64) {
            const double s = a[k][c];
            a[k][c] = a[p][c];
            a[p][c] = s;
        }
        __syncthreads();
        const double d = a[k][k];
        __syncthreads();
        for (int c = t; c < w; c += 64) a[k][c] /= d;
        __syncthreads();
        if (t < nc && t != k) {
            const double f = a[t][k];
            for (int c = 0; c < w; ++c) a[t][c] -= f * a[k][c];
        }
        __syncthreads();
    }
    if (t < nc)
        for (int c = 0; c < nc; ++c) cinv[(size_t)t * nc + c] = a[t][nc + c];
}

// x = C^-1 b on the coarsest level, one wavefront
__global__ void __launch_bounds__(64) mg_coarse_solve(const double* __restrict__ cinv, int nc,
                                                      const double* __restrict__ b, double* __restrict__ x) {
    const int t = threadIdx.x;
    if (t >= nc) return;
    double s = 0.0;
    for (int k = 0; k < nc; ++k) s += cinv[(size_t)t * nc + k] * b[k];
    x[t] = s;
}

// rp_i = u_i[0] (the pressure components of a block vector)
__global__ void __launch_bounds__(256) cpr_gather(int32_t n, const double* __restrict__ u, double* __restrict__ rp) {
    const int32_t i = (int32_t)(blockIdx.x * 256 + threadIdx.x);
    if (i < n) rp[i] = u[(size_t)i * NU];
}

// Stage-1 correction: w1 = A E e_p (E e_p holds e_p in the pressure slots) and
// r2 = u - w1; eight threads per cell, thread r forming row r over the
// row's blocks in ascending order (the diagonal block is the identity).
__global__ void __launch_bounds__(256) cpr_stage1(int32_t n, const int32_t* __restrict__ row_ptr,
                                                  const int32_t* __restrict__ col_idx,
                                                  const int32_t* __restrict__ diag_pos,
                                                  const double* __restrict__ pc, const double* __restrict__ ep,
                                                  const double* __restrict__ u, double* __restrict__ w1,
                                                  double* __restrict__ r2) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int32_t i = (int32_t)(t >> 3);
    const int r = (int)(t & 7);
    if (i >= n) return;
    const int32_t dp = diag_pos[i];
    double acc = 0.0;
    for (int32_t b = row_ptr[i]; b < row_ptr[i + 1]; ++b) {
        if (b == dp) {
            if (r == 0) acc += ep[i];
        } else {
            acc += pc[(size_t)b * 8 + r] * ep[col_idx[b]];
        }
    }
    w1[t] = acc;
    r2[t] = u[t] - acc;
}

// z += E e_p and w += w1 (the two stages combined)
__global__ void __launch_bounds__(256) cpr_combine(int32_t n, const double* __restrict__ ep, double* __restrict__ z,
                                                   double* __restrict__ w, const double* __restrict__ w1) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= (int64_t)n * NU) return;
    if ((t & 7) == 0) z[t] += ep[t >> 3];
    w[t] += w1[t];
}

static inline MgLev lev_of(const isc_ctx* ctx, int l) {
    const isc_ctx::MgLevel& L = ctx->mg[l];
    return MgLev{L.co, L.nx, L.ny, L.nz, L.n};
}

static inline dim3 grid_of(int64_t threads) { return dim3((unsigned)((threads + 255) / 256)); }

}  // namespace isc

// Levels of the pressure multigrid for the context's grid (host only).
void isc_cpr_plan(isc_ctx* ctx) {
    ctx->mg.clear();
    int32_t nx = ctx->g.nx, ny = ctx->g.ny, nz = ctx->g.nz;
    while (true) {
        isc_ctx::MgLevel L{};
        L.nx = nx;
        L.ny = ny;
        L.nz = nz;
        L.n = nx * ny * nz;
        ctx->mg.push_back(L);
        if (L.n <= ISC_CPR_COARSEST || (nx == 1 && ny == 1 && nz == 1)) break;
        nx = (nx + 1) / 2;
        ny = (ny + 1) / 2;
        nz = (nz + 1) / 2;
    }
}

// Builds stage 1 for the decoupled matrix A: the pressure stencil, the
// block-column pack, every coarse level and the coarsest inverse.  Launches
// only; a singular coarsest matrix raises *bad_dev (set to 0).
hipError_t isc_cpr_setup(isc_ctx* ctx, const double* A, int32_t* bad_dev) {
    using namespace isc;
    const int32_t n = ctx->n;
    hipLaunchKernelGGL(cpr_extract, grid_of((int64_t)n * 8), dim3(256), 0, ctx->stream, n, ctx->g.nx, ctx->g.ny,
                       ctx->row_ptr, ctx->col_idx, A, ctx->mg[0].co, ctx->cpr_pc);
    const int nl = (int)ctx->mg.size();
    for (int l = 0; l + 1 < nl; ++l) {
        const isc_ctx::MgLevel& C = ctx->mg[l + 1];
        hipLaunchKernelGGL(mg_galerkin, grid_of(C.n), dim3(256), 0, ctx->stream, lev_of(ctx, l), C.co, C.nx, C.ny,
                           C.nz);
    }
    hipLaunchKernelGGL(mg_coarse_invert, dim3(1), dim3(64), 0, ctx->stream, lev_of(ctx, nl - 1), ctx->mg_cinv,
                       bad_dev);
    return hipGetLastError();
}

// x = one V-cycle from level l applied to b (x is overwritten)
static void vcycle(isc_ctx* ctx, int l, const double* b, double* x) {
    using namespace isc;
    const int nl = (int)ctx->mg.size();
    const isc_ctx::MgLevel& L = ctx->mg[l];
    hipStream_t s = ctx->stream;
    if (l == nl - 1) {
        hipLaunchKernelGGL(mg_coarse_solve, dim3(1), dim3(64), 0, s, ctx->mg_cinv, L.n, b, x);
        return;
    }
    const MgLev A = lev_of(ctx, l);
    const dim3 gh = grid_of((int64_t)((L.nx + 1) / 2) * L.ny * L.nz);
    hipLaunchKernelGGL(mg_zero, grid_of(L.n), dim3(256), 0, s, L.n, x);
    for (int k = 0; k < ISC_CPR_NU; ++k) {
        hipLaunchKernelGGL(mg_smooth, gh, dim3(256), 0, s, A, b, x, 0);
        hipLaunchKernelGGL(mg_smooth, gh, dim3(256), 0, s, A, b, x, 1);
    }
    const isc_ctx::MgLevel& C = ctx->mg[l + 1];
    hipLaunchKernelGGL(mg_restrict, grid_of(C.n), dim3(256), 0, s, A, b, (const double*)x, C.b, C.nx, C.ny, C.nz);
    vcycle(ctx, l + 1, C.b, C.x);
    hipLaunchKernelGGL(mg_prolong, grid_of(L.n), dim3(256), 0, s, L.nx, L.ny, L.nz, x, (const double*)C.x, C.nx,
                       C.ny, ISC_CPR_CF);
    for (int k = 0; k < ISC_CPR_NU; ++k) {
        hipLaunchKernelGGL(mg_smooth, gh, dim3(256), 0, s, A, b, x, 1);
        hipLaunchKernelGGL(mg_smooth, gh, dim3(256), 0, s, A, b, x, 0);
    }
}

void isc_cpr_vcycle(isc_ctx* ctx, const double* b, double* x) { vcycle(ctx, 0, b, x); }

// y = A_p x (level 0)
void isc_cpr_pressure_apply(isc_ctx* ctx, const double* x, double* y) {
    hipLaunchKernelGGL(isc::mg_apply, isc::grid_of(ctx->n), dim3(256), 0, ctx->stream, isc::lev_of(ctx, 0), x, y);
}

void isc_cpr_gather(isc_ctx* ctx, const double* u, double* rp) {
    hipLaunchKernelGGL(isc::cpr_gather, isc::grid_of(ctx->n), dim3(256), 0, ctx->stream, ctx->n, u, rp);
}

// w1 = A E e_p, r2 = u - w1
void isc_cpr_stage1(isc_ctx* ctx, const double* ep, const double* u, double* w1, double* r2) {
    hipLaunchKernelGGL(isc::cpr_stage1, isc::grid_of((int64_t)ctx->n * 8), dim3(256), 0, ctx->stream, ctx->n,
                       ctx->row_ptr, ctx->col_idx, ctx->diag_pos, (const double*)ctx->cpr_pc, ep, u, w1, r2);
}

// z += E e_p, w += w1
void isc_cpr_combine(isc_ctx* ctx, const double* ep, double* z, double* w, const double* w1) {
    hipLaunchKernelGGL(isc::cpr_combine, isc::grid_of((int64_t)ctx->n * 8), dim3(256), 0, ctx->stream, ctx->n, ep, z,
                       w, w1);
}
