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
// Storage: every level keeps its cells colour by colour.  In a grid row
// (y, z) the cells of one colour are every other cell, so cell (x, y, z) sits
// in its colour's array at position (y + ny z) hx + x/2, hx = ceil(nx/2), and
// the colour arrays follow each other (lh = hx ny nz entries each; when nx is
// odd a row's last pair has one cell, and the empty position is a hole that
// holds zeros).  A colour sweep then streams its own colour's coefficients
// and right-hand side, and its neighbours are the other colour's entries at
// the same position (y and z neighbours), or that position and the one before
// or after it (x neighbours).  The stencil is structure-of-arrays over these
// positions, co[d * 2 lh + s] with d = 0 the diagonal and 1..6 the couplings
// to the -x, +x, -y, +y, -z, +z neighbours (0 outside the grid).  Sums over a
// row run in ascending neighbour order (-z, -y, -x, self, +x, +y, +z).  The
// pressure vectors of the GMRES steps use the same order.  Stage 1 also keeps
// column 0 of every off-diagonal block (cpr_pc[nnzb][8]) so that A E e_p
// reads 64 bytes per block instead of 512.
#include <cstdlib>

#include "common.h"

namespace isc {

enum { ST_D = 0, ST_XM, ST_XP, ST_YM, ST_YP, ST_ZM, ST_ZP };

struct MgLev {
    const double* co;   // [7][2 lh]
    int32_t nx, ny, nz;
    int32_t hx;         // positions per grid row and colour
    int32_t lh;         // positions per colour
};

// position of cell (x, y, z) in the colour-split order
__device__ __forceinline__ int32_t sidx(const MgLev& A, int32_t x, int32_t y, int32_t z) {
    return ((x + y + z) & 1) * A.lh + (y + A.ny * z) * A.hx + (x >> 1);
}

// cell of position p of colour c; false for a hole
__device__ __forceinline__ bool sdecode(const MgLev& A, int c, int32_t p, int32_t& x, int32_t& y, int32_t& z) {
    const int32_t row = p / A.hx, k = p - row * A.hx;
    y = row % A.ny;
    z = row / A.ny;
    x = 2 * k + ((c + y + z) & 1);
    return x < A.nx;
}

// Neighbour positions of cell (x, y, z) at position p (within its colour's
// array) in the other colour's array, and whether each neighbour exists.
struct Nbr {
    int32_t zm, ym, xm, xp, yp, zp;
    bool hzm, hym, hxm, hxp, hyp, hzp;
};
__device__ __forceinline__ Nbr neighbours(const MgLev& A, int32_t p, int32_t x, int32_t y, int32_t z) {
    Nbr q;
    const int32_t plane = A.ny * A.hx;
    q.zm = p - plane;
    q.ym = p - A.hx;
    q.xm = (x & 1) ? p : p - 1;
    q.xp = (x & 1) ? p + 1 : p;
    q.yp = p + A.hx;
    q.zp = p + plane;
    q.hzm = z > 0;
    q.hym = y > 0;
    q.hxm = x > 0;
    q.hxp = x + 1 < A.nx;
    q.hyp = y + 1 < A.ny;
    q.hzp = z + 1 < A.nz;
    return q;
}

// Pressure stencil of level 0 and column 0 of the off-diagonal blocks; eight
// threads per cell, thread r reads row r of each block's column 0.
__global__ void __launch_bounds__(256) cpr_extract(int32_t n, MgLev L0, const int32_t* __restrict__ row_ptr,
                                                   const int32_t* __restrict__ col_idx,
                                                   const double* __restrict__ A, double* __restrict__ co,
                                                   double* __restrict__ pc) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int32_t i = (int32_t)(t >> 3);
    const int r = (int)(t & 7);
    if (i >= n) return;
    const int32_t nx = L0.nx, nxy = L0.nx * L0.ny;
    const int32_t ix = i % nx, iy = (i / nx) % L0.ny, iz = i / nxy;
    double c[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int32_t b = row_ptr[i]; b < row_ptr[i + 1]; ++b) {
        const int32_t j = col_idx[b];
        const double v = A[(size_t)b * BS + r * 8];
        int d = ST_D;
        if (j != i) {
            pc[(size_t)b * 8 + r] = v;
            const int32_t jx = j % nx, jy = (j / nx) % L0.ny, jz = j / nxy;
            d = jx < ix ? ST_XM : jx > ix ? ST_XP : jy < iy ? ST_YM : jy > iy ? ST_YP : jz < iz ? ST_ZM : ST_ZP;
        }
#pragma unroll
        for (int k = 0; k < 7; ++k) c[k] = d == k ? v : c[k];
    }
    if (r == 0) {
        const int32_t s = sidx(L0, ix, iy, iz);
        const int64_t ld = 2 * (int64_t)L0.lh;
#pragma unroll
        for (int k = 0; k < 7; ++k) co[k * ld + s] = c[k];
    }
}

// Galerkin product of one level: coarse cell I sums the entries of the fine
// rows in its box; a coupling to a cell of the same box goes to the
// diagonal, one to another box to the coarse coupling in that direction.
// Fine cells (in ascending cell order) and each row's entries are taken in
// ascending order.  One thread per coarse position, both colours.
__global__ void __launch_bounds__(256) mg_galerkin(MgLev f, MgLev C, double* __restrict__ cco) {
    const int32_t t = (int32_t)(blockIdx.x * 256 + threadIdx.x);
    if (t >= 2 * C.lh) return;
    const int cc = t >= C.lh;
    int32_t cx, cy, cz;
    if (!sdecode(C, cc, t - cc * C.lh, cx, cy, cz)) return;
    const int64_t ld = 2 * (int64_t)f.lh;
    double a[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int32_t z = 2 * cz; z < 2 * cz + 2 && z < f.nz; ++z)
        for (int32_t y = 2 * cy; y < 2 * cy + 2 && y < f.ny; ++y)
            for (int32_t x = 2 * cx; x < 2 * cx + 2 && x < f.nx; ++x) {
                const double* c = f.co + sidx(f, x, y, z);
                // -z, -y, -x: inside the box when the coordinate is odd
                if (z & 1) a[ST_D] += c[ST_ZM * ld]; else a[ST_ZM] += c[ST_ZM * ld];
                if (y & 1) a[ST_D] += c[ST_YM * ld]; else a[ST_YM] += c[ST_YM * ld];
                if (x & 1) a[ST_D] += c[ST_XM * ld]; else a[ST_XM] += c[ST_XM * ld];
                a[ST_D] += c[0];
                // +x, +y, +z: inside the box when the coordinate is even and the neighbour exists
                if (!(x & 1) && x + 1 < f.nx) a[ST_D] += c[ST_XP * ld]; else a[ST_XP] += c[ST_XP * ld];
                if (!(y & 1) && y + 1 < f.ny) a[ST_D] += c[ST_YP * ld]; else a[ST_YP] += c[ST_YP * ld];
                if (!(z & 1) && z + 1 < f.nz) a[ST_D] += c[ST_ZP * ld]; else a[ST_ZP] += c[ST_ZP * ld];
            }
    const int64_t cld = 2 * (int64_t)C.lh;
#pragma unroll
    for (int k = 0; k < 7; ++k) cco[k * cld + t] = a[k];
}

// (A v)_s of the cell at position s = cb + p, summed in ascending column order
// from 0; ob is the base of the other colour's array
__device__ __forceinline__ double row_dot(const MgLev& A, int32_t s, const Nbr& q, int32_t ob,
                                          const double* __restrict__ v) {
    const int64_t ld = 2 * (int64_t)A.lh;
    double acc = 0.0;
    if (q.hzm) acc += A.co[ST_ZM * ld + s] * v[ob + q.zm];
    if (q.hym) acc += A.co[ST_YM * ld + s] * v[ob + q.ym];
    if (q.hxm) acc += A.co[ST_XM * ld + s] * v[ob + q.xm];
    acc += A.co[s] * v[s];
    if (q.hxp) acc += A.co[ST_XP * ld + s] * v[ob + q.xp];
    if (q.hyp) acc += A.co[ST_YP * ld + s] * v[ob + q.yp];
    if (q.hzp) acc += A.co[ST_ZP * ld + s] * v[ob + q.zp];
    return acc;
}

// Where the prolongation is folded into a sweep: the coarse correction of a
// fine neighbour, cf x_c[coarse position of the neighbour's box].
struct Prolong {
    const double* xc;
    MgLev C;
    double cf;
};
__device__ __forceinline__ double corrected(const Prolong& P, const double* __restrict__ v, int32_t pos, int32_t x,
                                            int32_t y, int32_t z) {
    return v[pos] + P.cf * P.xc[sidx(P.C, x >> 1, y >> 1, z >> 1)];
}

// One colour of a red-black Gauss-Seidel sweep: the cells of that colour
// take x_i = (b_i - sum_{j != i} a_ij x_j) / a_ii.  mode 0: as written; mode 1
// (the first sweep of a cycle, from x = 0): x_i = b_i / a_ii, no neighbour is
// read; mode 2 (the first sweep after the coarse correction): the neighbours'
// values are read with the correction cf x_c added, which is never stored --
// the other colour's cells are overwritten by the next sweep before anything
// else reads them.
template <int MODE>
__device__ __forceinline__ void smooth_at(const MgLev& A, const double* __restrict__ b, double* __restrict__ xv,
                                          int colour, int32_t p, const Prolong& P) {
    int32_t x, y, z;
    if (!sdecode(A, colour, p, x, y, z)) return;
    const int32_t s = colour * A.lh + p;
    const int32_t ob = (1 - colour) * A.lh;
    double acc = b[s];
    if (MODE != 1) {
        const int64_t ld = 2 * (int64_t)A.lh;
        const Nbr q = neighbours(A, p, x, y, z);
        if (MODE == 0) {
            if (q.hzm) acc -= A.co[ST_ZM * ld + s] * xv[ob + q.zm];
            if (q.hym) acc -= A.co[ST_YM * ld + s] * xv[ob + q.ym];
            if (q.hxm) acc -= A.co[ST_XM * ld + s] * xv[ob + q.xm];
            if (q.hxp) acc -= A.co[ST_XP * ld + s] * xv[ob + q.xp];
            if (q.hyp) acc -= A.co[ST_YP * ld + s] * xv[ob + q.yp];
            if (q.hzp) acc -= A.co[ST_ZP * ld + s] * xv[ob + q.zp];
        } else {
            if (q.hzm) acc -= A.co[ST_ZM * ld + s] * corrected(P, xv, ob + q.zm, x, y, z - 1);
            if (q.hym) acc -= A.co[ST_YM * ld + s] * corrected(P, xv, ob + q.ym, x, y - 1, z);
            if (q.hxm) acc -= A.co[ST_XM * ld + s] * corrected(P, xv, ob + q.xm, x - 1, y, z);
            if (q.hxp) acc -= A.co[ST_XP * ld + s] * corrected(P, xv, ob + q.xp, x + 1, y, z);
            if (q.hyp) acc -= A.co[ST_YP * ld + s] * corrected(P, xv, ob + q.yp, x, y + 1, z);
            if (q.hzp) acc -= A.co[ST_ZP * ld + s] * corrected(P, xv, ob + q.zp, x, y, z + 1);
        }
    }
    xv[s] = acc / A.co[s];
}

template <int MODE>
__global__ void __launch_bounds__(256) mg_smooth(MgLev A, const double* __restrict__ b, double* __restrict__ xv,
                                                 int colour, Prolong P) {
    const int32_t p = (int32_t)(blockIdx.x * 256 + threadIdx.x);
    if (p < A.lh) smooth_at<MODE>(A, b, xv, colour, p, P);
}

// Residual of level l restricted to level l + 1.  The pre-smoothing ends with
// a sweep of colour 1, after which every colour-1 cell satisfies its own
// equation with its neighbours' current values, so the residual is b - A x
// on the colour-0 cells and zero on the others:
// bc_I = sum over the box's colour-0 cells (ascending) of b_i - (A x)_i.
__device__ __forceinline__ void restrict_at(const MgLev& A, const double* __restrict__ b,
                                            const double* __restrict__ xv, double* __restrict__ bc, const MgLev& C,
                                            int32_t t) {
    const int cc = t >= C.lh;
    int32_t cx, cy, cz;
    if (!sdecode(C, cc, t - cc * C.lh, cx, cy, cz)) return;
    double acc = 0.0;
    for (int32_t z = 2 * cz; z < 2 * cz + 2 && z < A.nz; ++z)
        for (int32_t y = 2 * cy; y < 2 * cy + 2 && y < A.ny; ++y)
            for (int32_t x = 2 * cx; x < 2 * cx + 2 && x < A.nx; ++x) {
                if ((x + y + z) & 1) continue;
                const int32_t p = (y + A.ny * z) * A.hx + (x >> 1);
                const Nbr q = neighbours(A, p, x, y, z);
                acc += b[p] - row_dot(A, p, q, A.lh, xv);
            }
    bc[t] = acc;
}

__global__ void __launch_bounds__(256) mg_restrict(MgLev A, const double* __restrict__ b,
                                                   const double* __restrict__ xv, double* __restrict__ bc, MgLev C) {
    const int32_t t = (int32_t)(blockIdx.x * 256 + threadIdx.x);
    if (t < 2 * C.lh) restrict_at(A, b, xv, bc, C, t);
}

// y = A x on one level, every position (holes skipped)
__global__ void __launch_bounds__(256) mg_apply(MgLev A, const double* __restrict__ xv, double* __restrict__ y) {
    const int32_t t = (int32_t)(blockIdx.x * 256 + threadIdx.x);
    if (t >= 2 * A.lh) return;
    const int c = t >= A.lh;
    const int32_t p = t - c * A.lh;
    int32_t x, yy, z;
    if (!sdecode(A, c, p, x, yy, z)) return;
    const Nbr q = neighbours(A, p, x, yy, z);
    y[t] = row_dot(A, t, q, (1 - c) * A.lh, xv);
}

// Inverse of the coarsest matrix (at most ISC_CPR_COARSEST cells, natural
// cell order) by Gauss-Jordan elimination with partial pivoting on [A | I],
// one wavefront, lane t owning row t.  A zero pivot raises *bad.
__global__ void __launch_bounds__(64) mg_coarse_invert(MgLev A, double* __restrict__ cinv,
                                                       int32_t* __restrict__ bad) {
    __shared__ double a[ISC_CPR_COARSEST][2 * ISC_CPR_COARSEST];
    const int t = threadIdx.x;
    const int nxy = A.nx * A.ny;
    const int nc = nxy * A.nz;
    const int w = 2 * nc;
    const int64_t ld = 2 * (int64_t)A.lh;
    for (int r = 0; r < nc; ++r)
        for (int c = t; c < w; c += 64) a[r][c] = c == nc + r ? 1.0 : 0.0;
    __syncthreads();
    if (t < nc) {
        const int32_t x = t % A.nx, y = (t / A.nx) % A.ny, z = t / nxy;
        const int32_t s = sidx(A, x, y, z);
        a[t][t] = A.co[s];
        if (x > 0) a[t][t - 1] = A.co[ST_XM * ld + s];
        if (x + 1 < A.nx) a[t][t + 1] = A.co[ST_XP * ld + s];
        if (y > 0) a[t][t - A.nx] = A.co[ST_YM * ld + s];
        if (y + 1 < A.ny) a[t][t + A.nx] = A.co[ST_YP * ld + s];
        if (z > 0) a[t][t - nxy] = A.co[ST_ZM * ld + s];
        if (z + 1 < A.nz) a[t][t + nxy] = A.co[ST_ZP * ld + s];
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

// x = C^-1 b on the coarsest level, one wavefront; lane t takes the cell t
// of natural order, reading and writing the colour-split positions
__device__ __forceinline__ void coarse_solve_at(const MgLev& A, const double* __restrict__ cinv,
                                                const double* __restrict__ b, double* __restrict__ xv, int t) {
    const int nxy = A.nx * A.ny, nc = nxy * A.nz;
    if (t >= nc) return;
    double s = 0.0;
    for (int k = 0; k < nc; ++k) s += cinv[(size_t)t * nc + k] * b[sidx(A, k % A.nx, (k / A.nx) % A.ny, k / nxy)];
    xv[sidx(A, t % A.nx, (t / A.nx) % A.ny, t / nxy)] = s;
}

__global__ void __launch_bounds__(64) mg_coarse_solve(MgLev A, const double* __restrict__ cinv,
                                                      const double* __restrict__ b, double* __restrict__ xv) {
    coarse_solve_at(A, cinv, b, xv, threadIdx.x);
}

// The V-cycle from level `first` down to the coarsest in one workgroup, for
// levels small enough that one launch per sweep would cost more in launch
// latency than in work.  The same steps as the per-level launches (zero
// start in the first sweep, residual of colour 0, prolongation folded into
// the first post-smoothing sweep), each followed by a workgroup barrier,
// which also makes the global-memory writes of the step visible to the
// whole workgroup.
struct MgChain {
    MgLev lev[ISC_CPR_MAXLEV];
    double* x[ISC_CPR_MAXLEV];
    const double* b[ISC_CPR_MAXLEV];
    double* bw[ISC_CPR_MAXLEV];   // writable right-hand sides of the levels below `first`
    const double* cinv;
    int first, last;
};

constexpr int FUSED_THREADS = 1024;

template <int MODE>
__device__ __forceinline__ void sweep_all(const MgLev& A, const double* b, double* x, int colour, const Prolong& P) {
    for (int32_t p = threadIdx.x; p < A.lh; p += FUSED_THREADS) smooth_at<MODE>(A, b, x, colour, p, P);
    __syncthreads();
}

__global__ void __launch_bounds__(FUSED_THREADS) mg_cycle_fused(MgChain ch) {
    const Prolong none{nullptr, MgLev{}, 0.0};
    for (int l = ch.first; l < ch.last; ++l) {
        const MgLev& A = ch.lev[l];
        sweep_all<1>(A, ch.b[l], ch.x[l], 0, none);
        sweep_all<0>(A, ch.b[l], ch.x[l], 1, none);
        for (int k = 1; k < ISC_CPR_NU; ++k) {
            sweep_all<0>(A, ch.b[l], ch.x[l], 0, none);
            sweep_all<0>(A, ch.b[l], ch.x[l], 1, none);
        }
        const MgLev& C = ch.lev[l + 1];
        for (int32_t t = threadIdx.x; t < 2 * C.lh; t += FUSED_THREADS)
            restrict_at(A, ch.b[l], ch.x[l], ch.bw[l + 1], C, t);
        __syncthreads();
    }
    for (int t = threadIdx.x; t < ISC_CPR_COARSEST; t += FUSED_THREADS)
        coarse_solve_at(ch.lev[ch.last], ch.cinv, ch.b[ch.last], ch.x[ch.last], t);
    __syncthreads();
    for (int l = ch.last - 1; l >= ch.first; --l) {
        const MgLev& A = ch.lev[l];
        const Prolong pro{ch.x[l + 1], ch.lev[l + 1], ISC_CPR_CF};
        sweep_all<2>(A, ch.b[l], ch.x[l], 1, pro);
        sweep_all<0>(A, ch.b[l], ch.x[l], 0, none);
        for (int k = 1; k < ISC_CPR_NU; ++k) {
            sweep_all<0>(A, ch.b[l], ch.x[l], 1, none);
            sweep_all<0>(A, ch.b[l], ch.x[l], 0, none);
        }
    }
}

// rp = the pressure components of a block vector, in colour-split order
__global__ void __launch_bounds__(256) cpr_gather(int32_t n, MgLev L0, const double* __restrict__ u,
                                                  double* __restrict__ rp) {
    const int32_t i = (int32_t)(blockIdx.x * 256 + threadIdx.x);
    if (i >= n) return;
    const int32_t nxy = L0.nx * L0.ny;
    rp[sidx(L0, i % L0.nx, (i / L0.nx) % L0.ny, i / nxy)] = u[(size_t)i * NU];
}

// Stage-1 correction: w1 = A E e_p (E e_p holds e_p in the pressure slots) and
// r2 = u - w1; eight threads per cell, thread r forming row r over the
// row's blocks in ascending order (the diagonal block is the identity).
__global__ void __launch_bounds__(256) cpr_stage1(int32_t n, MgLev L0, const int32_t* __restrict__ row_ptr,
                                                  const int32_t* __restrict__ col_idx,
                                                  const int32_t* __restrict__ diag_pos,
                                                  const double* __restrict__ pc, const double* __restrict__ ep,
                                                  const double* __restrict__ u, double* __restrict__ w1,
                                                  double* __restrict__ r2) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int32_t i = (int32_t)(t >> 3);
    const int r = (int)(t & 7);
    if (i >= n) return;
    const int32_t nxy = L0.nx * L0.ny;
    const int32_t dp = diag_pos[i];
    double acc = 0.0;
    for (int32_t b = row_ptr[i]; b < row_ptr[i + 1]; ++b) {
        const int32_t j = col_idx[b];
        const double e = ep[sidx(L0, j % L0.nx, (j / L0.nx) % L0.ny, j / nxy)];
        if (b == dp) {
            if (r == 0) acc += e;
        } else {
            acc += pc[(size_t)b * 8 + r] * e;
        }
    }
    w1[t] = acc;
    r2[t] = u[t] - acc;
}

// z += E e_p and w += w1 (the two stages combined)
__global__ void __launch_bounds__(256) cpr_combine(int32_t n, MgLev L0, const double* __restrict__ ep,
                                                   double* __restrict__ z, double* __restrict__ w,
                                                   const double* __restrict__ w1) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= (int64_t)n * NU) return;
    if ((t & 7) == 0) {
        const int32_t i = (int32_t)(t >> 3), nxy = L0.nx * L0.ny;
        z[t] += ep[sidx(L0, i % L0.nx, (i / L0.nx) % L0.ny, i / nxy)];
    }
    w[t] += w1[t];
}

// natural order -> colour-split order (TO_SPLIT) or back
template <bool TO_SPLIT>
__global__ void __launch_bounds__(256) cpr_permute(int32_t n, MgLev L0, const double* __restrict__ src,
                                                   double* __restrict__ dst) {
    const int32_t i = (int32_t)(blockIdx.x * 256 + threadIdx.x);
    if (i >= n) return;
    const int32_t nxy = L0.nx * L0.ny;
    const int32_t s = sidx(L0, i % L0.nx, (i / L0.nx) % L0.ny, i / nxy);
    if (TO_SPLIT) dst[s] = src[i];
    else dst[i] = src[s];
}

static inline MgLev lev_of(const isc_ctx* ctx, int l) {
    const isc_ctx::MgLevel& L = ctx->mg[l];
    return MgLev{L.co, L.nx, L.ny, L.nz, L.hx, L.lh};
}

static inline dim3 grid_of(int64_t threads) { return dim3((unsigned)((threads + 255) / 256)); }

}  // namespace isc

// first level cycled by the one-workgroup kernel: the largest level with
// at most ISC_CPR_FUSED_MAX positions, or the coarsest
static void choose_fused(isc_ctx* ctx) {
    const int nl = (int)ctx->mg.size();
    int64_t lim = ISC_CPR_FUSED_MAX;
    if (const char* e = getenv("ISC_CPR_FUSED_MAX")) lim = strtoll(e, nullptr, 10);
    ctx->mg_fused_first = nl - 1;
    for (int l = 0; l < nl; ++l)
        if (2 * (int64_t)ctx->mg[l].lh <= lim) {
            ctx->mg_fused_first = l;
            break;
        }
}

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
        L.hx = (nx + 1) / 2;
        L.lh = L.hx * ny * nz;
        ctx->mg.push_back(L);
        if (L.n <= ISC_CPR_COARSEST || (nx == 1 && ny == 1 && nz == 1)) break;
        if ((int)ctx->mg.size() >= ISC_CPR_MAXLEV) break;
        nx = (nx + 1) / 2;
        ny = (ny + 1) / 2;
        nz = (nz + 1) / 2;
    }
    choose_fused(ctx);
}

// Builds stage 1 for the decoupled matrix A: the pressure stencil, the
// block-column pack, every coarse level and the coarsest inverse.  Launches
// only; a singular coarsest matrix raises *bad_dev (set to 0).
hipError_t isc_cpr_setup(isc_ctx* ctx, const double* A, int32_t* bad_dev) {
    using namespace isc;
    const int32_t n = ctx->n;
    hipLaunchKernelGGL(cpr_extract, grid_of((int64_t)n * 8), dim3(256), 0, ctx->stream, n, lev_of(ctx, 0),
                       ctx->row_ptr, ctx->col_idx, A, ctx->mg[0].co, ctx->cpr_pc);
    const int nl = (int)ctx->mg.size();
    for (int l = 0; l + 1 < nl; ++l) {
        const isc_ctx::MgLevel& C = ctx->mg[l + 1];
        hipLaunchKernelGGL(mg_galerkin, grid_of(2 * (int64_t)C.lh), dim3(256), 0, ctx->stream, lev_of(ctx, l),
                           lev_of(ctx, l + 1), C.co);
    }
    hipLaunchKernelGGL(mg_coarse_invert, dim3(1), dim3(64), 0, ctx->stream, lev_of(ctx, nl - 1), ctx->mg_cinv,
                       bad_dev);
    return hipGetLastError();
}

// x = one V-cycle from level l applied to b (x is overwritten)
static void vcycle(isc_ctx* ctx, int l, const double* b, double* x) {
    using namespace isc;
    static_assert(ISC_CPR_NU >= 1, "the sweeps carry the zero start and the prolongation");
    const int nl = (int)ctx->mg.size();
    const isc_ctx::MgLevel& L = ctx->mg[l];
    hipStream_t s = ctx->stream;
    const MgLev A = lev_of(ctx, l);
    if (l >= ctx->mg_fused_first) {   // this level and all below in one workgroup
        MgChain ch{};
        for (int k = l; k < nl; ++k) {
            ch.lev[k] = lev_of(ctx, k);
            ch.x[k] = k == l ? x : ctx->mg[k].x;
            ch.b[k] = k == l ? b : ctx->mg[k].b;
            ch.bw[k] = ctx->mg[k].b;
        }
        ch.cinv = ctx->mg_cinv;
        ch.first = l;
        ch.last = nl - 1;
        hipLaunchKernelGGL(mg_cycle_fused, dim3(1), dim3(FUSED_THREADS), 0, s, ch);
        return;
    }
    const dim3 gh = grid_of(L.lh);
    const Prolong none{nullptr, MgLev{}, 0.0};
    // pre-smoothing from x = 0: colours 0, 1, then nu - 1 more pairs
    hipLaunchKernelGGL(mg_smooth<1>, gh, dim3(256), 0, s, A, b, x, 0, none);
    hipLaunchKernelGGL(mg_smooth<0>, gh, dim3(256), 0, s, A, b, x, 1, none);
    for (int k = 1; k < ISC_CPR_NU; ++k) {
        hipLaunchKernelGGL(mg_smooth<0>, gh, dim3(256), 0, s, A, b, x, 0, none);
        hipLaunchKernelGGL(mg_smooth<0>, gh, dim3(256), 0, s, A, b, x, 1, none);
    }
    const isc_ctx::MgLevel& C = ctx->mg[l + 1];
    const MgLev Cl = lev_of(ctx, l + 1);
    hipLaunchKernelGGL(mg_restrict, grid_of(2 * (int64_t)C.lh), dim3(256), 0, s, A, b, (const double*)x, C.b, Cl);
    vcycle(ctx, l + 1, C.b, C.x);
    // post-smoothing: colours 1, 0 (the first reading the corrected colour-0 values), nu - 1 more pairs
    const Prolong pro{C.x, Cl, ISC_CPR_CF};
    hipLaunchKernelGGL(mg_smooth<2>, gh, dim3(256), 0, s, A, b, x, 1, pro);
    hipLaunchKernelGGL(mg_smooth<0>, gh, dim3(256), 0, s, A, b, x, 0, none);
    for (int k = 1; k < ISC_CPR_NU; ++k) {
        hipLaunchKernelGGL(mg_smooth<0>, gh, dim3(256), 0, s, A, b, x, 1, none);
        hipLaunchKernelGGL(mg_smooth<0>, gh, dim3(256), 0, s, A, b, x, 0, none);
    }
}

void isc_cpr_vcycle(isc_ctx* ctx, const double* b, double* x) { vcycle(ctx, 0, b, x); }

// y = A_p x (level 0, colour-split order)
void isc_cpr_pressure_apply(isc_ctx* ctx, const double* x, double* y) {
    hipLaunchKernelGGL(isc::mg_apply, isc::grid_of(2 * (int64_t)ctx->mg[0].lh), dim3(256), 0, ctx->stream,
                       isc::lev_of(ctx, 0), x, y);
}

void isc_cpr_gather(isc_ctx* ctx, const double* u, double* rp) {
    hipLaunchKernelGGL(isc::cpr_gather, isc::grid_of(ctx->n), dim3(256), 0, ctx->stream, ctx->n,
                       isc::lev_of(ctx, 0), u, rp);
}

// a pressure vector between natural cell order ([n]) and the colour-split order
void isc_cpr_to_split(isc_ctx* ctx, const double* nat, double* split) {
    hipLaunchKernelGGL(isc::cpr_permute<true>, isc::grid_of(ctx->n), dim3(256), 0, ctx->stream, ctx->n,
                       isc::lev_of(ctx, 0), nat, split);
}
void isc_cpr_from_split(isc_ctx* ctx, const double* split, double* nat) {
    hipLaunchKernelGGL(isc::cpr_permute<false>, isc::grid_of(ctx->n), dim3(256), 0, ctx->stream, ctx->n,
                       isc::lev_of(ctx, 0), split, nat);
}

// w1 = A E e_p, r2 = u - w1
void isc_cpr_stage1(isc_ctx* ctx, const double* ep, const double* u, double* w1, double* r2) {
    hipLaunchKernelGGL(isc::cpr_stage1, isc::grid_of((int64_t)ctx->n * 8), dim3(256), 0, ctx->stream, ctx->n,
                       isc::lev_of(ctx, 0), ctx->row_ptr, ctx->col_idx, ctx->diag_pos, (const double*)ctx->cpr_pc, ep,
                       u, w1, r2);
}

// z += E e_p, w += w1
void isc_cpr_combine(isc_ctx* ctx, const double* ep, double* z, double* w, const double* w1) {
    hipLaunchKernelGGL(isc::cpr_combine, isc::grid_of((int64_t)ctx->n * 8), dim3(256), 0, ctx->stream, ctx->n,
                       isc::lev_of(ctx, 0), ep, z, w, w1);
}
