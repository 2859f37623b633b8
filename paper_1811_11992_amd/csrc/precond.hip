// Block ILU(0) preconditioner and block sparse matrix-vector product for the
// decoupled system A = C_L J (unit diagonal blocks).
//
// On the 7-point stencil two distinct neighbours of a cell are never
// neighbours of each other, so ILU(0) in natural cell order only modifies the
// diagonal blocks: M = (D + L) D^-1 (D + U) with L, U the strict lower and
// upper block parts of A and
//     D_i = I - sum_{k lower neighbour of i} A_ik D_k^-1 A_ki.
// The factor keeps D_i^-1 and the products Lt_ik = A_ik D_k^-1 it forms on the
// way, and the apply uses M = (I + Lt)(D + U):
//     forward   y_i = r_i - sum_{k lower} Lt_ik y_k
//     backward  z_i = D_i^-1 (y_i - sum_{j upper} A_ij z_j),
// which reads seven blocks per row instead of eight (D^-1 once).
// The factor is one cooperative launch over the rows in hyperplane order
// (ix + iy + iz = s), each row awaiting the D_k^-1 of its lower neighbours;
// the triangular sweeps of the apply run as one launch each over 4x4x2 bricks
// of 256 threads (below).  One launch per hyperplane is kept for both as the
// reference schedule.  Every schedule gives the natural-order factorisation
// exactly, bit for bit the same.
//
// Mappings: factor - one wavefront per row, lane (r, c) with LDS-staged 8x8
// products and a column-per-lane Gauss-Jordan inverse; sweeps - one workgroup
// per brick, eight lanes per cell; SpMV - eight lanes per block row, lane r
// owns output row r.
#include <type_traits>

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

// Lt_ik = A_ik D_k^-1 for every lower neighbour k of i, from a given factor
// (the factor kernel forms them itself; this serves an apply with a factor
// computed elsewhere).  One wavefront per row, lane (r, c).
template <class T>
__global__ void __launch_bounds__(256) form_ltilde(int32_t n, int32_t nx, int32_t ny, const int32_t* __restrict__ row_ptr,
                                                   const T* __restrict__ A, const T* __restrict__ Dinv,
                                                   T* __restrict__ Lt, const int32_t* __restrict__ lt_slot) {
    __shared__ double sm[4][2][64];
    const int w = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int32_t i = (int32_t)blockIdx.x * 4 + w;
    if (i >= n) return;
    const int r = lane >> 3, c = lane & 7;
    double* sA = sm[w][0];
    double* sK = sm[w][1];
    const int32_t nxy = nx * ny;
    const int32_t ix = i % nx, iy = (i / nx) % ny, iz = i / nxy;
    const int32_t lower[3] = {iz > 0 ? i - nxy : -1, iy > 0 ? i - nx : -1, ix > 0 ? i - 1 : -1};
    int32_t blk = row_ptr[i];
    for (int q = 0; q < 3; ++q) {
        const int32_t k = lower[q];
        if (k < 0) continue;
        sA[lane] = (double)A[(size_t)blk * BS + lane];
        sK[lane] = (double)Dinv[(size_t)k * BS + lane];
        ++blk;
        __builtin_amdgcn_wave_barrier();
        double p = 0.0;
#pragma unroll
        for (int j = 0; j < 8; ++j) p += sA[r * 8 + j] * sK[j * 8 + c];
        Lt[((size_t)lt_slot[i] * 3 + q) * BS + lane] = (T)p;
        __builtin_amdgcn_wave_barrier();
    }
}

// The backward sweep's and the SpMV's blocks of each cell, copied into the
// packs at the cell's backward-list slot: U x+, U y+, U z+, D^-1 into the
// backward pack, the lower blocks z-, y-, x- into the SpMV pack (a missing
// neighbour's slot is left as it is; the sweeps mask it).  One wavefront per
// cell, one lane per block entry.
template <class T>
__global__ void __launch_bounds__(256) form_packs(int32_t n, int32_t nx, int32_t ny, int32_t nz,
                                                  const int32_t* __restrict__ row_ptr,
                                                  const int32_t* __restrict__ diag_pos, const T* __restrict__ A,
                                                  const T* __restrict__ Dinv, const int32_t* __restrict__ b_slot,
                                                  T* __restrict__ bpack, T* __restrict__ spack) {
    const int w = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int32_t i = (int32_t)blockIdx.x * 4 + w;
    if (i >= n) return;
    const int32_t nxy = nx * ny;
    const int32_t ix = i % nx, iy = (i / nx) % ny, iz = i / nxy;
    const size_t s = (size_t)b_slot[i];
    const bool up[3] = {ix + 1 < nx, iy + 1 < ny, iz + 1 < nz};
    int32_t blk = diag_pos[i] + 1;
    for (int q = 0; q < 3; ++q) {
        if (!up[q]) continue;
        bpack[(s * 4 + q) * BS + lane] = A[(size_t)blk * BS + lane];
        ++blk;
    }
    bpack[(s * 4 + 3) * BS + lane] = Dinv[(size_t)i * BS + lane];
    const bool lo[3] = {iz > 0, iy > 0, ix > 0};
    blk = row_ptr[i];
    for (int q = 0; q < 3; ++q) {
        if (!lo[q]) continue;
        spack[(s * 3 + q) * BS + lane] = A[(size_t)blk * BS + lane];
        ++blk;
    }
}

// Forward sweep of one level: y_i = r_i - sum_{k lower} Lt_ik y_k.
template <class T, class TV>
__global__ void __launch_bounds__(256) bilu0_fwd_level(
    const int32_t* __restrict__ rows, int32_t cnt, int32_t nx, int32_t ny, const T* __restrict__ Lt,
    const int32_t* __restrict__ lt_slot, const TV* rin, TV* y) {
    const int32_t t = (int32_t)((blockIdx.x * blockDim.x + threadIdx.x) >> 3);
    const int r = threadIdx.x & 7;
    if (t >= cnt) return;
    const int32_t i = rows[t];
    const int32_t nxy = nx * ny;
    const int32_t ix = i % nx, iy = (i / nx) % ny, iz = i / nxy;
    double acc = (double)rin[(size_t)i * NU + r];
    const int32_t lower[3] = {iz > 0 ? i - nxy : -1, iy > 0 ? i - nx : -1, ix > 0 ? i - 1 : -1};
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        const int32_t k = lower[q];
        if (k < 0) continue;
        const T* a = Lt + ((size_t)lt_slot[i] * 3 + q) * BS + r * 8;
        const TV* x = y + (size_t)k * NU;
#pragma unroll
        for (int c = 0; c < 8; ++c) acc -= (double)a[c] * (double)x[c];
    }
    y[(size_t)i * NU + r] = (TV)acc;
}

// Backward sweep of one level (in place over y): z_i = D_i^-1 (y_i - sum_{j upper} A_ij z_j),
// the sum formed on its own and then subtracted (as the sync-free sweep does).
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
    double su = 0.0;
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
        for (int c = 0; c < 8; ++c) su += (double)a[c] * (double)x[c];
        ++blk;
    }
    const double acc = (double)z[(size_t)i * NU + r] - su;
    const T* d = Dinv + (size_t)i * BS + r * 8;
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < 8; ++c) s += (double)d[c] * __shfl(acc, gbase + c);
    z[(size_t)i * NU + r] = (TV)s;
}

// The eight entries of a block row or of a cell's vector block, by 16-byte
// loads (a row is 64-byte aligned in FP64 and 32-byte aligned in FP32).
__device__ __forceinline__ void row8(const double* a, double* out) {
    const double2* p = reinterpret_cast<const double2*>(a);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const double2 t = p[k];
        out[2 * k] = t.x;
        out[2 * k + 1] = t.y;
    }
}
__device__ __forceinline__ void row8(const float* a, double* out) {
    const float4* p = reinterpret_cast<const float4*>(a);
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const float4 t = p[k];
        out[4 * k] = (double)t.x;
        out[4 * k + 1] = (double)t.y;
        out[4 * k + 2] = (double)t.z;
        out[4 * k + 3] = (double)t.w;
    }
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
        double a[8], xx[8];
        row8(A + (size_t)b * BS + r * 8, a);
        row8(x + (size_t)col_idx[b] * NU, xx);
#pragma unroll
        for (int c = 0; c < 8; ++c) acc += a[c] * xx[c];
    }
    y[(size_t)i * NU + r] = (TV)acc;
}

// ------------------------------------------------------------ sync-free sweeps
// One kernel per triangular sweep.  The grid is cut into bricks of
// BRICK_X x BRICK_Y x BRICK_Z cells (4x4x2: one workgroup of 256 threads, eight
// per cell), the bricks are listed by brick level bx + by + bz, and the
// workgroups take them in that order: statically under a cooperative launch
// (workgroup b takes entries b, b + grid, ...) or by ticket, so every brick a
// workgroup waits for belongs to one that is already running or finished.
// Inside a brick the cells go through in wavefront steps dx + dy + dz over
// LDS.  No flags: the
// sweep's output buffer holds a NaN sentinel before the sweep, a row's result
// is published with device-coherent 64-/32-bit stores, and a consumer lane
// polls its element of each predecessor with device-coherent loads until the
// sentinel is gone.  The forward sweep writes into a private buffer and sets
// the rows of z back to the sentinel; the backward sweep reads the private
// buffer, restores its sentinel for the next forward sweep, and writes z.
// Every wait is bounded in wall-clock time and stops early once any wait has
// timed out (error flag), so a sweep always terminates.
constexpr uint64_t SENTINEL64 = 0x7FF4DEC0DE5EED01ull;   // NaN payload no arithmetic produces
constexpr uint32_t SENTINEL32 = 0x7FA5EED1u;
#ifndef ISC_SWEEP_SLEEP
#define ISC_SWEEP_SLEEP 1      // s_sleep argument between polls (units of 64 clocks)
#endif
#ifndef ISC_SWEEP_LDS
#define ISC_SWEEP_LDS 0        // dynamic LDS per workgroup: caps resident sweep workgroups per CU
#endif

template <class TV> struct Bits;
template <> struct Bits<double> {
    using U = unsigned long long;
    static constexpr U sentinel = SENTINEL64;
};
template <> struct Bits<float> {
    using U = unsigned int;
    static constexpr U sentinel = SENTINEL32;
};

template <class TV> __device__ __forceinline__ TV from_bits(typename Bits<TV>::U u) {
    return __builtin_bit_cast(TV, u);
}
template <class TV> __device__ __forceinline__ void publish(TV* p, TV v) {
    __hip_atomic_store(reinterpret_cast<typename Bits<TV>::U*>(p), __builtin_bit_cast(typename Bits<TV>::U, v),
                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class TV> __device__ __forceinline__ typename Bits<TV>::U peek(const TV* p) {
    return __hip_atomic_load(reinterpret_cast<const typename Bits<TV>::U*>(p), __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
}
// Given a first read u of *p, polls *p until it no longer holds the sentinel
// (bounded in time: the limit in wall-clock ticks is the uint64 stored right
// after the error flag); returns the value, or 0 after a timeout.
template <class TV> __device__ __forceinline__ TV await_value(const TV* p, typename Bits<TV>::U u, int32_t* err) {
    if (u != Bits<TV>::sentinel) return from_bits<TV>(u);
    const uint64_t t0 = wall_clock64();
    for (int k = 1;; ++k) {
        __builtin_amdgcn_s_sleep(ISC_SWEEP_SLEEP);
        u = peek(p);
        if (u != Bits<TV>::sentinel) return from_bits<TV>(u);
        if ((k & 63) == 0) {
            if (wall_clock64() - t0 > *reinterpret_cast<const uint64_t*>(err + 1)) {
                atomicOr(err, 1);
                return TV(0);
            }
            if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return TV(0);
        }
    }
}

// The workgroup's ticket: its index among the launch's workgroups in the
// order they started.  A ticket below base (a counter that fell behind the
// host's count) reads as n, past every work item, so such a launch does
// nothing rather than index out of range.
__device__ __forceinline__ int32_t take_ticket(unsigned long long* ticket, unsigned long long base, int32_t n) {
    __shared__ int32_t s_t;
    if (threadIdx.x == 0) {
        const unsigned long long d = atomicAdd(ticket, 1ULL) - base;
        s_t = d < (unsigned long long)n ? (int32_t)d : n;
    }
    __syncthreads();
    return s_t;
}

// The work groups of a launch: by ticket (any grid), or, under a cooperative
// launch whose workgroups are all resident at once, statically: workgroup b
// takes groups b, b + grid, ... in order.  The static order needs no atomic:
// the lowest unfinished group's workgroup has finished all its earlier
// groups, so it is working on that group, whose predecessors are all lower.
template <bool STATIC, class Body>
__device__ __forceinline__ void for_each_group(unsigned long long* ticket, unsigned long long base, int32_t n,
                                               Body&& body) {
    if constexpr (STATIC) {
        for (int32_t k = (int32_t)blockIdx.x; k < n; k += (int32_t)gridDim.x) {
            body(k);
            __syncthreads();   // the next group reuses the LDS
        }
    } else {
        const int32_t k = take_ticket(ticket, base, n);
        if (k < n) body(k);
    }
}

// Bricks: a workgroup owns a BRICK_X x BRICK_Y x BRICK_Z brick of cells
// (thread = 8 * g + r, brick cell g = dx + BRICK_X (dy + BRICK_Y dz), block
// row r; the eight rows of a cell share one wavefront).  A brick depends only
// on the bricks below it in x, y and z, so the chain of waits is
// bx + by + bz long (123 on the 200x200x50 grid) instead of ix + iy + iz (448).
// Inside the brick the cells are finished in BRICK_STEPS steps
// (dx + dy + dz = 0, 1, ...), taking in-brick predecessors from LDS; each cell
// still subtracts its neighbours in the order z-, y-, x- (forward) and x+,
// y+, z+ (backward), as the level launches do.
constexpr int BRICK_CELLS = BRICK_X * BRICK_Y * BRICK_Z;
constexpr int BRICK_STEPS = BRICK_X + BRICK_Y + BRICK_Z - 2;
static_assert(BRICK_THREADS % 64 == 0 && BRICK_THREADS <= 1024, "one brick per workgroup of whole wavefronts");

struct BrickCell {
    int32_t i;      // row, or -1 outside the grid
    int32_t ii;     // row clamped to 0
    int g, r, step, dx, dy, dz;
};
__device__ __forceinline__ BrickCell brick_cell(int32_t b, int32_t nbx, int32_t nby, int32_t nx, int32_t ny,
                                                int32_t nz) {
    BrickCell bc;
    // thread within the brick, behind an empty asm so that what derives from it
    // is formed per brick rather than held in registers across a loop over bricks
    int tid = (int)(threadIdx.x % BRICK_THREADS);
    asm volatile("" : "+v"(tid));
    bc.g = tid >> 3;
    bc.r = tid & 7;
    const int32_t bx = b % nbx, by = (b / nbx) % nby, bz = b / (nbx * nby);
    bc.dx = bc.g % BRICK_X;
    bc.dy = (bc.g / BRICK_X) % BRICK_Y;
    bc.dz = bc.g / (BRICK_X * BRICK_Y);
    const int32_t ix = BRICK_X * bx + bc.dx, iy = BRICK_Y * by + bc.dy, iz = BRICK_Z * bz + bc.dz;
    bc.step = bc.dx + bc.dy + bc.dz;
    bc.i = (ix < nx && iy < ny && iz < nz) ? ix + nx * (iy + ny * iz) : -1;
    bc.ii = bc.i >= 0 ? bc.i : 0;
    return bc;
}

// In-brick exchange through LDS: results of the previous steps (double
// buffered, one block barrier per step), accumulators before the D^-1 product
// (exchanged inside a wavefront: LDS operations of one wavefront complete in
// issue order, so a wavefront-scope fence is enough), and the values taken
// from other bricks.
struct alignas(16) BrickLds {
    double v[2][BRICK_CELLS * 8];
    double acc[BRICK_CELLS * 8];
    double ext[3][BRICK_CELLS * 8];
};
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
// the eight doubles at x (LDS, 16-byte aligned)
__device__ __forceinline__ void lds_row8(const double* x, double* out8) {
    const double2* p = reinterpret_cast<const double2*>(x);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const double2 t = p[k];
        out8[2 * k] = t.x;
        out8[2 * k + 1] = t.y;
    }
}

// forward: y_i = r_i - sum_{k lower} Lt_ik y_k for brick b, the entry at
// position pos of the forward list (its L D^-1 blocks are stored there); y is
// the private buffer (sentinel on entry), z_i is reset to the sentinel for the
// backward sweep, and so is w_i when w is given (the fused SpMV's partial sums
// are published there)
template <class T, class TV, bool UPDATE = false>
__device__ __forceinline__ void fwd_brick(int32_t pos, int32_t b, int32_t nbx, int32_t nby, int32_t nx, int32_t ny,
                                          int32_t nz, const T* __restrict__ Lt, const TV* __restrict__ rin, TV* y,
                                          TV* __restrict__ z, TV* w, int32_t* err, BrickLds& L,
                                          const LagUpdateT<TV>& lu = LagUpdateT<TV>{}) {
    const BrickCell bc = brick_cell(b, nbx, nby, nx, ny, nz);
    const int r = bc.r;
    const bool act = bc.i >= 0;
    const int32_t ii = bc.ii;
    const int32_t nxy = nx * ny;
    const int32_t ix = ii % nx, iy = (ii / nx) % ny, iz = ii / nxy;
    const int32_t lower[3] = {iz > 0 ? ii - nxy : -1, iy > 0 ? ii - nx : -1, ix > 0 ? ii - 1 : -1};
    // in-brick predecessor (brick cell index) or -1
    const int inb[3] = {bc.dz > 0 ? bc.g - BRICK_X * BRICK_Y : -1, bc.dy > 0 ? bc.g - BRICK_X : -1,
                        bc.dx > 0 ? bc.g - 1 : -1};
    // everything that does not depend on other rows is loaded first, without
    // branches (the slot of a missing neighbour is read and masked)
    double arow[3][8];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        double x[8];
        row8(Lt + (((size_t)pos * BRICK_CELLS + bc.g) * 3 + q) * BS + r * 8, x);
#pragma unroll
        for (int c = 0; c < 8; ++c) arow[q][c] = lower[q] >= 0 ? x[c] : 0.0;
    }
    double rv;
    if constexpr (UPDATE) {
        const size_t e = (size_t)ii * NU + r;
        const double uo = (double)lu.u[e], wo = (double)lu.w[e];
        double sx = 0.0, zx = 0.0;
        // eight basis rows in flight at a time (the index is clamped so the
        // loads need no branch); summed in the order k = 0, 1, ...
        for (int k0 = 0; k0 < lu.jq; k0 += 8) {
            double q[8];
#pragma unroll
            for (int t = 0; t < 8; ++t) q[t] = (double)lu.Q[(size_t)min(k0 + t, lu.jq - 1) * lu.ldv + e];
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                if (k0 + t < lu.jq) {
                    sx += lu.s[k0 + t] * q[t];
                    zx += lu.z[k0 + t] * q[t];
                }
            }
        }
        const double rom = lu.omz[0] > 0.0 ? 1.0 / lu.omz[0] : 0.0, zeta = lu.omz[1];
        const double qj = (uo - sx) * rom;
        const double un = (wo - zx - zeta * qj) * rom;
        if (act) {
            lu.Q[(size_t)lu.jq * lu.ldv + e] = (TV)qj;
            lu.u[e] = (TV)un;
        }
        rv = act ? (double)(TV)un : 0.0;   // the stored u, as a separate update pass leaves it
    } else {
        rv = act ? (double)rin[(size_t)ii * NU + r] : 0.0;
    }
    if (act) z[(size_t)ii * NU + r] = from_bits<TV>(Bits<TV>::sentinel);
    if (act && w) w[(size_t)ii * NU + r] = from_bits<TV>(Bits<TV>::sentinel);
    // predecessors in other bricks: first reads go out together, then wait
    bool ext[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) ext[q] = act && lower[q] >= 0 && inb[q] < 0;
    typename Bits<TV>::U first[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) first[q] = ext[q] ? peek(y + (size_t)lower[q] * NU + r) : 0;
    double xg[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) xg[q] = ext[q] ? (double)await_value(y + (size_t)lower[q] * NU + r, first[q], err) : 0.0;
    const int me = bc.g * 8 + r;
#pragma unroll
    for (int q = 0; q < 3; ++q) L.ext[q][me] = xg[q];
    double yout = 0.0;
    for (int s = 0; s < BRICK_STEPS; ++s) {
        const int buf = s & 1;
        L.v[buf][me] = yout;
        __syncthreads();
        if (bc.step != s) continue;   // a wavefront with no cell on this step skips it
        double acc = rv;
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const double* src = (lower[q] >= 0 && inb[q] >= 0) ? &L.v[buf][inb[q] * 8] : &L.ext[q][bc.g * 8];
            double x[8];
            lds_row8(src, x);
#pragma unroll
            for (int c = 0; c < 8; ++c) acc -= arow[q][c] * x[c];
        }
        yout = acc;
    }
    if (act) publish(y + (size_t)ii * NU + r, (TV)yout);
}

// backward: z_i = D_i^-1 (y_i - sum_{j upper} A_ij z_j); z holds the sentinel on
// entry, y_i is reset to the sentinel for the next forward sweep.  With w
// given (sentinel on entry), also publishes w_i = z_i + sum_{j upper} A_ij z_j,
// the part of (A z)_i that the sweep has in hand (the diagonal block of the
// decoupled matrix is the identity); the SpMV bricks add the lower part.  The
// blocks U x+, U y+, U z+ and D^-1 of the brick's cells come from the backward
// pack, at the brick's position in the backward list (rank).
template <class T, class TV>
__device__ __forceinline__ void bwd_brick(int32_t rank, int32_t b, int32_t nbx, int32_t nby, int32_t nx, int32_t ny,
                                          int32_t nz, const T* __restrict__ bpack, TV* __restrict__ y, TV* z, TV* w,
                                          int32_t* err, BrickLds& L) {
    const BrickCell bc = brick_cell(b, nbx, nby, nx, ny, nz);
    const int r = bc.r;
    const bool act = bc.i >= 0;
    const int32_t ii = bc.ii;
    const int32_t nxy = nx * ny;
    const int32_t ix = ii % nx, iy = (ii / nx) % ny, iz = ii / nxy;
    const int32_t upper[3] = {ix + 1 < nx ? ii + 1 : -1, iy + 1 < ny ? ii + nx : -1, iz + 1 < nz ? ii + nxy : -1};
    const int inb[3] = {bc.dx < BRICK_X - 1 ? bc.g + 1 : -1, bc.dy < BRICK_Y - 1 ? bc.g + BRICK_X : -1,
                        bc.dz < BRICK_Z - 1 ? bc.g + BRICK_X * BRICK_Y : -1};
    // the slot of a missing neighbour is read and masked
    const T* pk = bpack + ((size_t)rank * BRICK_CELLS + bc.g) * 4 * BS + r * 8;
    double arow[3][8];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        double x[8];
        row8(pk + q * BS, x);
#pragma unroll
        for (int c = 0; c < 8; ++c) arow[q][c] = upper[q] >= 0 ? x[c] : 0.0;
    }
    double drow[8];
    row8(pk + 3 * BS, drow);
    const double yi = act ? (double)y[(size_t)ii * NU + r] : 0.0;
    if (act) y[(size_t)ii * NU + r] = from_bits<TV>(Bits<TV>::sentinel);
    bool ext[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) ext[q] = act && upper[q] >= 0 && inb[q] < 0;
    typename Bits<TV>::U first[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) first[q] = ext[q] ? peek(z + (size_t)upper[q] * NU + r) : 0;
    double xg[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) xg[q] = ext[q] ? (double)await_value(z + (size_t)upper[q] * NU + r, first[q], err) : 0.0;
    const int me = bc.g * 8 + r;
#pragma unroll
    for (int q = 0; q < 3; ++q) L.ext[q][me] = xg[q];
    const int mystep = BRICK_STEPS - 1 - bc.step;
    double zout = 0.0, uz = 0.0;
    for (int s = 0; s < BRICK_STEPS; ++s) {
        const int buf = s & 1;
        L.v[buf][me] = zout;
        __syncthreads();
        if (mystep != s) continue;   // a wavefront with no cell on this step skips it
        // (U z)_i on its own: the fused SpMV reuses it without cancellation
        double su = 0.0;
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const double* src = (upper[q] >= 0 && inb[q] >= 0) ? &L.v[buf][inb[q] * 8] : &L.ext[q][bc.g * 8];
            double x[8];
            lds_row8(src, x);
#pragma unroll
            for (int c = 0; c < 8; ++c) su += arow[q][c] * x[c];
        }
        const double acc = yi - su;
        L.acc[me] = acc;
        wave_lds_sync();
        double a8[8];
        lds_row8(&L.acc[bc.g * 8], a8);
        double t = 0.0;
#pragma unroll
        for (int c = 0; c < 8; ++c) t += drow[c] * a8[c];
        zout = t;
        uz = su;
        wave_lds_sync();
    }
    if (act) publish(z + (size_t)ii * NU + r, (TV)zout);
    if (act && w) publish(w + (size_t)ii * NU + r, (TV)(zout + uz));
}

// w_i += sum_{k lower} A_ik z_k for the cells of one brick: w_i holds the
// sentinel until the backward sweep publishes z_i + sum_{j upper} A_ij z_j
// there, and the lower neighbours' z are read as the sweep publishes them
// (the work list puts the brick after the backward bricks of all its lower
// neighbours).  The three lower rows go through LDS, eight lanes per cell;
// the blocks are added in ascending column order.  The lower blocks come from
// the SpMV pack, at the brick's position in the backward list (rank).
template <class T, class TV>
__device__ __forceinline__ void spmv_lower_brick(int32_t rank, int32_t b, int32_t nbx, int32_t nby, int32_t nx,
                                                 int32_t ny, int32_t nz, const T* __restrict__ spack, const TV* z,
                                                 TV* w, int32_t* err, BrickLds& L) {
    const BrickCell bc = brick_cell(b, nbx, nby, nx, ny, nz);
    const int r = bc.r;
    const bool act = bc.i >= 0;
    const int32_t ii = bc.ii;
    const int32_t nxy = nx * ny;
    const int32_t ix = ii % nx, iy = (ii / nx) % ny, iz = ii / nxy;
    const int32_t lower[3] = {iz > 0 ? ii - nxy : -1, iy > 0 ? ii - nx : -1, ix > 0 ? ii - 1 : -1};
    const int me = bc.g * 8 + r;
    const T* pk = spack + ((size_t)rank * BRICK_CELLS + bc.g) * 3 * BS + r * 8;
    double arow[3][8];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        double x[8];
        row8(pk + k * BS, x);
#pragma unroll
        for (int c = 0; c < 8; ++c) arow[k][c] = lower[k] >= 0 ? x[c] : 0.0;
    }
    typename Bits<TV>::U first[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) first[k] = (act && lower[k] >= 0) ? peek(z + (size_t)lower[k] * NU + r) : 0;
    const typename Bits<TV>::U own0 = act ? peek(w + (size_t)ii * NU + r) : 0;
#pragma unroll
    for (int k = 0; k < 3; ++k)
        L.ext[k][me] =
            (act && lower[k] >= 0) ? (double)await_value(z + (size_t)lower[k] * NU + r, first[k], err) : 0.0;
    double acc = act ? (double)await_value(w + (size_t)ii * NU + r, own0, err) : 0.0;
    wave_lds_sync();
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        double x[8];
        lds_row8(&L.ext[k][bc.g * 8], x);
#pragma unroll
        for (int c = 0; c < 8; ++c) acc += arow[k][c] * x[c];
    }
    if (act) w[(size_t)ii * NU + r] = (TV)acc;
}

// One row of the factor, one wavefront, lane (r, c): D_i = I - sum_k Lt_ik A_ki
// with Lt_ik = A_ik D_k^-1 for the lower neighbours k (stored in sweep order),
// then D_i^-1 by Gauss-Jordan with partial pivoting, a column per lane.  The
// blocks of A that the row needs are loaded first, all six at once, then the
// three D_k^-1: with SF (sync-free) awaited element by element, all three in
// flight together (Dinv holds the sentinel until a row publishes its block),
// and D_i^-1 is published; a singular row publishes zeros so that its
// dependants finish, and reports itself through bad.  Same arithmetic either
// way.  The row also writes the sweep packs (the layout of form_packs): its
// lower blocks, the upper block of each lower neighbour that points at it,
// and D_i^-1.  sm holds 12 tiles of 64 doubles.  The matrix may come in a
// wider type TA than the factor's storage T: its blocks are then rounded to T
// as they are loaded, the values a converted copy would hold.
template <class TA, class T, bool SF>
__device__ __forceinline__ void factor_row(int32_t i, int32_t nx, int32_t ny, int32_t nz,
                                           const int32_t* __restrict__ row_ptr,
                                           const int32_t* __restrict__ diag_pos, const TA* __restrict__ A, T* Dinv,
                                           T* __restrict__ Lt, const int32_t* __restrict__ lt_slot,
                                           const int32_t* __restrict__ b_slot, T* __restrict__ bpack,
                                           T* __restrict__ spack, int32_t* __restrict__ bad, int32_t* err,
                                           double (*sm)[64]) {
    const int lane = threadIdx.x & 63;
    const int r = lane >> 3, c = lane & 7;
    const int32_t nxy = nx * ny;
    const int32_t ix = i % nx, iy = (i / nx) % ny, iz = i / nxy;
    const int32_t lower[3] = {iz > 0 ? i - nxy : -1, iy > 0 ? i - nx : -1, ix > 0 ? i - 1 : -1};
    const int ldir[3] = {2, 1, 0};
    T av[3], bv[3], kv[3];
    int32_t blk = row_ptr[i];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        av[q] = bv[q] = T(0);
        if (lower[q] < 0) continue;
        av[q] = (T)A[(size_t)blk * BS + lane];   // A_ik: the row's lower blocks come first, in this order
        bv[q] = (T)A[(size_t)upper_block(lower[q], ldir[q], nx, ny, nz, diag_pos) * BS + lane];   // A_ki
        ++blk;
    }
    if constexpr (SF) {
        typename Bits<T>::U first[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) first[q] = lower[q] >= 0 ? peek(Dinv + (size_t)lower[q] * BS + lane) : 0;
#pragma unroll
        for (int q = 0; q < 3; ++q)
            kv[q] = lower[q] >= 0 ? await_value(Dinv + (size_t)lower[q] * BS + lane, first[q], err) : T(0);
    } else {
#pragma unroll
        for (int q = 0; q < 3; ++q) kv[q] = lower[q] >= 0 ? Dinv[(size_t)lower[q] * BS + lane] : T(0);
    }
    const size_t si = (size_t)b_slot[i];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        sm[q][lane] = (double)av[q];
        sm[3 + q][lane] = (double)kv[q];
        sm[6 + q][lane] = (double)bv[q];
        if (lower[q] < 0) continue;
        spack[(si * 3 + q) * BS + lane] = av[q];
        bpack[((size_t)b_slot[lower[q]] * 4 + ldir[q]) * BS + lane] = bv[q];
    }
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        if (lower[q] < 0) continue;
        double p = 0.0;
#pragma unroll
        for (int j = 0; j < 8; ++j) p += sm[q][r * 8 + j] * sm[3 + q][j * 8 + c];
        sm[9 + q][lane] = p;
        Lt[((size_t)lt_slot[i] * 3 + q) * BS + lane] = (T)p;
    }
    __builtin_amdgcn_wave_barrier();
    double D = (r == c) ? 1.0 : 0.0;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        if (lower[q] < 0) continue;
        double q2 = 0.0;
#pragma unroll
        for (int j = 0; j < 8; ++j) q2 += sm[9 + q][r * 8 + j] * sm[6 + q][j * 8 + c];
        D -= q2;
    }
    __builtin_amdgcn_wave_barrier();
    double* sP = sm[0];
    // invert D: lanes 0..15 hold the columns of [D | I]
    sP[lane] = D;
    __builtin_amdgcn_wave_barrier();
    double a[8];
#pragma unroll
    for (int rr = 0; rr < 8; ++rr) a[rr] = lane < 8 ? sP[rr * 8 + lane] : ((lane - 8) == rr ? 1.0 : 0.0);
    __builtin_amdgcn_wave_barrier();   // the LDS is reused by the wavefront's next row
    bool singular = false;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        double col[8];
#pragma unroll
        for (int rr = 0; rr < 8; ++rr) col[rr] = read_lane(a[rr], k);
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
        if constexpr (SF) {
            if (lane >= 8 && lane < 16) {
#pragma unroll
                for (int rr = 0; rr < 8; ++rr) publish(Dinv + (size_t)i * BS + rr * 8 + (lane - 8), T(0));
            }
        }
        return;
    }
    if (lane >= 8 && lane < 16) {
#pragma unroll
        for (int rr = 0; rr < 8; ++rr) {
            const T v = (T)a[rr];
            if constexpr (SF)
                publish(Dinv + (size_t)i * BS + rr * 8 + (lane - 8), v);
            else
                Dinv[(size_t)i * BS + rr * 8 + (lane - 8)] = v;
            bpack[(si * 4 + 3) * BS + rr * 8 + (lane - 8)] = v;
        }
    }
}

// The factor by hyperplanes ix + iy + iz = s, one launch each (the reference
// schedule): one wavefront per row of the hyperplane.
template <class T>
__global__ void __launch_bounds__(256) bilu0_factor_level(
    const int32_t* __restrict__ rows, int32_t cnt, int32_t nx, int32_t ny, int32_t nz,
    const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ diag_pos, const T* __restrict__ A,
    T* __restrict__ Dinv, T* __restrict__ Lt, const int32_t* __restrict__ lt_slot,
    const int32_t* __restrict__ b_slot, T* __restrict__ bpack, T* __restrict__ spack, int32_t* __restrict__ bad) {
    __shared__ double sm[4][12][64];
    const int w = threadIdx.x >> 6;
    const int32_t t = blockIdx.x * 4 + w;
    if (t >= cnt) return;
    factor_row<T, T, false>(rows[t], nx, ny, nz, row_ptr, diag_pos, A, Dinv, Lt, lt_slot, b_slot, bpack, spack,
                            bad, nullptr, sm[w]);
}

// The whole factor in one cooperative launch (every wavefront resident): the
// rows in hyperplane order, wavefront t of the grid taking rows t, t + W,
// t + 2W, ... (W = the grid's wavefronts).  The lowest unfinished row's
// wavefront has finished its earlier rows, so it is working on that row, and
// the rows it waits for lie on earlier hyperplanes: no deadlock.  Dinv must
// hold the sentinel on entry.
template <class TA, class T>
__global__ void __launch_bounds__(256) bilu0_factor_syncfree(
    const int32_t* __restrict__ rows, int32_t n, int32_t nx, int32_t ny, int32_t nz,
    const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ diag_pos, const TA* __restrict__ A, T* Dinv,
    T* __restrict__ Lt, const int32_t* __restrict__ lt_slot, const int32_t* __restrict__ b_slot,
    T* __restrict__ bpack, T* __restrict__ spack, int32_t* __restrict__ bad, int32_t* err) {
    __shared__ double sm[4][12][64];
    const int w = threadIdx.x >> 6;
    const int32_t nwave = (int32_t)gridDim.x * 4;
    for (int32_t t = (int32_t)blockIdx.x * 4 + w; t < n; t += nwave)
        factor_row<TA, T, true>(rows[t], nx, ny, nz, row_ptr, diag_pos, A, Dinv, Lt, lt_slot, b_slot, bpack, spack,
                                bad, err, sm[w]);
}

// b = a, element by element, in b's type
template <class TA, class T>
__global__ void __launch_bounds__(256) convert_copy(int64_t len, const TA* __restrict__ a, T* __restrict__ b) {
    for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < len; t += (int64_t)gridDim.x * 256) b[t] = (T)a[t];
}

// One workgroup per group of BPW bricks, taken in brick-list order (statically
// under a cooperative launch, else by ticket).
template <class T, class TV, int BPW, bool STATIC>
__global__ void __launch_bounds__(BRICK_THREADS * BPW) bilu0_fwd_syncfree(
    const int32_t* __restrict__ bricks, int32_t ngroup, int32_t nbx, int32_t nby, int32_t nx, int32_t ny, int32_t nz,
    const T* __restrict__ Lt, const TV* __restrict__ rin, TV* y, TV* __restrict__ z, TV* wreset,
    unsigned long long* ticket, unsigned long long base, int32_t* err) {
    __shared__ BrickLds L[BPW];
    const int h = (int)(threadIdx.x / BRICK_THREADS);
    for_each_group<STATIC>(ticket, base, ngroup, [&](int32_t k) {
        fwd_brick<T, TV>(k * BPW + h, bricks[k * BPW + h], nbx, nby, nx, ny, nz, Lt, rin, y, z, wreset, err, L[h]);
    });
}

// forward sweep preceded, row by row, by the lagged Gram-Schmidt update
template <class T, class TV, int BPW, bool STATIC>
__global__ void __launch_bounds__(BRICK_THREADS * BPW) bilu0_fwd_update_syncfree(
    const int32_t* __restrict__ bricks, int32_t ngroup, int32_t nbx, int32_t nby, int32_t nx, int32_t ny, int32_t nz,
    const T* __restrict__ Lt, LagUpdateT<TV> lu, TV* y, TV* __restrict__ z, TV* wreset,
    unsigned long long* ticket, unsigned long long base, int32_t* err) {
    __shared__ BrickLds L[BPW];
    const int h = (int)(threadIdx.x / BRICK_THREADS);
    for_each_group<STATIC>(ticket, base, ngroup, [&](int32_t k) {
        fwd_brick<T, TV, true>(k * BPW + h, bricks[k * BPW + h], nbx, nby, nx, ny, nz, Lt, nullptr, y, z, wreset,
                               err, L[h], lu);
    });
}

template <class T, class TV, int BPW, bool STATIC>
__global__ void __launch_bounds__(BRICK_THREADS * BPW) bilu0_bwd_syncfree(
    const int32_t* __restrict__ bricks, int32_t ngroup, int32_t nbx, int32_t nby, int32_t nx, int32_t ny, int32_t nz,
    const T* __restrict__ bpack, TV* __restrict__ y, TV* z, unsigned long long* ticket, unsigned long long base,
    int32_t* err) {
    __shared__ BrickLds L[BPW];
    const int h = (int)(threadIdx.x / BRICK_THREADS);
    for_each_group<STATIC>(ticket, base, ngroup, [&](int32_t k) {
        bwd_brick<T, TV>(k * BPW + h, bricks[k * BPW + h], nbx, nby, nx, ny, nz, bpack, y, z, nullptr, err, L[h]);
    });
}

// Backward sweep and w = A z in one launch: the work list interleaves the
// backward bricks (level by level, descending) with SpMV bricks (flag
// SPMV_ITEM), each SpMV brick after the backward bricks of all its
// neighbours, so the SpMV work fills the gaps of the wait chain.  The bricks
// of one workgroup come from one padded group, so they are all backward
// bricks (same block barriers) or all SpMV bricks (none).
constexpr int32_t SPMV_ITEM = 1 << 30;
template <class T, class TV, int BPW, bool STATIC>
__global__ void __launch_bounds__(BRICK_THREADS * BPW) bilu0_bwd_spmv_syncfree(
    const int32_t* __restrict__ items, int32_t ngroup, int32_t nbx, int32_t nby, int32_t nx, int32_t ny, int32_t nz,
    const int32_t* __restrict__ items_rank, const T* __restrict__ bpack, const T* __restrict__ spack,
    TV* __restrict__ y, TV* z, TV* w, unsigned long long* ticket, unsigned long long base, int32_t* err) {
    __shared__ BrickLds L[BPW];
    const int h = (int)(threadIdx.x / BRICK_THREADS);
    for_each_group<STATIC>(ticket, base, ngroup, [&](int32_t k) {
        const int32_t it = items[k * BPW + h];
        const int32_t rank = items_rank[k * BPW + h];
        if (it & SPMV_ITEM)
            spmv_lower_brick<T, TV>(rank, it & (SPMV_ITEM - 1), nbx, nby, nx, ny, nz, spack, z, w, err, L[h]);
        else
            bwd_brick<T, TV>(rank, it, nbx, nby, nx, ny, nz, bpack, y, z, w, err, L[h]);
    });
}

template <class U>
__global__ void fill_bits(int64_t len, U* p, U pattern) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < len) p[k] = pattern;
}

}  // namespace isc

namespace isc {
template <class TV> TV* sweep_buffer(isc_ctx* ctx);
template <> double* sweep_buffer<double>(isc_ctx* ctx) { return ctx->sweep64; }
template <> float* sweep_buffer<float>(isc_ctx* ctx) { return ctx->sweep32; }
// the Lt = L D^-1 blocks of the last factor in each precision
template <class T> T* lt_buffer(isc_ctx* ctx);
template <> double* lt_buffer<double>(isc_ctx* ctx) { return ctx->Lt; }
template <> float* lt_buffer<float>(isc_ctx* ctx) { return ctx->Lt32; }
// the backward and SpMV packs of the last factor in each precision
template <class T> T* bpack_buffer(isc_ctx* ctx);
template <> double* bpack_buffer<double>(isc_ctx* ctx) { return ctx->bpack64; }
template <> float* bpack_buffer<float>(isc_ctx* ctx) { return ctx->bpack32; }
template <class T> T* spack_buffer(isc_ctx* ctx);
template <> double* spack_buffer<double>(isc_ctx* ctx) { return ctx->spack64; }
template <> float* spack_buffer<float>(isc_ctx* ctx) { return ctx->spack32; }
template <class T>
void launch_form_packs(isc_ctx* ctx, const T* A, const T* Dinv) {
    hipLaunchKernelGGL(isc::form_packs<T>, dim3((ctx->n + 3) / 4), dim3(256), 0, ctx->stream, ctx->n, ctx->g.nx,
                       ctx->g.ny, ctx->g.nz, ctx->row_ptr, ctx->diag_pos, A, Dinv, ctx->b_slot,
                       isc::bpack_buffer<T>(ctx), isc::spack_buffer<T>(ctx));
}
}  // namespace isc

// Fills the private sweep buffers with the sentinel (at creation and after a
// sweep gave up, when they may hold stale values).
hipError_t isc_reset_sweep_buffers(isc_ctx* ctx) {
    const int64_t len = (int64_t)ctx->n * isc::NU;
    const int nb = (int)((len + 255) / 256);
    hipLaunchKernelGGL((isc::fill_bits<unsigned long long>), dim3(nb), dim3(256), 0, ctx->stream, len,
                       reinterpret_cast<unsigned long long*>(ctx->sweep64), (unsigned long long)isc::SENTINEL64);
    hipLaunchKernelGGL((isc::fill_bits<unsigned int>), dim3(nb), dim3(256), 0, ctx->stream, len,
                       reinterpret_cast<unsigned int*>(ctx->sweep32), (unsigned int)isc::SENTINEL32);
    return hipGetLastError();
}

// ------------------------------------------------------------------ launchers

// One launch of each sync-free sweep kernel with `BPW` bricks per workgroup
// (the context's choice); each workgroup takes one group of the list at a time.
namespace {
int32_t bricks_x(const isc_ctx* ctx) { return (ctx->g.nx + isc::BRICK_X - 1) / isc::BRICK_X; }
int32_t bricks_y(const isc_ctx* ctx) { return (ctx->g.ny + isc::BRICK_Y - 1) / isc::BRICK_Y; }

// Workgroups of `kernel` that fit on the device at once (cached per context).
int32_t coresident(isc_ctx* ctx, const void* kernel, int threads) {
    for (const auto& e : ctx->grid_cache)
        if (e.first == kernel) return e.second;
    int dev = 0, ncu = 0, per_cu = 0;
    int32_t g = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, ISC_SWEEP_LDS) == hipSuccess)
        g = ncu * per_cu;
    (void)hipGetLastError();
    ctx->grid_cache.emplace_back(kernel, g);
    return g;
}

// One launch of a sync-free sweep kernel over `ngroup` workgroup-sized groups:
// cooperative with a static schedule (grid = the co-resident workgroups, at
// most ngroup) when the context uses it, else one workgroup per group taking
// tickets.  The kernel's arguments after the group count are `args`; the
// ticket pointer, its base and the error flag are appended here.
template <class... Args>
void launch_sweep(isc_ctx* ctx, const void* ticket_kernel, const void* static_kernel, int threads, int32_t ngroup,
                  const int32_t* list, Args... args) {
    unsigned long long* ticket = ctx->ticket;
    unsigned long long base = ctx->ticket_base;
    int32_t* err = ctx->flags + ISC_FLAG_SWEEP;
    int32_t n = ngroup;
    if (ctx->coop) {
        const int32_t cap = coresident(ctx, static_kernel, threads);
        if (cap > 0) {
            const int32_t grid = cap < ngroup ? cap : (ngroup > 0 ? ngroup : 1);
            void* argv[] = {(void*)&list, (void*)&n, (void*)&args..., (void*)&ticket, (void*)&base, (void*)&err};
            if (hipLaunchCooperativeKernel(static_kernel, dim3(grid), dim3(threads), argv, ISC_SWEEP_LDS,
                                           ctx->stream) == hipSuccess)
                return;
            (void)hipGetLastError();   // fall back to tickets
        }
    }
    void* argv[] = {(void*)&list, (void*)&n, (void*)&args..., (void*)&ticket, (void*)&base, (void*)&err};
    (void)hipLaunchKernel(ticket_kernel, dim3(ngroup), dim3(threads), argv, ISC_SWEEP_LDS, ctx->stream);
    ctx->ticket_base += (unsigned long long)ngroup;
}

template <int BPW, class T, class TV>
void launch_fwd(isc_ctx* ctx, const TV* r, TV* v, TV* z, TV* w) {
    const T* Lt = isc::lt_buffer<T>(ctx);
    launch_sweep(ctx, reinterpret_cast<const void*>(&isc::bilu0_fwd_syncfree<T, TV, BPW, false>),
                 reinterpret_cast<const void*>(&isc::bilu0_fwd_syncfree<T, TV, BPW, true>),
                 isc::BRICK_THREADS * BPW, ctx->nfwd_items / BPW, (const int32_t*)ctx->bricks_fwd, bricks_x(ctx),
                 bricks_y(ctx), ctx->g.nx, ctx->g.ny, ctx->g.nz, Lt, r, v, z, w);
}
template <int BPW, class T>
void launch_fwd_update(isc_ctx* ctx, const isc::LagUpdateT<T>& lu, T* v, T* z, T* w) {
    const T* Lt = isc::lt_buffer<T>(ctx);
    launch_sweep(ctx, reinterpret_cast<const void*>(&isc::bilu0_fwd_update_syncfree<T, T, BPW, false>),
                 reinterpret_cast<const void*>(&isc::bilu0_fwd_update_syncfree<T, T, BPW, true>),
                 isc::BRICK_THREADS * BPW, ctx->nfwd_items / BPW, (const int32_t*)ctx->bricks_fwd, bricks_x(ctx),
                 bricks_y(ctx), ctx->g.nx, ctx->g.ny, ctx->g.nz, Lt, lu, v, z, w);
}
template <int BPW, class T, class TV>
void launch_bwd(isc_ctx* ctx, TV* v, TV* z) {
    const T* bpack = isc::bpack_buffer<T>(ctx);
    launch_sweep(ctx, reinterpret_cast<const void*>(&isc::bilu0_bwd_syncfree<T, TV, BPW, false>),
                 reinterpret_cast<const void*>(&isc::bilu0_bwd_syncfree<T, TV, BPW, true>),
                 isc::BRICK_THREADS * BPW, ctx->nbwd_items / BPW, (const int32_t*)ctx->bricks_bwd, bricks_x(ctx),
                 bricks_y(ctx), ctx->g.nx, ctx->g.ny, ctx->g.nz, bpack, v, z);
}
template <int BPW, class T, class TV>
void launch_bwd_spmv(isc_ctx* ctx, TV* v, TV* z, TV* w) {
    const T* bpack = isc::bpack_buffer<T>(ctx);
    const T* spack = isc::spack_buffer<T>(ctx);
    launch_sweep(ctx, reinterpret_cast<const void*>(&isc::bilu0_bwd_spmv_syncfree<T, TV, BPW, false>),
                 reinterpret_cast<const void*>(&isc::bilu0_bwd_spmv_syncfree<T, TV, BPW, true>),
                 isc::BRICK_THREADS * BPW, ctx->nfused_items / BPW, (const int32_t*)ctx->items_bwd_spmv,
                 bricks_x(ctx), bricks_y(ctx), ctx->g.nx, ctx->g.ny, ctx->g.nz, (const int32_t*)ctx->items_rank,
                 bpack, spack, v, z, w);
}
}  // namespace

// The factor of A (type TA) stored in T.  With TA wider than T, At receives A
// converted to T only if the per-hyperplane schedule runs (its sweeps read
// the converted matrix); the sync-free factor rounds the blocks as it loads
// them and leaves At alone.
template <class TA, class T>
hipError_t isc_launch_bilu0_factor_t(isc_ctx* ctx, const TA* A, T* Dinv, int32_t* bad_dev, T* At) {
    bool done = false;
    if (ctx->syncfree) {   // one cooperative launch; Dinv starts as the sentinel
        const int64_t len = (int64_t)ctx->n * isc::BS;
        const int nb = (int)((len + 255) / 256);
        if (sizeof(T) == 8)
            hipLaunchKernelGGL((isc::fill_bits<unsigned long long>), dim3(nb), dim3(256), 0, ctx->stream, len,
                               reinterpret_cast<unsigned long long*>(Dinv), (unsigned long long)isc::SENTINEL64);
        else
            hipLaunchKernelGGL((isc::fill_bits<unsigned int>), dim3(nb), dim3(256), 0, ctx->stream, len,
                               reinterpret_cast<unsigned int*>(Dinv), (unsigned int)isc::SENTINEL32);
        const void* k = reinterpret_cast<const void*>(&isc::bilu0_factor_syncfree<TA, T>);
        const int32_t cap = coresident(ctx, k, 256);
        if (cap > 0) {
            const int32_t rows_n = ctx->n;
            const int32_t grid = cap < (rows_n + 3) / 4 ? cap : (rows_n + 3) / 4;
            const int32_t* rows = ctx->lvl_rows;
            int32_t nx = ctx->g.nx, ny = ctx->g.ny, nz = ctx->g.nz, n = rows_n;
            const int32_t* row_ptr = ctx->row_ptr;
            const int32_t* diag_pos = ctx->diag_pos;
            T* Lt = isc::lt_buffer<T>(ctx);
            const int32_t* lt_slot = ctx->lt_slot;
            const int32_t* b_slot = ctx->b_slot;
            T* bpack = isc::bpack_buffer<T>(ctx);
            T* spack = isc::spack_buffer<T>(ctx);
            int32_t* err = ctx->flags + ISC_FLAG_SWEEP;
            void* argv[] = {(void*)&rows, (void*)&n, (void*)&nx, (void*)&ny, (void*)&nz, (void*)&row_ptr,
                            (void*)&diag_pos, (void*)&A, (void*)&Dinv, (void*)&Lt, (void*)&lt_slot,
                            (void*)&b_slot, (void*)&bpack, (void*)&spack, (void*)&bad_dev, (void*)&err};
            done = hipLaunchCooperativeKernel(k, dim3(grid), dim3(256), argv, 0, ctx->stream) == hipSuccess;
            if (!done) (void)hipGetLastError();   // the level launches below
        }
    }
    if (!done) {
        const T* Al;
        if constexpr (std::is_same<TA, T>::value) {
            Al = A;
        } else {
            const int64_t len = (int64_t)ctx->nnzb * isc::BS;
            hipLaunchKernelGGL((isc::convert_copy<TA, T>), dim3(2048), dim3(256), 0, ctx->stream, len, A, At);
            Al = At;
        }
        for (int32_t s = 0; s < ctx->nlev; ++s) {
            const int32_t off = ctx->lvl_off_h[s], cnt = ctx->lvl_off_h[s + 1] - off;
            hipLaunchKernelGGL(isc::bilu0_factor_level<T>, dim3((cnt + 3) / 4), dim3(256), 0, ctx->stream,
                               ctx->lvl_rows + off, cnt, ctx->g.nx, ctx->g.ny, ctx->g.nz, ctx->row_ptr,
                               ctx->diag_pos, Al, Dinv, isc::lt_buffer<T>(ctx), ctx->lt_slot, ctx->b_slot,
                               isc::bpack_buffer<T>(ctx), isc::spack_buffer<T>(ctx), bad_dev);
        }
    }
    return hipGetLastError();   // the factor wrote the packs
}

template <class T, class TV>
hipError_t isc_launch_bilu0_apply_t(isc_ctx* ctx, const T* A, const T* Dinv, const TV* r, TV* z) {
    if (ctx->syncfree) {
        TV* v = isc::sweep_buffer<TV>(ctx);
        if (ctx->bpw == 2) {
            launch_fwd<2, T, TV>(ctx, r, v, z, (TV*)nullptr);
            launch_bwd<2, T, TV>(ctx, v, z);
        } else {
            launch_fwd<1, T, TV>(ctx, r, v, z, (TV*)nullptr);
            launch_bwd<1, T, TV>(ctx, v, z);
        }
        return hipGetLastError();
    }
    for (int32_t s = 0; s < ctx->nlev; ++s) {
        const int32_t off = ctx->lvl_off_h[s], cnt = ctx->lvl_off_h[s + 1] - off;
        hipLaunchKernelGGL((isc::bilu0_fwd_level<T, TV>), dim3((cnt + 31) / 32), dim3(256), 0, ctx->stream,
                           ctx->lvl_rows + off, cnt, ctx->g.nx, ctx->g.ny, (const T*)isc::lt_buffer<T>(ctx),
                           (const int32_t*)ctx->lt_slot, r, z);
    }
    for (int32_t s = ctx->nlev - 1; s >= 0; --s) {
        const int32_t off = ctx->lvl_off_h[s], cnt = ctx->lvl_off_h[s + 1] - off;
        hipLaunchKernelGGL((isc::bilu0_bwd_level<T, TV>), dim3((cnt + 31) / 32), dim3(256), 0, ctx->stream,
                           ctx->lvl_rows + off, cnt, ctx->g.nx, ctx->g.ny, ctx->g.nz, ctx->diag_pos, A,
                           Dinv, z);
    }
    return hipGetLastError();
}

// z = M^-1 r and w = A z; forward sweep, then the fused backward sweep + SpMV
// (level launches followed by the SpMV when the sync-free sweeps are off).
template <class T, class TV>
hipError_t isc_launch_spmv_t(isc_ctx* ctx, const T* A, const TV* x, TV* y);
template <class T, class TV>
hipError_t isc_launch_bilu0_apply_spmv_t(isc_ctx* ctx, const T* A, const T* Dinv, const TV* r, TV* z, TV* w) {
    if (!ctx->syncfree) {
        const hipError_t e = isc_launch_bilu0_apply_t<T, TV>(ctx, A, Dinv, r, z);
        if (e != hipSuccess) return e;
        return isc_launch_spmv_t<T, TV>(ctx, A, z, w);
    }
    TV* v = isc::sweep_buffer<TV>(ctx);
    if (ctx->bpw == 2) {
        launch_fwd<2, T, TV>(ctx, r, v, z, w);
        launch_bwd_spmv<2, T, TV>(ctx, v, z, w);
    } else {
        launch_fwd<1, T, TV>(ctx, r, v, z, w);
        launch_bwd_spmv<1, T, TV>(ctx, v, z, w);
    }
    return hipGetLastError();
}

// A GMRES iteration with the previous iteration's delayed Gram-Schmidt update
// folded into the forward sweep: writes Q_jq and the new u, then z = M^-1 u
// and w = A z (FP64, or FP32 storage for the inner solver).  Sync-free sweeps
// only.
template <class T>
hipError_t isc_launch_update_apply_spmv_t(isc_ctx* ctx, const T* A, const T* Dinv, const isc::LagUpdateT<T>& lu,
                                          T* z, T* w) {
    T* v = isc::sweep_buffer<T>(ctx);
    if (ctx->bpw == 2) {
        launch_fwd_update<2, T>(ctx, lu, v, z, w);
        launch_bwd_spmv<2, T, T>(ctx, v, z, w);
    } else {
        launch_fwd_update<1, T>(ctx, lu, v, z, w);
        launch_bwd_spmv<1, T, T>(ctx, v, z, w);
    }
    return hipGetLastError();
}
hipError_t isc_launch_update_apply_spmv(isc_ctx* ctx, const double* A, const double* Dinv, const isc::LagUpdate& lu,
                                        double* z, double* w) {
    return isc_launch_update_apply_spmv_t<double>(ctx, A, Dinv, lu, z, w);
}
hipError_t isc_launch_update_apply_spmv32(isc_ctx* ctx, const float* A, const float* Dinv,
                                          const isc::LagUpdateT<float>& lu, float* z, float* w) {
    return isc_launch_update_apply_spmv_t<float>(ctx, A, Dinv, lu, z, w);
}

template <class T, class TV>
hipError_t isc_launch_spmv_t(isc_ctx* ctx, const T* A, const TV* x, TV* y) {
    const int blocks = (int)(((int64_t)ctx->n * 8 + 255) / 256);
    hipLaunchKernelGGL((isc::spmv_unitdiag<T, TV>), dim3(blocks), dim3(256), 0, ctx->stream, ctx->n,
                       ctx->row_ptr, ctx->col_idx, ctx->diag_pos, A, x, y);
    return hipGetLastError();
}

hipError_t isc_launch_bilu0_factor(isc_ctx* ctx, const double* A, double* Dinv, int32_t* bad) {
    return isc_launch_bilu0_factor_t<double, double>(ctx, A, Dinv, bad, nullptr);
}
// FP32 factor of the FP64 matrix A; A32 gets A in FP32 when the
// per-hyperplane schedule needs it (see isc_launch_bilu0_factor_t).
hipError_t isc_launch_bilu0_factor32_from64(isc_ctx* ctx, const double* A, float* A32, float* Dinv, int32_t* bad) {
    return isc_launch_bilu0_factor_t<double, float>(ctx, A, Dinv, bad, A32);
}
// Lt of the context from a factor computed elsewhere (FP64).
hipError_t isc_launch_form_ltilde(isc_ctx* ctx, const double* A, const double* Dinv) {
    hipLaunchKernelGGL(isc::form_ltilde<double>, dim3((ctx->n + 3) / 4), dim3(256), 0, ctx->stream, ctx->n,
                       ctx->g.nx, ctx->g.ny, ctx->row_ptr, A, Dinv, ctx->Lt, (const int32_t*)ctx->lt_slot);
    isc::launch_form_packs<double>(ctx, A, Dinv);
    return hipGetLastError();
}
hipError_t isc_launch_bilu0_apply(isc_ctx* ctx, const double* A, const double* Dinv, const double* r, double* z) {
    return isc_launch_bilu0_apply_t<double, double>(ctx, A, Dinv, r, z);
}
hipError_t isc_launch_bilu0_apply_spmv(isc_ctx* ctx, const double* A, const double* Dinv, const double* r,
                                       double* z, double* w) {
    return isc_launch_bilu0_apply_spmv_t<double, double>(ctx, A, Dinv, r, z, w);
}
hipError_t isc_launch_spmv(isc_ctx* ctx, const double* A, const double* x, double* y) {
    return isc_launch_spmv_t<double, double>(ctx, A, x, y);
}
hipError_t isc_launch_bilu0_apply_spmv32(isc_ctx* ctx, const float* A, const float* Dinv, const float* r, float* z,
                                         float* w) {
    return isc_launch_bilu0_apply_spmv_t<float, float>(ctx, A, Dinv, r, z, w);
}
