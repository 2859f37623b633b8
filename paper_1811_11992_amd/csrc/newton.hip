// Newton update with safeguards and the scaled convergence norm.
//
// Update (saturation treatment of the PER subsection): a saturation driven
// negative by the Newton step is replaced by half of its previous value; the
// same rule is used for the primary mole fractions (and, at the top, half way
// to one) and for C_c; if S_o = 1 - S_w - S_g would become negative the
// (S_w, S_g) increments are scaled so that S_o halves.  Before these rules
// each increment is clipped to a per-variable step limit (|dp| <= 0.2 |p|,
// |dT| <= 50 K, fractions and saturations 0.2, C_c 1000 mol/m^3) - a reading:
// the paper names only the saturation treatment.
//
// Norm: max over cells and rows of |F| / s with s = V phi_ref rho_ref,W / dt
// for molar and coke rows and s = V (1 - phi_ref) cp_rock (1 K) / dt for the
// energy row.
#include <cmath>
#include <mutex>
#include <string>

#include "common.h"

namespace isc {

__global__ void __launch_bounds__(256) update_kernel(int32_t n, double* __restrict__ u,
                                                     const double* __restrict__ du, int32_t* __restrict__ flag) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double lim[8] = {0.2, 0.2, 0.2, 0.2, 50.0, 0.2, 0.2, 1000.0};
    double o[8], v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        o[k] = u[(size_t)k * n + i];
        double d = du[(size_t)i * NU + k];
        const double L = k == 0 ? lim[0] * fabs(o[0]) : lim[k];
        d = d > L ? L : (d < -L ? -L : d);
        v[k] = o[k] + d;
    }
#pragma unroll
    for (int k = 1; k <= 3; ++k) {
        if (v[k] < 0.0) v[k] = 0.5 * o[k];
        else if (v[k] > 1.0) v[k] = 0.5 * (1.0 + o[k]);
    }
    if (v[5] < 0.0) v[5] = 0.5 * o[5];
    if (v[6] < 0.0) v[6] = 0.5 * o[6];
    if (1.0 - v[5] - v[6] < 0.0) {
        const double th = 0.5 * (1.0 - o[5] - o[6]) / ((v[5] - o[5]) + (v[6] - o[6]));
        v[5] = o[5] + th * (v[5] - o[5]);
        v[6] = o[6] + th * (v[6] - o[6]);
    }
    if (v[7] < 0.0) v[7] = 0.5 * o[7];
    bool bad = false;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        bad |= !isfinite(v[k]);
        u[(size_t)k * n + i] = v[k];
    }
    if (bad) atomicOr(flag, 1);
}

__device__ __forceinline__ double nanmax(double a, double b) { return (b > a || isnan(b)) ? b : a; }

// max over the eight rows of cell i of |F_e,i| / s_e,i, folded into m
__device__ __forceinline__ double cell_scaled_max(double m, const double* __restrict__ F,
                                                  const double* __restrict__ poro, int32_t i, double v_dt,
                                                  double rho_w, double cp_rock) {
    const double ph = poro[i];
    const double sm = v_dt * ph * rho_w, se = v_dt * (1.0 - ph) * cp_rock;
#pragma unroll
    for (int e = 0; e < 8; ++e) m = nanmax(m, fabs(F[(size_t)i * NU + e]) / (e == 6 ? se : sm));
    return m;
}

// workgroup maximum of m (256 threads), written to partial[blockIdx.x]
__device__ __forceinline__ void block_max_store(double m, double* __restrict__ partial) {
    __shared__ double red[4];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = nanmax(m, __shfl_xor(m, o));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) partial[blockIdx.x] = nanmax(nanmax(red[0], red[1]), nanmax(red[2], red[3]));
}

__global__ void __launch_bounds__(256) scaled_norm_partial(int32_t n, const double* __restrict__ F,
                                                           const double* __restrict__ poro, double v_dt,
                                                           double rho_w, double cp_rock,
                                                           double* __restrict__ partial) {
    double m = 0.0;
    for (int32_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256)
        m = cell_scaled_max(m, F, poro, i, v_dt, rho_w, cp_rock);
    block_max_store(m, partial);
}

// The same partial maxima with a fixed share per workgroup: workgroup b
// covers cells [b NORM_CELLS_PER_WG, (b + 1) NORM_CELLS_PER_WG), so the
// number of partials, ceil(n / NORM_CELLS_PER_WG), grows with the grid.
constexpr int32_t NORM_CELLS_PER_WG = 2048;
__global__ void __launch_bounds__(256) scaled_norm_partial_fixed(int32_t n, const double* __restrict__ F,
                                                                 const double* __restrict__ poro, double v_dt,
                                                                 double rho_w, double cp_rock,
                                                                 double* __restrict__ partial) {
    double m = 0.0;
    const int32_t base = blockIdx.x * NORM_CELLS_PER_WG;
#pragma unroll
    for (int k = 0; k < NORM_CELLS_PER_WG / 256; ++k) {
        const int32_t i = base + k * 256 + (int32_t)threadIdx.x;
        if (i < n) m = cell_scaled_max(m, F, poro, i, v_dt, rho_w, cp_rock);
    }
    block_max_store(m, partial);
}

__global__ void __launch_bounds__(256) max_partials(const double* __restrict__ partial, int nblk,
                                                    double* __restrict__ out) {
    __shared__ double red[4];
    double m = 0.0;
    for (int b = threadIdx.x; b < nblk; b += 256) m = nanmax(m, partial[b]);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = nanmax(m, __shfl_xor(m, o));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) *out = nanmax(nanmax(red[0], red[1]), nanmax(red[2], red[3]));
}

__global__ void __launch_bounds__(256) negate_copy(int64_t len, const double* __restrict__ x, double* __restrict__ y) {
    for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < len; t += (int64_t)gridDim.x * 256) y[t] = -x[t];
}

}  // namespace isc

hipError_t isc_launch_update(isc_ctx* ctx, double* u, const double* du, int32_t* flag_dev) {
    hipLaunchKernelGGL(isc::update_kernel, dim3((ctx->n + 255) / 256), dim3(256), 0, ctx->stream, ctx->n, u,
                       du, flag_dev);
    return hipGetLastError();
}

hipError_t isc_launch_scaled_norm(isc_ctx* ctx, const double* F, double dt, double* out_dev) {
    const double V = ctx->g.dx * ctx->g.dy * ctx->g.dz;
    int nb = (ctx->n + 255) / 256;
    nb = nb > isc::NPART ? isc::NPART : nb;
    hipLaunchKernelGGL(isc::scaled_norm_partial, dim3(nb), dim3(256), 0, ctx->stream, ctx->n, F, ctx->poro,
                       V / dt, ctx->fluid_h.rho_ref[0], ctx->fluid_h.cp_rock, ctx->partial);
    hipLaunchKernelGGL(isc::max_partials, dim3(1), dim3(256), 0, ctx->stream, ctx->partial, nb, out_dev);
    return hipGetLastError();
}

hipError_t isc_launch_negate(isc_ctx* ctx, const double* x, double* y) {
    const int64_t len = (int64_t)ctx->n * isc::NU;
    int64_t nb = (len + 255) / 256;
    nb = nb > isc::NPART ? isc::NPART : nb;
    hipLaunchKernelGGL(isc::negate_copy, dim3((int)nb), dim3(256), 0, ctx->stream, len, x, y);
    return hipGetLastError();
}

// ------------------------------------------------ allocation-free scaled norm
// For callers that cannot allocate device memory: the partial maxima live in
// a file-scope device array instead of a context's workspace.  Each device
// the library runs on holds its own copy until the process ends.
namespace isc {
constexpr int32_t NOALLOC_PARTIALS = ISC_NOALLOC_MAX_CELLS / NORM_CELLS_PER_WG;   // 8192 doubles, 64 KiB
static_assert(ISC_NOALLOC_MAX_CELLS % NORM_CELLS_PER_WG == 0, "whole workgroups");
static __device__ __align__(256) double scratch[NOALLOC_PARTIALS];
}  // namespace isc

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double* g_scratch_dev[MAX_DEVICES] = {};   // device address of isc::scratch, per device

// Device address of the scratch array on device dev (current), resolved once
// per device.  The array's name is only a host-side stand-in: host code uses
// this address, never the name.
hipError_t scratch_on(int dev, double** out) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(isc::scratch));
        if (e != hipSuccess) return e;
        g_scratch_dev[dev] = static_cast<double*>(p);
    }
    *out = g_scratch_dev[dev];
    return hipSuccess;
}
}  // namespace

extern "C" isc_status isc_scaled_norm_noalloc(const isc_grid* grid_h, const isc_fluid* fluid_h, const double* poro,
                                              const double* F, double dt, double* res, void* hip_stream) {
    if (!grid_h || !fluid_h || !poro || !F || !res || !(dt > 0)) {
        isc_set_noctx_error("isc_scaled_norm_noalloc: null argument or dt <= 0");
        return ISC_ERR_ARG;
    }
    const isc_grid& g = *grid_h;
    if (g.nx < 1 || g.ny < 1 || g.nz < 1 || !(g.dx > 0) || !(g.dy > 0) || !(g.dz > 0)) {
        isc_set_noctx_error("isc_scaled_norm_noalloc: invalid grid");
        return ISC_ERR_ARG;
    }
    const int64_t n = (int64_t)g.nx * g.ny * g.nz;
    if (n > ISC_NOALLOC_MAX_CELLS) {
        isc_set_noctx_error(("isc_scaled_norm_noalloc: " + std::to_string(n) + " cells exceed the maximum of " +
                             std::to_string(ISC_NOALLOC_MAX_CELLS) + " (the fixed partial-maximum buffer)")
                                .c_str());
        return ISC_ERR_ARG;
    }
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) {
        isc_set_noctx_error("isc_scaled_norm_noalloc: no usable current HIP device");
        return ISC_ERR_HIP;
    }
    double* part = nullptr;
    hipError_t e = scratch_on(dev, &part);
    if (e != hipSuccess) {
        isc_set_noctx_error((std::string("isc_scaled_norm_noalloc: hipGetSymbolAddress: ") + hipGetErrorString(e)).c_str());
        return ISC_ERR_HIP;
    }
    const int32_t nb = (int32_t)((n + isc::NORM_CELLS_PER_WG - 1) / isc::NORM_CELLS_PER_WG);
    const hipStream_t s = (hipStream_t)hip_stream;
    const double V = g.dx * g.dy * g.dz;
    // every partial that max_partials reads is written by this launch first,
    // so the scratch needs no clearing
    hipLaunchKernelGGL(isc::scaled_norm_partial_fixed, dim3(nb), dim3(256), 0, s, (int32_t)n, F, poro, V / dt,
                       fluid_h->rho_ref[0], fluid_h->cp_rock, part);
    hipLaunchKernelGGL(isc::max_partials, dim3(1), dim3(256), 0, s, part, nb, res);
    e = hipGetLastError();
    if (e != hipSuccess) {
        isc_set_noctx_error((std::string("isc_scaled_norm_noalloc: launch: ") + hipGetErrorString(e)).c_str());
        return ISC_ERR_HIP;
    }
    return ISC_OK;
}
