// Differentiation form: discrete adjoint of one implicit step.
//
// Objective J_obj = sum_n dt_n q_oil(u^n), q_oil = sum over producer
// perforations of WI lambda_o (p - p_wf)^+ (oil-phase molar rate); parameters
// m = (ln k per cell, A_R).  With J^n = dR^n/du^n and the accumulation
// coupling dR^{n+1}/du^n = -(V/dt_{n+1}) dA/du(u^n):
//   (J^n)^T lam^n = rhs,  rhs = dt_n dq/du + (V/dt_{n+1}) (dA/du)^T lam^{n+1},
//   g_lnk += dt_n dq/dlnk - lam . dR/dlnk,  g_A += -lam . dR/dA.
// The 7-point pattern is symmetric, so J^T is formed in place (block (i, j)
// of J^T is J_ji^T); J^T is then decoupled by its own diagonal blocks
// (Gauss-Jordan, as for the forward system) and solved with the same BILU(0)
// GMRES, giving lam directly.
// dR/dln k acts through the harmonic transmissibilities (dT/dln k_i =
// T k_f/(k_i + k_f)), the producer well indices (proportional to k) and the
// injector split (q_p proportional to WI_p / sum WI); dR/dA_R through r_R.
#include <cmath>

#include "common.h"

hipError_t isc_launch_props(isc_ctx*, const double* u, const double* u_old, double dt);
hipError_t isc_launch_assemble(isc_ctx*, const double* u, double* F, double* J);
hipError_t isc_launch_accgrad(isc_ctx*, const double* u);
hipError_t isc_launch_decouple(isc_ctx*, double* J, double* F, int32_t* bad_dev);
hipError_t isc_launch_bilu0_factor(isc_ctx*, const double* A, double* Dinv, int32_t* bad);
isc_status isc_gmres_fp64(isc_ctx*, const double* A, const double* Dinv, const double* b, double* x,
                          const isc_solve_opts* o, isc_solve_info* info);

namespace isc {

__global__ void __launch_bounds__(256) adj_rhs(int32_t n, double dt_n, double v_dt1, const double* __restrict__ qg,
                                               const double* __restrict__ accJ, const double* __restrict__ lam1,
                                               double* __restrict__ rhs) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= (int64_t)n * 8) return;
    const int32_t i = (int32_t)(t >> 3);
    const int v = (int)(t & 7);
    double s = dt_n * qg[t];
    if (lam1) {
        const double* a = accJ + (size_t)i * 64 + v;
        const double* l = lam1 + (size_t)i * 8;
#pragma unroll
        for (int e = 0; e < 8; ++e) s += v_dt1 * a[e * 8] * l[e];
    }
    rhs[t] = s;
}

// In-place block transpose of a matrix with a symmetric block pattern: one
// wavefront per stored block (i, j) with j >= i swaps it with block (j, i),
// both transposed; lane (r, c) moves entry (r, c).
__global__ void __launch_bounds__(256) block_transpose(int32_t n, int32_t nx, int32_t ny,
                                                       const int32_t* __restrict__ row_ptr,
                                                       const int32_t* __restrict__ col_idx,
                                                       const int32_t* __restrict__ diag_pos, double* __restrict__ J) {
    const int32_t b = (int32_t)(blockIdx.x * 4 + (threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    if (b >= row_ptr[n]) return;
    // row of block b: binary search in row_ptr
    int32_t lo = 0, hi = n;
    while (hi - lo > 1) {
        const int32_t mid = (lo + hi) >> 1;
        if (row_ptr[mid] <= b) lo = mid; else hi = mid;
    }
    const int32_t i = lo, j = col_idx[b];
    if (j < i) return;
    const int r = lane >> 3, c = lane & 7;
    if (j == i) {
        const double x = J[(size_t)b * 64 + c * 8 + r];
        __builtin_amdgcn_wave_barrier();
        J[(size_t)b * 64 + r * 8 + c] = x;
        return;
    }
    // block (j, i): i is j's lower neighbour; its slot in row j (lower
    // neighbours are stored z-, y-, x-); the direction comes from the
    // coordinates, which stays unambiguous when nx or ny is 1
    const int32_t nxy = nx * ny;
    const int32_t jy = (j / nx) % ny, jz = j / nxy;
    const int32_t iy = (i / nx) % ny, iz = i / nxy;
    int32_t bt = row_ptr[j];
    if (iz == jz) bt += (jz > 0) + (iy == jy ? (jy > 0) : 0);
    (void)diag_pos;
    const double x = J[(size_t)b * 64 + c * 8 + r];
    const double y = J[(size_t)bt * 64 + c * 8 + r];
    __builtin_amdgcn_wave_barrier();
    J[(size_t)bt * 64 + r * 8 + c] = x;
    J[(size_t)b * 64 + r * 8 + c] = y;
}

// g_lnk[i] -= sum over the faces of i of (lam_lo - lam_hi) . F_conv * k_other / (k_i + k_other),
// F_conv = T sum_a (lambda_a xi_{e,a})_up dPhi_a (values of the assembly's face flux without conduction)
__global__ void __launch_bounds__(256) grad_faces(int32_t n, int32_t nx, int32_t ny, int32_t nz,
                                                  const double* __restrict__ u, const double* __restrict__ payload,
                                                  const double* __restrict__ trans, const double* __restrict__ logk,
                                                  double dz, const double* __restrict__ lam,
                                                  double* __restrict__ g) {
    const int32_t i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const int32_t nxy = nx * ny;
    const int32_t ix = i % nx, iy = (i / nx) % ny, iz = i / nxy;
    const int32_t nb[6] = {iz > 0 ? i - nxy : -1, iy > 0 ? i - nx : -1, ix > 0 ? i - 1 : -1,
                           ix + 1 < nx ? i + 1 : -1, iy + 1 < ny ? i + nx : -1, iz + 1 < nz ? i + nxy : -1};
    const int dirs[6] = {2, 1, 0, 0, 1, 2};
    const double ki = exp(logk[i]);
    double acc = 0.0;
    for (int q = 0; q < 6; ++q) {
        const int32_t f = nb[q];
        if (f < 0) continue;
        const bool i_lo = q >= 3;
        const int32_t lo = i_lo ? i : f, hi = i_lo ? f : i;
        const double* Pl = payload + (size_t)lo * PL;
        const double* Ph = payload + (size_t)hi * PL;
        const double dzlh = dirs[q] == 2 ? -dz : 0.0;
        const double tr = trans[(size_t)dirs[q] * n + lo];
        const double dp = u[lo] - u[hi];
        double s = 0.0;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const double dphi = dp - 0.5 * (Pl[PL_GAM + 9 * a] + Ph[PL_GAM + 9 * a]) * dzlh;
            const double* Pu = !(dphi < 0.0) ? Pl : Ph;
#pragma unroll
            for (int e = 0; e < 7; ++e) {
                const int sl = mob_slot(a, e);
                if (sl < 0) continue;
                s += (lam[(size_t)lo * 8 + e] - lam[(size_t)hi * 8 + e]) * (tr * Pu[PL_MOB + 9 * sl] * dphi);
            }
        }
        const double kf = exp(logk[f]);
        acc += s * kf / (ki + kf);
    }
    g[i] -= acc;
}

// wells (one thread; perforation counts are small): producers
// g += lam . W + dt_n q (W proportional to WI), injectors through the split
__global__ void grad_wells(int32_t nwells, const int32_t* __restrict__ well_off, const int32_t* __restrict__ pcell,
                           const double* __restrict__ perf, const double* __restrict__ u, int32_t n,
                           const double* __restrict__ payload, const double* __restrict__ qv, double dt_n,
                           const double* __restrict__ lam, double* __restrict__ g) {
    for (int32_t w = 0; w < nwells; ++w) {
        const int32_t p0 = well_off[w], p1 = well_off[w + 1];
        if (perf[(size_t)p0 * PERF_W] == 1.0) {
            for (int32_t p = p0; p < p1; ++p) {
                const int32_t i = pcell[p];
                const double* pf = perf + (size_t)p * PERF_W;
                const double pres = u[i];
                if (!(pres > pf[2])) continue;
                const double dpw = pf[1] * (pf[2] - pres);
                const double* P = payload + (size_t)i * PL;
                double s = 0.0;
                for (int a = 0; a < 3; ++a)
                    for (int e = 0; e < 7; ++e) {
                        const int sl = mob_slot(a, e);
                        if (sl >= 0) s += lam[(size_t)i * 8 + e] * dpw * P[PL_MOB + 9 * sl];
                    }
                g[i] += s + dt_n * qv[i];
            }
        } else {
            double sum_wi = 0.0, sum_s = 0.0;
            for (int32_t p = p0; p < p1; ++p) {
                const double* pf = perf + (size_t)p * PERF_W;
                const int32_t i = pcell[p];
                double s = lam[(size_t)i * 8 + 6] * pf[10];
                for (int c = 0; c < 6; ++c) s += lam[(size_t)i * 8 + c] * pf[3 + c];
                sum_wi += pf[1];
                sum_s += s;
            }
            for (int32_t p = p0; p < p1; ++p) {
                const double* pf = perf + (size_t)p * PERF_W;
                const int32_t i = pcell[p];
                double s = lam[(size_t)i * 8 + 6] * pf[10];
                for (int c = 0; c < 6; ++c) s += lam[(size_t)i * 8 + c] * pf[3 + c];
                g[i] += s - pf[1] / sum_wi * sum_s;
            }
        }
    }
    (void)n;
}

__device__ __forceinline__ double wsum(double x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
    return x;
}

// partial[r * nblk + b] = sum over cells of r_R lam . (s_R, H_R); partial[4 * nblk + b] = sum q_oil
__global__ void __launch_bounds__(256) grad_A_partial(int32_t n, const double* __restrict__ rates,
                                                      const double* __restrict__ lam, const double* __restrict__ qv,
                                                      const isc_fluid* __restrict__ fl, double* __restrict__ partial) {
    __shared__ double red[4][5];
    double acc[5] = {0, 0, 0, 0, 0};
    for (int32_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
        const double* l = lam ? lam + (size_t)i * 8 : nullptr;
        if (l) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                double s = fl->Hreac[r] * l[6];
#pragma unroll
                for (int c = 0; c < 6; ++c) s += fl->stoich[r][c] * l[c];
                s += fl->stoich[r][6] * l[7];
                acc[r] += rates[(size_t)i * 4 + r] * s;
            }
        }
        acc[4] += qv[i];
    }
    const int w = threadIdx.x >> 6;
#pragma unroll
    for (int r = 0; r < 5; ++r) {
        const double s = wsum(acc[r]);
        if ((threadIdx.x & 63) == 0) red[w][r] = s;
    }
    __syncthreads();
    if (threadIdx.x < 5)
        partial[(size_t)threadIdx.x * gridDim.x + blockIdx.x] =
            (red[0][threadIdx.x] + red[1][threadIdx.x]) + (red[2][threadIdx.x] + red[3][threadIdx.x]);
}

__global__ void __launch_bounds__(256) sum5(const double* __restrict__ partial, int nblk, double* __restrict__ out) {
    __shared__ double red[4];
    const int r = blockIdx.x;
    double s = 0.0;
    for (int b = threadIdx.x; b < nblk; b += 256) s += partial[(size_t)r * nblk + b];
    s = wsum(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) out[r] = (red[0] + red[1]) + (red[2] + red[3]);
}

}  // namespace isc

// accJ, qg, qv, rates at u; sums of (rate x lam) and q_oil into ctx->small[3008..3012]
static isc_status reduce_rates(isc_ctx* ctx, const double* lam, double* out5_h) {
    int nb = (ctx->n + 255) / 256;
    nb = nb > isc::NPART ? isc::NPART : nb;
    hipLaunchKernelGGL(isc::grad_A_partial, dim3(nb), dim3(256), 0, ctx->stream, ctx->n, ctx->rates, lam, ctx->qv,
                       ctx->fluid_d, ctx->partial);
    hipLaunchKernelGGL(isc::sum5, dim3(5), dim3(256), 0, ctx->stream, ctx->partial, nb, ctx->small + 3008);
    ISC_HIP(hipMemcpyAsync(ctx->hscratch, ctx->small + 3008, 5 * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    ISC_HIP(hipStreamSynchronize(ctx->stream));
    for (int k = 0; k < 5; ++k) out5_h[k] = ctx->hscratch[k];
    return ISC_OK;
}

isc_status isc_oil_rate_impl(isc_ctx* ctx, const double* u, double* q_h) {
    ISC_HIP(isc_launch_accgrad(ctx, u));
    double out[5];
    isc_status st = reduce_rates(ctx, nullptr, out);
    if (st != ISC_OK) return st;
    *q_h = out[4];
    return ISC_OK;
}

__global__ static void fill_bad(int32_t* f) { f[0] = INT32_MAX; }

isc_status isc_adjoint_impl(isc_ctx* ctx, const double* u_n, const double* u_nm1, double dt_n, const double* lam_np1,
                            double dt_np1, double* lam_n, double* g_logk, double* g_A_h, const isc_solve_opts* o,
                            isc_solve_info* info_h) {
    using namespace isc;
    if (!u_n || !u_nm1 || !lam_n || !g_logk || !g_A_h || !(dt_n > 0) || (lam_np1 && !(dt_np1 > 0))) {
        ctx->err = "isc_adjoint: invalid argument";
        return ISC_ERR_ARG;
    }
    const isc_solve_opts def{30, 200, ISC_FP64, 0, ISC_PC_BILU0, 0, 1e-12};
    isc_solve_opts opts = o ? *o : def;
    opts.precision = ISC_FP64;
    opts.precond = ISC_PC_BILU0;
    if (opts.restart < 1 || opts.restart > ctx->mmax) opts.restart = ctx->mmax;
    const int32_t n = ctx->n;
    const double V = ctx->g.dx * ctx->g.dy * ctx->g.dz;
    // Jacobian at (u^n, u^{n-1}) and the per-cell adjoint inputs at u^n
    ISC_HIP(isc_launch_props(ctx, u_n, u_nm1, dt_n));
    ISC_HIP(isc_launch_assemble(ctx, u_n, ctx->F, ctx->J));
    ISC_HIP(isc_launch_accgrad(ctx, u_n));
    const int64_t n8 = (int64_t)n * 8;
    hipLaunchKernelGGL(adj_rhs, dim3((unsigned)((n8 + 255) / 256)), dim3(256), 0, ctx->stream, n, dt_n,
                       lam_np1 ? V / dt_np1 : 0.0, ctx->qg, ctx->accJ, lam_np1, ctx->rhs);
    // J^T in place, then decouple J^T with rhs and solve for lam directly
    hipLaunchKernelGGL(block_transpose, dim3((ctx->nnzb + 3) / 4), dim3(256), 0, ctx->stream, n, ctx->g.nx,
                       ctx->g.ny, ctx->row_ptr, ctx->col_idx, ctx->diag_pos, ctx->J);
    int32_t* bad = ctx->flags + 2;
    hipLaunchKernelGGL(fill_bad, dim3(1), dim3(1), 0, ctx->stream, bad);
    ISC_HIP(isc_launch_decouple(ctx, ctx->J, ctx->rhs, bad));
    ISC_HIP(isc_launch_bilu0_factor(ctx, ctx->J, ctx->Dinv, bad));
    ISC_HIP(hipMemcpyAsync(ctx->hflags + 2, bad, sizeof(int32_t), hipMemcpyDeviceToHost, ctx->stream));
    ISC_HIP(hipStreamSynchronize(ctx->stream));
    if (ctx->hflags[2] != INT32_MAX) {
        ctx->err = "isc_adjoint: singular block at cell " + std::to_string(ctx->hflags[2]);
        return ISC_ERR_SINGULAR;
    }
    isc_status st = isc_gmres_fp64(ctx, ctx->J, ctx->Dinv, ctx->rhs, lam_n, &opts, info_h);
    if (st != ISC_OK) return st;
    // gradient
    hipLaunchKernelGGL(grad_faces, dim3((n + 255) / 256), dim3(256), 0, ctx->stream, n, ctx->g.nx, ctx->g.ny,
                       ctx->g.nz, u_n, ctx->payload, ctx->trans, ctx->logk, ctx->g.dz, lam_n, g_logk);
    hipLaunchKernelGGL(grad_wells, dim3(1), dim3(1), 0, ctx->stream, (int32_t)ctx->wells.size(), ctx->well_off,
                       ctx->perf_cell, ctx->perf, u_n, n, ctx->payload, ctx->qv, dt_n, lam_n, g_logk);
    double out[5];
    st = reduce_rates(ctx, lam_n, out);
    if (st != ISC_OK) return st;
    for (int r = 0; r < 4; ++r)
        if (ctx->fluid_h.Afreq[r] != 0.0) g_A_h[r] += V * out[r] / ctx->fluid_h.Afreq[r];
    return ISC_OK;
}
