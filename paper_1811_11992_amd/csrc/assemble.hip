// Residual and Jacobian assembly over the 7-point stencil (Section 3.1):
// F_i = local terms + sum over the six faces of the outflow
//   T_f * sum_a (lambda_a xi_{e,a})_upstream * dPhi_a  (+ conduction on the
//   energy row: (A/h) K_T,harmonic (T_i - T_f)),
// with harmonic transmissibilities and the upstream cell of each phase chosen
// by potential (ties: the lower cell index is upstream).
//
// Mapping: one wavefront per cell, lane (e, v) = (row, unknown) owns entry
// (e, v) of every block of the cell's block row.  A face is evaluated with
// its cells ordered (lo, hi) = (min, max), so the two cells sharing a face
// compute bitwise identical fluxes and derivatives.
#include "common.h"

namespace isc {

struct FaceOut {
    double f;    // flux of row e from lo to hi
    double dl;   // d f / d u_lo[v]
    double dh;   // d f / d u_hi[v]
};

__device__ __forceinline__ FaceOut face_eval(const double* __restrict__ Plo,
                                             const double* __restrict__ Phi, double plo,
                                             double phi_, double Tlo, double Thi, double trans,
                                             double area_h, double dz_lh, int e, int v) {
    // The loads come in two independent batches: first the values every
    // lane shares (the phases' gravity terms, the conductivities), which
    // decide the upstream cell of each phase; then each lane's entries (the
    // derivatives, and the upstream mobilities).  The arithmetic below is
    // the same, in the same order, as evaluating phase by phase.
    double gl[3], gh[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        gl[a] = Plo[PL_GAM + 9 * a];
        gh[a] = Phi[PL_GAM + 9 * a];
    }
    const double dp = plo - phi_;
    double dphi[3];
    bool up_lo[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        dphi[a] = dp - 0.5 * (gl[a] + gh[a]) * dz_lh;
        up_lo[a] = !(dphi[a] < 0.0);
    }
    double dgl[3], dgh[3], m[3], md[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int s = mob_slot(a, e);
        dgl[a] = Plo[PL_GAM + 9 * a + 1 + v];
        dgh[a] = Phi[PL_GAM + 9 * a + 1 + v];
        const double* Pu = up_lo[a] ? Plo : Phi;
        m[a] = s >= 0 ? Pu[PL_MOB + 9 * s] : 0.0;
        md[a] = s >= 0 ? Pu[PL_MOB + 9 * s + 1 + v] : 0.0;
    }
    FaceOut o{0.0, 0.0, 0.0};
    const double ip = (v == 0) ? 1.0 : 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (mob_slot(a, e) < 0) continue;
        const double ddl = ip - 0.5 * dgl[a] * dz_lh;
        const double ddh = -ip - 0.5 * dgh[a] * dz_lh;
        const double tm = trans * m[a];
        o.f += tm * dphi[a];
        if (up_lo[a]) {
            o.dl += trans * md[a] * dphi[a] + tm * ddl;
            o.dh += tm * ddh;
        } else {
            o.dl += tm * ddl;
            o.dh += trans * md[a] * dphi[a] + tm * ddh;
        }
    }
    if (e == 6) {  // conduction with a harmonic bulk conductivity
        const double kl = Plo[PL_KT], kh = Phi[PL_KT];
        const double sum = kl + kh;
        const double kbar = 2.0 * kl * kh / sum;
        const double dT = Tlo - Thi;
        const double it = (v == 4) ? 1.0 : 0.0;
        const double gl2 = 2.0 * kh * kh / (sum * sum), gh2 = 2.0 * kl * kl / (sum * sum);
        o.f += area_h * kbar * dT;
        o.dl += area_h * (gl2 * Plo[PL_KT + 1 + v] * dT + kbar * it);
        o.dh += area_h * (gh2 * Phi[PL_KT + 1 + v] * dT - kbar * it);
    }
    return o;
}

__global__ void __launch_bounds__(256) assemble_kernel(
    int32_t n, int32_t nx, int32_t ny, int32_t nz, const double* __restrict__ u,
    const double* __restrict__ payload, const double* __restrict__ trans, double ah_x, double ah_y,
    double ah_z, double dz, const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ diag_pos,
    double* __restrict__ F, double* __restrict__ J) {
    // the cell is the same on all lanes of the wavefront; saying so lets the
    // values the lanes share (its neighbours' pressures, transmissibilities,
    // gravity terms) come through scalar loads into scalar registers
    const int32_t i = __builtin_amdgcn_readfirstlane((int32_t)(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)));
    const int lane = threadIdx.x & 63;
    const int e = lane >> 3, v = lane & 7;
    if (i >= n) return;
    const int32_t nxy = nx * ny;
    const int32_t ix = i % nx, iy = (i / nx) % ny, iz = i / nxy;
    const double* Pi = payload + (size_t)i * PL;
    double Fe = Pi[PL_LOCAL + 9 * e];
    double Jii = Pi[PL_LOCAL + 9 * e + 1 + v];
    const double pi_ = u[i], Ti = u[(size_t)4 * n + i];
    int32_t blk = row_ptr[i];
    const int32_t dpos = diag_pos[i];
    // neighbours in ascending column order: z-, y-, x-, (self), x+, y+, z+
    const int32_t nbr[6] = {iz > 0 ? i - nxy : -1, iy > 0 ? i - nx : -1, ix > 0 ? i - 1 : -1,
                            ix + 1 < nx ? i + 1 : -1, iy + 1 < ny ? i + nx : -1,
                            iz + 1 < nz ? i + nxy : -1};
    const int dirs[6] = {2, 1, 0, 0, 1, 2};
#pragma unroll
    for (int q = 0; q < 6; ++q) {
        const int32_t f = nbr[q];
        if (q == 3) blk = dpos + 1;
        if (f < 0) continue;
        const int d = dirs[q];
        const bool i_lo = q >= 3;
        const int32_t lo = i_lo ? i : f;
        const double* Pf = payload + (size_t)f * PL;
        const double pf = u[f], Tf = u[(size_t)4 * n + f];
        const double tr = trans[(size_t)d * n + lo];
        const double ah = d == 0 ? ah_x : (d == 1 ? ah_y : ah_z);
        const double dz_lh = d == 2 ? -dz : 0.0;
        // one call site: both cells of the face run the same instructions
        FaceOut o = face_eval(i_lo ? Pi : Pf, i_lo ? Pf : Pi, i_lo ? pi_ : pf, i_lo ? pf : pi_,
                              i_lo ? Ti : Tf, i_lo ? Tf : Ti, tr, ah, dz_lh, e, v);
        double jf;
        if (i_lo) {
            Fe += o.f;
            Jii += o.dl;
            jf = o.dh;
        } else {
            Fe -= o.f;
            Jii -= o.dh;
            jf = -o.dl;
        }
        J[(size_t)blk * BS + lane] = jf;
        ++blk;
    }
    J[(size_t)dpos * BS + lane] = Jii;
    if (v == 0) F[(size_t)i * NU + e] = Fe;
}

}  // namespace isc

hipError_t isc_launch_assemble(isc_ctx* ctx, const double* u, double* F, double* J) {
    const isc_grid& g = ctx->g;
    const int threads = 256;  // 4 cells per workgroup
    const int blocks = (ctx->n + 3) / 4;
    hipLaunchKernelGGL(isc::assemble_kernel, dim3(blocks), dim3(threads), 0, ctx->stream, ctx->n,
                       g.nx, g.ny, g.nz, u, ctx->payload, ctx->trans, g.dy * g.dz / g.dx,
                       g.dx * g.dz / g.dy, g.dx * g.dy / g.dz, g.dz, ctx->row_ptr, ctx->diag_pos, F, J);
    return hipGetLastError();
}
