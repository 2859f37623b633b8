// C-ABI of libisc: context management and the hot-path entry points.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <unordered_map>
#include <vector>

#include "common.h"

// launchers defined in the kernel sources
hipError_t isc_launch_props(isc_ctx*, const double* u, const double* u_old, double dt);
hipError_t isc_launch_assemble(isc_ctx*, const double* u, double* F, double* J);
hipError_t isc_launch_decouple(isc_ctx*, double* J, double* F, int32_t* bad_dev);
hipError_t isc_launch_bilu0_factor(isc_ctx*, const double* A, double* Dinv, int32_t* bad);
hipError_t isc_launch_bilu0_apply(isc_ctx*, const double* A, const double* Dinv, const double* r, double* z);
hipError_t isc_launch_form_ltilde(isc_ctx*, const double* A, const double* Dinv);
hipError_t isc_launch_bilu0_apply_spmv(isc_ctx*, const double* A, const double* Dinv, const double* r, double* z,
                                       double* w);
hipError_t isc_launch_spmv(isc_ctx*, const double* A, const double* x, double* y);
hipError_t isc_launch_update(isc_ctx*, double* u, const double* du, int32_t* flag_dev);
hipError_t isc_launch_scaled_norm(isc_ctx*, const double* F, double dt, double* out_dev);
hipError_t isc_launch_negate(isc_ctx*, const double* x, double* y);
hipError_t isc_launch_well_line(isc_ctx*, const double* u, int mode);
hipError_t isc_launch_well_rows(isc_ctx*, const double* u);
hipError_t isc_launch_well_fold(isc_ctx*, double* J);
hipError_t isc_launch_well_reduce(isc_ctx*, double dt);
hipError_t isc_launch_well_rhs(isc_ctx*, double* rhs);
hipError_t isc_launch_well_update(isc_ctx*, const double* du, int32_t* nonfinite_dev);
isc_status isc_gmres_fp64(isc_ctx*, const double* A, const double* Dinv, const double* b, double* x,
                          const isc_solve_opts* o, isc_solve_info* info);
isc_status isc_fgmres(isc_ctx*, const double* A, const double* b, double* x, const isc_solve_opts* o,
                      isc_solve_info* info);
isc_status isc_prepare_mixed_dev(isc_ctx*, const double* A, int32_t* bad_dev);
isc_status isc_bicgstab_run(isc_ctx*, const double* A, const double* b, double* x, int32_t max_iters, double rtol,
                            isc_solve_info* info);
void isc_cpr_pressure_gmres(isc_ctx*, const double* rp, double* e, int k);
void isc_apply_spmv32_from64(isc_ctx*, const double* r, double* z, double* w);
void isc_cpr_apply_w(isc_ctx*, const double* A, const double* u, double* z, double* w, int k);
isc_status isc_adjoint_impl(isc_ctx*, const double* u_n, const double* u_nm1, double dt_n,
                            const double* lam_np1, double dt_np1, double* lam_n, double* g_logk,
                            double* g_A_h, const isc_solve_opts* o, isc_solve_info* info_h);
isc_status isc_oil_rate_impl(isc_ctx*, const double* u, double* q_h);

#ifndef ISC_SPMV_LAG
#define ISC_SPMV_LAG 0   // brick levels between the sweep front and the SpMV bricks of the fused kernel
#endif

namespace {

constexpr int FLAG_BAD = 0;      // int32 slot: singular cell (INT32_MAX = none)
constexpr int FLAG_NONFIN = 1;   // int32 slot: non-finite update

// gas enthalpy of species c at T (host copy of the cp integral, for the
// injected-gas energy rate)
double host_hgas(const isc_fluid& f, int c, double T) {
    double h = 0.0, Tp = T, Rp = f.T_ref;
    for (int j = 0; j < 4; ++j) {
        h += f.cpg[c][j] / (j + 1) * (Tp - Rp);
        Tp *= T;
        Rp *= f.T_ref;
    }
    return h;
}

template <class T>
isc_status dalloc(isc_ctx* ctx, T** p, size_t count) {
    if (count == 0) count = 1;
    hipError_t e = hipMalloc((void**)p, count * sizeof(T));
    if (e != hipSuccess) {
        ctx->err = "hipMalloc of " + std::to_string(count * sizeof(T)) + " bytes failed: " + hipGetErrorString(e);
        return ISC_ERR_OOM;
    }
    return ISC_OK;
}

#define TRY(x)                          \
    do {                                \
        isc_status s_ = (x);            \
        if (s_ != ISC_OK) return s_;    \
    } while (0)

// transmissibilities of the +x, +y, +z faces (harmonic mean of A k / h)
// and the perforation table (Peaceman well index, injection split)
isc_status rebuild_static(isc_ctx* ctx) {
    const isc_grid& g = ctx->g;
    const int32_t n = ctx->n, nx = g.nx, ny = g.ny, nz = g.nz, nxy = nx * ny;
    std::vector<double> tr((size_t)3 * n, 0.0);
    const double ah[3] = {g.dy * g.dz / g.dx, g.dx * g.dz / g.dy, g.dx * g.dy / g.dz};
    for (int32_t i = 0; i < n; ++i) {
        const int32_t ix = i % nx, iy = (i / nx) % ny, iz = i / nxy;
        const bool has[3] = {ix + 1 < nx, iy + 1 < ny, iz + 1 < nz};
        const int32_t st[3] = {1, nx, nxy};
        for (int d = 0; d < 3; ++d) {
            if (!has[d]) continue;
            const int32_t f = i + st[d];
            const double ki = std::exp(ctx->logk_h[i]) * (d == 2 ? ctx->kvkh : 1.0);
            const double kf = std::exp(ctx->logk_h[f]) * (d == 2 ? ctx->kvkh : 1.0);
            const double ai = ah[d] * ki, af = ah[d] * kf;
            tr[(size_t)d * n + i] = 2.0 * ai * af / (ai + af);
        }
    }
    ISC_HIP(hipMemcpyAsync(ctx->trans, tr.data(), tr.size() * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
    // wells
    std::vector<int32_t> slot(n, -1);
    ctx->perf_h.assign((size_t)std::max(ctx->npf, 1) * isc::PERF_W, 0.0);
    const double re = 0.14 * std::sqrt(g.dx * g.dx + g.dy * g.dy);
    int32_t p = 0, cwi = -1;
    for (size_t w = 0; w < ctx->wells.size(); ++w) {
        const isc_well& W = ctx->wells[w];
        if (W.kind == ISC_WELL_PRODUCER || W.kind == ISC_WELL_INJECTOR) ++cwi;
        const std::vector<int32_t>& cells = ctx->well_cells[w];
        std::vector<double> wi(cells.size());
        double sum = 0.0;
        for (size_t k = 0; k < cells.size(); ++k) {
            wi[k] = 2.0 * M_PI * g.dz * std::exp(ctx->logk_h[cells[k]]) / (std::log(re / W.rw) + W.skin);
            sum += wi[k];
        }
        double hinj = 0.0;
        for (int c = 0; c < 6; ++c) hinj += W.z_inj[c] * host_hgas(ctx->fluid_h, c, W.T_inj);
        const bool controlled = W.kind == ISC_WELL_PRODUCER || W.kind == ISC_WELL_INJECTOR;
        for (size_t k = 0; k < cells.size(); ++k, ++p) {
            double* pf = ctx->perf_h.data() + (size_t)p * isc::PERF_W;
            if (slot[cells[k]] >= 0) {
                ctx->err = "isc_create: a cell is perforated by more than one well";
                return ISC_ERR_ARG;
            }
            slot[cells[k]] = p;
            pf[0] = (double)W.kind;
            pf[1] = wi[k];
            if (controlled) {
                pf[2] = (double)cwi;
                for (int c = 0; c < 7; ++c) pf[3 + c] = W.z_inj[c];
                pf[10] = hinj;
                pf[11] = (double)(ctx->cw_h[cwi].c0 + (int32_t)k);
            } else if (W.kind == ISC_WELL_BHP_PRODUCER) {
                pf[2] = W.target;
            } else {
                const double q = W.target * wi[k] / sum;
                for (int c = 0; c < 7; ++c) pf[3 + c] = q * W.z_inj[c];
                pf[10] = q * hinj;
                pf[11] = q;
            }
        }
    }
    ISC_HIP(hipMemcpyAsync(ctx->well_slot, slot.data(), slot.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                           ctx->stream));
    ISC_HIP(hipMemcpyAsync(ctx->perf, ctx->perf_h.data(), ctx->perf_h.size() * sizeof(double),
                           hipMemcpyHostToDevice, ctx->stream));
    ISC_HIP(hipStreamSynchronize(ctx->stream));
    return ISC_OK;
}

isc_status read_flag(isc_ctx* ctx, int slot, int32_t* out) {
    ISC_HIP(hipMemcpyAsync(ctx->hflags + slot, ctx->flags + slot, sizeof(int32_t), hipMemcpyDeviceToHost,
                           ctx->stream));
    ISC_HIP(hipStreamSynchronize(ctx->stream));
    *out = ctx->hflags[slot];
    isc_prof_drain(ctx);
    return ISC_OK;
}

__global__ void fill_flags(int32_t* f) {
    f[FLAG_BAD] = INT32_MAX;
    f[FLAG_NONFIN] = 0;
}

isc_status reset_flags(isc_ctx* ctx) {
    hipLaunchKernelGGL(fill_flags, dim3(1), dim3(1), 0, ctx->stream, ctx->flags);
    ISC_HIP(hipGetLastError());
    return ISC_OK;
}

isc_status check_ctx(const isc_ctx* ctx) { return ctx ? ISC_OK : ISC_ERR_ARG; }

// the preconditioner and precision options against what the context holds
isc_status check_precond(isc_ctx* ctx, const isc_solve_opts* o, const char* who) {
    if (o->precond != ISC_PC_BILU0 && o->precond != ISC_PC_CPR) {
        ctx->err = std::string(who) + ": unknown preconditioner";
        return ISC_ERR_ARG;
    }
    if (o->krylov != ISC_KRYLOV_GMRES && o->krylov != ISC_KRYLOV_BICGSTAB) {
        ctx->err = std::string(who) + ": unknown Krylov method";
        return ISC_ERR_ARG;
    }
    if (o->krylov == ISC_KRYLOV_BICGSTAB &&
        (o->precision != ISC_FP64 || o->precond != ISC_PC_BILU0 || ctx->mmax < 6)) {
        ctx->err = std::string(who) + ": BiCGSTAB runs in FP64 with BILU(0), on a context of max restart >= 6";
        return ISC_ERR_ARG;
    }
    if (o->precond == ISC_PC_CPR) {
        if (o->precision != ISC_FP64) {
            ctx->err = std::string(who) + ": the CPR preconditioner runs in FP64 only";
            return ISC_ERR_ARG;
        }
        if (ctx->cpr_kmax < 0 || o->p_iters < 0 || o->p_iters > ctx->cpr_kmax) {
            ctx->err = std::string(who) + ": CPR needs a context created for it with max p_iters >= p_iters >= 0";
            return ISC_ERR_ARG;
        }
    } else if (o->precision == ISC_MIXED && (o->inner_iters < 1 || o->inner_iters > ctx->inner_max)) {
        ctx->err = std::string(who) + ": mixed precision needs 1 <= inner_iters <= the context's maximum";
        return ISC_ERR_ARG;
    }
    return ISC_OK;
}

thread_local std::string g_noctx_err;   // last error of a context-free call on this thread

}  // namespace

void isc_set_noctx_error(const char* msg) { g_noctx_err = msg; }

extern "C" {

isc_status isc_create(const isc_grid* grid_h, const isc_fluid* fluid_h, const double* logk, double kv_over_kh,
                      const double* poro, const isc_well* wells_h, int32_t nwells,
                      const isc_solve_opts* max_opts_h, void* hip_stream, isc_ctx** out_h) {
    if (!out_h) return ISC_ERR_ARG;
    *out_h = nullptr;
    isc_ctx* ctx = new isc_ctx();
    auto fail = [&](isc_status s) {
        // keep the message reachable through a leaked-on-error context is not
        // possible; print it so the caller sees why creation failed
        fprintf(stderr, "isc_create: %s\n", ctx->err.c_str());
        isc_destroy(ctx);
        return s;
    };
    if (!grid_h || !fluid_h || !logk || !poro || (nwells > 0 && !wells_h) || nwells < 0) {
        ctx->err = "null argument";
        return fail(ISC_ERR_ARG);
    }
    const isc_grid& g = *grid_h;
    if (g.nx < 1 || g.ny < 1 || g.nz < 1 || !(g.dx > 0) || !(g.dy > 0) || !(g.dz > 0) || !(kv_over_kh > 0)) {
        ctx->err = "invalid grid";
        return fail(ISC_ERR_ARG);
    }
    const int64_t n64 = (int64_t)g.nx * g.ny * g.nz;
    if (n64 * 7 > INT32_MAX / 2) {
        ctx->err = "grid too large for 32-bit block indices";
        return fail(ISC_ERR_ARG);
    }
    ctx->g = g;
    ctx->n = (int32_t)n64;
    ctx->kvkh = kv_over_kh;
    ctx->fluid_h = *fluid_h;
    ctx->stream = (hipStream_t)hip_stream;
    if (hipGetDevice(&ctx->dev) != hipSuccess) {
        ctx->err = "no HIP device";
        return fail(ISC_ERR_HIP);
    }
    isc_solve_opts mo{30, 20, ISC_FP64, 0, ISC_PC_BILU0, 0, 1e-8};
    if (max_opts_h) mo = *max_opts_h;
    if (mo.restart < 1 || mo.restart > 31) {
        ctx->err = "max restart must be in [1, 31]";
        return fail(ISC_ERR_ARG);
    }
    if (mo.inner_iters < 0 || mo.inner_iters > 31) {
        ctx->err = "max inner_iters must be in [0, 31]";
        return fail(ISC_ERR_ARG);
    }
    if (mo.precond == ISC_PC_CPR && (mo.p_iters < 0 || mo.p_iters > ISC_CPR_MAX_K)) {
        ctx->err = "max p_iters must be in [0, 16]";
        return fail(ISC_ERR_ARG);
    }
    ctx->mmax = mo.restart;
    ctx->inner_max = mo.inner_iters;
    const int32_t n = ctx->n, nx = g.nx, ny = g.ny, nz = g.nz, nxy = nx * ny;

    // block CSR pattern of the 7-point stencil, columns ascending
    ctx->row_ptr_h.assign(n + 1, 0);
    ctx->diag_pos_h.assign(n, 0);
    ctx->col_idx_h.reserve((size_t)7 * n);
    for (int32_t i = 0; i < n; ++i) {
        const int32_t ix = i % nx, iy = (i / nx) % ny, iz = i / nxy;
        const int32_t cand[7] = {iz > 0 ? i - nxy : -1, iy > 0 ? i - nx : -1, ix > 0 ? i - 1 : -1, i,
                                 ix + 1 < nx ? i + 1 : -1, iy + 1 < ny ? i + nx : -1, iz + 1 < nz ? i + nxy : -1};
        for (int k = 0; k < 7; ++k) {
            if (cand[k] < 0) continue;
            if (cand[k] == i) ctx->diag_pos_h[i] = (int32_t)ctx->col_idx_h.size();
            ctx->col_idx_h.push_back(cand[k]);
        }
        ctx->row_ptr_h[i + 1] = (int32_t)ctx->col_idx_h.size();
    }
    ctx->nnzb = ctx->row_ptr_h[n];
    // hyperplane levels s = ix + iy + iz, rows ascending inside a level
    ctx->nlev = nx + ny + nz - 2;
    ctx->lvl_off_h.assign(ctx->nlev + 1, 0);
    for (int32_t i = 0; i < n; ++i) {
        const int32_t s = i % nx + (i / nx) % ny + i / nxy;
        ctx->lvl_off_h[s + 1]++;
    }
    for (int32_t s = 0; s < ctx->nlev; ++s) ctx->lvl_off_h[s + 1] += ctx->lvl_off_h[s];
    std::vector<int32_t> lvl_rows(n), fillp(ctx->lvl_off_h.begin(), ctx->lvl_off_h.end() - 1);
    for (int32_t i = 0; i < n; ++i) lvl_rows[fillp[i % nx + (i / nx) % ny + i / nxy]++] = i;

    // bricks by brick level (sync-free sweeps), ascending brick index inside a level
    const int32_t nbx = (nx + isc::BRICK_X - 1) / isc::BRICK_X, nby = (ny + isc::BRICK_Y - 1) / isc::BRICK_Y,
                  nbz = (nz + isc::BRICK_Z - 1) / isc::BRICK_Z;
    ctx->nbrick = nbx * nby * nbz;
    std::vector<int32_t> chf, chb, items, items_rank;
    {
        const int32_t nbl = nbx + nby + nbz - 2;
        const int32_t dummy = ctx->nbrick;   // past the last brick layer: every cell inactive
        // pads a group of mutually independent items to whole workgroups
        auto pad = [](std::vector<int32_t>& v, int32_t fill) {
            while (v.size() % isc::MAX_BRICKS_PER_WG) v.push_back(fill);
        };
        auto level_of = [&](int32_t b) { return b % nbx + (b / nbx) % nby + b / (nbx * nby); };
        std::vector<std::vector<int32_t>> by_level(nbl);   // ascending brick index
        for (int32_t b = 0; b < ctx->nbrick; ++b) by_level[level_of(b)].push_back(b);
        for (int32_t L = 0; L < nbl; ++L) {
            chf.insert(chf.end(), by_level[L].begin(), by_level[L].end());
            pad(chf, dummy);
        }
        for (int32_t L = nbl - 1; L >= 0; --L) {
            chb.insert(chb.end(), by_level[L].rbegin(), by_level[L].rend());
            pad(chb, dummy);
        }
        // fused backward sweep + SpMV: after the backward bricks of level L come the
        // SpMV bricks of level L + 1 + ISC_SPMV_LAG (their neighbours are at levels
        // L + ISC_SPMV_LAG .. L + 2 + ISC_SPMV_LAG, all swept before them); the lag
        // keeps SpMV bricks from waiting on the sweep front
        items.reserve((size_t)2 * ctx->nbrick + 2 * nbl * isc::MAX_BRICKS_PER_WG);
        // Each item also records its rank: the position of its brick in the
        // backward list, where the brick's backward and SpMV data are stored
        // (both kinds of groups come in the backward list's order and padding).
        int32_t rank_b = 0, rank_s = 0;
        auto push_group = [&](int32_t L, int32_t flag, int32_t& rank) {
            for (auto it = by_level[L].rbegin(); it != by_level[L].rend(); ++it) {
                items.push_back(*it | flag);
                items_rank.push_back(rank++);
            }
            while (items.size() % isc::MAX_BRICKS_PER_WG) {
                items.push_back(dummy | flag);
                items_rank.push_back(rank++);
            }
        };
        int32_t next_spmv = nbl - 1;   // highest level whose SpMV bricks are not listed yet
        for (int32_t L = nbl - 1; L >= 0; --L) {
            push_group(L, 0, rank_b);
            for (; next_spmv >= 0 && next_spmv >= L + 1 + ISC_SPMV_LAG; --next_spmv)
                push_group(next_spmv, 1 << 30, rank_s);
        }
        for (; next_spmv >= 0; --next_spmv) push_group(next_spmv, 1 << 30, rank_s);
        if (rank_b != (int32_t)chb.size() || rank_s != (int32_t)chb.size()) {
            ctx->err = "internal: fused work list out of step with the backward list";
            return fail(ISC_ERR_ARG);
        }
    }
    {
        // cooperative static schedule unless switched off (ISC_SWEEP_COOP=0);
        // under tickets, one atomic per workgroup costs about 12 ns of
        // serialised atomic throughput, so bricks are paired once those exceed
        // a fraction of the wait chain (about 200 bricks per brick level)
        if (const char* e = getenv("ISC_SWEEP_COOP")) ctx->coop = e[0] != '0';
        if (const char* e = getenv("ISC_FOLD_UPDATE")) ctx->fold_update = e[0] == '1';
        const int32_t nbl = nbx + nby + nbz - 2;
        ctx->bpw = (!ctx->coop && ctx->nbrick >= 200 * nbl) ? 2 : 1;
        if (const char* e = getenv("ISC_BRICKS_PER_WG")) ctx->bpw = e[0] == '2' ? 2 : 1;
    }
    ctx->nfwd_items = (int32_t)chf.size();
    // slot of each cell's L D^-1 blocks: its brick's position in the forward
    // list; slot of its backward and SpMV data: the position in the backward list
    std::vector<int32_t> lt_slot(n), b_slot(n);
    {
        std::vector<int32_t> pos((size_t)ctx->nbrick, 0), posb((size_t)ctx->nbrick, 0);
        for (size_t k = 0; k < chf.size(); ++k)
            if (chf[k] < ctx->nbrick) pos[chf[k]] = (int32_t)k;
        for (size_t k = 0; k < chb.size(); ++k)
            if (chb[k] < ctx->nbrick) posb[chb[k]] = (int32_t)k;
        for (int32_t i = 0; i < n; ++i) {
            const int32_t ix = i % nx, iy = (i / nx) % ny, iz = i / nxy;
            const int32_t b = ix / isc::BRICK_X + nbx * (iy / isc::BRICK_Y + nby * (iz / isc::BRICK_Z));
            const int32_t g = ix % isc::BRICK_X + isc::BRICK_X * (iy % isc::BRICK_Y + isc::BRICK_Y * (iz % isc::BRICK_Z));
            lt_slot[i] = pos[b] * (isc::BRICK_X * isc::BRICK_Y * isc::BRICK_Z) + g;
            b_slot[i] = posb[b] * (isc::BRICK_X * isc::BRICK_Y * isc::BRICK_Z) + g;
        }
    }
    ctx->nbwd_items = (int32_t)chb.size();
    ctx->nfused_items = (int32_t)items.size();
    if (const char* e = getenv("ISC_LEVEL_SWEEPS")) ctx->syncfree = !(e[0] == '1');

    // wells
    int32_t npf = 0;
    for (int32_t w = 0; w < nwells; ++w) {
        const isc_well& W = wells_h[w];
        const bool controlled = W.kind == ISC_WELL_PRODUCER || W.kind == ISC_WELL_INJECTOR;
        const bool ctrl_ok = !controlled ||
                             (W.nperf <= isc::CW_MAXPERF && std::isfinite(W.target) && std::isfinite(W.limit) &&
                              W.target > 0 && (W.control == ISC_CTRL_BHP || W.limit > 0) &&
                              (W.kind == ISC_WELL_INJECTOR || (W.control >= 0 && W.control <= 7)));
        if (W.nperf < 1 || !W.perf_cells_h || !(W.kind >= ISC_WELL_BHP_PRODUCER && W.kind <= ISC_WELL_INJECTOR) ||
            !(W.rw > 0) || !ctrl_ok) {
            ctx->err = "invalid well " + std::to_string(w);
            return fail(ISC_ERR_ARG);
        }
        if (controlled) {
            isc::CWell C{};
            C.kind = W.kind;
            C.control = W.kind == ISC_WELL_INJECTOR && W.control != ISC_CTRL_BHP ? 7 : W.control;
            C.c0 = ctx->ncp;
            C.np = W.nperf;
            C.target = W.target;
            C.limit = W.limit;
            C.bhp = W.control == ISC_CTRL_BHP ? W.target : W.limit;
            C.D = 1.0;
            ctx->cw_h.push_back(C);
            ctx->ncp += W.nperf;
            ctx->cw_maxnp = std::max(ctx->cw_maxnp, W.nperf);
        }
        std::vector<int32_t> cells(W.perf_cells_h, W.perf_cells_h + W.nperf);
        for (int32_t c : cells)
            if (c < 0 || c >= n) {
                ctx->err = "well perforation outside the grid";
                return fail(ISC_ERR_ARG);
            }
        ctx->wells.push_back(W);
        ctx->wells.back().perf_cells_h = nullptr;
        ctx->well_cells.push_back(cells);
        npf += W.nperf;
    }
    ctx->npf = npf;
    ctx->ncw = (int32_t)ctx->cw_h.size();

    // device allocations (all workspace lives for the context's lifetime)
    const size_t nv = (size_t)n * isc::NU;
    isc_status s = ISC_OK;
#define ALLOC(p, cnt) if ((s = dalloc(ctx, &(p), (cnt))) != ISC_OK) return fail(s)
    ALLOC(ctx->fluid_d, 1);
    ALLOC(ctx->logk, n);
    ALLOC(ctx->poro, n);
    ALLOC(ctx->trans, (size_t)3 * n);
    ALLOC(ctx->row_ptr, (size_t)n + 1);
    ALLOC(ctx->col_idx, (size_t)ctx->nnzb);
    ALLOC(ctx->diag_pos, (size_t)n);
    ALLOC(ctx->well_slot, (size_t)n);
    ALLOC(ctx->perf, (size_t)std::max(npf, 1) * isc::PERF_W);
    ALLOC(ctx->lvl_rows, (size_t)n);
    ALLOC(ctx->payload, (size_t)n * isc::PL);
    ALLOC(ctx->F, nv);
    ALLOC(ctx->J, (size_t)ctx->nnzb * isc::BS);
    ALLOC(ctx->Dinv, (size_t)n * isc::BS);
    ALLOC(ctx->du, nv);
    ALLOC(ctx->rhs, nv);
    ALLOC(ctx->V, nv * (ctx->mmax + 1));
    ALLOC(ctx->w, nv);
    ALLOC(ctx->tvec, nv);
    ALLOC(ctx->acc_old, nv);
    ALLOC(ctx->partial, (size_t)65 * isc::NPART);   // 64 rows of dot partials + one norm row
    ALLOC(ctx->small, (size_t)4096 + 32 * 32);   // scalars, Hessenberg, delayed-CGS2 state; Rs past 4096
    ALLOC(ctx->flags, (size_t)16);
    ALLOC(ctx->accJ, (size_t)n * isc::BS);
    ALLOC(ctx->qg, nv);
    ALLOC(ctx->qv, (size_t)n);
    ALLOC(ctx->rates, (size_t)n * 4);
    ALLOC(ctx->perf_cell, (size_t)std::max(npf, 1));
    ALLOC(ctx->bricks_fwd, chf.size());
    ALLOC(ctx->bricks_bwd, chb.size());
    ALLOC(ctx->items_bwd_spmv, items.size());
    ALLOC(ctx->sweep64, (size_t)n * isc::NU);
    const size_t lt_cells = (size_t)ctx->nfwd_items * isc::BRICK_X * isc::BRICK_Y * isc::BRICK_Z;
    ALLOC(ctx->Lt, lt_cells * 3 * isc::BS);
    ALLOC(ctx->lt_slot, (size_t)n);
    ALLOC(ctx->b_slot, (size_t)n);
    ALLOC(ctx->items_rank, items_rank.size());
    const size_t b_cells = (size_t)ctx->nbwd_items * isc::BRICK_X * isc::BRICK_Y * isc::BRICK_Z;
    ALLOC(ctx->bpack64, b_cells * 4 * isc::BS);
    ALLOC(ctx->spack64, b_cells * 3 * isc::BS);
    ALLOC(ctx->sweep32, (size_t)n * isc::NU);
    ALLOC(ctx->ticket, (size_t)1);
    ALLOC(ctx->well_off, (size_t)nwells + 1);
    ALLOC(ctx->cw, (size_t)ctx->ncw);
    ALLOC(ctx->cwp, (size_t)ctx->ncp * isc::CWP_W);
    ALLOC(ctx->cwp_cell, (size_t)ctx->ncp);
    ALLOC(ctx->cwp_well, (size_t)ctx->ncp);
    ALLOC(ctx->cwp_nb, (size_t)ctx->ncp * isc::CW_NB * 2);
    ALLOC(ctx->wres, (size_t)1);
    ALLOC(ctx->wsw, (size_t)1);
    ALLOC(ctx->Z, nv * ctx->mmax);
    if (ctx->inner_max > 0) {
        ALLOC(ctx->J32, (size_t)ctx->nnzb * isc::BS);
        ALLOC(ctx->Dinv32, (size_t)n * isc::BS);
        ALLOC(ctx->Lt32, lt_cells * 3 * isc::BS);
        ALLOC(ctx->bpack32, b_cells * 4 * isc::BS);
        ALLOC(ctx->spack32, b_cells * 3 * isc::BS);
        ALLOC(ctx->V32, nv * (ctx->inner_max + 1));
        ALLOC(ctx->w32, nv);
        ALLOC(ctx->t32, nv);
        ALLOC(ctx->small32, (size_t)4096 + 32 * 32);   // as small: Rs past 4096
        ALLOC(ctx->Z32, nv * ctx->inner_max);
    }
    if (mo.precond == ISC_PC_CPR) {   // CPR: multigrid levels and stage-1 buffers
        isc_cpr_plan(ctx);
        if (ctx->mg.back().n > ISC_CPR_COARSEST) {
            ctx->err = "grid too large for the pressure multigrid's level count";
            return fail(ISC_ERR_ARG);
        }
        size_t words = 0;
        for (size_t l = 0; l < ctx->mg.size(); ++l) words += (size_t)2 * ctx->mg[l].lh * (l == 0 ? 7 : 9);
        ALLOC(ctx->mg_store, words);
        // the holes of the colour-split order stay zero in every stencil and vector
        if (hipMemsetAsync(ctx->mg_store, 0, words * sizeof(double), ctx->stream) != hipSuccess) {
            ctx->err = "clearing the CPR levels failed";
            return fail(ISC_ERR_HIP);
        }
        double* p = ctx->mg_store;
        for (size_t l = 0; l < ctx->mg.size(); ++l) {
            isc_ctx::MgLevel& L = ctx->mg[l];
            const size_t ns = (size_t)2 * L.lh;
            L.co = p;
            p += 7 * ns;
            if (l > 0) {
                L.x = p;
                p += ns;
                L.b = p;
                p += ns;
            }
        }
        ctx->cpr_kmax = mo.p_iters;
        ctx->cpr_npad = (int32_t)((2 * (int64_t)ctx->mg[0].lh + 7) & ~7);
        const size_t np = (size_t)ctx->cpr_npad;
        ALLOC(ctx->mg_cinv, (size_t)ISC_CPR_COARSEST * ISC_CPR_COARSEST);
        ALLOC(ctx->cpr_pc, (size_t)ctx->nnzb * 8);
        ALLOC(ctx->cpr_V, np * (ctx->cpr_kmax + 1));
        ALLOC(ctx->cpr_Z, np * std::max(ctx->cpr_kmax, 1));
        ALLOC(ctx->cpr_w, np);
        ALLOC(ctx->cpr_rp, np);
        ALLOC(ctx->cpr_ep, np);
        ALLOC(ctx->cpr_w1, nv);
        ALLOC(ctx->cpr_r2, nv);
        ALLOC(ctx->small_p, (size_t)4096 + 32 * 32);
        // the pressure vectors' padding is read by the Gram-Schmidt passes and must stay zero
        double* zero_bufs[] = {ctx->cpr_V, ctx->cpr_Z, ctx->cpr_w, ctx->cpr_rp, ctx->cpr_ep};
        const size_t zero_len[] = {np * (ctx->cpr_kmax + 1), np * std::max(ctx->cpr_kmax, 1), np, np, np};
        for (int k = 0; k < 5; ++k)
            if (hipMemsetAsync(zero_bufs[k], 0, zero_len[k] * sizeof(double), ctx->stream) != hipSuccess) {
                ctx->err = "clearing the CPR buffers failed";
                return fail(ISC_ERR_HIP);
            }
    }
#undef ALLOC
    if (hipHostMalloc((void**)&ctx->hscratch, 64 * sizeof(double), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&ctx->hflags, 16 * sizeof(int32_t), hipHostMallocDefault) != hipSuccess) {
        ctx->err = "hipHostMalloc failed";
        return fail(ISC_ERR_OOM);
    }
    for (auto& e : ctx->ev)
        if (hipEventCreate(&e) != hipSuccess) {
            ctx->err = "hipEventCreate failed";
            return fail(ISC_ERR_HIP);
        }
    auto h2d = [&](void* dst, const void* src, size_t bytes) {
        return hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, ctx->stream) == hipSuccess;
    };
    ctx->logk_h.resize(n);
    ctx->poro_h.resize(n);
    if (hipMemcpyAsync(ctx->logk_h.data(), logk, (size_t)n * sizeof(double), hipMemcpyDeviceToHost, ctx->stream) !=
            hipSuccess ||
        hipMemcpyAsync(ctx->poro_h.data(), poro, (size_t)n * sizeof(double), hipMemcpyDeviceToHost, ctx->stream) !=
            hipSuccess ||
        hipStreamSynchronize(ctx->stream) != hipSuccess) {
        ctx->err = "cannot read logk/poro (device pointers expected)";
        return fail(ISC_ERR_ARG);
    }
    // wait limit of the sweeps (ISC_SWEEP_WAIT_TICKS overrides it, e.g. to test the timeout path)
    uint64_t wait_ticks = ISC_SWEEP_WAIT_DEFAULT;
    if (const char* e = getenv("ISC_SWEEP_WAIT_TICKS")) wait_ticks = strtoull(e, nullptr, 10);
    if (isc_reset_sweep_buffers(ctx) != hipSuccess ||
        hipMemsetAsync(ctx->ticket, 0, sizeof(unsigned long long), ctx->stream) != hipSuccess ||
        hipMemsetAsync(ctx->flags, 0, 16 * sizeof(int32_t), ctx->stream) != hipSuccess ||
        !h2d(ctx->flags + ISC_FLAG_WAIT, &wait_ticks, sizeof(uint64_t)) ||
        !h2d(ctx->bricks_fwd, chf.data(), chf.size() * sizeof(int32_t)) ||
        !h2d(ctx->bricks_bwd, chb.data(), chb.size() * sizeof(int32_t)) ||
        !h2d(ctx->items_bwd_spmv, items.data(), items.size() * sizeof(int32_t))) {
        ctx->err = "initialising the sweep schedule failed";
        return fail(ISC_ERR_HIP);
    }
    if (!h2d(ctx->fluid_d, &ctx->fluid_h, sizeof(isc_fluid)) ||
        !h2d(ctx->logk, ctx->logk_h.data(), (size_t)n * sizeof(double)) ||
        !h2d(ctx->poro, ctx->poro_h.data(), (size_t)n * sizeof(double)) ||
        !h2d(ctx->row_ptr, ctx->row_ptr_h.data(), ((size_t)n + 1) * sizeof(int32_t)) ||
        !h2d(ctx->col_idx, ctx->col_idx_h.data(), (size_t)ctx->nnzb * sizeof(int32_t)) ||
        !h2d(ctx->diag_pos, ctx->diag_pos_h.data(), (size_t)n * sizeof(int32_t)) ||
        !h2d(ctx->lvl_rows, lvl_rows.data(), (size_t)n * sizeof(int32_t)) ||
        !h2d(ctx->lt_slot, lt_slot.data(), (size_t)n * sizeof(int32_t)) ||
        !h2d(ctx->b_slot, b_slot.data(), (size_t)n * sizeof(int32_t)) ||
        !h2d(ctx->items_rank, items_rank.data(), items_rank.size() * sizeof(int32_t))) {
        ctx->err = "host to device copy failed";
        return fail(ISC_ERR_HIP);
    }
    {
        std::vector<int32_t> pcell, woff(1, 0);
        for (auto& cells : ctx->well_cells) {
            pcell.insert(pcell.end(), cells.begin(), cells.end());
            woff.push_back((int32_t)pcell.size());
        }
        if ((!pcell.empty() && !h2d(ctx->perf_cell, pcell.data(), pcell.size() * sizeof(int32_t))) ||
            !h2d(ctx->well_off, woff.data(), woff.size() * sizeof(int32_t))) {
            ctx->err = "host to device copy failed";
            return fail(ISC_ERR_HIP);
        }
    }
    if (ctx->ncw > 0) {   // controlled wells: perforation lists and the initial state
        std::vector<int32_t> ccell, cwell;
        const double vol = ctx->g.dx * ctx->g.dy * ctx->g.dz;
        int32_t w = 0;
        for (size_t k = 0; k < ctx->wells.size(); ++k) {
            const isc_well& W = ctx->wells[k];
            if (W.kind != ISC_WELL_PRODUCER && W.kind != ISC_WELL_INJECTOR) continue;
            const std::vector<int32_t>& cells = ctx->well_cells[k];
            ccell.insert(ccell.end(), cells.begin(), cells.end());
            cwell.insert(cwell.end(), cells.size(), w);
            ctx->cw_h[w].rscale = vol * ctx->poro_h[cells[0]] * ctx->fluid_h.rho_ref[0];
            ++w;
        }
        // each perforation's in-pattern partners: the same well's perforations
        // at the columns of its cell's stencil row, and those blocks of J
        std::vector<int32_t> nb((size_t)ctx->ncp * isc::CW_NB * 2, -1);
        std::unordered_map<int32_t, int32_t> perf_of;
        for (int32_t p = 0; p < ctx->ncp; ++p) perf_of[ccell[p]] = p;
        for (int32_t p = 0; p < ctx->ncp; ++p) {
            int32_t slot = 0;
            for (int32_t b = ctx->row_ptr_h[ccell[p]]; b < ctx->row_ptr_h[ccell[p] + 1]; ++b) {
                const auto it = perf_of.find(ctx->col_idx_h[b]);
                if (it == perf_of.end() || cwell[it->second] != cwell[p]) continue;
                nb[((size_t)p * isc::CW_NB + slot) * 2] = it->second;
                nb[((size_t)p * isc::CW_NB + slot) * 2 + 1] = b;
                ++slot;
            }
        }
        if (!h2d(ctx->cwp_cell, ccell.data(), ccell.size() * sizeof(int32_t)) ||
            !h2d(ctx->cwp_well, cwell.data(), cwell.size() * sizeof(int32_t)) ||
            !h2d(ctx->cwp_nb, nb.data(), nb.size() * sizeof(int32_t)) ||
            !h2d(ctx->cw, ctx->cw_h.data(), ctx->cw_h.size() * sizeof(isc::CWell)) ||
            hipMemsetAsync(ctx->cwp, 0, (size_t)ctx->ncp * isc::CWP_W * sizeof(double), ctx->stream) != hipSuccess) {
            ctx->err = "host to device copy failed";
            return fail(ISC_ERR_HIP);
        }
    }
    if ((s = rebuild_static(ctx)) != ISC_OK) return fail(s);
    if (hipStreamSynchronize(ctx->stream) != hipSuccess) {
        ctx->err = "stream synchronisation failed";
        return fail(ISC_ERR_HIP);
    }
    *out_h = ctx;
    return ISC_OK;
}

isc_status isc_destroy(isc_ctx* ctx) {
    if (!ctx) return ISC_OK;
    if (ctx->stream) hipStreamSynchronize(ctx->stream);
    else hipDeviceSynchronize();
    void* ptrs[] = {ctx->fluid_d, ctx->logk,  ctx->poro,    ctx->trans,  ctx->row_ptr, ctx->col_idx,
                    ctx->diag_pos, ctx->well_slot, ctx->perf, ctx->lvl_rows, ctx->lt_slot, ctx->b_slot, ctx->items_rank,
                    ctx->bpack64, ctx->spack64, ctx->bpack32, ctx->spack32, ctx->payload, ctx->F,
                    ctx->J,       ctx->Dinv,  ctx->du,      ctx->rhs,    ctx->V,       ctx->Z,
                    ctx->w,       ctx->tvec,  ctx->acc_old, ctx->partial, ctx->small,  ctx->flags,
                    ctx->J32,     ctx->Dinv32, ctx->V32,    ctx->w32,    ctx->t32,
                    ctx->small32, ctx->Z32, ctx->accJ,   ctx->qg,     ctx->qv,     ctx->rates,
                    ctx->perf_cell, ctx->well_off, ctx->bricks_fwd, ctx->bricks_bwd, ctx->sweep64,
                    ctx->sweep32, ctx->ticket, ctx->Lt, ctx->Lt32, ctx->items_bwd_spmv,
                    ctx->mg_store, ctx->mg_cinv, ctx->cpr_pc, ctx->cpr_V, ctx->cpr_Z, ctx->cpr_w,
                    ctx->cpr_rp, ctx->cpr_ep, ctx->cpr_w1, ctx->cpr_r2, ctx->small_p, ctx->cw, ctx->cwp,
                    ctx->cwp_cell, ctx->cwp_well, ctx->cwp_nb, ctx->wres, ctx->wsw};
    for (void* p : ptrs)
        if (p) hipFree(p);
    if (ctx->hscratch) hipHostFree(ctx->hscratch);
    if (ctx->hflags) hipHostFree(ctx->hflags);
    for (auto& e : ctx->ev)
        if (e) hipEventDestroy(e);
    isc_prof_drain(ctx);
    for (auto& e : ctx->prof_pool) hipEventDestroy(e);
    delete ctx;
    return ISC_OK;
}

isc_status isc_set_params(isc_ctx* ctx, const double* logk, const double* A_h) {
    TRY(check_ctx(ctx));
    if (logk) {
        ISC_HIP(hipMemcpyAsync(ctx->logk_h.data(), logk, (size_t)ctx->n * sizeof(double), hipMemcpyDeviceToHost,
                               ctx->stream));
        ISC_HIP(hipStreamSynchronize(ctx->stream));
        ISC_HIP(hipMemcpyAsync(ctx->logk, ctx->logk_h.data(), (size_t)ctx->n * sizeof(double),
                               hipMemcpyHostToDevice, ctx->stream));
        TRY(rebuild_static(ctx));
    }
    if (A_h) {
        for (int r = 0; r < ISC_NREAC; ++r) ctx->fluid_h.Afreq[r] = A_h[r];
        ISC_HIP(hipMemcpyAsync(ctx->fluid_d, &ctx->fluid_h, sizeof(isc_fluid), hipMemcpyHostToDevice, ctx->stream));
        ISC_HIP(hipStreamSynchronize(ctx->stream));
    }
    return ISC_OK;
}

isc_status isc_set_heater(isc_ctx* ctx, int32_t cell, double rate_W) {
    TRY(check_ctx(ctx));
    if (cell >= ctx->n || !std::isfinite(rate_W)) {
        ctx->err = "isc_set_heater: cell outside the grid or rate not finite";
        return ISC_ERR_ARG;
    }
    const bool on = cell >= 0 && rate_W != 0.0;
    ctx->heater_cell = on ? cell : -1;
    ctx->heater_W = on ? rate_W : 0.0;
    return ISC_OK;
}

isc_status isc_bcsr_pattern(const isc_ctx* ctx, const int32_t** row_ptr, const int32_t** col_idx,
                            int32_t* nnzb_h) {
    if (!ctx) return ISC_ERR_ARG;
    if (row_ptr) *row_ptr = ctx->row_ptr;
    if (col_idx) *col_idx = ctx->col_idx;
    if (nnzb_h) *nnzb_h = ctx->nnzb;
    return ISC_OK;
}

isc_status isc_assemble(isc_ctx* ctx, const double* u, const double* u_old, double dt, double* F, double* Jval) {
    TRY(check_ctx(ctx));
    if (!u || !u_old || !F || !Jval || !(dt > 0)) {
        ctx->err = "isc_assemble: invalid argument";
        return ISC_ERR_ARG;
    }
    ISC_HIP(isc_launch_props(ctx, u, u_old, dt));
    ISC_HIP(isc_launch_assemble(ctx, u, F, Jval));
    return ISC_OK;
}

isc_status isc_decouple(isc_ctx* ctx, double* Jval, double* F, int32_t* bad_cell_h) {
    TRY(check_ctx(ctx));
    if (!Jval || !F) {
        ctx->err = "isc_decouple: invalid argument";
        return ISC_ERR_ARG;
    }
    ISC_HIP(isc_launch_decouple(ctx, Jval, F, ctx->flags + FLAG_BAD));
    int32_t bad;
    TRY(read_flag(ctx, FLAG_BAD, &bad));
    if (bad_cell_h) *bad_cell_h = bad == INT32_MAX ? -1 : bad;
    if (bad != INT32_MAX) {
        ctx->err = "isc_decouple: singular diagonal block at cell " + std::to_string(bad);
        return ISC_ERR_SINGULAR;
    }
    return ISC_OK;
}

isc_status isc_bilu0(isc_ctx* ctx, const double* Jdec, double* Dinv) {
    TRY(check_ctx(ctx));
    TRY(reset_flags(ctx));
    ISC_HIP(isc_launch_bilu0_factor(ctx, Jdec, Dinv, ctx->flags + FLAG_BAD));
    int32_t bad;
    TRY(read_flag(ctx, FLAG_BAD, &bad));
    if (bad != INT32_MAX) {
        ctx->err = "block ILU(0): singular pivot block at cell " + std::to_string(bad);
        (void)isc_check_sweeps(ctx);
        return ISC_ERR_SINGULAR;
    }
    return isc_check_sweeps(ctx);
}

isc_status isc_bilu0_apply(isc_ctx* ctx, const double* Jdec, const double* Dinv, const double* r, double* z) {
    TRY(check_ctx(ctx));
    if (r == z) {
        ctx->err = "isc_bilu0_apply: r and z must not alias";
        return ISC_ERR_ARG;
    }
    ISC_HIP(isc_launch_form_ltilde(ctx, Jdec, Dinv));
    ISC_HIP(isc_launch_bilu0_apply(ctx, Jdec, Dinv, r, z));
    return isc_check_sweeps(ctx);
}

isc_status isc_bilu0_apply_spmv(isc_ctx* ctx, const double* Jdec, const double* Dinv, const double* r, double* z,
                                double* w) {
    TRY(check_ctx(ctx));
    if (!Jdec || !Dinv || !r || !z || !w || r == z || r == w || z == w) {
        ctx->err = "isc_bilu0_apply_spmv: null or aliased arrays";
        return ISC_ERR_ARG;
    }
    ISC_HIP(isc_launch_form_ltilde(ctx, Jdec, Dinv));
    ISC_HIP(isc_launch_bilu0_apply_spmv(ctx, Jdec, Dinv, r, z, w));
    return isc_check_sweeps(ctx);
}

isc_status isc_bilu0_apply_spmv32(isc_ctx* ctx, const double* Jdec, const double* r, double* z, double* w) {
    TRY(check_ctx(ctx));
    if (!Jdec || !r || !z || !w || r == z || r == w || z == w) {
        ctx->err = "isc_bilu0_apply_spmv32: null or aliased arrays";
        return ISC_ERR_ARG;
    }
    TRY(reset_flags(ctx));
    TRY(isc_prepare_mixed_dev(ctx, Jdec, ctx->flags + FLAG_BAD));
    int32_t bad;
    TRY(read_flag(ctx, FLAG_BAD, &bad));
    if (bad != INT32_MAX) {
        ctx->err = "block ILU(0) (FP32): singular pivot block at cell " + std::to_string(bad);
        return ISC_ERR_SINGULAR;
    }
    isc_apply_spmv32_from64(ctx, r, z, w);
    ISC_HIP(hipGetLastError());
    return isc_check_sweeps(ctx);
}

isc_status isc_spmv(isc_ctx* ctx, const double* Jdec, const double* x, double* y) {
    TRY(check_ctx(ctx));
    if (x == y) {
        ctx->err = "isc_spmv: x and y must not alias";
        return ISC_ERR_ARG;
    }
    ISC_HIP(isc_launch_spmv(ctx, Jdec, x, y));
    return ISC_OK;
}

isc_status isc_solve(isc_ctx* ctx, const double* Jdec, const double* b, double* x, const isc_solve_opts* o,
                     isc_solve_info* info_h) {
    TRY(check_ctx(ctx));
    if (!Jdec || !b || !x || !o || x == b) {
        ctx->err = "isc_solve: invalid argument";
        return ISC_ERR_ARG;
    }
    if (o->restart < 1 || o->restart > ctx->mmax || o->max_restarts < 1 || !(o->rtol > 0)) {
        ctx->err = "isc_solve: restart must be in [1, max restart of the context], max_restarts >= 1, rtol > 0";
        return ISC_ERR_ARG;
    }
    TRY(check_precond(ctx, o, "isc_solve"));
    if (o->krylov == ISC_KRYLOV_BICGSTAB)
        return isc_solve_bicgstab(ctx, Jdec, b, x, o->restart * o->max_restarts, o->rtol, info_h);
    if (o->precond == ISC_PC_CPR) {
        TRY(isc_bilu0(ctx, Jdec, ctx->Dinv));
        TRY(reset_flags(ctx));
        ISC_HIP(isc_cpr_setup(ctx, Jdec, ctx->flags + FLAG_BAD));
        int32_t bad;
        TRY(read_flag(ctx, FLAG_BAD, &bad));
        if (bad != INT32_MAX) {
            ctx->err = "CPR: the coarsest pressure matrix is singular";
            return ISC_ERR_SINGULAR;
        }
        return isc_fgmres(ctx, Jdec, b, x, o, info_h);
    }
    if (o->precision == ISC_MIXED) {
        TRY(reset_flags(ctx));
        TRY(isc_prepare_mixed_dev(ctx, Jdec, ctx->flags + FLAG_BAD));
        int32_t bad;
        TRY(read_flag(ctx, FLAG_BAD, &bad));
        if (bad != INT32_MAX) {
            ctx->err = "block ILU(0) (FP32): singular pivot block at cell " + std::to_string(bad);
            return ISC_ERR_SINGULAR;
        }
        return isc_fgmres(ctx, Jdec, b, x, o, info_h);
    }
    TRY(isc_bilu0(ctx, Jdec, ctx->Dinv));
    return isc_gmres_fp64(ctx, Jdec, ctx->Dinv, b, x, o, info_h);
}

// factor + CPR set-up for Jdec (component entry points below)
static isc_status cpr_prepare(isc_ctx* ctx, const double* Jdec, int32_t p_iters, const char* who) {
    isc_solve_opts o{1, 1, ISC_FP64, 0, ISC_PC_CPR, p_iters, 1e-8};
    TRY(check_precond(ctx, &o, who));
    TRY(isc_bilu0(ctx, Jdec, ctx->Dinv));
    TRY(reset_flags(ctx));
    ISC_HIP(isc_cpr_setup(ctx, Jdec, ctx->flags + FLAG_BAD));
    int32_t bad;
    TRY(read_flag(ctx, FLAG_BAD, &bad));
    if (bad != INT32_MAX) {
        ctx->err = std::string(who) + ": the coarsest pressure matrix is singular";
        return ISC_ERR_SINGULAR;
    }
    return ISC_OK;
}

isc_status isc_cpr_pressure_solve(isc_ctx* ctx, const double* Jdec, int32_t p_iters, const double* rp, double* e) {
    TRY(check_ctx(ctx));
    if (!Jdec || !rp || !e) {
        ctx->err = "isc_cpr_pressure_solve: null argument";
        return ISC_ERR_ARG;
    }
    TRY(cpr_prepare(ctx, Jdec, p_iters, "isc_cpr_pressure_solve"));
    isc_cpr_to_split(ctx, rp, ctx->cpr_rp);
    isc_cpr_pressure_gmres(ctx, ctx->cpr_rp, ctx->cpr_ep, p_iters);
    isc_cpr_from_split(ctx, ctx->cpr_ep, e);
    ISC_HIP(hipStreamSynchronize(ctx->stream));
    return isc_check_sweeps(ctx);
}

isc_status isc_cpr_apply(isc_ctx* ctx, const double* Jdec, int32_t p_iters, const double* r, double* z, double* w) {
    TRY(check_ctx(ctx));
    if (!Jdec || !r || !z || !w || r == z || r == w || z == w) {
        ctx->err = "isc_cpr_apply: null or aliased arrays";
        return ISC_ERR_ARG;
    }
    TRY(cpr_prepare(ctx, Jdec, p_iters, "isc_cpr_apply"));
    isc_cpr_apply_w(ctx, Jdec, r, z, w, p_iters);
    ISC_HIP(hipGetLastError());
    return isc_check_sweeps(ctx);
}

isc_status isc_update(isc_ctx* ctx, double* u, const double* du) {
    TRY(check_ctx(ctx));
    TRY(reset_flags(ctx));
    ISC_HIP(isc_launch_update(ctx, u, du, ctx->flags + FLAG_NONFIN));
    int32_t nf;
    TRY(read_flag(ctx, FLAG_NONFIN, &nf));
    if (nf) {
        ctx->err = "isc_update: non-finite state after the Newton update";
        return ISC_ERR_NONFINITE;
    }
    return ISC_OK;
}

isc_status isc_scaled_norm(isc_ctx* ctx, const double* F, double dt, double* res_h) {
    TRY(check_ctx(ctx));
    ISC_HIP(isc_launch_scaled_norm(ctx, F, dt, ctx->small + 3000));
    ISC_HIP(hipMemcpyAsync(ctx->hscratch, ctx->small + 3000, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    ISC_HIP(hipStreamSynchronize(ctx->stream));
    *res_h = ctx->hscratch[0];
    isc_prof_drain(ctx);
    return ISC_OK;
}

isc_status isc_newton_step(isc_ctx* ctx, double* u, const double* u_old, double dt, const isc_newton_opts* o,
                           isc_newton_info* info_h) {
    TRY(check_ctx(ctx));
    if (!u || !u_old || !o || !(dt > 0)) {
        ctx->err = "isc_newton_step: invalid argument";
        return ISC_ERR_ARG;
    }
    isc_newton_info inf{};
    inf.bad_cell = -1;
    hipEvent_t* ev = ctx->ev;
    const bool wells = ctx->ncw > 0;
    ISC_HIP(hipEventRecord(ev[0], ctx->stream));
    int tk = isc_prof_begin(ctx, ISC_PROF_ASSEMBLE);
    if (wells) ISC_HIP(isc_launch_well_line(ctx, u, 0));   // the rate wells' equations alone, for bhp
    ISC_HIP(isc_launch_props(ctx, u, u_old, dt));
    ISC_HIP(isc_launch_assemble(ctx, u, ctx->F, ctx->J));
    if (wells) {
        ISC_HIP(isc_launch_well_rows(ctx, u));
        ISC_HIP(isc_launch_well_reduce(ctx, dt));
    }
    isc_prof_end(ctx, tk);
    ISC_HIP(hipEventRecord(ev[1], ctx->stream));
    double res;
    TRY(isc_scaled_norm(ctx, ctx->F, dt, &res));
    if (wells) {
        ISC_HIP(hipMemcpyAsync(ctx->hscratch + 16, ctx->wres, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
        ISC_HIP(hipStreamSynchronize(ctx->stream));
        const double rw = ctx->hscratch[16];
        if (!(rw <= res)) res = rw;
    }
    inf.res_scaled = res;
    if (!std::isfinite(res)) {
        ctx->err = "isc_newton_step: non-finite residual";
        if (info_h) *info_h = inf;
        return ISC_ERR_NONFINITE;
    }
    if (res <= o->tol) {
        inf.converged = 1;
        ISC_HIP(hipEventElapsedTime(&inf.ms_assemble, ev[0], ev[1]));
        if (info_h) *info_h = inf;
        return ISC_OK;
    }
    TRY(reset_flags(ctx));
    tk = isc_prof_begin(ctx, ISC_PROF_DECOUPLE);
    if (wells) ISC_HIP(isc_launch_well_fold(ctx, ctx->J));
    ISC_HIP(isc_launch_decouple(ctx, ctx->J, ctx->F, ctx->flags + FLAG_BAD));
    isc_prof_end(ctx, tk);
    ISC_HIP(isc_launch_negate(ctx, ctx->F, ctx->rhs));
    if (wells) ISC_HIP(isc_launch_well_rhs(ctx, ctx->rhs));
    ISC_HIP(hipEventRecord(ev[2], ctx->stream));
    isc_status st;
    TRY(check_precond(ctx, &o->lin, "isc_newton_step"));
    const bool cpr = o->lin.precond == ISC_PC_CPR;
    if (o->lin.precision == ISC_MIXED && !cpr) {
        tk = isc_prof_begin(ctx, ISC_PROF_ILU_FACTOR);
        TRY(isc_prepare_mixed_dev(ctx, ctx->J, ctx->flags + FLAG_BAD));
        isc_prof_end(ctx, tk);
    } else {
        tk = isc_prof_begin(ctx, ISC_PROF_ILU_FACTOR);
        ISC_HIP(isc_launch_bilu0_factor(ctx, ctx->J, ctx->Dinv, ctx->flags + FLAG_BAD));
        isc_prof_end(ctx, tk);
        if (cpr) {   // a singular coarsest pressure matrix reports cell 0
            tk = isc_prof_begin(ctx, ISC_PROF_CPR_SETUP);
            ISC_HIP(isc_cpr_setup(ctx, ctx->J, ctx->flags + FLAG_BAD));
            isc_prof_end(ctx, tk);
        }
    }
    ISC_HIP(hipEventRecord(ev[3], ctx->stream));
    int32_t bad;
    TRY(read_flag(ctx, FLAG_BAD, &bad));
    if (bad != INT32_MAX) {
        inf.bad_cell = bad;
        ctx->err = "isc_newton_step: singular block at cell " + std::to_string(bad);
        if (info_h) *info_h = inf;
        return ISC_ERR_SINGULAR;
    }
    if (o->lin.restart < 1 || o->lin.restart > ctx->mmax) {
        ctx->err = "isc_newton_step: restart exceeds the context's maximum";
        return ISC_ERR_ARG;
    }
    ctx->border = wells;   // the Krylov operator takes the eliminated well rows
    if (o->lin.krylov == ISC_KRYLOV_BICGSTAB)
        st = isc_bicgstab_run(ctx, ctx->J, ctx->rhs, ctx->du, o->lin.restart * o->lin.max_restarts, o->lin.rtol,
                              &inf.lin);
    else if (o->lin.precision == ISC_MIXED || cpr)
        st = isc_fgmres(ctx, ctx->J, ctx->rhs, ctx->du, &o->lin, &inf.lin);
    else
        st = isc_gmres_fp64(ctx, ctx->J, ctx->Dinv, ctx->rhs, ctx->du, &o->lin, &inf.lin);
    ctx->border = false;
    ISC_HIP(hipEventRecord(ev[4], ctx->stream));
    if (st != ISC_OK) {
        if (info_h) *info_h = inf;
        return st;
    }
    ISC_HIP(isc_launch_update(ctx, u, ctx->du, ctx->flags + FLAG_NONFIN));
    if (wells) ISC_HIP(isc_launch_well_update(ctx, ctx->du, ctx->flags + FLAG_NONFIN));
    ISC_HIP(hipEventRecord(ev[5], ctx->stream));
    int32_t nf;
    TRY(read_flag(ctx, FLAG_NONFIN, &nf));
    ISC_HIP(hipEventElapsedTime(&inf.ms_assemble, ev[0], ev[1]));
    ISC_HIP(hipEventElapsedTime(&inf.ms_decouple, ev[1], ev[2]));
    ISC_HIP(hipEventElapsedTime(&inf.ms_precond, ev[2], ev[3]));
    ISC_HIP(hipEventElapsedTime(&inf.ms_krylov, ev[3], ev[4]));
    ISC_HIP(hipEventElapsedTime(&inf.ms_update, ev[4], ev[5]));
    if (info_h) *info_h = inf;
    if (nf) {
        ctx->err = "isc_newton_step: non-finite state after the update";
        return ISC_ERR_NONFINITE;
    }
    return ISC_OK;
}

isc_status isc_adjoint(isc_ctx* ctx, const double* u_n, const double* u_nm1, double dt_n, const double* lam_np1,
                       double dt_np1, double* lam_n, double* g_logk, double* g_A_h, const isc_solve_opts* opts_h,
                       isc_solve_info* info_h) {
    TRY(check_ctx(ctx));
    if (ctx->ncw > 0) {
        ctx->err = "isc_adjoint: the well rows of bhp unknowns are not part of the adjoint";
        return ISC_ERR_ARG;
    }
    return isc_adjoint_impl(ctx, u_n, u_nm1, dt_n, lam_np1, dt_np1, lam_n, g_logk, g_A_h, opts_h, info_h);
}

isc_status isc_oil_rate(isc_ctx* ctx, const double* u, double* q_h) {
    TRY(check_ctx(ctx));
    if (!u || !q_h) {
        ctx->err = "isc_oil_rate: invalid argument";
        return ISC_ERR_ARG;
    }
    return isc_oil_rate_impl(ctx, u, q_h);
}

// ---- controlled wells

namespace {
isc_status read_wells(isc_ctx* ctx, std::vector<isc::CWell>& cw) {
    cw.resize((size_t)ctx->ncw);
    if (ctx->ncw == 0) return ISC_OK;
    ISC_HIP(hipMemcpyAsync(cw.data(), ctx->cw, cw.size() * sizeof(isc::CWell), hipMemcpyDeviceToHost, ctx->stream));
    ISC_HIP(hipStreamSynchronize(ctx->stream));
    return ISC_OK;
}

isc_status well_line(isc_ctx* ctx, const double* u, int mode, int32_t* nswitch_h, const char* who) {
    TRY(check_ctx(ctx));
    if (!u) {
        ctx->err = std::string(who) + ": invalid argument";
        return ISC_ERR_ARG;
    }
    if (ctx->ncw == 0) {
        if (nswitch_h) *nswitch_h = 0;
        return ISC_OK;
    }
    ISC_HIP(hipMemsetAsync(ctx->wsw, 0, sizeof(int32_t), ctx->stream));
    ISC_HIP(isc_launch_well_line(ctx, u, mode));
    int32_t nsw = 0;
    ISC_HIP(hipMemcpyAsync(&nsw, ctx->wsw, sizeof(int32_t), hipMemcpyDeviceToHost, ctx->stream));
    ISC_HIP(hipStreamSynchronize(ctx->stream));
    if (nswitch_h) *nswitch_h = nsw;
    return ISC_OK;
}
}  // namespace

isc_status isc_well_count(const isc_ctx* ctx, int32_t* ncw_h, int32_t* ncp_h) {
    TRY(check_ctx(ctx));
    if (ncw_h) *ncw_h = ctx->ncw;
    if (ncp_h) *ncp_h = ctx->ncp;
    return ISC_OK;
}

isc_status isc_well_state(isc_ctx* ctx, double* bhp_h, int32_t* on_limit_h) {
    TRY(check_ctx(ctx));
    std::vector<isc::CWell> cw;
    TRY(read_wells(ctx, cw));
    for (size_t w = 0; w < cw.size(); ++w) {
        if (bhp_h) bhp_h[w] = cw[w].bhp;
        if (on_limit_h) on_limit_h[w] = cw[w].on_limit;
    }
    return ISC_OK;
}

isc_status isc_set_well_state(isc_ctx* ctx, const double* bhp_h, const int32_t* on_limit_h) {
    TRY(check_ctx(ctx));
    std::vector<isc::CWell> cw;
    TRY(read_wells(ctx, cw));
    for (size_t w = 0; w < cw.size(); ++w) {
        if (bhp_h) {
            if (!std::isfinite(bhp_h[w])) {
                ctx->err = "isc_set_well_state: non-finite bhp";
                return ISC_ERR_ARG;
            }
            cw[w].bhp = bhp_h[w];
        }
        if (on_limit_h) cw[w].on_limit = on_limit_h[w] ? 1 : 0;
    }
    if (!cw.empty()) {
        ISC_HIP(hipMemcpyAsync(ctx->cw, cw.data(), cw.size() * sizeof(isc::CWell), hipMemcpyHostToDevice,
                               ctx->stream));
        ISC_HIP(hipStreamSynchronize(ctx->stream));
    }
    return ISC_OK;
}

isc_status isc_well_controls(isc_ctx* ctx, const double* u, int32_t* nswitch_h) {
    return well_line(ctx, u, 1, nswitch_h, "isc_well_controls");
}

isc_status isc_well_solve(isc_ctx* ctx, const double* u, int32_t* nswitch_h) {
    return well_line(ctx, u, 0, nswitch_h, "isc_well_solve");
}

isc_status isc_well_border(isc_ctx* ctx, const double* u, const double* u_old, double dt, double* R_h, double* D_h,
                           double* B, double* C) {
    TRY(check_ctx(ctx));
    if (!u || !u_old || !(dt > 0)) {
        ctx->err = "isc_well_border: invalid argument";
        return ISC_ERR_ARG;
    }
    if (ctx->ncw == 0) return ISC_OK;
    ISC_HIP(isc_launch_props(ctx, u, u_old, dt));
    ISC_HIP(isc_launch_assemble(ctx, u, ctx->F, ctx->J));
    ISC_HIP(isc_launch_well_rows(ctx, u));
    ISC_HIP(isc_launch_well_reduce(ctx, dt));
    const size_t pitch = (size_t)isc::CWP_W * sizeof(double);
    if (B) ISC_HIP(hipMemcpy2DAsync(B, 8 * sizeof(double), ctx->cwp + isc::CWP_B, pitch, 8 * sizeof(double),
                                    (size_t)ctx->ncp, hipMemcpyDeviceToDevice, ctx->stream));
    if (C) ISC_HIP(hipMemcpy2DAsync(C, 8 * sizeof(double), ctx->cwp + isc::CWP_C, pitch, 8 * sizeof(double),
                                    (size_t)ctx->ncp, hipMemcpyDeviceToDevice, ctx->stream));
    std::vector<isc::CWell> cw;
    TRY(read_wells(ctx, cw));
    for (size_t w = 0; w < cw.size(); ++w) {
        if (R_h) R_h[w] = cw[w].R;
        if (D_h) D_h[w] = cw[w].D;
    }
    return ISC_OK;
}

isc_status isc_profile(isc_ctx* ctx, int32_t enable, double* ms_h, int32_t* count_h) {
    TRY(check_ctx(ctx));
    ISC_HIP(hipStreamSynchronize(ctx->stream));
    isc_prof_drain(ctx);
    if (enable == 1) {
        for (int c = 0; c < ISC_PROF_NCLASS; ++c) {
            ctx->prof_ms[c] = 0.0;
            ctx->prof_cnt[c] = 0;
            ctx->prof_vec[c] = 0.0;
        }
        ctx->prof = true;
    } else if (enable == 0) {
        ctx->prof = false;
    }
    for (int c = 0; c < ISC_PROF_NCLASS; ++c) {
        if (ms_h) ms_h[c] = ctx->prof_ms[c];
        if (count_h) count_h[c] = ctx->prof_cnt[c];
    }
    return ISC_OK;
}

isc_status isc_profile_vectors(isc_ctx* ctx, double* vec_h) {
    TRY(check_ctx(ctx));
    if (!vec_h) {
        ctx->err = "isc_profile_vectors: null output";
        return ISC_ERR_ARG;
    }
    for (int c = 0; c < ISC_PROF_NCLASS; ++c) vec_h[c] = ctx->prof_vec[c];
    return ISC_OK;
}

const char* isc_last_error(const isc_ctx* ctx) {
    if (ctx) return ctx->err.c_str();
    return g_noctx_err.empty() ? "null context" : g_noctx_err.c_str();
}

}  // extern "C"
