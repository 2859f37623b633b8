// Shared device/host definitions of libisc (HIP, gfx950).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/isc.h"

namespace isc {

constexpr int NU = 8;        // unknowns per cell
constexpr int BS = 64;       // 8x8 block
// cells of one brick of the sync-free triangular sweeps (one workgroup, eight
// threads per cell)
#ifndef ISC_BRICK_X
#define ISC_BRICK_X 4
#endif
#ifndef ISC_BRICK_Y
#define ISC_BRICK_Y 4
#endif
#ifndef ISC_BRICK_Z
#define ISC_BRICK_Z 2
#endif
constexpr int BRICK_X = ISC_BRICK_X, BRICK_Y = ISC_BRICK_Y, BRICK_Z = ISC_BRICK_Z;
constexpr int BRICK_THREADS = BRICK_X * BRICK_Y * BRICK_Z * 8;
// A sweep workgroup takes one brick, or two side by side under one ticket
// (the work lists are padded for two)
constexpr int MAX_BRICKS_PER_WG = 2;

// Lane l's value, read into a scalar register (l the same on every lane).
__device__ __forceinline__ double read_lane(double v, int l) {
    const uint64_t b = (uint64_t)__double_as_longlong(v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), l);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// The delayed Gram-Schmidt update of the previous GMRES iteration, done by
// the forward sweep for its own rows before sweeping:
//   q_{j-1} = (u - sum_{k<j-1} s_k Q_k) / omega,
//   u      <- (w - sum_{k<j-1} z_k Q_k - zeta q_{j-1}) / omega,
// the new u being the sweep's right-hand side.  jq = j - 1 is the index of
// the basis vector written; s, z: coefficients; omz = (omega, zeta).  TV is
// the storage of the basis and the vectors (the arithmetic is FP64).
template <class TV>
struct LagUpdateT {
    TV* Q;
    int64_t ldv;
    int jq;
    const double* s;
    const double* z;
    const double* omz;
    TV* u;
    const TV* w;
};
using LagUpdate = LagUpdateT<double>;

// A well whose bottom-hole pressure is an unknown (kinds ISC_WELL_PRODUCER
// and ISC_WELL_INJECTOR), device resident: its control, its state (bhp and
// whether it is held at its BHP limit) and its row of the last assembly.
struct CWell {
    int32_t kind, control;    // 3 / 4; ISC_CTRL_BHP or a phase mask
    int32_t c0, np;           // its perforations [c0, c0 + np) of the controlled-perforation list
    double target, limit;
    double bhp;               // state
    int32_t on_limit;         // state: rate control suspended at the BHP limit
    int32_t pad;
    double R, D;              // well equation's residual and dR/dbhp at the last assembly
    double rscale;            // rate rows: V phi rho_ref,W of its first perforated cell (divided by dt)
};
// per controlled perforation: B = dF_cell/dbhp, C = dq/du_cell, the rate q
// and dq/dbhp it adds to its well, Bt = J_ii^-1 B (J_ii after the fold of
// the well's in-pattern couplings)
constexpr int CWP_B = 0, CWP_C = 8, CWP_Q = 16, CWP_DQ = 17, CWP_BT = 18, CWP_W = 26;
constexpr int CW_MAXPERF = 2048;   // perforations of one controlled well (LDS of the well-line solve)
constexpr int CW_NB = 8;           // slots of a perforation's in-pattern partner list (stencil of 7)
// Per-cell property payload written by the property pass and read by the
// face-flux assembly (doubles, value followed by the 8 partial derivatives):
//   [0, 72)     local residual terms of the 8 rows (accumulation change,
//               reactions, wells)
//   [72, 180)   12 mobility-weighted carried quantities lambda_a * xi_{e,a}
//   [180, 207)  specific weights gamma_w, gamma_o, gamma_g
//   [207, 216)  bulk thermal conductivity K_T
constexpr int PL_LOCAL = 0;
constexpr int PL_MOB = 72;
constexpr int PL_GAM = 180;
constexpr int PL_KT = 207;
constexpr int PL = 216;
constexpr int NMOB = 12;
// carried-quantity slot of (phase, row), -1 if the row's species is absent
// from the phase.  Phases: 0 water, 1 oil, 2 gas.
__host__ __device__ constexpr int mob_slot(int a, int e) {
    return a == 0 ? (e == 0 ? 0 : e == 6 ? 1 : -1)
         : a == 1 ? (e == 1 ? 2 : e == 2 ? 3 : e == 6 ? 4 : -1)
                  : (e <= 5 ? 5 + e : e == 6 ? 11 : -1);
}

// Value and one directional derivative.  The property pass runs eight lanes
// per cell; lane k carries d/du_k, so a cell's full 8-gradient is spread over
// its eight lanes and every lane computes the same values (the branch taken
// therefore agrees across the lanes of a cell).
struct G1 {
    double v, d;
};
__device__ __forceinline__ G1 gconst(double x) { return G1{x, 0.0}; }
__device__ __forceinline__ G1 operator+(G1 a, G1 b) { return G1{a.v + b.v, a.d + b.d}; }
__device__ __forceinline__ G1 operator-(G1 a, G1 b) { return G1{a.v - b.v, a.d - b.d}; }
__device__ __forceinline__ G1 operator-(G1 a) { return G1{-a.v, -a.d}; }
__device__ __forceinline__ G1 operator*(G1 a, G1 b) { return G1{a.v * b.v, a.d * b.v + a.v * b.d}; }
__device__ __forceinline__ G1 operator*(double s, G1 a) { return G1{s * a.v, s * a.d}; }
__device__ __forceinline__ G1 operator*(G1 a, double s) { return G1{s * a.v, s * a.d}; }
__device__ __forceinline__ G1 operator+(G1 a, double s) { return G1{a.v + s, a.d}; }
__device__ __forceinline__ G1 operator+(double s, G1 a) { return G1{a.v + s, a.d}; }
__device__ __forceinline__ G1 operator-(G1 a, double s) { return G1{a.v - s, a.d}; }
__device__ __forceinline__ G1 operator-(double s, G1 a) { return G1{s - a.v, -a.d}; }
__device__ __forceinline__ G1 operator/(G1 a, G1 b) {
    const double q = a.v / b.v;
    return G1{q, (a.d - q * b.d) / b.v};
}
__device__ __forceinline__ G1 operator/(G1 a, double s) { return G1{a.v / s, a.d / s}; }
__device__ __forceinline__ G1 operator/(double s, G1 b) {
    const double q = s / b.v;
    return G1{q, -q * b.d / b.v};
}
__device__ __forceinline__ G1 gexp(G1 a) { const double e = exp(a.v); return G1{e, e * a.d}; }
__device__ __forceinline__ G1 gpow(G1 a, double c) {
    const double p = pow(a.v, c);
    return G1{p, c * p / a.v * a.d};
}

}  // namespace isc

// ---------------------------------------------------------------- context
struct isc_ctx {
    int dev = 0;
    hipStream_t stream = nullptr;
    isc_grid g{};
    int32_t n = 0, nnzb = 0;
    double kvkh = 1.0;
    isc_fluid fluid_h{};
    isc_fluid* fluid_d = nullptr;
    // static fields
    double* logk = nullptr;
    double* poro = nullptr;
    double* trans = nullptr;        // [3][N]: +x, +y, +z face transmissibility of cell i
    std::vector<double> logk_h, poro_h;
    // pattern
    int32_t *row_ptr = nullptr, *col_idx = nullptr, *diag_pos = nullptr;
    std::vector<int32_t> row_ptr_h, col_idx_h, diag_pos_h;
    // wells
    std::vector<isc_well> wells;
    std::vector<std::vector<int32_t>> well_cells;
    int32_t npf = 0;
    int32_t heater_cell = -1;       // heat source into one cell's energy balance (isc_set_heater)
    double heater_W = 0.0;
    int32_t* well_slot = nullptr;   // [N] perforation index or -1
    // controlled wells (bhp unknowns): their perforations are listed in well
    // order; the Krylov operator of isc_newton_step subtracts the eliminated
    // well rows while `border` is set
    int32_t ncw = 0, ncp = 0, cw_maxnp = 0;   // wells, perforations, most perforations of one well
    std::vector<isc::CWell> cw_h;   // set-up copy (the state lives on the device)
    isc::CWell* cw = nullptr;       // [ncw]
    double* cwp = nullptr;          // [ncp][CWP_W]
    int32_t* cwp_cell = nullptr;    // [ncp] perforated cell
    int32_t* cwp_well = nullptr;    // [ncp] its well
    int32_t* cwp_nb = nullptr;      // [ncp][CW_NB][2] the same well's perforations whose cells
                                    // are in this cell's stencil row (itself included): the
                                    // perforation and the block of J between them; -1 past the end
    double* wres = nullptr;         // [1] scaled residual of the well rows
    int32_t* wsw = nullptr;         // [1] wells switched by the last well-line pass
    bool border = false;
    double* perf = nullptr;         // [npf][PERF_W]
    std::vector<double> perf_h;
    // hyperplane level schedule for the ILU recurrences
    int32_t nlev = 0;
    std::vector<int32_t> lvl_off_h;
    int32_t* lvl_rows = nullptr;
    // sync-free triangular sweeps: bricks listed by ascending (forward) and
    // descending (backward) brick level; tickets order the workgroups
    bool syncfree = true;
    int32_t nbrick = 0;
    // lengths of the three sweep work lists: each group of mutually independent
    // items (a brick level, or the SpMV bricks of one level) is padded with
    // inactive bricks to a multiple of MAX_BRICKS_PER_WG, so bricks sharing a
    // workgroup never wait for one another
    int32_t nfwd_items = 0, nbwd_items = 0, nfused_items = 0;
    // L D^-1 blocks are stored in forward-sweep order: cell i's three blocks
    // sit at slot lt_slot[i] = (position of its brick in the forward list) x
    // brick cells + its index in the brick, so the sweep streams them
    int32_t* lt_slot = nullptr;
    // The backward sweep's blocks (U x+, U y+, U z+, D^-1) and the SpMV's lower
    // blocks (z-, y-, x-) are written by the factor (or copied for a factor
    // given from outside) into packs in
    // backward-list order: cell i at slot b_slot[i] (its brick's position in
    // the backward list x brick cells + its index in the brick).  items_rank
    // gives each fused work item that position.
    int32_t* b_slot = nullptr;
    int32_t* items_rank = nullptr;
    double* bpack64 = nullptr;   // [slots][4][64]
    double* spack64 = nullptr;   // [slots][3][64]
    float* bpack32 = nullptr;
    float* spack32 = nullptr;
    // Sync-free sweeps run as cooperative launches with a static schedule (no
    // ticket atomics); if a cooperative launch is refused they take tickets.
    bool coop = true;
    // FP64 GMRES: fold the delayed Gram-Schmidt update into the forward sweep
    // (off: a separate pass launched while the host reads the residual
    // estimate, which measured faster under the static sweep schedule)
    bool fold_update = false;
    // bricks per sweep workgroup under tickets: 2 halves the ticket atomics,
    // which bound the sweeps on large grids; 1 keeps bricks uncoupled where the
    // chain of waits dominates (small grids), and always under the static
    // schedule
    int32_t bpw = 1;
    // co-resident workgroups per sweep kernel
    std::vector<std::pair<const void*, int32_t>> grid_cache;
    int32_t* bricks_fwd = nullptr;
    int32_t* bricks_bwd = nullptr;
    int32_t* items_bwd_spmv = nullptr;   // [2 nbrick] backward bricks interleaved with SpMV bricks
    double* Lt = nullptr;        // [N][3][8][8] L D^-1 blocks of the last BILU(0) factor (z-, y-, x-)
    float* Lt32 = nullptr;       // the same for the FP32 factor of the precision form
    double* sweep64 = nullptr;   // private forward-sweep buffers, sentinel-filled between sweeps
    float* sweep32 = nullptr;
    unsigned long long* ticket = nullptr;
    unsigned long long ticket_base = 0;
    // workspace
    double* payload = nullptr;      // [N][PL]
    double* F = nullptr;            // [N][8]
    double* J = nullptr;            // [nnzb][64]
    double* Dinv = nullptr;         // [N][64]
    double* du = nullptr;           // [N][8]
    double* rhs = nullptr;          // [N][8]
    // Krylov
    int32_t mmax = 30, inner_max = 0;
    double* V = nullptr;            // [(mmax+1)][N*8]
    double* Z = nullptr;            // [mmax][N*8] preconditioned lagged vectors z_j = P(u_j)
    double* w = nullptr;            // [N*8]
    double* tvec = nullptr;         // [N*8]
    double* acc_old = nullptr;      // [N][8] accumulation at the previous time level (property pass)
    double* partial = nullptr;      // [65][NPART] block partial sums
    double* small = nullptr;        // device scalars: reductions, Hessenberg, Givens, g, y, delayed-CGS2 state
    int32_t* flags = nullptr;       // device ints: [0] error/bad cell
    // FP32 copies (mixed precision)
    float* J32 = nullptr;           // [nnzb][64]
    float* Dinv32 = nullptr;        // [N][64]
    float* V32 = nullptr;           // [(inner+1)][N*8]
    float* w32 = nullptr;
    float* t32 = nullptr;
    double* small32 = nullptr;
    float* Z32 = nullptr;           // [inner][N*8] the inner solver's z_j = P(u_j)
    // CPR preconditioner (cpr.hip): the levels of the pressure multigrid and
    // the stage-1 buffers; allocated when the context's maximum options ask
    // for CPR (cpr_kmax = the most pressure GMRES steps, -1 = not allocated)
    struct MgLevel {
        int32_t nx, ny, nz, n;
        int32_t hx, lh;   // colour-split order: positions per row and colour, per colour
        double* co;       // [7][2 lh] stencil
        double* x;        // [2 lh] (levels >= 1; level 0 uses the caller's vectors)
        double* b;        // [2 lh]
    };
    std::vector<MgLevel> mg;
    int32_t cpr_kmax = -1;
    int32_t mg_fused_first = 0;    // levels from this one down run in one workgroup launch
    int32_t cpr_npad = 0;          // pressure vector length (colour-split order), padded to a multiple of 8
    double* mg_store = nullptr;    // all levels' stencils and vectors
    double* mg_cinv = nullptr;     // [nc][nc] inverse of the coarsest matrix
    double* cpr_pc = nullptr;      // [nnzb][8] column 0 of every block of the decoupled matrix
    double* cpr_V = nullptr;       // pressure GMRES basis [(kmax + 1)][npad]
    double* cpr_Z = nullptr;       // [kmax][npad] its preconditioned vectors
    double* cpr_w = nullptr;       // [npad]
    double* cpr_rp = nullptr;      // [npad] pressure part of the residual
    double* cpr_ep = nullptr;      // [npad] stage-1 pressure correction
    double* cpr_w1 = nullptr;      // [N][8] A E e_p
    double* cpr_r2 = nullptr;      // [N][8] stage-2 residual
    double* small_p = nullptr;     // small dense state of the pressure GMRES
    // adjoint workspace
    double* accJ = nullptr;         // [N][64] accumulation Jacobian
    double* qg = nullptr;           // [N][8]  producer oil-rate gradient
    double* qv = nullptr;           // [N]     producer oil rate
    double* rates = nullptr;        // [N][4]  reaction rates
    int32_t* perf_cell = nullptr;   // [npf]
    int32_t* well_off = nullptr;    // [nwells + 1] perforation ranges
    // host pinned scratch
    double* hscratch = nullptr;     // 64 doubles
    int32_t* hflags = nullptr;
    hipEvent_t ev[8] = {};
    std::string err;
    // kernel-class timing (isc_profile)
    bool prof = false;
    double prof_ms[ISC_PROF_NCLASS] = {};
    int32_t prof_cnt[ISC_PROF_NCLASS] = {};
    double prof_vec[ISC_PROF_NCLASS] = {};   // isc_profile_vectors
    struct Pending { int cls; hipEvent_t a, b; };
    std::vector<Pending> prof_pending;
    std::vector<hipEvent_t> prof_pool;
};

namespace isc {
// perforation table: kind, wi, bhp, q[7], qE, q_total (kinds 1, 2);
// kinds 3, 4: kind, wi, controlled well, z_inj[7], H_inj, controlled perforation
constexpr int PERF_W = 12;
#ifndef ISC_NPART
#define ISC_NPART 4096
#endif
constexpr int NPART = ISC_NPART;  // partial sums per reduction (block count of the reducing kernels)
}

// CPR pressure multigrid: smoothing sweeps before and after the coarse
// correction, its scale, and the size at which coarsening stops
#define ISC_CPR_NU 2
#define ISC_CPR_CF 1.5
#define ISC_CPR_COARSEST 64
#define ISC_CPR_MAX_K 16      // most GMRES steps of the pressure solve
#define ISC_CPR_MAXLEV 16     // most multigrid levels
#define ISC_CPR_FUSED_MAX 8192   // levels of at most this many positions are cycled by one workgroup

void isc_cpr_plan(isc_ctx* ctx);
hipError_t isc_cpr_setup(isc_ctx* ctx, const double* A, int32_t* bad_dev);
void isc_cpr_vcycle(isc_ctx* ctx, const double* b, double* x);
void isc_cpr_pressure_apply(isc_ctx* ctx, const double* x, double* y);
void isc_cpr_gather(isc_ctx* ctx, const double* u, double* rp);
void isc_cpr_stage1(isc_ctx* ctx, const double* ep, const double* u, double* w1, double* r2);
void isc_cpr_combine(isc_ctx* ctx, const double* ep, double* z, double* w, const double* w1);
void isc_cpr_to_split(isc_ctx* ctx, const double* nat, double* split);
void isc_cpr_from_split(isc_ctx* ctx, const double* split, double* nat);

// Profiling helpers (host).  prof_begin/prof_end bracket a kernel class on the
// context stream; prof_drain converts finished pairs to milliseconds and must
// only run after the stream has been synchronised.
inline int isc_prof_begin(isc_ctx* ctx, int cls) {
    if (!ctx->prof) return -1;
    auto take = [&]() {
        hipEvent_t e;
        if (!ctx->prof_pool.empty()) { e = ctx->prof_pool.back(); ctx->prof_pool.pop_back(); }
        else if (hipEventCreate(&e) != hipSuccess) e = nullptr;
        return e;
    };
    isc_ctx::Pending p{cls, take(), take()};
    if (!p.a || !p.b) return -1;
    (void)hipEventRecord(p.a, ctx->stream);
    ctx->prof_pending.push_back(p);
    return (int)ctx->prof_pending.size() - 1;
}
// full-length vectors a profiled launch of class cls streams beyond the
// class's fixed access pattern (isc_profile_vectors)
inline void isc_prof_vectors(isc_ctx* ctx, int cls, double nvec) {
    if (ctx->prof) ctx->prof_vec[cls] += nvec;
}
inline void isc_prof_end(isc_ctx* ctx, int tok) {
    if (tok >= 0) (void)hipEventRecord(ctx->prof_pending[tok].b, ctx->stream);
}
inline void isc_prof_drain(isc_ctx* ctx) {
    for (auto& p : ctx->prof_pending) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
            ctx->prof_ms[p.cls] += ms;
            ctx->prof_cnt[p.cls] += 1;
        }
        ctx->prof_pool.push_back(p.a);
        ctx->prof_pool.push_back(p.b);
    }
    ctx->prof_pending.clear();
}

hipError_t isc_reset_sweep_buffers(isc_ctx* ctx);

// Error text of the last failed context-free call on this thread (returned by
// isc_last_error(NULL)).
void isc_set_noctx_error(const char* msg);

// Slot of ctx->flags raised when a sync-free triangular sweep gave up waiting;
// the two slots after it hold the wait limit (uint64, wall-clock ticks).
constexpr int ISC_FLAG_SWEEP = 3;
constexpr int ISC_FLAG_WAIT = 4;
constexpr uint64_t ISC_SWEEP_WAIT_DEFAULT = 1ull << 24;   // ~0.17 s of the 100 MHz wall clock

// Reads (and clears) the sweep error flag; waits for the stream.
inline isc_status isc_check_sweeps(isc_ctx* ctx) {
    if (hipMemcpyAsync(ctx->hflags + ISC_FLAG_SWEEP, ctx->flags + ISC_FLAG_SWEEP, sizeof(int32_t),
                       hipMemcpyDeviceToHost, ctx->stream) != hipSuccess ||
        hipStreamSynchronize(ctx->stream) != hipSuccess) {
        ctx->err = "reading the sweep status failed";
        return ISC_ERR_HIP;
    }
    if (ctx->hflags[ISC_FLAG_SWEEP] != 0) {
        ctx->hflags[ISC_FLAG_SWEEP] = 0;
        (void)hipMemcpyAsync(ctx->flags + ISC_FLAG_SWEEP, ctx->hflags + ISC_FLAG_SWEEP, sizeof(int32_t),
                             hipMemcpyHostToDevice, ctx->stream);
        (void)hipStreamSynchronize(ctx->stream);
        (void)isc_reset_sweep_buffers(ctx);
        (void)hipStreamSynchronize(ctx->stream);
        ctx->err = "triangular sweep: a row waited too long for its predecessors";
        return ISC_ERR_HIP;
    }
    return ISC_OK;
}

// error helpers for host code
#define ISC_HIP(call)                                                          \
    do {                                                                       \
        hipError_t e_ = (call);                                                \
        if (e_ != hipSuccess) {                                                \
            ctx->err = std::string(#call) + ": " + hipGetErrorString(e_);      \
            return ISC_ERR_HIP;                                                \
        }                                                                      \
    } while (0)
