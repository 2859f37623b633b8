/* libisc — MI355X (gfx950) Newton hot path of a fully implicit in-situ
 * combustion (ISC) simulator.
 *
 * The operations follow He, Yang, Liu, Chen, "A New In-Situ Combustion
 * Simulator for Parallel Computers":
 *   - the PDE system of Section 2 (molar balances eq. 4.2, coke eq. 4.8,
 *     energy eq. 4.3, constraints eqs. 4.4-4.7) reduced to eight unknowns per
 *     cell (table "Modified mathematical system for ISC", with the two
 *     composition constraints substituted);
 *   - the implicit-Euler, 7-point finite-difference discretisation with harmonic
 *     transmissibilities and upstream weighting of Section 3.1;
 *   - Newton's method with an analytical Jacobian, J du = -f (abstract, Sec. 3);
 *   - Gauss-Jordan decoupling C_L J du = -C_L f, C_L = blockdiag(J_ii^-1)
 *     (Section 3.2);
 *   - a block-ILU(0)-preconditioned restarted GMRES solve of the decoupled
 *     system (the paper's own solver is BiCGSTAB with RAS or CPR-PF).
 *
 * Conventions
 *   N = nx*ny*nz cells; cell i = ix + nx*(iy + ny*iz); iz grows with depth.
 *   Unknowns (u):  0 p [Pa], 1 x_LO, 2 y_O2, 3 y_CO2, 4 T [K], 5 S_w, 6 S_g,
 *                  7 C_c [mol/m^3]  — stored structure-of-arrays, u[8][N].
 *   Rows (F, J):   0..5 molar balances of W, LO, HO, O2, CO2, N2 [mol/s],
 *                  6 energy [W], 7 coke [mol/s] — stored F[N][8].
 *   Jacobian:      block CSR with 8x8 row-major blocks Jval[nnzb][8][8];
 *                  block (e, v) = dF_e/du_v.  Each row lists its existing
 *                  neighbours in ascending cell order (z-, y-, x-, self, x+,
 *                  y+, z+).  The pattern is owned by the context
 *                  (isc_bcsr_pattern).
 *   Pointers are device pointers on the context's device unless their name
 *   ends in _h (host).  The caller owns every array passed in; the context
 *   owns all workspace (Krylov bases, ILU factors, FP32 copies, scratch),
 *   allocated once by isc_create and never during the hot calls.  Every call
 *   is enqueued on the context's HIP stream; calls with a host (_h) output
 *   synchronise that stream before returning.  A context is not thread-safe.
 *   Errors: every function returns an isc_status; on error the outputs are
 *   undefined and isc_last_error() describes the failure.
 *
 * Schedules
 *   The BILU(0) factor and the triangular sweeps of its apply run as single
 *   launches in which each row (factor) or brick of cells (sweeps) waits for
 *   the rows it depends on; every such wait is bounded in wall-clock time.  A
 *   wait that runs out ends the launch early and the call returns ISC_ERR_HIP
 *   ("a row waited too long"); the context stays usable.  Every schedule
 *   computes the natural-order factorisation and its apply bit for bit alike.
 *   Environment switches, read by isc_create:
 *     ISC_LEVEL_SWEEPS=1      one launch per hyperplane ix+iy+iz = s instead;
 *     ISC_SWEEP_COOP=0        workgroups take sweep work by ticket instead of
 *                             the static cooperative order;
 *     ISC_BRICKS_PER_WG=2     two bricks per workgroup (ticket order only);
 *     ISC_FOLD_UPDATE=1       the FP64 GMRES does its Gram-Schmidt update inside
 *                             the next forward sweep;
 *     ISC_SWEEP_WAIT_TICKS=t  the wait limit in 100 MHz wall-clock ticks.
 */
#ifndef ISC_H
#define ISC_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t isc_status;
enum {
    ISC_OK = 0,
    ISC_ERR_ARG = -1,             /* invalid argument */
    ISC_ERR_HIP = -2,             /* HIP runtime error */
    ISC_ERR_OOM = -3,             /* device allocation failed */
    ISC_ERR_SINGULAR = -4,        /* singular diagonal block (bad_cell set) */
    ISC_ERR_NONFINITE = -5,       /* NaN/Inf in the state or residual */
    ISC_ERR_LINEAR_NOCONV = -6,   /* Krylov solve missed its tolerance */
    ISC_ERR_NEWTON_NOCONV = -7    /* Newton missed its tolerance */
};

enum { ISC_NSPEC = 7, ISC_NGAS = 6, ISC_NREAC = 4, ISC_NTAB = 101 };

/* SI physics card.  Species order W, LO, HO, O2, CO2, N2, coke; liquids
 * W, LO, HO.  All correlations take T in K and p in Pa (Section 2.2). */
typedef struct {
    double M[ISC_NSPEC];               /* molar masses, kg/mol */
    double Tc[ISC_NGAS], pc[ISC_NGAS]; /* critical T (K) and p (Pa) */
    double rho_ref[3];                 /* liquid reference molar densities, mol/m^3 */
    double cp_liq[3], ct1_liq[3];      /* liquid compressibility 1/Pa, expansivity 1/K */
    double rho_coke;                   /* mol/m^3 */
    double cpg[ISC_NGAS][4];           /* gas cp(T) = sum_j cpg[j] T^j, J/(mol K) */
    double hvr[3], ev[3];              /* Hv(T) = hvr (Tc-T)^ev for T < Tc, J/mol */
    double avisc[3], bvisc[3];         /* liquid mu = avisc exp(bvisc/T), Pa s */
    double avg[ISC_NGAS], bvg[ISC_NGAS]; /* gas mu_c = avg T^bvg, Pa s */
    double kv1[3], kv4[3], kv5[3];     /* K = kv1/p exp(kv4/(T - kv5)) */
    double stoich[ISC_NREAC][ISC_NSPEC]; /* molar stoichiometry, reactants < 0 */
    double Afreq[ISC_NREAC];           /* frequency factors (r1,r2,r4 1/(Pa s); r3 1/s) */
    double Eact[ISC_NREAC];            /* activation energies, J/mol */
    double Hreac[ISC_NREAC];           /* reaction enthalpies, J/mol, + exothermic */
    double eps;                        /* PER correction constant */
    double Ccmax;                      /* coke concentration limit, mol/m^3 */
    double p_ref, T_ref;               /* reference state */
    double cpor;                       /* rock compressibility 1/Pa (linear law) */
    double cp_rock;                    /* rock volumetric heat capacity J/(m^3 K) */
    double cp_coke;                    /* coke heat capacity J/(mol K) */
    double Kcond[4];                   /* conductivities W/(m K): water, oil, gas, rock */
    double grav, Rgas;                 /* m/s^2, J/(mol K) */
    double krocw;                      /* k_ro at connate water (Stone II) */
    double krw[ISC_NTAB], krow[ISC_NTAB]; /* SWT table at S_w = k/100 */
    double krg[ISC_NTAB], krog[ISC_NTAB]; /* SLT table at S_g = k/100 */
} isc_fluid;

typedef struct { int32_t nx, ny, nz; double dx, dy, dz; } isc_grid;

enum { ISC_WELL_BHP_PRODUCER = 1, ISC_WELL_RATE_INJECTOR = 2, ISC_WELL_PRODUCER = 3, ISC_WELL_INJECTOR = 4 };
/* Well controls of kinds 3 and 4: BHP, or a molar rate (a producer's: of the
 * phases in the mask; an injector's: any nonzero value, the injected total). */
enum { ISC_CTRL_BHP = 0, ISC_CTRL_WATER = 1, ISC_CTRL_OIL = 2, ISC_CTRL_GAS = 4 };
/* One vertical well (well-modelling subsection, Peaceman index).
 * Kind 1 producers hold a fixed bottom-hole pressure (target, Pa) with no
 * backflow; kind 2 injectors inject a fixed molar rate (target, mol/s) of gas
 * of composition z_inj at T_inj, split over the perforations in proportion to
 * their well index.  Kinds 3 (producer) and 4 (injector) make the bottom-hole
 * pressure an unknown with a well equation: control ISC_CTRL_BHP holds
 * bhp = target (Pa); otherwise the well holds a molar rate target (mol/s) --
 * the sum over perforations of WI lambda_a (p - bhp) over the phases a in the
 * mask for a producer (lambda_a = rho_a k_ra / mu_a, molar), or of
 * WI (lambda_w + lambda_o + lambda_g) (bhp - p) of gas z_inj at T_inj for an
 * injector -- and is held at its BHP limit `limit` (producer minimum,
 * injector maximum) when the rate cannot be met within it.  No backflow.
 * isc_create refuses (ISC_ERR_ARG) a kind 3/4 well with more than 2048
 * perforations, a target that is not finite and positive (a well that is to
 * stay shut is left out: at a zero rate its row has no bhp derivative), a
 * limit that is not finite (under rate control: not finite and positive), or
 * an unknown control. */
typedef struct {
    int32_t kind;
    int32_t nperf;
    const int32_t* perf_cells_h;      /* host array of perforated cell indices */
    double target;
    double T_inj;
    double z_inj[ISC_NSPEC];
    double rw, skin;                  /* wellbore radius (m), skin */
    int32_t control;                  /* kinds 3/4 */
    double limit;                     /* kinds 3/4 under rate control: BHP limit, Pa */
} isc_well;

enum { ISC_FP64 = 0, ISC_MIXED = 1 };
enum { ISC_PC_BILU0 = 0, ISC_PC_CPR = 1 };
enum { ISC_KRYLOV_GMRES = 0, ISC_KRYLOV_BICGSTAB = 1 };
typedef struct {
    int32_t restart;       /* GMRES restart length m (<= max_opts.restart) */
    int32_t max_restarts;  /* cycles before ISC_ERR_LINEAR_NOCONV */
    int32_t precision;     /* ISC_FP64, or ISC_MIXED: FP32 preconditioner and
                              inner SpMV inside an FP64 flexible GMRES */
    int32_t inner_iters;   /* ISC_MIXED: FP32 inner GMRES iterations per outer one */
    int32_t precond;       /* ISC_PC_BILU0: block ILU(0) (right-preconditioned
                              GMRES, or the inner solver of ISC_MIXED);
                              ISC_PC_CPR (FP64 only): the two-stage CPR
                              preconditioner (Section 4.3, Example 2) inside an
                              FP64 flexible GMRES -- stage 1 a pressure solve,
                              stage 2 block ILU(0) on the remaining residual */
    int32_t p_iters;       /* ISC_PC_CPR: GMRES steps of the pressure solve, each
                              preconditioned by one V-cycle of the pressure
                              multigrid (0: the V-cycle alone); at most
                              max_opts.p_iters */
    double rtol;           /* stop when ||b - A x||_2 <= rtol ||b||_2 */
    int32_t krylov;        /* ISC_KRYLOV_GMRES, or ISC_KRYLOV_BICGSTAB (ISC_FP64 with
                              ISC_PC_BILU0 only): the BiCGSTAB of isc_solve_bicgstab
                              with at most restart x max_restarts iterations */
} isc_solve_opts;

typedef struct {
    int32_t iters;               /* outer Krylov iterations (columns of the solutions formed) */
    int32_t inner_iters_total;   /* ISC_MIXED: inner iterations executed, including the one
                                    preconditioner application per cycle whose residual test
                                    ended the cycle (its column is not used); ISC_PC_CPR: the
                                    pressure GMRES steps executed */
    int32_t restarts;
    int32_t reserved;
    double relres_est;           /* Arnoldi residual estimate / ||b|| */
    double relres_true;          /* ||b - A x|| / ||b|| recomputed at exit */
} isc_solve_info;

typedef struct {
    isc_solve_opts lin;
    double tol;                  /* convergence: scaled max-norm of F <= tol */
} isc_newton_opts;

typedef struct {
    int32_t converged;           /* 1 if F already met tol (no solve was done) */
    int32_t bad_cell;            /* singular cell, or -1 */
    double res_scaled;           /* scaled max-norm of F at entry */
    isc_solve_info lin;
    float ms_assemble, ms_decouple, ms_precond, ms_krylov, ms_update;
} isc_newton_info;

typedef struct isc_ctx isc_ctx;

/* Create a context for one grid.  logk: ln(k_h / m^2) per cell (device, [N]);
 * kz = kv_over_kh * kh; poro: reference porosity per cell (device, [N]);
 * wells_h: host array of nwells wells.  max_opts fixes the largest restart
 * length and inner iteration count the context will be asked for (workspace
 * is sized from it; max_opts.precond = ISC_PC_CPR also allocates the CPR
 * preconditioner for up to max_opts.p_iters <= 16 pressure steps).
 * hip_stream: a hipStream_t (NULL = default stream). */
isc_status isc_create(const isc_grid* grid_h, const isc_fluid* fluid_h, const double* logk,
                      double kv_over_kh, const double* poro, const isc_well* wells_h,
                      int32_t nwells, const isc_solve_opts* max_opts_h, void* hip_stream,
                      isc_ctx** out_h);
isc_status isc_destroy(isc_ctx* ctx);

/* Replace ln k (device [N], or NULL) and/or the reaction frequency factors
 * (host [4], or NULL); transmissibilities and well indices are recomputed. */
isc_status isc_set_params(isc_ctx* ctx, const double* logk, const double* A_h);

/* A heat source of rate_W watts in the energy balance of one cell, as the
 * ignition heater of the combustion tube (Section 4.1, well table: "heat
 * rate" and "heat stop time"), independent of the state; it enters every
 * later residual until changed.  cell < 0 or rate_W = 0 removes it.  The
 * caller switches it off at the stop time.  ISC_ERR_ARG for a cell outside
 * the grid or a non-finite rate. */
isc_status isc_set_heater(isc_ctx* ctx, int32_t cell, double rate_W);

/* Block CSR pattern (device pointers owned by the context) and its size. */
isc_status isc_bcsr_pattern(const isc_ctx* ctx, const int32_t** row_ptr, const int32_t** col_idx,
                            int32_t* nnzb_h);

/* Residual F[N][8] and analytical Jacobian Jval[nnzb][8][8] of the implicit
 * Euler step u_old -> u over dt seconds (Section 3.1 residuals F_W, F_O[i],
 * F_G[i], F_E, F_Coke with the constraints substituted).  u, u_old: [8][N]. */
isc_status isc_assemble(isc_ctx* ctx, const double* u, const double* u_old, double dt, double* F,
                        double* Jval);

/* Gauss-Jordan decoupling in place (Section 3.2): every block row
 * [J_ii | J_i,nbr | F_i] becomes [I | J_ii^-1 J_i,nbr | J_ii^-1 F_i] by
 * elimination with partial pivoting (row exchanges = dynamic equation
 * alignment).  On a singular J_ii returns ISC_ERR_SINGULAR and *bad_cell_h. */
isc_status isc_decouple(isc_ctx* ctx, double* Jval, double* F, int32_t* bad_cell_h);

/* Solve Jdec x = b for a decoupled matrix (unit diagonal blocks, as left by
 * isc_decouple) from x0 = 0.  b, x: [N][8].  info_h may be NULL.
 * opts->precond = ISC_PC_BILU0: block-ILU(0) (natural cell order)
 * right-preconditioned restarted GMRES (FP64), or with ISC_MIXED the FP64
 * flexible GMRES around FP32 inner GMRES.  ISC_PC_CPR: FP64 flexible GMRES
 * with the two-stage CPR preconditioner.  Stage 1 takes the pressure equation
 * of the decoupled system, the scalar matrix A_p of the (pressure row,
 * pressure column) entries (Jdec_ij)[0][0], and solves it for the pressure
 * part of the residual by opts->p_iters GMRES steps (from 0, no restart), each
 * preconditioned by one V-cycle of a multigrid on the grid: levels lump 2x2x2
 * boxes, the coarse matrices are the Galerkin products P^T A P for
 * piecewise-constant P, smoothing is two red-black Gauss-Seidel sweeps before
 * and after a coarse correction scaled by 1.5, and the coarsest level (at
 * most 64 cells) is solved with its inverse.  Stage 2 applies block ILU(0) to
 * what the pressure correction leaves of the residual:
 *   z = E e_p + M^-1 (r - A E e_p),  e_p ~= A_p^-1 (E^T r),
 * E^T r the pressure components of r.  opts->krylov = ISC_KRYLOV_BICGSTAB
 * (FP64, ISC_PC_BILU0) runs isc_solve_bicgstab with restart x max_restarts
 * iterations instead.  ISC_ERR_SINGULAR if the factor or the coarsest matrix
 * is singular. */
isc_status isc_solve(isc_ctx* ctx, const double* Jdec, const double* b, double* x,
                     const isc_solve_opts* opts_h, isc_solve_info* info_h);

/* Solve Jdec x = b (decoupled matrix, unit diagonal blocks) with
 * right-preconditioned BiCGSTAB and block ILU(0) from x0 = 0: the
 * stabilised bi-conjugate gradient method of the paper's experiments
 * (Section 4, where it runs with RAS or CPR-PF preconditioning).  Stops when
 * the updated residual meets ||r||_2 <= rtol ||b||_2, then checks the true
 * residual and, if it is still above, restarts from it.  A breakdown --
 * |(r~, r)| <= 1e-12 ||r~|| ||r||, |(r~, v)| <= 1e-12 ||r~|| ||v||, (t, t) = 0
 * (after keeping the half step x += alpha p^, whose residual is s) or
 * omega = 0 -- also restarts from the true residual, which becomes the new
 * shadow vector r~, at most 8 times.  b, x: [N][8] (distinct).  Uses seven
 * of the context's Krylov vectors (max restart >= 6).  info_h (may be NULL):
 * iters = iterations (two preconditioned products each), restarts,
 * relres_est = the last updated residual / ||b||, relres_true.  Returns
 * ISC_ERR_LINEAR_NOCONV after max_iters iterations or a ninth breakdown
 * unless the true residual already meets the tolerance; ISC_ERR_SINGULAR
 * from the factor. */
isc_status isc_solve_bicgstab(isc_ctx* ctx, const double* Jdec, const double* b, double* x,
                              int32_t max_iters, double rtol, isc_solve_info* info_h);

/* One Newton iteration at (u, u_old, dt): assemble, scaled-norm test (if
 * res <= tol: converged = 1, u unchanged), else decouple, the preconditioner
 * set-up and the linear solve of opts->lin (as isc_solve), and the
 * safeguarded update of u in place (saturation halving rule of the PER
 * subsection plus per-variable step limits).
 * With controlled wells (kinds 3, 4) the system is bordered by one row per
 * well in its bhp (well-modelling subsection; the bhp row of the table of
 * unknowns and equations):
 *   [J  B] [du  ]     [F]    B = dF/dbhp, C = dR/du, D = dR/dbhp,
 *   [C  D] [dbhp] = - [R],   R = bhp - held BHP, or q - target (rate).
 * First isc_well_solve sets each rate-controlled well's bhp from its own
 * equation at the current cells (or moves it onto its BHP limit); the well
 * rows count in res (isc_well_border's scaling); they are eliminated,
 *   (J - B D^-1 C) du = -(F - B D^-1 R),  dbhp = -D^-1 (R + C du),
 * with the part of B D^-1 C that the 7-point pattern holds (a perforated
 * cell with itself and its stencil neighbours in the same well) subtracted
 * from J before the decoupling, so that the preconditioners see it, and the
 * rest applied matrix-free in every Krylov product; bhp takes its Newton
 * step with the cells. */
isc_status isc_newton_step(isc_ctx* ctx, double* u, const double* u_old, double dt,
                           const isc_newton_opts* opts_h, isc_newton_info* info_h);

/* Controlled wells (kinds 3, 4), numbered in the order of the wells given to
 * isc_create; their perforations are listed in the same order.  The state of
 * each is its bhp (Pa) and on_limit (1 while a rate-controlled well is held
 * at its BHP limit); isc_create starts it at bhp = target under BHP control,
 * else at the limit, with on_limit = 0.  Host arrays of isc_well_count's
 * ncw entries; every call synchronises the context stream. */
isc_status isc_well_count(const isc_ctx* ctx, int32_t* ncw_h, int32_t* ncp_h);
isc_status isc_well_state(isc_ctx* ctx, double* bhp_h, int32_t* on_limit_h);
isc_status isc_set_well_state(isc_ctx* ctx, const double* bhp_h, const int32_t* on_limit_h);
/* Control switching.  With the cells at u, the rate a controlled well holds
 * is piecewise linear and monotone in its bhp.  isc_well_solve (run by
 * isc_newton_step first): a well on its rate whose rate at the BHP limit
 * falls short of the target is held at the limit, else its bhp is set to the
 * root of its rate equation.  isc_well_controls, to be called at the start of
 * every time step (and every retry of one): a well held at its limit returns
 * to its rate when it would move more than the target at the limit.  A well
 * thus leaves its limit only between steps, which keeps a Newton iteration
 * from cycling between controls.  *nswitch_h (may be NULL): wells switched.
 * u: [8][N] device. */
isc_status isc_well_controls(isc_ctx* ctx, const double* u, int32_t* nswitch_h);
isc_status isc_well_solve(isc_ctx* ctx, const double* u, int32_t* nswitch_h);
/* The well rows at (u, u_old, dt) and the current well state (assembles):
 * R_h[ncw], D_h[ncw] (host) and B[ncp][8] = dF_cell/dbhp, C[ncp][8] =
 * dR_w/du_cell (device; either may be NULL).  Under BHP control or at the
 * limit R = bhp - held, D = 1, C = 0.  The Newton test scales |R| by
 * V phi rho_ref,W / dt of the well's first perforated cell (rate rows) or by
 * the pressure held, at least 1 Pa (BHP rows). */
isc_status isc_well_border(isc_ctx* ctx, const double* u, const double* u_old, double dt, double* R_h,
                           double* D_h, double* B, double* C);

/* Component steps exposed for testing and profiling. */
isc_status isc_spmv(isc_ctx* ctx, const double* Jdec, const double* x, double* y);
/* D^-1 of the block ILU(0) of Jdec in natural cell order (D-ILU form:
 * D_i = I - sum over lower neighbours k of A_ik D_k^-1 A_ki).  A singular D_i
 * returns ISC_ERR_SINGULAR, naming the lowest such cell in the error text. */
isc_status isc_bilu0(isc_ctx* ctx, const double* Jdec, double* Dinv /* [N][8][8] */);
isc_status isc_bilu0_apply(isc_ctx* ctx, const double* Jdec, const double* Dinv, const double* r,
                           double* z);
/* z = M^-1 r and w = Jdec z in one call (the preconditioned operator of the
 * GMRES iteration): the backward sweep of the BILU(0) apply and the SpMV run as
 * one launch, each SpMV brick scheduled after the sweep of its neighbours.
 * r, z, w: [N][8], pairwise distinct. */
isc_status isc_bilu0_apply_spmv(isc_ctx* ctx, const double* Jdec, const double* Dinv, const double* r,
                                double* z, double* w);
/* CPR components (the preconditioner of isc_solve with ISC_PC_CPR), for
 * testing: each call factors Jdec and builds the pressure multigrid first
 * (the context must have been created for CPR with max p_iters >= p_iters).
 * isc_cpr_pressure_solve: e [N] = the stage-1 pressure solve of rp [N] (the
 * p_iters V-cycle-preconditioned GMRES steps on A_p e = rp).
 * isc_cpr_apply: z = CPR r and w = Jdec z (r, z, w: [N][8], distinct). */
isc_status isc_cpr_pressure_solve(isc_ctx* ctx, const double* Jdec, int32_t p_iters, const double* rp, double* e);
isc_status isc_cpr_apply(isc_ctx* ctx, const double* Jdec, int32_t p_iters, const double* r, double* z, double* w);
/* The precision form's product z = M32^-1 r, w = A32 z, as its inner
 * iteration runs it (block ILU(0) factored from the FP32-rounded blocks of
 * Jdec, FP32 storage of the factor, the matrix data and the vectors; the
 * backward sweep fused with the SpMV), for testing: r, z, w are FP64 [N][8],
 * rounded to FP32 on entry and widened on exit.  Needs a context with max
 * inner_iters >= 1; ISC_ERR_SINGULAR for a singular pivot block. */
isc_status isc_bilu0_apply_spmv32(isc_ctx* ctx, const double* Jdec, const double* r, double* z, double* w);
isc_status isc_update(isc_ctx* ctx, double* u, const double* du /* [N][8] */);
isc_status isc_scaled_norm(isc_ctx* ctx, const double* F, double dt, double* res_h);

/* Allocation-free variant of isc_scaled_norm, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  It needs no context: grid_h and fluid_h
 * (host) give the cell volume, rho_ref[0] and cp_rock; poro [N] and F [N][8]
 * are device arrays; *res (device, one double) receives max over cells and
 * rows of |F_e,i| / s_e,i with the scales of isc_scaled_norm.  The call only
 * enqueues two kernels on hip_stream (a stream of the current device, NULL =
 * default) and returns; it calls no allocating routine.  Its partial maxima
 * live in a fixed device array of ISC_NOALLOC_MAX_CELLS / 2048 doubles
 * (64 KiB) that each device holds until the process ends, so grids above
 * ISC_NOALLOC_MAX_CELLS cells are rejected with ISC_ERR_ARG.  All calls on one
 * device share that array: calls that overlap in time on one device (on
 * different streams, or from several threads) race and must be serialised by
 * the caller.  Every partial read is written by the same call first, so
 * nothing needs clearing between calls.  The first call on a device resolves
 * the array's address (hipGetSymbolAddress); a caller that captures graphs
 * makes one call before capturing.  Errors: ISC_ERR_ARG (null pointer,
 * dt <= 0, invalid or too large grid), ISC_ERR_HIP; isc_last_error(NULL)
 * returns the message of the last failed context-free call on the thread. */
enum { ISC_NOALLOC_MAX_CELLS = 16777216 };
isc_status isc_scaled_norm_noalloc(const isc_grid* grid_h, const isc_fluid* fluid_h, const double* poro,
                                   const double* F, double dt, double* res, void* hip_stream);

/* Differentiation form.  Objective J_obj = sum_n dt_n q_oil(u^n) with
 * q_oil(u) = sum over producer perforations of WI lambda_o (p - p_wf) for
 * p > p_wf (oil-phase molar rate, mol/s); parameters m = (ln k per cell,
 * frequency factors A_R).  One backward step of the discrete adjoint:
 *   (dR^n/du^n)^T lam^n = dt_n (dq_oil/du^n)^T + (V/dt_{n+1}) (dA/du(u^n))^T lam^{n+1}
 * (A: accumulation per bulk volume; lam_np1 = NULL at the last step, then
 * dt_np1 is ignored), solved by transposing J in place (the 7-point pattern is
 * symmetric), decoupling J^T by its own diagonal blocks and running the
 * BILU(0)-preconditioned GMRES on it (opts_h may be NULL: restart 30, 200
 * cycles, rtol 1e-12); then g_logk[N] += dt_n dq/dln k - lam^n . dR^n/dln k (device)
 * and g_A_h[4] += -lam^n . dR^n/dA_R (host).  u_n, u_nm1: [8][N]; lam: [N][8]. */
isc_status isc_adjoint(isc_ctx* ctx, const double* u_n, const double* u_nm1, double dt_n,
                       const double* lam_np1, double dt_np1, double* lam_n, double* g_logk,
                       double* g_A_h, const isc_solve_opts* opts_h, isc_solve_info* info_h);

/* q_oil(u) defined above, summed over the kind 1 producers (host output,
 * mol/s).  isc_adjoint returns ISC_ERR_ARG for a context with controlled
 * wells: their rows are not part of this adjoint. */
isc_status isc_oil_rate(isc_ctx* ctx, const double* u, double* q_h);

/* Kernel-class timing with HIP events on the context's stream, for
 * profiling.  enable = 1 clears the accumulators and starts timing; every
 * launch of a class inside the calls above is then bracketed by an event
 * pair; enable = 0 stops.  Always returns the accumulated milliseconds and
 * launch counts (host arrays of ISC_PROF_NCLASS, may be NULL).  Classes:
 * 0 SpMV, 1 BILU(0) apply (one forward plus one backward sweep), 2 assembly
 * (property pass + face assembly), 3 decoupling, 4 BILU(0) factor (all
 * levels), 5 Krylov vector work (orthogonalisation, updates, norms, in both
 * precisions), 6 the CPR pressure stage (pressure extraction of the
 * residual, the V-cycles, the pressure SpMV and GMRES vector work, the stage-1
 * correction A E e_p and the combination of the stages), 7 the CPR set-up
 * (pressure stencil and block-column pack, coarse matrices, coarsest
 * inverse), 8 BILU(0) apply fused with the SpMV (z = M^-1 r, w = A z; the
 * FP64 GMRES iteration, with its folded Gram-Schmidt update, and stage 2 of
 * CPR), 9 the same in FP32 (the inner GMRES iteration of the precision form). */
enum { ISC_PROF_SPMV = 0, ISC_PROF_ILU_APPLY, ISC_PROF_ASSEMBLE, ISC_PROF_DECOUPLE, ISC_PROF_ILU_FACTOR,
       ISC_PROF_KRYLOV, ISC_PROF_CPR_PRESSURE, ISC_PROF_CPR_SETUP, ISC_PROF_ILU_SPMV, ISC_PROF_ILU_SPMV32,
       ISC_PROF_NCLASS = 10 };
isc_status isc_profile(isc_ctx* ctx, int32_t enable, double* ms_h, int32_t* count_h);

/* Per class, the number of full-length vectors (n x 8 values in the class's
 * precision) that the profiled launches streamed on top of the class's fixed
 * access pattern, accumulated over the same window as isc_profile.  Nonzero
 * only for classes 8 and 9: the GMRES iterations (FP64, and the FP32 inner
 * one of the precision form) fold the previous iteration's delayed
 * Gram-Schmidt update into the forward sweep, which then reads j - 1 basis
 * vectors and w and writes q_{j-1} and u (j + 2 vectors at iteration j).
 * vec_h: host array of ISC_PROF_NCLASS.  ISC_ERR_ARG if it is NULL. */
isc_status isc_profile_vectors(isc_ctx* ctx, double* vec_h);

const char* isc_last_error(const isc_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif
