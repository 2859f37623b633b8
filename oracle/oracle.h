/* CPU oracle for the in-situ-combustion Newton hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, serial FP64 implementation
 * written from the paper (He, Yang, Liu, Chen, "A New In-Situ Combustion
 * Simulator for Parallel Computers").  It exists to check the GPU library; it
 * shares no code, header, table or helper with it, and the product path never
 * calls it.  Only the test suite, the smoke check and the CPU-baseline leg of
 * the benchmark load it.
 *
 * Layouts (same meaning as the GPU library's public header, declared here
 * independently):
 *   cell i = ix + nx*(iy + ny*iz), iz grows with depth
 *   u[8][N]   structure of arrays, unknowns (p, x_LO, y_O2, y_CO2, T, S_w, S_g, C_c)
 *   F[N][8]   residual, rows (W, LO, HO, O2, CO2, N2, energy, coke)
 *   J[nnzb][8][8] block CSR, row-major blocks, columns ascending in each row
 */
#ifndef ISC_ORACLE_H
#define ISC_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_NSPEC = 7, ORC_NGAS = 6, ORC_NREAC = 4, ORC_NTAB = 101 };

typedef struct {
    double M[ORC_NSPEC];
    double Tc[ORC_NGAS], pc[ORC_NGAS];
    double rho_ref[3], cp_liq[3], ct1_liq[3];
    double rho_coke;
    double cpg[ORC_NGAS][4];
    double hvr[3], ev[3];
    double avisc[3], bvisc[3];
    double avg[ORC_NGAS], bvg[ORC_NGAS];
    double kv1[3], kv4[3], kv5[3];
    double stoich[ORC_NREAC][ORC_NSPEC];
    double Afreq[ORC_NREAC], Eact[ORC_NREAC], Hreac[ORC_NREAC];
    double eps, Ccmax, p_ref, T_ref, cpor, cp_rock, cp_coke;
    double Kcond[4];
    double grav, Rgas, krocw;
    double krw[ORC_NTAB], krow[ORC_NTAB], krg[ORC_NTAB], krog[ORC_NTAB];
} orc_fluid;

typedef struct { int32_t nx, ny, nz; double dx, dy, dz; } orc_grid;

/* Kinds 1 and 2 are local sources (fixed BHP producer, fixed-rate injector
 * split over the perforations by WI).  Kinds 3 and 4 make the bottom-hole
 * pressure an unknown with a well equation of its own (well-modelling
 * subsection): control 0 holds bhp = target; otherwise the well holds a
 * molar rate, target mol/s -- for a producer the sum over perforations of the
 * phases in the mask control (1 water, 2 oil, 4 gas; 7 = total), for an
 * injector the injected total -- and falls back to its BHP limit `limit`
 * (producer minimum, injector maximum) when the rate would need a bhp
 * beyond it. */
typedef struct {
    int32_t kind;            /* 1 BHP producer, 2 rate injector, 3 controlled producer, 4 controlled injector */
    int32_t nperf;
    const int32_t* perf_cells;
    double target;           /* kind 1, kinds 3/4 at control 0: BHP (Pa); otherwise mol/s */
    double T_inj;
    double z_inj[ORC_NSPEC];
    double rw, skin;
    int32_t control;         /* kinds 3/4: 0 BHP control, else rate control (producer: phase mask) */
    double limit;            /* kinds 3/4 under rate control: BHP limit (Pa) */
} orc_well;

typedef struct {
    int32_t iters;           /* Krylov iterations */
    int32_t restarts;
    double relres_est, relres_true;
} orc_solve_info;

typedef struct orc_model orc_model;

/* setup */
orc_model* orc_create(const orc_grid* g, const orc_fluid* fl, const double* logk,
                      double kv_over_kh, const double* poro, const orc_well* wells,
                      int32_t nwells);
void orc_destroy(orc_model* m);
int32_t orc_ncell(const orc_model* m);
int32_t orc_nnzb(const orc_model* m);
void orc_pattern(const orc_model* m, int32_t* row_ptr, int32_t* col_idx);
/* replace ln k (may be NULL) and/or the frequency factors A_R (may be NULL) */
void orc_set_params(orc_model* m, const double* logk, const double* A);
void orc_perf_info(const orc_model* m, int32_t* cells, int32_t* kinds, double* wi, double* q);
/* heat source rate_W (W) in the energy balance of one cell; cell < 0 or
 * rate 0: none.  It counts with the well terms in orc_sources. */
void orc_set_heater(orc_model* m, int32_t cell, double rate_W);

/* diagnostics for the pins: per-cell secondary quantities at state u.
 * out[N][ORC_NDIAG], see ORC_DIAG_* */
enum {
    ORC_DIAG_SO, ORC_DIAG_XHO, ORC_DIAG_Y0, /* y[6] at 2..7 */
    ORC_DIAG_Z = 8, ORC_DIAG_RHOW, ORC_DIAG_RHOO, ORC_DIAG_RHOG,
    ORC_DIAG_MUW, ORC_DIAG_MUO, ORC_DIAG_MUG, ORC_DIAG_PHI, ORC_DIAG_PHIF,
    ORC_DIAG_KRW, ORC_DIAG_KRO, ORC_DIAG_KRG, ORC_DIAG_HW, ORC_DIAG_HO, ORC_DIAG_HG,
    ORC_DIAG_KT, ORC_DIAG_R0 /* rates 4 at 24..27 */, ORC_DIAG_ACC0 = 28 /* acc 8 at 28..35 */,
    ORC_DIAG_KW = 36, ORC_DIAG_KLO, ORC_DIAG_KHO, ORC_DIAG_HVW, ORC_DIAG_HGO2,
    ORC_NDIAG = 41
};
void orc_diag(const orc_model* m, const double* u, double* out);
/* Z-factor of a gas of composition y[6] at (p, T); also returns pseudo-criticals */
double orc_zfactor(const orc_fluid* fl, double p, double T, const double* y, double* Tcm, double* pcm);

/* gas-phase viscosity of composition y[6] at T (Pa s) */
double orc_gas_viscosity(const orc_fluid* fl, double T, const double* y);

/* Wells of kinds 3 and 4 ("controlled wells", in the order given): their
 * state is bhp (Pa) and on_limit (1 while a rate-controlled well is held at
 * its BHP limit).  At creation bhp = target under BHP control, else the limit,
 * and on_limit = 0. */
int32_t orc_ncwell(const orc_model* m);
void orc_well_state(const orc_model* m, double* bhp, int32_t* on_limit);
void orc_set_well_state(orc_model* m, const double* bhp, const int32_t* on_limit);
/* Control switching and the well equations alone.  orc_well_solve, before
 * every Newton iteration assembles: with the cells at state u, a
 * rate-controlled well's rate is piecewise linear and monotone in bhp; if it
 * falls short of the target at the BHP limit the well is held at the limit
 * for the rest of the time step, else bhp is set to the root of its rate
 * equation.  orc_well_controls, at the start of a time step: a well held at
 * its limit returns to its rate when, at state u, it would move more than
 * the target there.  (Switching back only between steps keeps a Newton
 * iteration from cycling between the two controls.)  Both return the number
 * of wells switched. */
int32_t orc_well_controls(orc_model* m, const double* u);
int32_t orc_well_solve(orc_model* m, const double* u);
/* The well rows at state u and the current well state (as orc_well_controls
 * left it).  Per controlled well w: R[w] its equation's residual and D[w] =
 * dR_w/dbhp_w; per perforation k of the controlled wells (in well order):
 * B[k][8] = dF_cell/dbhp and C[k][8] = dR_w/du_cell.  Newton's system is
 *   [J  B] [du  ]     [F]
 *   [C  D] [dbhp] = - [R]. */
void orc_well_border(orc_model* m, const double* u, double* R, double* D, double* B, double* C);
/* |R_w| scaled like the cell rows: rate rows by V phi rho_ref,W / dt of the
 * well's first perforated cell, BHP rows by the pressure held (at least 1 Pa) */
double orc_well_scaled_norm(orc_model* m, const double* R, double dt);

/* hot-path steps */
int orc_residual(orc_model* m, const double* u, const double* u_old, double dt, double* F);
int orc_assemble(orc_model* m, const double* u, const double* u_old, double dt,
                 double* F, double* J);
/* well and reaction source terms at state u: src[N][8] (the amounts subtracted in F) */
void orc_sources(orc_model* m, const double* u, double* wells_out, double* reac_out);
/* J -> C_L J (diagonal blocks := I), F -> C_L F.  Returns 0 or -4 (singular, *bad_cell set). */
int orc_decouple(orc_model* m, double* J, double* F, int32_t* bad_cell);
/* block ILU(0) of a decoupled matrix: Lblk (lower blocks, L_ik) and Dinv [N][64] */
int orc_bilu0(orc_model* m, const double* Jdec, double* LU, double* Dinv);
void orc_bilu0_apply(orc_model* m, const double* LU, const double* Dinv, const double* r, double* z);
void orc_spmv(orc_model* m, const double* J, const double* x, double* y);
int orc_gmres(orc_model* m, const double* Jdec, const double* b, double* x, int32_t restart,
              int32_t max_restarts, double rtol, orc_solve_info* info);
/* right-preconditioned BiCGSTAB with block ILU(0), x0 = 0; returns 0 or -6 */
int orc_bicgstab(orc_model* m, const double* Jdec, const double* b, double* x, int32_t max_iters, double rtol,
                 orc_solve_info* info);
/* scaled max-norm of F for convergence */
double orc_scaled_norm(orc_model* m, const double* F, double dt);
/* Newton update with the saturation/fraction safeguards; returns 0 or -5 (non-finite) */
int orc_update(orc_model* m, double* u, const double* du);

typedef struct {
    int32_t converged, iters_lin, status;
    double res_scaled, relres_true;
} orc_newton_info;
/* One Newton iteration (assemble, converged if res <= tol, else decouple,
 * GMRES, update).  With controlled wells: orc_well_solve first, the well
 * rows count in res (orc_well_scaled_norm), and they are eliminated from the
 * bordered system (Schur complement) before GMRES; bhp takes its Newton
 * step with the cells. */
int orc_newton_step(orc_model* m, double* u, const double* u_old, double dt, double tol,
                    int32_t restart, int32_t max_restarts, double rtol, orc_newton_info* info);

/* time loop: u [8][N] in/out; per step records NI and linear iterations;
 * every attempt at a step starts with orc_well_controls; a failed step
 * restores u and the well state and halves dt (at most four times); returns
 * number of successful steps or a negative status */
typedef struct {
    int32_t newton_its, lin_its, cuts;
    double dt_used, res_final;
} orc_step_info;
int orc_run(orc_model* m, double* u, double dt, int32_t nsteps, double tol, int32_t max_newton,
            int32_t restart, int32_t max_restarts, double rtol, orc_step_info* steps,
            double* u_hist /* [nsteps+1][8][N] or NULL */);

/* CPR two-stage preconditioner of a decoupled matrix (see oracle/cpr.cpp):
 * stage 1 an approximate solve of the pressure equation (p_iters GMRES steps
 * preconditioned by an aggregation multigrid V-cycle with nu red-black
 * Gauss-Seidel sweeps before and after a coarse correction scaled by cf),
 * stage 2 block ILU(0) on the remaining residual. */
enum { ORC_CPR_COARSEST = 64 };
typedef struct orc_cpr orc_cpr;
orc_cpr* orc_cpr_create(orc_model* m, const double* Jdec, int32_t p_iters, int32_t nu, double cf);
void orc_cpr_destroy(orc_cpr* c);
int32_t orc_cpr_nlevels(const orc_cpr* c);
int32_t orc_cpr_level_dims(const orc_cpr* c, int32_t l, int32_t* dims);
void orc_cpr_level_dense(const orc_cpr* c, int32_t l, double* out);
void orc_cpr_smooth(const orc_cpr* c, int32_t l, const double* b, double* x, int32_t first);
void orc_cpr_vcycle(const orc_cpr* c, const double* b, double* x);
void orc_cpr_pressure(const orc_cpr* c, const double* rp, double* e);
void orc_cpr_apply(const orc_cpr* c, const double* r, double* z);
int orc_fgmres_cpr(orc_model* m, const double* Jdec, const double* b, double* x, int32_t restart,
                   int32_t max_restarts, double rtol, int32_t p_iters, int32_t nu, double cf, orc_solve_info* info);

/* discrete adjoint (see oracle/adjoint.cpp); orc_adjoint_step returns -2 for
 * a model with controlled wells (their rows are not in this adjoint) */
double orc_oil_rate(orc_model* m, const double* u);
int orc_adjoint_step(orc_model* m, const double* u_n, const double* u_nm1, double dt_n,
                     const double* lam_np1, const double* u_np1_unused, double dt_np1,
                     double* lam_n, double* g_logk, double* g_A);

#ifdef __cplusplus
}
#endif
#endif
