/* CPU oracle: cell properties, residual and analytical Jacobian.
 *
 * TEST INFRASTRUCTURE ONLY.  Plain serial FP64, written from the paper's model
 * (Section 2) and discretisation (Section 3.1).  Readings of passages that are
 * silent or garbled are stated where they are used.
 */
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "dual.h"
#include "model.h"

namespace orc {

using D8 = Dual<8>;
using D16 = Dual<16>;

/* ---------------------------------------------------------------- helpers */
inline double lift(double x, int) { return x; }
inline D16 lift(const D8& x, int off) {
    D16 r(x.v);
    for (int k = 0; k < 8; ++k) r.d[off + k] = x.d[k];
    return r;
}
template <class S> S seed(double x, int k);
template <> double seed<double>(double x, int) { return x; }
template <> D8 seed<D8>(double x, int k) { return D8::var(x, k); }

template <class S> inline S clamp0(const S& x) { return val(x) < 0.0 ? S(0.0) : x; }

/* Linear interpolation in a 101-row table with knots S = k/100 (the SWT/SLT
 * tables of the relative-permeability subsection).  Constant outside [0, 1];
 * at an exact interior knot the right-hand segment is used. */
template <class S> S table(const double* a, const S& s) {
    double x = val(s) * 100.0;
    if (x < 0.0) return S(a[0]);
    if (x >= 100.0) return S(a[100]);
    int k = (int)std::floor(x);
    if (k > 99) k = 99;
    S t = s * 100.0 - (double)k;
    return a[k] + t * (a[k + 1] - a[k]);
}

/* Largest real root of Z^3 - Z^2 + c1 Z + c0 (Redlich-Kwong cubic; the paper
 * takes the biggest real root).  Cardano / trigonometric form, then two
 * Newton polishing steps. */
static double cubic_largest_root(double c1, double c0) {
    const double a2 = -1.0;
    double pp = c1 - a2 * a2 / 3.0;
    double qq = 2.0 * a2 * a2 * a2 / 27.0 - a2 * c1 / 3.0 + c0;
    double disc = 0.25 * qq * qq + pp * pp * pp / 27.0;
    double t;
    if (disc > 0.0) {
        double s = std::sqrt(disc);
        t = std::cbrt(-0.5 * qq + s) + std::cbrt(-0.5 * qq - s);
    } else if (pp == 0.0) {
        t = 0.0;
    } else {
        double r = std::sqrt(-pp / 3.0);
        double arg = (3.0 * qq / (2.0 * pp)) * std::sqrt(-3.0 / pp);
        arg = std::max(-1.0, std::min(1.0, arg));
        t = 2.0 * r * std::cos(std::acos(arg) / 3.0);
    }
    double z = t - a2 / 3.0;
    for (int it = 0; it < 2; ++it) {
        double P = ((z - 1.0) * z + c1) * z + c0;
        double dP = (3.0 * z - 2.0) * z + c1;
        if (dP != 0.0) z -= P / dP;
    }
    return z;
}
static double zroot(double A, double B) { return cubic_largest_root(A - B - B * B, -A * B); }
/* derivative of the root by implicit differentiation of P(Z; A, B) = 0 */
template <int N> Dual<N> zroot(const Dual<N>& A, const Dual<N>& B) {
    double z = zroot(A.v, B.v);
    double dPdZ = (3.0 * z - 2.0) * z + (A.v - B.v - B.v * B.v);
    double dPdA = z - B.v;
    double dPdB = -z - 2.0 * B.v * z - A.v;
    Dual<N> r(z);
    for (int k = 0; k < N; ++k) r.d[k] = -(dPdA * A.d[k] + dPdB * B.d[k]) / dPdZ;
    return r;
}

/* ------------------------------------------------------------- properties */
/* Secondary quantities of one cell (Section 2.2), T in K, p in Pa.
 * Readings:
 *  - unknowns (p, x_LO, y_O2, y_CO2, T, S_w, S_g, C_c): S_o from the saturation
 *    constraint, x_HO from the oil composition constraint, y_N2 from the gas
 *    composition constraint (both constraint rows substituted);
 *  - modified PER: pseudo K only on water (S_w/(S_w+eps)) and on the heaviest
 *    oil component (S_o/(S_o+eps)); the light oil uses its plain K-value;
 *  - Redlich-Kwong mixing with a = sum y Tc^1.25/sqrt(pc), b = sum y Tc/pc,
 *    Tcm = (a^2/b)^(2/3), pcm = Tcm/b (exact in the pure-component limit);
 *  - capillary pressure zero, so every phase pressure is p;
 *  - phi_f = phi - C_c/rho_coke in the fluid accumulation and the reaction
 *    concentrations, (1 - phi) for the rock, C_c U_c for coke. */
template <class S> struct Props {
    S So, xHO, K[3], y[6];
    S Z, rho[3], mu[3], kr[3], H[3], U[3], mob[3], gam[3];
    S phi, phif, KT, Ur, Uc, rate[4], acc[8];
    S Hgc[6], Hv[3];
    S xi[3][8];   /* [phase w,o,g][row]: fraction carried (component rows), enthalpy (energy row) */
    S Tcm, pcm;
};

template <class S> S kvalue(const orc_fluid& f, int c, const S& p, const S& T) {
    return (f.kv1[c] / p) * exp(f.kv4[c] / (T - f.kv5[c]));
}

/* gas-phase molar enthalpy of species c: integral of cp from T_ref to T */
template <class S> S gas_enthalpy(const orc_fluid& f, int c, const S& T) {
    S h(0.0);
    S Tj = T;  /* T^(j+1) */
    double Rj = f.T_ref;
    for (int j = 0; j < 4; ++j) {
        h = h + (f.cpg[c][j] / (j + 1)) * (Tj - Rj);
        Tj = Tj * T;
        Rj *= f.T_ref;
    }
    return h;
}

/* gas-phase viscosity (viscosity subsection): component viscosities
 * avg_c T^bvg_c mixed with weights y_c sqrt(M_c) */
template <class S> S gas_viscosity(const orc_fluid& f, const S& T, const S* y) {
    S num(0.0), den(0.0);
    for (int c = 0; c < 6; ++c) {
        double sm = std::sqrt(f.M[c]);
        S mgc = f.avg[c] * pow(T, f.bvg[c]);
        num = num + mgc * y[c] * sm;
        den = den + y[c] * sm;
    }
    return num / den;
}

template <class S> S vap_heat(const orc_fluid& f, int c, const S& T) {
    if (val(T) < f.Tc[c]) return f.hvr[c] * pow(f.Tc[c] - T, f.ev[c]);
    return S(0.0);
}

template <class S> void props(const orc_fluid& f, double phi_ref, const S* u, Props<S>& P) {
    const S& p = u[0]; const S& xLO = u[1]; const S& yO2 = u[2]; const S& yCO2 = u[3];
    const S& T = u[4]; const S& Sw = u[5]; const S& Sg = u[6]; const S& Cc = u[7];
    P.So = 1.0 - Sw - Sg;
    P.xHO = 1.0 - xLO;
    for (int c = 0; c < 3; ++c) P.K[c] = kvalue(f, c, p, T);
    S fw = Sw / (Sw + f.eps);
    S fo = P.So / (P.So + f.eps);
    P.y[0] = fw * P.K[0];
    P.y[1] = P.K[1] * xLO;
    P.y[2] = fo * P.K[2] * P.xHO;
    P.y[3] = yO2;
    P.y[4] = yCO2;
    P.y[5] = 1.0 - P.y[0] - P.y[1] - P.y[2] - P.y[3] - P.y[4];

    /* Z factor */
    S a(0.0), b(0.0);
    for (int c = 0; c < 6; ++c) {
        a = a + P.y[c] * (std::pow(f.Tc[c], 1.25) / std::sqrt(f.pc[c]));
        b = b + P.y[c] * (f.Tc[c] / f.pc[c]);
    }
    P.Tcm = pow(a * a / b, 2.0 / 3.0);
    P.pcm = P.Tcm / b;
    S Ar = 0.42748 * (p / P.pcm) * pow(P.Tcm / T, 2.5);
    S Br = 0.08664 * (p / P.pcm) * (P.Tcm / T);
    P.Z = zroot(Ar, Br);

    /* densities */
    P.rho[2] = p / (P.Z * f.Rgas * T);
    S rl[3];
    for (int c = 0; c < 3; ++c)
        rl[c] = f.rho_ref[c] * exp(f.cp_liq[c] * (p - f.p_ref) - f.ct1_liq[c] * (T - f.T_ref));
    P.rho[0] = rl[0];
    P.rho[1] = 1.0 / (xLO / rl[1] + P.xHO / rl[2]);

    /* viscosities */
    P.mu[0] = f.avisc[0] * exp(f.bvisc[0] / T);
    S lnLO = std::log(f.avisc[1]) + f.bvisc[1] / T;
    S lnHO = std::log(f.avisc[2]) + f.bvisc[2] / T;
    P.mu[1] = exp(xLO * lnLO + P.xHO * lnHO);
    P.mu[2] = gas_viscosity(f, T, P.y);

    /* porosity */
    P.phi = phi_ref * (1.0 + f.cpor * (p - f.p_ref));
    P.phif = P.phi - Cc / f.rho_coke;

    /* relative permeabilities, Stone II */
    S krw = table(f.krw, Sw), krow = table(f.krow, Sw);
    S krg = table(f.krg, Sg), krog = table(f.krog, Sg);
    S kro = f.krocw * ((krow / f.krocw + krw) * (krog / f.krocw + krg) - krw - krg);
    P.kr[0] = krw;
    P.kr[1] = clamp0(kro);
    P.kr[2] = krg;

    /* enthalpies and internal energies */
    for (int c = 0; c < 6; ++c) P.Hgc[c] = gas_enthalpy(f, c, T);
    for (int c = 0; c < 3; ++c) P.Hv[c] = vap_heat(f, c, T);
    P.H[0] = P.Hgc[0] - P.Hv[0];
    P.H[1] = xLO * (P.Hgc[1] - P.Hv[1]) + P.xHO * (P.Hgc[2] - P.Hv[2]);
    P.H[2] = P.y[0] * P.Hgc[0];
    for (int c = 1; c < 6; ++c) P.H[2] = P.H[2] + P.y[c] * P.Hgc[c];
    for (int a2 = 0; a2 < 3; ++a2) P.U[a2] = P.H[a2] - p / P.rho[a2];
    P.Ur = f.cp_rock * (T - f.T_ref);
    P.Uc = f.cp_coke * (T - f.T_ref);

    /* bulk conductivity (coke term dropped: no coke conductivity is given) */
    P.KT = P.phif * (Sw * f.Kcond[0] + P.So * f.Kcond[1] + Sg * f.Kcond[2]) +
           (1.0 - P.phi) * f.Kcond[3];

    /* Arrhenius rates with concentrations per bulk volume */
    S ek[4];
    for (int r = 0; r < 4; ++r) ek[r] = f.Afreq[r] * exp(-f.Eact[r] / (f.Rgas * T));
    S conc_o = P.phif * P.So * P.rho[1];
    S pO2 = yO2 * p;
    P.rate[0] = ek[0] * pO2 * conc_o * xLO;
    P.rate[1] = ek[1] * pO2 * conc_o * P.xHO;
    S ratio = Cc / f.Ccmax;
    S r2 = ratio * ratio;
    S limiter = clamp0(1.0 - r2 * r2 * ratio);
    P.rate[2] = ek[2] * conc_o * P.xHO * limiter;
    P.rate[3] = ek[3] * pO2 * Cc;

    /* accumulation per unit bulk volume */
    S gw = P.rho[0] * Sw, go = P.rho[1] * P.So, gg = P.rho[2] * Sg;
    P.acc[0] = P.phif * (gw + gg * P.y[0]);
    P.acc[1] = P.phif * (go * xLO + gg * P.y[1]);
    P.acc[2] = P.phif * (go * P.xHO + gg * P.y[2]);
    P.acc[3] = P.phif * gg * P.y[3];
    P.acc[4] = P.phif * gg * P.y[4];
    P.acc[5] = P.phif * gg * P.y[5];
    P.acc[6] = P.phif * (gw * P.U[0] + go * P.U[1] + gg * P.U[2]) + (1.0 - P.phi) * P.Ur +
               Cc * P.Uc;
    P.acc[7] = Cc;

    /* mobilities and specific weights */
    for (int a2 = 0; a2 < 3; ++a2) P.mob[a2] = P.kr[a2] * P.rho[a2] / P.mu[a2];
    P.gam[0] = f.grav * P.rho[0] * f.M[0];
    P.gam[1] = f.grav * P.rho[1] * (xLO * f.M[1] + P.xHO * f.M[2]);
    S Mg = P.y[0] * f.M[0];
    for (int c = 1; c < 6; ++c) Mg = Mg + P.y[c] * f.M[c];
    P.gam[2] = f.grav * P.rho[2] * Mg;

    for (int a2 = 0; a2 < 3; ++a2)
        for (int e = 0; e < 8; ++e) P.xi[a2][e] = S(0.0);
    P.xi[0][0] = S(1.0);
    P.xi[0][6] = P.H[0];
    P.xi[1][1] = xLO;
    P.xi[1][2] = P.xHO;
    P.xi[1][6] = P.H[1];
    for (int c = 0; c < 6; ++c) P.xi[2][c] = P.y[c];
    P.xi[2][6] = P.H[2];
}

/* Row e of the equations owned by species c (rows 0..5 are W..N2, 7 is coke). */
static const int kSpeciesRow[ORC_NSPEC] = {0, 1, 2, 3, 4, 5, 7};

/* ------------------------------------------------------------- grid utils */
double cell_volume(const orc_model& m) { return m.g.dx * m.g.dy * m.g.dz; }
double depth(const orc_model& m, int32_t i) {
    int32_t iz = i / (m.g.nx * m.g.ny);
    return (iz + 0.5) * m.g.dz;
}
int32_t block_of(const orc_model& m, int32_t i, int32_t j) {
    for (int32_t b = m.row_ptr[i]; b < m.row_ptr[i + 1]; ++b)
        if (m.col_idx[b] == j) return b;
    return -1;
}

/* Peaceman inflow (well-modelling subsection): WI = 2 pi h sqrt(kx ky) /
 * (ln(re/rw) + s), re = 0.14 sqrt(dx^2 + dy^2).  Producers (kind 1): fixed
 * BHP, local inflow, no backflow.  Injectors (kind 2): fixed molar rate split
 * over perforations in proportion to WI, injected as gas at T_inj.  Kinds 3
 * and 4 take their bhp from the well state (orc_cwell); their perforations
 * keep only WI here. */
void compute_wells(orc_model& m) {
    m.perfs.clear();
    double re = 0.14 * std::sqrt(m.g.dx * m.g.dx + m.g.dy * m.g.dy);
    size_t ncw = 0;
    for (size_t w = 0; w < m.wells_in.size(); ++w) {
        const orc_well& W = m.wells_in[w];
        const std::vector<int32_t>& cells = m.well_cells[w];
        std::vector<double> wi(cells.size());
        double sum = 0.0;
        for (size_t k = 0; k < cells.size(); ++k) {
            double kh = m.kh[cells[k]];
            wi[k] = 2.0 * M_PI * m.g.dz * kh / (std::log(re / W.rw) + W.skin);
            sum += wi[k];
        }
        double Hinj = 0.0;
        for (int c = 0; c < 6; ++c) Hinj += W.z_inj[c] * gas_enthalpy(m.fl, c, W.T_inj);
        const bool controlled = W.kind == 3 || W.kind == 4;
        if (controlled) {
            orc_cwell& C = m.cw[ncw];
            C.p0 = (int32_t)m.perfs.size();
            C.np = (int32_t)cells.size();
            C.c0 = ncw == 0 ? 0 : m.cw[ncw - 1].c0 + m.cw[ncw - 1].np;
            for (int c = 0; c < ORC_NSPEC; ++c) C.z[c] = W.z_inj[c];
            C.Hinj = Hinj;
        }
        for (size_t k = 0; k < cells.size(); ++k) {
            orc_perf P;
            std::memset(&P, 0, sizeof(P));
            P.cell = cells[k];
            P.kind = W.kind;
            P.well = controlled ? (int32_t)ncw : -1;
            P.wi = wi[k];
            if (controlled) {
                /* bhp from the well state */
            } else if (W.kind == 1) {
                P.bhp = W.target;
            } else {
                double q = W.target * wi[k] / sum;
                P.q_total = q;
                for (int c = 0; c < ORC_NSPEC; ++c) P.q[c] = q * W.z_inj[c];
                P.qE = q * Hinj;
            }
            m.perfs.push_back(P);
        }
        if (controlled) ++ncw;
    }
}

/* Flow of one perforation of a controlled well at its cell's properties P,
 * cell pressure p and the well's bhp (well-modelling subsection): phase molar
 * rates Q_a = WI lambda_a (bhp - p), lambda_a = rho_a k_ra / mu_a, at a
 * producer while p > bhp; at an injector the injected gas enters with the
 * cell's total mobility, Q = WI (lambda_w + lambda_o + lambda_g) (bhp - p),
 * while bhp > p; no backflow either way.  Q < 0 is production.  dQ holds
 * dQ/dbhp. */
template <class S> struct PerfFlow {
    bool active = false;
    S Q[3];         /* producer phase rates */
    double dQ[3] = {0.0, 0.0, 0.0};
    S Qi;           /* injector total rate */
    double dQi = 0.0;
};
template <class S>
PerfFlow<S> perf_flow(const orc_perf& W, const orc_cwell& C, const Props<S>& P, const S& p) {
    PerfFlow<S> f;
    for (int a = 0; a < 3; ++a) f.Q[a] = S(0.0);
    f.Qi = S(0.0);
    if (W.kind == 3) {
        if (!(val(p) > C.bhp)) return f;
        f.active = true;
        for (int a = 0; a < 3; ++a) {
            f.Q[a] = W.wi * P.mob[a] * (C.bhp - p);
            f.dQ[a] = W.wi * val(P.mob[a]);
        }
    } else {
        if (!(C.bhp > val(p))) return f;
        f.active = true;
        S lt = P.mob[0] + P.mob[1] + P.mob[2];
        f.Qi = W.wi * lt * (C.bhp - p);
        f.dQi = W.wi * val(lt);
    }
    return f;
}

/* the amount that a controlled well's perforation takes out of row e */
template <class S> S perf_row(const orc_perf& W, const orc_cwell& C, const Props<S>& P, const PerfFlow<S>& f, int e) {
    S t(0.0);
    if (!f.active || e > 6) return t;
    if (W.kind == 3) {
        for (int a = 0; a < 3; ++a) t = t + f.Q[a] * P.xi[a][e];
    } else {
        t = f.Qi * (e == 6 ? C.Hinj : C.z[e]);
    }
    return t;
}

/* ------------------------------------------------------------- assembly */
struct FaceGeom { double area_over_h; double trans; double dz; };

/* dir: 0 = x, 1 = y, 2 = z face between lo and its +dir neighbour hi */
static FaceGeom face_geom(const orc_model& m, int32_t lo, int32_t hi, int dir) {
    const orc_grid& g = m.g;
    FaceGeom G;
    double klo, khi;
    if (dir == 0) { G.area_over_h = g.dy * g.dz / g.dx; klo = m.kh[lo]; khi = m.kh[hi]; G.dz = 0.0; }
    else if (dir == 1) { G.area_over_h = g.dx * g.dz / g.dy; klo = m.kh[lo]; khi = m.kh[hi]; G.dz = 0.0; }
    else { G.area_over_h = g.dx * g.dy / g.dz; klo = m.kz[lo]; khi = m.kz[hi]; G.dz = -g.dz; }
    double alo = G.area_over_h * klo, ahi = G.area_over_h * khi;
    G.trans = 2.0 * alo * ahi / (alo + ahi);  /* harmonic transmissibility */
    return G;
}

/* Molar/energy outflow from lo to hi for each row (Section 3.1 residuals).
 * Reading of the sign: outflow-positive, T * lambda_up * (Phi_lo - Phi_hi),
 * conduction (A/h) K_T,harm (T_lo - T_hi).  Upstream: the cell with the higher
 * potential; on a tie the lower cell index (lo). */
template <class S16, class S8>
void face_flux(const orc_model& m, const FaceGeom& G, const Props<S8>& Plo, const Props<S8>& Phi,
               const S8& plo, const S8& phi_, const S8& Tlo, const S8& Thi, S16* flow,
               bool conduction = true) {
    for (int e = 0; e < 8; ++e) flow[e] = S16(0.0);
    S16 dp = lift(plo, 0) - lift(phi_, 8);
    for (int a = 0; a < 3; ++a) {
        S16 gbar = 0.5 * (lift(Plo.gam[a], 0) + lift(Phi.gam[a], 8));
        S16 dphi = dp - gbar * G.dz;
        bool up_lo = !(val(dphi) < 0.0);
        const Props<S8>& U = up_lo ? Plo : Phi;
        int off = up_lo ? 0 : 8;
        S16 mob = lift(U.mob[a], off);
        S16 base = G.trans * mob * dphi;
        for (int e = 0; e < 7; ++e) {
            bool present = (a == 0 && (e == 0 || e == 6)) || (a == 1 && (e == 1 || e == 2 || e == 6)) ||
                           (a == 2);
            if (!present) continue;
            flow[e] = flow[e] + base * lift(U.xi[a][e], off);
        }
    }
    if (!conduction) return;
    S16 klo = lift(Plo.KT, 0), khi = lift(Phi.KT, 8);
    S16 kh = 2.0 * klo * khi / (klo + khi);
    flow[6] = flow[6] + G.area_over_h * kh * (lift(Tlo, 0) - lift(Thi, 8));
}

template <class S8> static void load_cell(const double* u, int32_t n, int32_t i, S8* ui) {
    for (int v = 0; v < 8; ++v) ui[v] = seed<S8>(u[(size_t)v * n + i], v);
}

static inline void add_block(double* J, int32_t b, double sgn, const D16& x, int off, int e) {
    for (int v = 0; v < 8; ++v) J[(size_t)b * 64 + e * 8 + v] += sgn * x.d[off + v];
}
static inline void add_block(double*, int32_t, double, double, int, int) {}
static inline void add_diag(double* J, int32_t b, double sgn, const D8& x, int e) {
    for (int v = 0; v < 8; ++v) J[(size_t)b * 64 + e * 8 + v] += sgn * x.d[v];
}
static inline void add_diag(double*, int32_t, double, double, int) {}

/* residual F (and Jacobian J when S8 is a dual type) at state u */
template <class S8, class S16>
static int assemble_impl(orc_model& m, const double* u, const double* u_old, double dt, double* F,
                         double* J) {
    const int32_t n = m.n;
    const orc_fluid& f = m.fl;
    const double V = cell_volume(m);
    std::fill(F, F + (size_t)n * 8, 0.0);
    if (J) std::fill(J, J + (size_t)m.row_ptr[n] * 64, 0.0);
    std::vector<Props<S8>> P(n);
    std::vector<S8> pp(n), TT(n);

    /* local terms: accumulation, reactions */
    for (int32_t i = 0; i < n; ++i) {
        S8 ui[8];
        load_cell(u, n, i, ui);
        props(f, m.poro[i], ui, P[i]);
        pp[i] = ui[0];
        TT[i] = ui[4];
        double uo[8];
        for (int v = 0; v < 8; ++v) uo[v] = u_old[(size_t)v * n + i];
        Props<double> Po;
        props(f, m.poro[i], uo, Po);
        S8 src[8];
        for (int e = 0; e < 8; ++e) src[e] = S8(0.0);
        for (int r = 0; r < 4; ++r) {
            for (int c = 0; c < ORC_NSPEC; ++c)
                if (f.stoich[r][c] != 0.0) src[kSpeciesRow[c]] = src[kSpeciesRow[c]] + f.stoich[r][c] * P[i].rate[r];
            src[6] = src[6] + f.Hreac[r] * P[i].rate[r];
        }
        for (int e = 0; e < 8; ++e) {
            S8 Fe = (V / dt) * (P[i].acc[e] - Po.acc[e]) - V * src[e];
            F[(size_t)i * 8 + e] += val(Fe);
            if (J) add_diag(J, m.diag_pos[i], 1.0, Fe, e);
        }
    }
    /* wells */
    for (const orc_perf& W : m.perfs) {
        int32_t i = W.cell;
        if (W.kind == 1) {
            if (!(val(pp[i]) > W.bhp)) continue;   /* no backflow */
            for (int a = 0; a < 3; ++a) {
                S8 Q = W.wi * P[i].mob[a] * (W.bhp - pp[i]);
                for (int e = 0; e < 7; ++e) {
                    S8 t = Q * P[i].xi[a][e];
                    F[(size_t)i * 8 + e] -= val(t);
                    if (J) add_diag(J, m.diag_pos[i], -1.0, t, e);
                }
            }
        } else if (W.kind == 2) {
            for (int c = 0; c < 6; ++c) F[(size_t)i * 8 + c] -= W.q[c];
            F[(size_t)i * 8 + 6] -= W.qE;
        } else {
            const orc_cwell& C = m.cw[W.well];
            PerfFlow<S8> fl = perf_flow(W, C, P[i], pp[i]);
            for (int e = 0; e < 7; ++e) {
                S8 t = perf_row(W, C, P[i], fl, e);
                F[(size_t)i * 8 + e] -= val(t);
                if (J) add_diag(J, m.diag_pos[i], -1.0, t, e);
            }
        }
    }
    /* heater: a fixed heat rate into one cell (the ignition heater of the
     * combustion tube, Section 4.1), independent of the state */
    if (m.heater_cell >= 0) F[(size_t)m.heater_cell * 8 + 6] -= m.heater_W;
    /* faces, each evaluated once with (lo, hi) = (min, max) cell index */
    const orc_grid& g = m.g;
    for (int32_t lo = 0; lo < n; ++lo) {
        int32_t ix = lo % g.nx, iy = (lo / g.nx) % g.ny, iz = lo / (g.nx * g.ny);
        int32_t nb[3] = {ix + 1 < g.nx ? lo + 1 : -1, iy + 1 < g.ny ? lo + g.nx : -1,
                         iz + 1 < g.nz ? lo + g.nx * g.ny : -1};
        for (int d = 0; d < 3; ++d) {
            int32_t hi = nb[d];
            if (hi < 0) continue;
            FaceGeom G = face_geom(m, lo, hi, d);
            S16 flow[8];
            face_flux<S16, S8>(m, G, P[lo], P[hi], pp[lo], pp[hi], TT[lo], TT[hi], flow);
            for (int e = 0; e < 7; ++e) {
                F[(size_t)lo * 8 + e] += val(flow[e]);
                F[(size_t)hi * 8 + e] -= val(flow[e]);
                if (J) {
                    add_block(J, m.diag_pos[lo], 1.0, flow[e], 0, e);
                    add_block(J, block_of(m, lo, hi), 1.0, flow[e], 8, e);
                    add_block(J, m.diag_pos[hi], -1.0, flow[e], 8, e);
                    add_block(J, block_of(m, hi, lo), -1.0, flow[e], 0, e);
                }
            }
        }
    }
    return 0;
}

/* ------------------------------------------------------------- adjoint helpers */
static const orc_perf* producer_at(const orc_model& m, int32_t i) {
    for (const orc_perf& P : m.perfs)
        if (P.cell == i && P.kind == 1) return &P;
    return nullptr;
}

/* accumulation Jacobian dA_e/du_v at u_i and the producer's oil-phase molar
 * rate q = WI lambda_o (p - p_wf) for p > p_wf with its gradient */
void props_acc_grad(const orc_model& m, int32_t i, const double* u_i, double* acc_jac, double* qoil,
                    double* qoil_grad, double* mob_o_val) {
    D8 ui[8];
    for (int v = 0; v < 8; ++v) ui[v] = D8::var(u_i[v], v);
    Props<D8> P;
    props(m.fl, m.poro[i], ui, P);
    for (int e = 0; e < 8; ++e)
        for (int v = 0; v < 8; ++v) acc_jac[e * 8 + v] = P.acc[e].d[v];
    *mob_o_val = P.mob[1].v;
    *qoil = 0.0;
    for (int v = 0; v < 8; ++v) qoil_grad[v] = 0.0;
    const orc_perf* W = producer_at(m, i);
    if (W && u_i[0] > W->bhp) {
        D8 q = W->wi * P.mob[1] * (ui[0] - W->bhp);
        *qoil = q.v;
        for (int v = 0; v < 8; ++v) qoil_grad[v] = q.d[v];
    }
}

double cell_oil_rate(const orc_model& m, int32_t i, const double* u_i) {
    const orc_perf* W = producer_at(m, i);
    if (!W || !(u_i[0] > W->bhp)) return 0.0;
    Props<double> P;
    props(m.fl, m.poro[i], u_i, P);
    return W->wi * P.mob[1] * (u_i[0] - W->bhp);
}

/* convective part of the face outflow (proportional to the transmissibility) */
void face_conv_flux(const orc_model& m, const double* u, int32_t lo, int32_t hi, int dir, double* flow) {
    double ul[8], uh[8];
    for (int v = 0; v < 8; ++v) {
        ul[v] = u[(size_t)v * m.n + lo];
        uh[v] = u[(size_t)v * m.n + hi];
    }
    Props<double> Pl, Ph;
    props(m.fl, m.poro[lo], ul, Pl);
    props(m.fl, m.poro[hi], uh, Ph);
    FaceGeom G = face_geom(m, lo, hi, dir);
    face_flux<double, double>(m, G, Pl, Ph, ul[0], uh[0], ul[4], uh[4], flow, false);
    flow[7] = 0.0;
}

void cell_rates(const orc_model& m, int32_t i, const double* u_i, double* rates) {
    Props<double> P;
    props(m.fl, m.poro[i], u_i, P);
    for (int r = 0; r < 4; ++r) rates[r] = P.rate[r];
}

/* producer well terms at cell i (the amounts subtracted from the residual) */
void well_terms(const orc_model& m, int32_t i, const double* u_i, double* W) {
    for (int e = 0; e < 8; ++e) W[e] = 0.0;
    const orc_perf* P = producer_at(m, i);
    if (!P || !(u_i[0] > P->bhp)) return;
    Props<double> Pr;
    props(m.fl, m.poro[i], u_i, Pr);
    for (int a = 0; a < 3; ++a) {
        double Q = P->wi * Pr.mob[a] * (P->bhp - u_i[0]);
        for (int e = 0; e < 7; ++e) W[e] += Q * Pr.xi[a][e];
    }
}

}  // namespace orc

using namespace orc;

extern "C" {

orc_model* orc_create(const orc_grid* g, const orc_fluid* fl, const double* logk, double kvkh,
                      const double* poro, const orc_well* wells, int32_t nwells) {
    orc_model* m = new orc_model();
    m->g = *g;
    m->fl = *fl;
    m->n = g->nx * g->ny * g->nz;
    m->kvkh = kvkh;
    m->logk.assign(logk, logk + m->n);
    m->poro.assign(poro, poro + m->n);
    m->kh.resize(m->n);
    m->kz.resize(m->n);
    for (int32_t i = 0; i < m->n; ++i) {
        m->kh[i] = std::exp(logk[i]);
        m->kz[i] = m->kh[i] * kvkh;
    }
    /* block CSR pattern: 7-point stencil, columns ascending */
    const int32_t nx = g->nx, nxy = g->nx * g->ny;
    m->row_ptr.assign(m->n + 1, 0);
    m->diag_pos.assign(m->n, 0);
    for (int32_t i = 0; i < m->n; ++i) {
        int32_t ix = i % nx, iy = (i / nx) % g->ny, iz = i / nxy;
        int32_t cand[7] = {iz > 0 ? i - nxy : -1, iy > 0 ? i - nx : -1, ix > 0 ? i - 1 : -1, i,
                           ix + 1 < nx ? i + 1 : -1, iy + 1 < g->ny ? i + nx : -1,
                           iz + 1 < g->nz ? i + nxy : -1};
        for (int k = 0; k < 7; ++k) {
            if (cand[k] < 0) continue;
            if (cand[k] == i) m->diag_pos[i] = (int32_t)m->col_idx.size();
            m->col_idx.push_back(cand[k]);
        }
        m->row_ptr[i + 1] = (int32_t)m->col_idx.size();
    }
    for (int32_t w = 0; w < nwells; ++w) {
        m->wells_in.push_back(wells[w]);
        m->well_cells.emplace_back(wells[w].perf_cells, wells[w].perf_cells + wells[w].nperf);
        if (wells[w].kind == 3 || wells[w].kind == 4) {
            orc_cwell C;
            C.kind = wells[w].kind;
            C.control = wells[w].control;
            C.target = wells[w].target;
            C.limit = wells[w].limit;
            C.bhp = C.control == 0 ? C.target : C.limit;
            m->cw.push_back(C);
        }
    }
    compute_wells(*m);
    return m;
}

void orc_destroy(orc_model* m) { delete m; }
int32_t orc_ncell(const orc_model* m) { return m->n; }
int32_t orc_nnzb(const orc_model* m) { return m->row_ptr[m->n]; }
void orc_pattern(const orc_model* m, int32_t* row_ptr, int32_t* col_idx) {
    std::copy(m->row_ptr.begin(), m->row_ptr.end(), row_ptr);
    std::copy(m->col_idx.begin(), m->col_idx.end(), col_idx);
}

void orc_set_heater(orc_model* m, int32_t cell, double rate_W) {
    m->heater_cell = (cell >= 0 && cell < m->n && rate_W != 0.0) ? cell : -1;
    m->heater_W = m->heater_cell >= 0 ? rate_W : 0.0;
}

void orc_set_params(orc_model* m, const double* logk, const double* A) {
    if (logk) {
        m->logk.assign(logk, logk + m->n);
        for (int32_t i = 0; i < m->n; ++i) {
            m->kh[i] = std::exp(logk[i]);
            m->kz[i] = m->kh[i] * m->kvkh;
        }
        compute_wells(*m);
    }
    if (A)
        for (int r = 0; r < ORC_NREAC; ++r) m->fl.Afreq[r] = A[r];
}

void orc_perf_info(const orc_model* m, int32_t* cells, int32_t* kinds, double* wi, double* q) {
    for (size_t k = 0; k < m->perfs.size(); ++k) {
        cells[k] = m->perfs[k].cell;
        kinds[k] = m->perfs[k].kind;
        wi[k] = m->perfs[k].wi;
        q[k] = m->perfs[k].q_total;
    }
}

void orc_diag(const orc_model* m, const double* u, double* out) {
    const int32_t n = m->n;
    for (int32_t i = 0; i < n; ++i) {
        double ui[8];
        for (int v = 0; v < 8; ++v) ui[v] = u[(size_t)v * n + i];
        Props<double> P;
        props(m->fl, m->poro[i], ui, P);
        double* o = out + (size_t)i * ORC_NDIAG;
        o[ORC_DIAG_SO] = P.So; o[ORC_DIAG_XHO] = P.xHO;
        for (int c = 0; c < 6; ++c) o[ORC_DIAG_Y0 + c] = P.y[c];
        o[ORC_DIAG_Z] = P.Z;
        o[ORC_DIAG_RHOW] = P.rho[0]; o[ORC_DIAG_RHOO] = P.rho[1]; o[ORC_DIAG_RHOG] = P.rho[2];
        o[ORC_DIAG_MUW] = P.mu[0]; o[ORC_DIAG_MUO] = P.mu[1]; o[ORC_DIAG_MUG] = P.mu[2];
        o[ORC_DIAG_PHI] = P.phi; o[ORC_DIAG_PHIF] = P.phif;
        o[ORC_DIAG_KRW] = P.kr[0]; o[ORC_DIAG_KRO] = P.kr[1]; o[ORC_DIAG_KRG] = P.kr[2];
        o[ORC_DIAG_HW] = P.H[0]; o[ORC_DIAG_HO] = P.H[1]; o[ORC_DIAG_HG] = P.H[2];
        o[ORC_DIAG_KT] = P.KT;
        for (int r = 0; r < 4; ++r) o[ORC_DIAG_R0 + r] = P.rate[r];
        for (int e = 0; e < 8; ++e) o[ORC_DIAG_ACC0 + e] = P.acc[e];
        o[ORC_DIAG_KW] = P.K[0]; o[ORC_DIAG_KLO] = P.K[1]; o[ORC_DIAG_KHO] = P.K[2];
        o[ORC_DIAG_HVW] = P.Hv[0];
        o[ORC_DIAG_HGO2] = P.Hgc[3];
    }
}

double orc_zfactor(const orc_fluid* fl, double p, double T, const double* y, double* Tcm, double* pcm) {
    double a = 0.0, b = 0.0;
    for (int c = 0; c < 6; ++c) {
        a += y[c] * (std::pow(fl->Tc[c], 1.25) / std::sqrt(fl->pc[c]));
        b += y[c] * (fl->Tc[c] / fl->pc[c]);
    }
    double tcm = std::pow(a * a / b, 2.0 / 3.0), pcm_ = tcm / b;
    double A = 0.42748 * (p / pcm_) * std::pow(tcm / T, 2.5);
    double B = 0.08664 * (p / pcm_) * (tcm / T);
    if (Tcm) *Tcm = tcm;
    if (pcm) *pcm = pcm_;
    return zroot(A, B);
}

double orc_gas_viscosity(const orc_fluid* fl, double T, const double* y) {
    return gas_viscosity(*fl, T, y);
}

int orc_residual(orc_model* m, const double* u, const double* u_old, double dt, double* F) {
    return assemble_impl<double, double>(*m, u, u_old, dt, F, nullptr);
}

int orc_assemble(orc_model* m, const double* u, const double* u_old, double dt, double* F, double* J) {
    return assemble_impl<D8, D16>(*m, u, u_old, dt, F, J);
}

void orc_sources(orc_model* m, const double* u, double* wells_out, double* reac_out) {
    const int32_t n = m->n;
    const double V = cell_volume(*m);
    std::vector<Props<double>> P(n);
    for (int32_t i = 0; i < n; ++i) {
        double ui[8];
        for (int v = 0; v < 8; ++v) ui[v] = u[(size_t)v * n + i];
        props(m->fl, m->poro[i], ui, P[i]);
    }
    if (reac_out) {
        std::fill(reac_out, reac_out + (size_t)n * 8, 0.0);
        for (int32_t i = 0; i < n; ++i)
            for (int r = 0; r < 4; ++r) {
                for (int c = 0; c < ORC_NSPEC; ++c)
                    reac_out[(size_t)i * 8 + kSpeciesRow[c]] += V * m->fl.stoich[r][c] * P[i].rate[r];
                reac_out[(size_t)i * 8 + 6] += V * m->fl.Hreac[r] * P[i].rate[r];
            }
    }
    if (wells_out) {
        std::fill(wells_out, wells_out + (size_t)n * 8, 0.0);
        for (const orc_perf& W : m->perfs) {
            int32_t i = W.cell;
            double p = u[i];
            if (W.kind == 1) {
                if (!(p > W.bhp)) continue;
                for (int a = 0; a < 3; ++a) {
                    double Q = W.wi * P[i].mob[a] * (W.bhp - p);
                    for (int e = 0; e < 7; ++e) wells_out[(size_t)i * 8 + e] += Q * P[i].xi[a][e];
                }
            } else if (W.kind == 2) {
                for (int c = 0; c < 6; ++c) wells_out[(size_t)i * 8 + c] += W.q[c];
                wells_out[(size_t)i * 8 + 6] += W.qE;
            } else {
                const orc_cwell& C = m->cw[W.well];
                PerfFlow<double> fl = perf_flow(W, C, P[i], p);
                for (int e = 0; e < 7; ++e) wells_out[(size_t)i * 8 + e] += perf_row(W, C, P[i], fl, e);
            }
        }
        if (m->heater_cell >= 0) wells_out[(size_t)m->heater_cell * 8 + 6] += m->heater_W;
    }
}

int32_t orc_ncwell(const orc_model* m) { return (int32_t)m->cw.size(); }

void orc_well_state(const orc_model* m, double* bhp, int32_t* on_limit) {
    for (size_t w = 0; w < m->cw.size(); ++w) {
        if (bhp) bhp[w] = m->cw[w].bhp;
        if (on_limit) on_limit[w] = m->cw[w].on_limit;
    }
}

void orc_set_well_state(orc_model* m, const double* bhp, const int32_t* on_limit) {
    for (size_t w = 0; w < m->cw.size(); ++w) {
        if (bhp) m->cw[w].bhp = bhp[w];
        if (on_limit) m->cw[w].on_limit = on_limit[w] ? 1 : 0;
    }
}

/* the controlled quantity of well C at state u and its current bhp: the
 * produced molar rate of the phases in the mask (producer) or the injected
 * molar rate (injector), with its gradient per perforation (C[k][8], may be
 * NULL) and its derivative in bhp */
static double controlled_rate(const orc_model& m, const orc_cwell& C, const double* u, double* Cg, double* dq) {
    double q = 0.0, d = 0.0;
    for (int32_t k = 0; k < C.np; ++k) {
        const orc_perf& W = m.perfs[C.p0 + k];
        D8 ui[8];
        load_cell(u, m.n, W.cell, ui);
        Props<D8> P;
        props(m.fl, m.poro[W.cell], ui, P);
        PerfFlow<D8> fl = perf_flow(W, C, P, ui[0]);
        D8 qk(0.0);
        double dk = 0.0;
        if (C.kind == 3) {
            for (int a = 0; a < 3; ++a)
                if (C.control & (1 << a)) {
                    qk = qk - fl.Q[a];
                    dk -= fl.dQ[a];
                }
        } else {
            qk = fl.Qi;
            dk = fl.dQi;
        }
        q += qk.v;
        d += dk;
        if (Cg)
            for (int v = 0; v < 8; ++v) Cg[(size_t)k * 8 + v] = qk.d[v];
    }
    if (dq) *dq = d;
    return q;
}

}  // extern "C"

/* The well equation of a rate-controlled well on its own.  With the cells'
 * state fixed, the controlled rate is g(b) = sum_k a_k (p_k - b)^+ for a
 * producer (a_k = WI times the mobilities of the phases in its mask) and
 * sum_k a_k (b - p_k)^+ for an injector (a_k = WI lambda_t): piecewise linear
 * and monotone in the bottom-hole pressure b, with breakpoints at the
 * perforated cells' pressures p_k. */
struct WellLine {
    std::vector<double> a, p;
    bool injector;
    double g(double b) const {
        double s = 0.0;
        for (size_t k = 0; k < a.size(); ++k) {
            const double d = injector ? b - p[k] : p[k] - b;
            if (d > 0.0) s += a[k] * d;
        }
        return s;
    }
};

static WellLine well_line(const orc_model& m, const orc_cwell& C, const double* u) {
    WellLine L;
    L.injector = C.kind == 4;
    for (int32_t k = 0; k < C.np; ++k) {
        const orc_perf& W = m.perfs[C.p0 + k];
        double ui[8];
        for (int v = 0; v < 8; ++v) ui[v] = u[(size_t)v * m.n + W.cell];
        Props<double> P;
        props(m.fl, m.poro[W.cell], ui, P);
        double lam = 0.0;
        for (int a = 0; a < 3; ++a)
            if (L.injector || (C.control & (1 << a))) lam += P.mob[a];
        L.a.push_back(W.wi * lam);
        L.p.push_back(ui[0]);
    }
    return L;
}

/* the b with g(b) = c, given g(lim) >= c: walk the breakpoints away from the
 * limit to the first segment whose far end has g <= c, and solve the linear
 * piece there (its active perforations are those beyond that end) */
static double well_line_root(const WellLine& L, double lim, double c) {
    const double s = L.injector ? -1.0 : 1.0;   /* an injector in a producer's form: b -> -b */
    std::vector<double> bp{s * lim};
    for (double x : L.p)
        if (s * x > s * lim) bp.push_back(s * x);
    std::sort(bp.begin(), bp.end());
    for (size_t i = 0; i + 1 < bp.size(); ++i) {
        if (L.g(s * bp[i + 1]) > c) continue;
        double sa = 0.0, sap = 0.0;
        for (size_t k = 0; k < L.a.size(); ++k)
            if (s * L.p[k] >= bp[i + 1]) {
                sa += L.a[k];
                sap += L.a[k] * s * L.p[k];
            }
        double b = sa > 0.0 ? (sap - c) / sa : bp[i];
        b = std::min(std::max(b, bp[i]), bp[i + 1]);
        return s * b;
    }
    return lim;   /* no perforation beyond the limit: g(lim) = 0 = c */
}

extern "C" {

int32_t orc_well_solve(orc_model* m, const double* u) {
    int32_t nsw = 0;
    for (orc_cwell& C : m->cw) {
        if (C.control == 0 || C.on_limit) continue;
        WellLine L = well_line(*m, C, u);
        if (L.g(C.limit) < C.target) {
            C.on_limit = 1;
            C.bhp = C.limit;
            ++nsw;
        } else {
            C.bhp = well_line_root(L, C.limit, C.target);
        }
    }
    return nsw;
}

int32_t orc_well_controls(orc_model* m, const double* u) {
    int32_t nsw = 0;
    for (orc_cwell& C : m->cw) {
        if (C.control == 0 || !C.on_limit) continue;
        if (well_line(*m, C, u).g(C.limit) > C.target) {
            C.on_limit = 0;
            ++nsw;
        }
    }
    return nsw;
}

void orc_well_border(orc_model* m, const double* u, double* R, double* D, double* B, double* Cg) {
    for (size_t w = 0; w < m->cw.size(); ++w) {
        const orc_cwell& C = m->cw[w];
        /* B: how the cell rows move with bhp */
        for (int32_t k = 0; k < C.np; ++k) {
            const orc_perf& W = m->perfs[C.p0 + k];
            double ui[8];
            for (int v = 0; v < 8; ++v) ui[v] = u[(size_t)v * m->n + W.cell];
            Props<double> P;
            props(m->fl, m->poro[W.cell], ui, P);
            PerfFlow<double> fl = perf_flow(W, C, P, ui[0]);
            double* b = B + (size_t)(C.c0 + k) * 8;
            for (int e = 0; e < 8; ++e) b[e] = 0.0;
            if (!fl.active) continue;
            for (int e = 0; e < 7; ++e) {
                if (C.kind == 3) {
                    for (int a = 0; a < 3; ++a) b[e] -= fl.dQ[a] * P.xi[a][e];
                } else {
                    b[e] = -fl.dQi * (e == 6 ? C.Hinj : C.z[e]);
                }
            }
        }
        double* cg = Cg + (size_t)C.c0 * 8;
        if (C.control == 0 || C.on_limit) {
            R[w] = C.bhp - (C.control == 0 ? C.target : C.limit);
            D[w] = 1.0;
            std::fill(cg, cg + (size_t)C.np * 8, 0.0);
        } else {
            double dq;
            R[w] = controlled_rate(*m, C, u, cg, &dq) - C.target;
            D[w] = dq;
        }
    }
}

double orc_well_scaled_norm(orc_model* m, const double* R, double dt) {
    const double V = cell_volume(*m);
    double mx = 0.0;
    for (size_t w = 0; w < m->cw.size(); ++w) {
        const orc_cwell& C = m->cw[w];
        double s;
        if (C.control == 0 || C.on_limit)
            s = std::max(std::fabs(C.control == 0 ? C.target : C.limit), 1.0);
        else
            s = V * m->poro[m->perfs[C.p0].cell] * m->fl.rho_ref[0] / dt;
        double v = std::fabs(R[w]) / s;
        if (!(v <= mx)) mx = v;
    }
    return mx;
}

}  // extern "C"
