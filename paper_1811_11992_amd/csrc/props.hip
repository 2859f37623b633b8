// Property pass: secondary variables and their derivatives per cell, the
// cell's local residual terms (accumulation change, reactions, wells) and the
// quantities the face fluxes need.  Eight lanes per cell, one derivative each.
//
// Model: Section 2.2 of the paper (K-values with the modified pseudo
// equilibrium ratio, Redlich-Kwong Z-factor, densities, viscosities, porosity
// with coke, Stone II relative permeability, enthalpies, internal energies,
// Arrhenius rates, Peaceman wells).  Readings where the paper is silent or
// garbled: x_HO = 1 - x_LO and y_N2 = 1 - sum of the other gas fractions
// (composition constraints substituted), pseudo K only on water and the
// heaviest oil, RK mixing a = sum y Tc^1.25/sqrt(pc), b = sum y Tc/pc,
// Tcm = (a^2/b)^(2/3), pcm = Tcm/b, zero capillary pressure, phi_f =
// phi - C_c/rho_coke in the fluid and reaction terms, no coke conductivity.
#include <algorithm>

#include "common.h"

namespace isc {

// ---- scalar-or-gradient overloads
__device__ __forceinline__ double vof(double x) { return x; }
__device__ __forceinline__ double vof(G1 x) { return x.v; }
__device__ __forceinline__ double xexp(double x) { return exp(x); }
__device__ __forceinline__ G1 xexp(G1 x) { return gexp(x); }
__device__ __forceinline__ double xpow(double x, double c) { return pow(x, c); }
__device__ __forceinline__ G1 xpow(G1 x, double c) { return gpow(x, c); }
template <class S> __device__ __forceinline__ S mk(double x);
template <> __device__ __forceinline__ double mk<double>(double x) { return x; }
template <> __device__ __forceinline__ G1 mk<G1>(double x) { return gconst(x); }

// Largest real root of Z^3 - Z^2 + c1 Z + c0 = 0 (closed form, then Newton).
__device__ double rk_root(double c1, double c0) {
    // Z = t + 1/3 turns it into t^3 + p t + q = 0
    const double p = c1 - 1.0 / 3.0;
    const double q = c1 / 3.0 + c0 - 2.0 / 27.0;
    const double disc = 0.25 * q * q + p * p * p / 27.0;
    double t;
    if (disc > 0.0) {
        const double s = sqrt(disc);
        t = cbrt(-0.5 * q + s) + cbrt(-0.5 * q - s);
    } else if (p == 0.0) {
        t = 0.0;
    } else {
        const double m = sqrt(-p / 3.0);
        double c = -0.5 * q / (m * m * m);
        c = fmin(1.0, fmax(-1.0, c));
        t = 2.0 * m * cos(acos(c) / 3.0);
    }
    double z = t + 1.0 / 3.0;
#pragma unroll
    for (int it = 0; it < 2; ++it) {
        const double P = ((z - 1.0) * z + c1) * z + c0;
        const double dP = (3.0 * z - 2.0) * z + c1;
        if (dP != 0.0) z -= P / dP;
    }
    return z;
}
__device__ __forceinline__ double zfac(double A, double B) { return rk_root(A - B - B * B, -A * B); }
__device__ __forceinline__ G1 zfac(G1 A, G1 B) {
    const double z = rk_root(A.v - B.v - B.v * B.v, -A.v * B.v);
    // P(Z; A, B) = Z^3 - Z^2 + (A - B - B^2) Z - A B = 0, implicit derivative
    const double Pz = (3.0 * z - 2.0) * z + (A.v - B.v - B.v * B.v);
    const double Pa = z - B.v;
    const double Pb = -(1.0 + 2.0 * B.v) * z - A.v;
    return G1{z, -(Pa * A.d + Pb * B.d) / Pz};
}

// piecewise-linear table with knots at S = k/100; constant outside [0, 1]
template <class S> __device__ __forceinline__ S interp(const double* tab, const S& s) {
    const double x = vof(s) * 100.0;
    if (x < 0.0) return mk<S>(tab[0]);
    if (x >= 100.0) return mk<S>(tab[100]);
    int k = (int)floor(x);
    k = k > 99 ? 99 : k;
    const double lo = tab[k], slope = tab[k + 1] - tab[k];
    return (s * 100.0 - (double)k) * slope + lo;
}

template <class S> __device__ __forceinline__ S pos_part(const S& x) { return vof(x) < 0.0 ? mk<S>(0.0) : x; }

// gas-phase enthalpy of species c relative to T_ref: integral of cp dT
template <class S> __device__ __forceinline__ S hgas(const isc_fluid& f, int c, const S& T) {
    const double Tr = f.T_ref;
    // sum_j cpg_j (T^{j+1} - Tr^{j+1}) / (j+1), Horner in T
    const double c0 = f.cpg[c][0], c1 = f.cpg[c][1] * 0.5, c2 = f.cpg[c][2] / 3.0,
                 c3 = f.cpg[c][3] * 0.25;
    const double href = Tr * (c0 + Tr * (c1 + Tr * (c2 + Tr * c3)));
    return T * (((T * c3 + c2) * T + c1) * T + c0) - href;
}

// heat of vaporisation, zero at and above the critical temperature
template <class S> __device__ __forceinline__ S hvap(const isc_fluid& f, int c, const S& T) {
    if (vof(T) < f.Tc[c]) return f.hvr[c] * xpow(f.Tc[c] - T, f.ev[c]);
    return mk<S>(0.0);
}

template <class S> struct Cell {
    S acc[8];      // accumulation per bulk volume
    S src[8];      // reaction source per bulk volume (rows; energy row: heat)
    S mx[NMOB];    // mobility times carried fraction/enthalpy, by mob_slot
    S gam[3];      // specific weights g rho M
    S KT;          // bulk thermal conductivity
    S rate[4];     // Arrhenius rates r_R per bulk volume
    S mob_w, mob_o, mob_g;   // phase mobilities k_ra rho_a / mu_a
};

// Secondary variables of one cell.  u = (p, x_LO, y_O2, y_CO2, T, S_w, S_g, C_c).
template <class S> __device__ void cell_eval(const isc_fluid& f, double phi_ref, const S* u,
                                             Cell<S>& c) {
    const S& p = u[0]; const S& xlo = u[1]; const S& yo2 = u[2]; const S& yco2 = u[3];
    const S& T = u[4]; const S& sw = u[5]; const S& sg = u[6]; const S& cc = u[7];
    const S so = 1.0 - sw - sg;
    const S xho = 1.0 - xlo;
    const S invT = 1.0 / T;

    // K-values (kv2 = kv3 = 0) and gas composition with the pseudo K of the
    // water and of the heaviest oil component
    S kw = (f.kv1[0] / p) * xexp(f.kv4[0] / (T - f.kv5[0]));
    S klo = (f.kv1[1] / p) * xexp(f.kv4[1] / (T - f.kv5[1]));
    S kho = (f.kv1[2] / p) * xexp(f.kv4[2] / (T - f.kv5[2]));
    S y[6];
    y[0] = (sw / (sw + f.eps)) * kw;
    y[1] = klo * xlo;
    y[2] = (so / (so + f.eps)) * kho * xho;
    y[3] = yo2;
    y[4] = yco2;
    y[5] = 1.0 - (y[0] + y[1] + y[2] + y[3] + y[4]);

    // Redlich-Kwong compressibility with pseudo-critical mixing
    S am = mk<S>(0.0), bm = mk<S>(0.0);
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        am = am + (pow(f.Tc[k], 1.25) / sqrt(f.pc[k])) * y[k];
        bm = bm + (f.Tc[k] / f.pc[k]) * y[k];
    }
    const S tcm = xpow(am * am / bm, 2.0 / 3.0);
    const S pr = p * bm / tcm;              // p / pcm
    const S tr = tcm * invT;                // Tcm / T
    const S Arr = 0.42748 * pr * xpow(tr, 2.5);
    const S Brr = 0.08664 * pr * tr;
    const S Z = zfac(Arr, Brr);

    // molar densities
    S rho[3];
    rho[2] = p / (f.Rgas * Z * T);
    S rl[3];
#pragma unroll
    for (int k = 0; k < 3; ++k)
        rl[k] = f.rho_ref[k] * xexp(f.cp_liq[k] * (p - f.p_ref) - f.ct1_liq[k] * (T - f.T_ref));
    rho[0] = rl[0];
    rho[1] = 1.0 / (xlo / rl[1] + xho / rl[2]);

    // viscosities: liquid exponential, oil log-mixing, gas sqrt(M) mixing
    S mu[3];
    mu[0] = f.avisc[0] * xexp(f.bvisc[0] * invT);
    mu[1] = xexp(xlo * (log(f.avisc[1]) + f.bvisc[1] * invT) + xho * (log(f.avisc[2]) + f.bvisc[2] * invT));
    {
        S num = mk<S>(0.0), den = mk<S>(0.0);
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const double sm = sqrt(f.M[k]);
            num = num + (sm * f.avg[k]) * (xpow(T, f.bvg[k]) * y[k]);
            den = den + sm * y[k];
        }
        mu[2] = num / den;
    }

    // porosity and the part left to fluids by coke
    const S phi = phi_ref + (phi_ref * f.cpor) * (p - f.p_ref);
    const S phif = phi - cc / f.rho_coke;

    // relative permeabilities (SWT by S_w, SLT by S_g) and Stone II
    const S krw = interp(f.krw, sw), krow = interp(f.krow, sw);
    const S krg = interp(f.krg, sg), krog = interp(f.krog, sg);
    const S kro = pos_part(f.krocw * ((krow / f.krocw + krw) * (krog / f.krocw + krg) - krw - krg));

    // enthalpies
    S hg[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) hg[k] = hgas(f, k, T);
    S H[3];
    H[0] = hg[0] - hvap(f, 0, T);
    H[1] = xlo * (hg[1] - hvap(f, 1, T)) + xho * (hg[2] - hvap(f, 2, T));
    H[2] = y[0] * hg[0] + y[1] * hg[1] + y[2] * hg[2] + y[3] * hg[3] + y[4] * hg[4] + y[5] * hg[5];

    // accumulation per bulk volume
    const S nw = phif * rho[0] * sw;            // water-phase moles per bulk volume
    const S no = phif * rho[1] * so;
    const S ng = phif * rho[2] * sg;
    c.acc[0] = nw + ng * y[0];
    c.acc[1] = no * xlo + ng * y[1];
    c.acc[2] = no * xho + ng * y[2];
    c.acc[3] = ng * y[3];
    c.acc[4] = ng * y[4];
    c.acc[5] = ng * y[5];
    // internal energies U = H - p/rho; rock and coke sensible heat
    const S Uw = H[0] - p / rho[0], Uo = H[1] - p / rho[1], Ug = H[2] - p / rho[2];
    c.acc[6] = nw * Uw + no * Uo + ng * Ug + (1.0 - phi) * (f.cp_rock * (T - f.T_ref)) +
               cc * (f.cp_coke * (T - f.T_ref));
    c.acc[7] = cc;

    // Arrhenius rates, concentrations per bulk volume
    S rr[4];
    {
        const S oil = phif * so * rho[1];
        const S po2 = yo2 * p;
        const double ER0 = f.Eact[0] / f.Rgas, ER1 = f.Eact[1] / f.Rgas;
        const double ER2 = f.Eact[2] / f.Rgas, ER3 = f.Eact[3] / f.Rgas;
        rr[0] = (f.Afreq[0] * xexp(-ER0 * invT)) * po2 * oil * xlo;
        rr[1] = (f.Afreq[1] * xexp(-ER1 * invT)) * po2 * oil * xho;
        const S ratio = cc / f.Ccmax;
        const S r2 = ratio * ratio;
        rr[2] = (f.Afreq[2] * xexp(-ER2 * invT)) * oil * xho * pos_part(1.0 - r2 * r2 * ratio);
        rr[3] = (f.Afreq[3] * xexp(-ER3 * invT)) * po2 * cc;
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) c.rate[r] = rr[r];
#pragma unroll
    for (int e = 0; e < 8; ++e) c.src[e] = mk<S>(0.0);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
#pragma unroll
        for (int k = 0; k < 6; ++k)
            if (f.stoich[r][k] != 0.0) c.src[k] = c.src[k] + f.stoich[r][k] * rr[r];
        if (f.stoich[r][6] != 0.0) c.src[7] = c.src[7] + f.stoich[r][6] * rr[r];
        c.src[6] = c.src[6] + f.Hreac[r] * rr[r];
    }

    // bulk conductivity
    c.KT = phif * (f.Kcond[0] * sw + f.Kcond[1] * so + f.Kcond[2] * sg) + (1.0 - phi) * f.Kcond[3];

    // mobilities times carried fraction (component rows) or enthalpy (energy)
    {
        const S mw = krw * rho[0] / mu[0];
        const S mo = kro * rho[1] / mu[1];
        c.mob_w = mw;
        c.mob_o = mo;
        const S mg = krg * rho[2] / mu[2];
        c.mob_g = mg;
        c.mx[mob_slot(0, 0)] = mw;
        c.mx[mob_slot(0, 6)] = mw * H[0];
        c.mx[mob_slot(1, 1)] = mo * xlo;
        c.mx[mob_slot(1, 2)] = mo * xho;
        c.mx[mob_slot(1, 6)] = mo * H[1];
#pragma unroll
        for (int k = 0; k < 6; ++k) c.mx[mob_slot(2, k)] = mg * y[k];
        c.mx[mob_slot(2, 6)] = mg * H[2];
    }
    c.gam[0] = (f.grav * f.M[0]) * rho[0];
    c.gam[1] = f.grav * rho[1] * (f.M[1] * xlo + f.M[2] * xho);
    c.gam[2] = f.grav * rho[2] *
               (f.M[0] * y[0] + f.M[1] * y[1] + f.M[2] * y[2] + f.M[3] * y[3] + f.M[4] * y[4] + f.M[5] * y[5]);
}

// store quantity x of a cell: lane k writes d/du_k, lane 0 also the value
__device__ __forceinline__ void put(double* rec, G1 x, int k) {
    rec[1 + k] = x.d;
    if (k == 0) rec[0] = x.v;
}

// Accumulation at the previous time level (values only), one thread per
// cell: acc_old[i][e].  The property pass reads it instead of evaluating it
// on each of a cell's eight lanes.
__global__ void __launch_bounds__(256) acc_old_kernel(int32_t n, const double* __restrict__ u_old,
                                                      const double* __restrict__ poro,
                                                      const isc_fluid* __restrict__ fl,
                                                      double* __restrict__ acc_old) {
    const int32_t i = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i >= n) return;
    double uo[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) uo[q] = u_old[(size_t)q * n + i];
    Cell<double> co;
    cell_eval<double>(*fl, poro[i], uo, co);
#pragma unroll
    for (int e = 0; e < 8; ++e) acc_old[(size_t)i * 8 + e] = co.acc[e];
}

// Eight lanes per cell (lane k of a cell carries d/du_k): local residual terms
// with their derivatives and the flux payload.  vol_dt = V/dt, vol = V.
__global__ void __launch_bounds__(256, 2) props_kernel(
    int32_t n, const double* __restrict__ u, const double* __restrict__ acc_old_in, double vol_dt,
    double vol, const double* __restrict__ poro, const int32_t* __restrict__ well_slot,
    const double* __restrict__ perf, const isc_fluid* __restrict__ fl, double* __restrict__ payload,
    int32_t heater_cell, double heater_W, const CWell* __restrict__ cw) {
    const int32_t i = (int32_t)((blockIdx.x * blockDim.x + threadIdx.x) >> 3);
    const int k = threadIdx.x & 7;
    if (i >= n) return;
    const isc_fluid& f = *fl;
    const double phi_ref = poro[i];
    double* out = payload + (size_t)i * PL;

    double acc_old[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) acc_old[e] = acc_old_in[(size_t)i * 8 + e];

    G1 ug[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) ug[q] = G1{u[(size_t)q * n + i], q == k ? 1.0 : 0.0};
    Cell<G1> c;
    cell_eval<G1>(f, phi_ref, ug, c);

    // local rows: V/dt (A - A_old) - V q_reac
    G1 loc[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) loc[e] = vol_dt * (c.acc[e] - acc_old[e]) - vol * c.src[e];

    // wells: producer inflow (Peaceman, no backflow) at a fixed BHP or at the
    // well's bhp unknown, fixed injection, or injection at the well's bhp
    // with the cell's total mobility
    const int32_t ws = well_slot[i];
    if (ws >= 0) {
        const double* pf = perf + (size_t)ws * PERF_W;
        if (pf[0] == 4.0) {
            const double wi = pf[1], bhp = cw[(int)pf[2]].bhp;
            if (bhp > ug[0].v) {
                const G1 Q = (wi * ((c.mob_w + c.mob_o) + c.mob_g)) * (bhp - ug[0]);   // > 0: injection
#pragma unroll
                for (int q = 0; q < 6; ++q) loc[q] = loc[q] - Q * pf[3 + q];
                loc[6] = loc[6] - Q * pf[10];
            }
        } else if (pf[0] != 2.0) {
            const double wi = pf[1], bhp = pf[0] == 1.0 ? pf[2] : cw[(int)pf[2]].bhp;
            if (ug[0].v > bhp) {
                const G1 dp = wi * (bhp - ug[0]);   // < 0: production
#pragma unroll
                for (int a = 0; a < 3; ++a)
#pragma unroll
                    for (int e = 0; e < 7; ++e)
                        if (mob_slot(a, e) >= 0) loc[e] = loc[e] - dp * c.mx[mob_slot(a, e)];
            }
        } else {
#pragma unroll
            for (int q = 0; q < 6; ++q) loc[q].v -= pf[3 + q];
            loc[6].v -= pf[10];
        }
    }
    // heater: a fixed heat rate into one cell's energy balance
    if (i == heater_cell) loc[6].v -= heater_W;
#pragma unroll
    for (int e = 0; e < 8; ++e) put(out + PL_LOCAL + 9 * e, loc[e], k);
#pragma unroll
    for (int s = 0; s < NMOB; ++s) put(out + PL_MOB + 9 * s, c.mx[s], k);
#pragma unroll
    for (int a = 0; a < 3; ++a) put(out + PL_GAM + 9 * a, c.gam[a], k);
    put(out + PL_KT, c.KT, k);
}

// Adjoint inputs at state u, eight lanes per cell (lane k carries d/du_k):
// accJ[i][e][k] = dA_e/du_k (accumulation per bulk volume), the producer's
// oil-phase molar rate q = WI lambda_o (p - p_wf) for p > p_wf with dq/du_k,
// and the reaction rates.
__global__ void __launch_bounds__(256) accgrad_kernel(
    int32_t n, const double* __restrict__ u, const double* __restrict__ poro, const int32_t* __restrict__ well_slot,
    const double* __restrict__ perf, const isc_fluid* __restrict__ fl, double* __restrict__ accJ,
    double* __restrict__ qg, double* __restrict__ qv, double* __restrict__ rates) {
    const int32_t i = (int32_t)((blockIdx.x * blockDim.x + threadIdx.x) >> 3);
    const int k = threadIdx.x & 7;
    if (i >= n) return;
    G1 ug[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) ug[q] = G1{u[(size_t)q * n + i], q == k ? 1.0 : 0.0};
    Cell<G1> c;
    cell_eval<G1>(*fl, poro[i], ug, c);
#pragma unroll
    for (int e = 0; e < 8; ++e) accJ[(size_t)i * 64 + e * 8 + k] = c.acc[e].d;
    G1 q = G1{0.0, 0.0};
    const int32_t ws = well_slot[i];
    if (ws >= 0) {
        const double* pf = perf + (size_t)ws * PERF_W;
        if (pf[0] == 1.0 && ug[0].v > pf[2]) q = (pf[1] * c.mob_o) * (ug[0] - pf[2]);
    }
    qg[(size_t)i * 8 + k] = q.d;
    if (k == 0) {
        qv[i] = q.v;
#pragma unroll
        for (int r = 0; r < 4; ++r) rates[(size_t)i * 4 + r] = c.rate[r].v;
    }
}

// ---- controlled wells

// the mobility a controlled well's rate is taken over: the phases of a
// producer's mask, the total at an injector
__device__ __forceinline__ double well_mobility(const CWell& W, const Cell<double>& c) {
    if (W.kind == ISC_WELL_INJECTOR) return (c.mob_w + c.mob_o) + c.mob_g;
    double lam = 0.0;
    if (W.control & ISC_CTRL_WATER) lam += c.mob_w;
    if (W.control & ISC_CTRL_OIL) lam += c.mob_o;
    if (W.control & ISC_CTRL_GAS) lam += c.mob_g;
    return lam;
}

// One wavefront per controlled well.  With the cells fixed at u, the rate a
// rate-controlled well holds is piecewise linear and monotone in its bhp b:
//   g(b) = sum_k a_k (p_k - b)^+   (producer, a_k = WI lambda of its phases)
//   g(b) = sum_k a_k (b - p_k)^+   (injector, a_k = WI lambda_t),
// evaluated here in the producer's form over s b, s = +1 / -1.
// mode 0, before a Newton iteration: a well on its rate moves to its limit if
// g(limit) < target, else b becomes the root of g(b) = target (the first
// breakpoint beyond the limit with g <= target closes the linear piece that
// holds it).  mode 1, at a time step's start: a well held at its limit
// returns to its rate if g(limit) > target.  a and p are staged in LDS.
__global__ void __launch_bounds__(64) well_line_kernel(int mode, const int32_t* __restrict__ pcell,
                                                      const double* __restrict__ u, int32_t n,
                                                      const double* __restrict__ poro,
                                                      const int32_t* __restrict__ well_slot,
                                                      const double* __restrict__ perf,
                                                      const isc_fluid* __restrict__ fl, CWell* cw,
                                                      int32_t* nswitch) {
    extern __shared__ double sh[];
    CWell& W = cw[blockIdx.x];
    if (W.control == ISC_CTRL_BHP) return;
    if ((mode == 0) == (W.on_limit != 0)) return;
    const int np = W.np;
    const double s = W.kind == ISC_WELL_INJECTOR ? -1.0 : 1.0;
    double* a = sh;
    double* sp = sh + np;   // s p_k
    for (int k = threadIdx.x; k < np; k += 64) {
        const int32_t i = pcell[W.c0 + k];
        double ui[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) ui[q] = u[(size_t)q * n + i];
        Cell<double> c;
        cell_eval<double>(*fl, poro[i], ui, c);
        a[k] = perf[(size_t)well_slot[i] * PERF_W + 1] * well_mobility(W, c);
        sp[k] = s * ui[0];
    }
    __syncthreads();
    auto g = [&](double x) {   // g at s b = x, summed in perforation order
        double t = 0.0;
        for (int k = 0; k < np; ++k) {
            const double d = sp[k] - x;
            if (d > 0.0) t += a[k] * d;
        }
        return t;
    };
    const double slim = s * W.limit, c = W.target;
    if (mode == 1) {
        if (threadIdx.x == 0 && g(slim) > c) {
            W.on_limit = 0;
            atomicAdd(nswitch, 1);
        }
        return;
    }
    const double glim = g(slim);   // every lane, same value
    if (glim < c) {
        if (threadIdx.x == 0) {
            W.on_limit = 1;
            W.bhp = W.limit;
            atomicAdd(nswitch, 1);
        }
        return;
    }
    // hi: the smallest breakpoint beyond the limit with g <= target
    double hi = INFINITY;
    for (int j = threadIdx.x; j < np; j += 64)
        if (sp[j] > slim && sp[j] < hi && g(sp[j]) <= c) hi = sp[j];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) hi = fmin(hi, __shfl_xor(hi, off, 64));
    if (threadIdx.x != 0) return;
    if (hi == INFINITY) {   // no perforation beyond the limit: g(limit) = 0 = target
        W.bhp = W.limit;
        return;
    }
    double lo = slim, sa = 0.0, sap = 0.0;
    for (int k = 0; k < np; ++k) {
        if (sp[k] < hi && sp[k] > lo) lo = sp[k];
        if (sp[k] >= hi) {
            sa += a[k];
            sap += a[k] * sp[k];
        }
    }
    double b = sa > 0.0 ? (sap - c) / sa : lo;
    b = fmin(fmax(b, lo), hi);
    W.bhp = s * b;
}

// Eight lanes per controlled perforation (lane k carries d/du_k): the
// perforation's entries of Newton's bordered system at the well's bhp --
// B = dF_cell/dbhp, C = dq/du_cell with q the rate it adds to its well's
// equation, dq/dbhp.
__global__ void __launch_bounds__(256) well_rows_kernel(
    int32_t ncp, const int32_t* __restrict__ pcell, const int32_t* __restrict__ pwell, const double* __restrict__ u,
    int32_t n, const double* __restrict__ poro, const int32_t* __restrict__ well_slot,
    const double* __restrict__ perf, const isc_fluid* __restrict__ fl, const CWell* __restrict__ cw,
    double* __restrict__ cwp) {
    const int32_t p = (int32_t)((blockIdx.x * blockDim.x + threadIdx.x) >> 3);
    const int k = threadIdx.x & 7;
    if (p >= ncp) return;
    double Bk = 0.0;
    const int32_t i = pcell[p];
    const double* pf = perf + (size_t)well_slot[i] * PERF_W;
    const CWell& W = cw[pwell[p]];
    G1 ug[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) ug[q] = G1{u[(size_t)q * n + i], q == k ? 1.0 : 0.0};
    Cell<G1> c;
    cell_eval<G1>(*fl, poro[i], ug, c);
    const double wi = pf[1];
    G1 q = G1{0.0, 0.0};
    double dq = 0.0;
    if (W.kind == ISC_WELL_PRODUCER) {
        if (ug[0].v > W.bhp) {
            const G1 dp = W.bhp - ug[0];
            if (W.control & ISC_CTRL_WATER) { q = q - (wi * c.mob_w) * dp; dq -= wi * c.mob_w.v; }
            if (W.control & ISC_CTRL_OIL) { q = q - (wi * c.mob_o) * dp; dq -= wi * c.mob_o.v; }
            if (W.control & ISC_CTRL_GAS) { q = q - (wi * c.mob_g) * dp; dq -= wi * c.mob_g.v; }
            if (k < 7) {
                double t = 0.0;
#pragma unroll
                for (int a = 0; a < 3; ++a)
                    if (mob_slot(a, k) >= 0) t += c.mx[mob_slot(a, k)].v;
                Bk = -wi * t;
            }
        }
    } else if (W.bhp > ug[0].v) {
        const G1 lt = (c.mob_w + c.mob_o) + c.mob_g;
        q = (wi * lt) * (W.bhp - ug[0]);
        dq = wi * lt.v;
        Bk = k < 6 ? -dq * pf[3 + k] : k == 6 ? -dq * pf[10] : 0.0;
    }
    double* o = cwp + (size_t)p * CWP_W;
    o[CWP_B + k] = Bk;
    o[CWP_C + k] = (W.control == ISC_CTRL_BHP || W.on_limit) ? 0.0 : q.d;   // a held row is bhp - c
    if (k == 0) {
        o[CWP_Q] = q.v;
        o[CWP_DQ] = dq;
    }
}

}  // namespace isc

hipError_t isc_launch_accgrad(isc_ctx* ctx, const double* u) {
    const int blocks = (int)(((int64_t)ctx->n * 8 + 255) / 256);
    hipLaunchKernelGGL(isc::accgrad_kernel, dim3(blocks), dim3(256), 0, ctx->stream, ctx->n, u, ctx->poro,
                       ctx->well_slot, ctx->perf, ctx->fluid_d, ctx->accJ, ctx->qg, ctx->qv, ctx->rates);
    return hipGetLastError();
}

hipError_t isc_launch_props(isc_ctx* ctx, const double* u, const double* u_old, double dt) {
    const double vol = ctx->g.dx * ctx->g.dy * ctx->g.dz;
    hipLaunchKernelGGL(isc::acc_old_kernel, dim3((ctx->n + 255) / 256), dim3(256), 0, ctx->stream, ctx->n, u_old,
                       ctx->poro, ctx->fluid_d, ctx->acc_old);
    const int threads = 256;                      // 32 cells x 8 lanes
    const int blocks = (int)(((int64_t)ctx->n * 8 + threads - 1) / threads);
    hipLaunchKernelGGL(isc::props_kernel, dim3(blocks), dim3(threads), 0, ctx->stream, ctx->n, u,
                       ctx->acc_old, vol / dt, vol, ctx->poro, ctx->well_slot, ctx->perf, ctx->fluid_d,
                       ctx->payload, ctx->heater_cell, ctx->heater_W, ctx->cw);
    return hipGetLastError();
}

// Controlled wells: the well line (bhp from its rate equation at fixed
// cells) and the well rows of Newton's bordered system.
hipError_t isc_launch_well_line(isc_ctx* ctx, const double* u, int mode) {
    if (ctx->ncw == 0) return hipSuccess;
    hipLaunchKernelGGL(isc::well_line_kernel, dim3(ctx->ncw), dim3(64), (size_t)2 * ctx->cw_maxnp * sizeof(double),
                       ctx->stream, mode, ctx->cwp_cell, u, ctx->n, ctx->poro, ctx->well_slot, ctx->perf,
                       ctx->fluid_d, ctx->cw, ctx->wsw);
    return hipGetLastError();
}

hipError_t isc_launch_well_rows(isc_ctx* ctx, const double* u) {
    if (ctx->ncp == 0) return hipSuccess;
    const int blocks = (int)(((int64_t)ctx->ncp * 8 + 255) / 256);
    hipLaunchKernelGGL(isc::well_rows_kernel, dim3(blocks), dim3(256), 0, ctx->stream, ctx->ncp, ctx->cwp_cell,
                       ctx->cwp_well, u, ctx->n, ctx->poro, ctx->well_slot, ctx->perf, ctx->fluid_d, ctx->cw,
                       ctx->cwp);
    return hipGetLastError();
}
