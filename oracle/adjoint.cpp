/* CPU oracle: discrete adjoint of the implicit time stepping.
 *
 * TEST INFRASTRUCTURE ONLY.  Reference for the differentiation form: the
 * gradient of cumulative oil-phase production
 *     J_obj = sum_n dt_n q_oil(u^n),
 *     q_oil(u) = sum over producer perforations of WI lambda_o (p - p_wf)^+
 * with respect to m = (ln k per cell, frequency factors A_R), where u^n solves
 * R^n(u^n, u^{n-1}, m) = 0 (the residual of Section 3.1).  With
 * L = J_obj - sum_n lam^n . R^n:
 *   (dR^n/du^n)^T lam^n = (dj^n/du^n)^T - (dR^{n+1}/du^n)^T lam^{n+1},
 *   dR^{n+1}/du^n = -(V/dt_{n+1}) dA/du(u^n)   (block diagonal),
 *   dJ/dm = sum_n dj^n/dm - lam^n . dR^n/dm.
 * The transposed system is built explicitly and solved by decoupling plus a
 * tight GMRES solve.
 */
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "dual.h"
#include "model.h"

/* property evaluation lives in physics.cpp; declare the pieces used here */
namespace orc {
using D8 = Dual<8>;
void props_acc_grad(const orc_model& m, int32_t i, const double* u_i, double* acc_jac /*64*/,
                    double* qoil /*value*/, double* qoil_grad /*8*/, double* mob_o_val);
double cell_oil_rate(const orc_model& m, int32_t i, const double* u_i);
void face_conv_flux(const orc_model& m, const double* u, int32_t lo, int32_t hi, int dir, double* flow /*8*/);
void cell_rates(const orc_model& m, int32_t i, const double* u_i, double* rates /*4*/);
void well_terms(const orc_model& m, int32_t i, const double* u_i, double* W /*8*/);
}  // namespace orc

using namespace orc;

extern "C" {

double orc_oil_rate(orc_model* m, const double* u) {
    double q = 0.0;
    for (const orc_perf& P : m->perfs) {
        if (P.kind != 1) continue;
        double ui[8];
        for (int v = 0; v < 8; ++v) ui[v] = u[(size_t)v * m->n + P.cell];
        q += cell_oil_rate(*m, P.cell, ui);
    }
    return q;
}

int orc_adjoint_step(orc_model* m, const double* u_n, const double* u_nm1, double dt_n, const double* lam_np1,
                     const double* /*u_np1_unused*/, double dt_np1, double* lam_n, double* g_logk, double* g_A) {
    if (!m->cw.empty()) return -2;   /* the well rows of bhp unknowns are not in this adjoint */
    const int32_t n = m->n;
    const size_t N8 = (size_t)n * 8;
    const double V = cell_volume(*m);
    const int32_t nnzb = m->row_ptr[n];
    std::vector<double> F(N8), J((size_t)nnzb * 64), JT((size_t)nnzb * 64), rhs(N8, 0.0), lam(N8, 0.0);
    orc_assemble(m, u_n, u_nm1, dt_n, F.data(), J.data());

    /* right-hand side: dt_n dq/du + (V/dt_{n+1}) (dA/du)^T lam^{n+1} */
    std::vector<double> qcell(n, 0.0);
    for (int32_t i = 0; i < n; ++i) {
        double ui[8], aj[64], q, qg[8], mo;
        for (int v = 0; v < 8; ++v) ui[v] = u_n[(size_t)v * n + i];
        props_acc_grad(*m, i, ui, aj, &q, qg, &mo);
        qcell[i] = q;
        for (int v = 0; v < 8; ++v) {
            double s = dt_n * qg[v];
            if (lam_np1)
                for (int e = 0; e < 8; ++e) s += (V / dt_np1) * aj[e * 8 + v] * lam_np1[(size_t)i * 8 + e];
            rhs[(size_t)i * 8 + v] = s;
        }
    }
    /* J^T in the same (symmetric) pattern: block (j, i) = J_ij^T */
    for (int32_t i = 0; i < n; ++i)
        for (int32_t b = m->row_ptr[i]; b < m->row_ptr[i + 1]; ++b) {
            int32_t j = m->col_idx[b];
            int32_t bt = block_of(*m, j, i);
            for (int r = 0; r < 8; ++r)
                for (int c = 0; c < 8; ++c) JT[(size_t)bt * 64 + c * 8 + r] = J[(size_t)b * 64 + r * 8 + c];
        }
    int32_t bad;
    int st = orc_decouple(m, JT.data(), rhs.data(), &bad);
    if (st) return st;
    orc_solve_info info;
    st = orc_gmres(m, JT.data(), rhs.data(), lam.data(), 30, 400, 1e-13, &info);
    if (st) return st;
    std::memcpy(lam_n, lam.data(), sizeof(double) * N8);

    /* gradient: dj/dlnk - lam . dR/dlnk, faces (harmonic transmissibility) */
    const orc_grid& g = m->g;
    for (int32_t lo = 0; lo < n; ++lo) {
        int32_t ix = lo % g.nx, iy = (lo / g.nx) % g.ny, iz = lo / (g.nx * g.ny);
        int32_t nb[3] = {ix + 1 < g.nx ? lo + 1 : -1, iy + 1 < g.ny ? lo + g.nx : -1,
                         iz + 1 < g.nz ? lo + g.nx * g.ny : -1};
        for (int d = 0; d < 3; ++d) {
            int32_t hi = nb[d];
            if (hi < 0) continue;
            double fc[8];
            face_conv_flux(*m, u_n, lo, hi, d, fc);
            double s = 0.0;
            for (int e = 0; e < 8; ++e) s += (lam[(size_t)lo * 8 + e] - lam[(size_t)hi * 8 + e]) * fc[e];
            double klo = d == 2 ? m->kz[lo] : m->kh[lo], khi = d == 2 ? m->kz[hi] : m->kh[hi];
            /* dT/dlnk_lo = T k_hi/(k_lo + k_hi) (A/h equal on both sides) */
            g_logk[lo] -= s * khi / (klo + khi);
            g_logk[hi] -= s * klo / (klo + khi);
        }
    }
    /* wells */
    std::vector<double> inj_s(m->perfs.size(), 0.0);
    for (size_t p = 0; p < m->perfs.size(); ++p) {
        const orc_perf& P = m->perfs[p];
        const int32_t i = P.cell;
        if (P.kind == 1) {
            double ui[8], W[8];
            for (int v = 0; v < 8; ++v) ui[v] = u_n[(size_t)v * n + i];
            well_terms(*m, i, ui, W);      /* amounts subtracted from R_i, proportional to WI */
            double s = 0.0;
            for (int e = 0; e < 8; ++e) s += lam[(size_t)i * 8 + e] * W[e];
            g_logk[i] += s + dt_n * qcell[i];
        } else {
            double s = 0.0;
            for (int c = 0; c < 6; ++c) s += lam[(size_t)i * 8 + c] * P.q[c];
            s += lam[(size_t)i * 8 + 6] * P.qE;
            inj_s[p] = s;
        }
    }
    /* injector split q_p = q WI_p / sum WI: d q_p / d lnk_j = q_p (delta_pj - WI_j / sum WI) */
    {
        size_t p0 = 0;
        for (size_t w = 0; w < m->wells_in.size(); ++w) {
            size_t np = m->well_cells[w].size();
            if (m->wells_in[w].kind == 2) {
                double sum_wi = 0.0, sum_s = 0.0;
                for (size_t p = p0; p < p0 + np; ++p) { sum_wi += m->perfs[p].wi; sum_s += inj_s[p]; }
                for (size_t p = p0; p < p0 + np; ++p)
                    g_logk[m->perfs[p].cell] += inj_s[p] - m->perfs[p].wi / sum_wi * sum_s;
            }
            p0 += np;
        }
    }
    /* frequency factors: r_R is proportional to A_R */
    for (int32_t i = 0; i < n; ++i) {
        double ui[8], rates[4];
        for (int v = 0; v < 8; ++v) ui[v] = u_n[(size_t)v * n + i];
        cell_rates(*m, i, ui, rates);
        const double* li = lam.data() + (size_t)i * 8;
        static const int rowof[7] = {0, 1, 2, 3, 4, 5, 7};
        for (int r = 0; r < 4; ++r) {
            if (m->fl.Afreq[r] == 0.0) continue;
            double s = m->fl.Hreac[r] * li[6];
            for (int c = 0; c < 7; ++c) s += m->fl.stoich[r][c] * li[rowof[c]];
            g_A[r] += V * rates[r] / m->fl.Afreq[r] * s;
        }
    }
    return 0;
}

}  // extern "C"
