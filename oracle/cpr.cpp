/* CPU oracle: the two-stage CPR preconditioner and the flexible GMRES it
 * drives.
 *
 * TEST INFRASTRUCTURE ONLY.  Plain serial FP64, written from the method's
 * definition; it shares nothing with the GPU library.
 *
 * CPR (constrained pressure residual, the CPR-PF preconditioner of the
 * paper's Section 4.3, Example 2), applied to the decoupled system A = C_L J
 * whose diagonal blocks are the identity:
 *   stage 1  the pressure equation: the scalar matrix A_p with entries
 *            (A_ij)[0][0] (pressure row, pressure column of every block),
 *            solved approximately for the pressure part of the residual,
 *            e_p ~= A_p^-1 (E^T r), where E^T takes component 0 of each cell;
 *   stage 2  z = E e_p + M^-1 (r - A E e_p), M the block ILU(0) of A.
 * The pressure solve is p_iters steps of right-preconditioned GMRES (from 0,
 * no restart) whose preconditioner is one V-cycle of an aggregation
 * multigrid; p_iters = 0 means the V-cycle alone.
 *
 * Multigrid: level l + 1 aggregates the cells of level l in 2 x 2 x 2 boxes
 * of the structured grid (ragged at odd sizes); P_l is the piecewise-constant
 * prolongation (P_l)_{iI} = 1 if cell i lies in aggregate I, and the coarse
 * matrix is the Galerkin product A_{l+1} = P_l^T A_l P_l.  Coarsening stops at
 * no more than ORC_CPR_COARSEST cells (or one cell), where the system is
 * solved directly.  Smoothing is red-black Gauss-Seidel, colour (ix+iy+iz)
 * mod 2 on each level's grid: nu sweeps before (red, then black) and nu after
 * (black, then red) the coarse correction, which is scaled by cf.
 */
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <vector>

#include "model.h"

using namespace orc;

namespace {

struct Level {
    int32_t nx, ny, nz, n;
    std::vector<int32_t> rp, ci;     /* CSR, columns ascending */
    std::vector<double> val;
    std::vector<int32_t> agg;        /* aggregate of each cell on the next level */
};

double dotv(const std::vector<double>& a, const std::vector<double>& b) {
    double s = 0.0;
    for (size_t i = 0; i < a.size(); ++i) s += a[i] * b[i];
    return s;
}

void csr_mv(const Level& L, const std::vector<double>& x, std::vector<double>& y) {
    for (int32_t i = 0; i < L.n; ++i) {
        double s = 0.0;
        for (int32_t k = L.rp[i]; k < L.rp[i + 1]; ++k) s += L.val[k] * x[L.ci[k]];
        y[i] = s;
    }
}

}  // namespace

struct orc_cpr {
    orc_model* m;
    int32_t p_iters, nu;
    double cf;
    std::vector<double> A;            /* copy of the decoupled matrix */
    std::vector<double> LU, Dinv;     /* its block ILU(0) */
    std::vector<Level> lv;
    std::vector<double> clu;          /* dense LU of the coarsest level, row-major */
    std::vector<int32_t> cpiv;
};

namespace {

/* Dense LU with partial pivoting of the coarsest level (in place). */
bool coarse_factor(orc_cpr& c) {
    const Level& L = c.lv.back();
    const int32_t n = L.n;
    c.clu.assign((size_t)n * n, 0.0);
    c.cpiv.assign(n, 0);
    for (int32_t i = 0; i < n; ++i)
        for (int32_t k = L.rp[i]; k < L.rp[i + 1]; ++k) c.clu[(size_t)i * n + L.ci[k]] = L.val[k];
    double* a = c.clu.data();
    for (int32_t k = 0; k < n; ++k) {
        int32_t p = k;
        for (int32_t r = k + 1; r < n; ++r)
            if (std::fabs(a[(size_t)r * n + k]) > std::fabs(a[(size_t)p * n + k])) p = r;
        c.cpiv[k] = p;
        if (!(std::fabs(a[(size_t)p * n + k]) > 0.0)) return false;
        if (p != k)
            for (int32_t j = 0; j < n; ++j) std::swap(a[(size_t)k * n + j], a[(size_t)p * n + j]);
        for (int32_t r = k + 1; r < n; ++r) {
            const double f = a[(size_t)r * n + k] / a[(size_t)k * n + k];
            a[(size_t)r * n + k] = f;
            for (int32_t j = k + 1; j < n; ++j) a[(size_t)r * n + j] -= f * a[(size_t)k * n + j];
        }
    }
    return true;
}

void coarse_solve(const orc_cpr& c, const std::vector<double>& b, std::vector<double>& x) {
    const int32_t n = c.lv.back().n;
    const double* a = c.clu.data();
    x = b;
    for (int32_t k = 0; k < n; ++k) std::swap(x[k], x[c.cpiv[k]]);
    for (int32_t i = 0; i < n; ++i)
        for (int32_t k = 0; k < i; ++k) x[i] -= a[(size_t)i * n + k] * x[k];
    for (int32_t i = n - 1; i >= 0; --i) {
        for (int32_t k = i + 1; k < n; ++k) x[i] -= a[(size_t)i * n + k] * x[k];
        x[i] /= a[(size_t)i * n + i];
    }
}

/* one red-black Gauss-Seidel sweep: cells of colour first, then the other;
 * each cell takes x_i = (b_i - sum_{j != i} a_ij x_j) / a_ii */
void rbgs(const Level& L, const std::vector<double>& b, std::vector<double>& x, int first) {
    for (int pass = 0; pass < 2; ++pass) {
        const int colour = pass == 0 ? first : 1 - first;
        for (int32_t i = 0; i < L.n; ++i) {
            const int32_t ix = i % L.nx, iy = (i / L.nx) % L.ny, iz = i / (L.nx * L.ny);
            if ((ix + iy + iz) % 2 != colour) continue;
            double s = b[i], d = 0.0;
            for (int32_t k = L.rp[i]; k < L.rp[i + 1]; ++k) {
                if (L.ci[k] == i) d = L.val[k];
                else s -= L.val[k] * x[L.ci[k]];
            }
            x[i] = s / d;
        }
    }
}

/* x = V-cycle on level l applied to b, from x = 0 */
void vcycle(const orc_cpr& c, size_t l, const std::vector<double>& b, std::vector<double>& x) {
    const Level& L = c.lv[l];
    if (l + 1 == c.lv.size()) {
        coarse_solve(c, b, x);
        return;
    }
    x.assign(L.n, 0.0);
    for (int s = 0; s < c.nu; ++s) rbgs(L, b, x, 0);
    std::vector<double> r(L.n);
    csr_mv(L, x, r);
    for (int32_t i = 0; i < L.n; ++i) r[i] = b[i] - r[i];
    const Level& C = c.lv[l + 1];
    std::vector<double> bc(C.n, 0.0), xc;
    for (int32_t i = 0; i < L.n; ++i) bc[L.agg[i]] += r[i];   /* P^T r */
    vcycle(c, l + 1, bc, xc);
    for (int32_t i = 0; i < L.n; ++i) x[i] += c.cf * xc[L.agg[i]];   /* x += cf P x_c */
    for (int s = 0; s < c.nu; ++s) rbgs(L, b, x, 1);
}

/* p_iters steps of GMRES (modified Gram-Schmidt, Givens rotations) on
 * A_p e = rp, right-preconditioned by the V-cycle, from e = 0 */
void pressure_solve(const orc_cpr& c, const std::vector<double>& rp, std::vector<double>& e) {
    const Level& L = c.lv[0];
    const int32_t n = L.n;
    if (c.p_iters == 0) {
        vcycle(c, 0, rp, e);
        return;
    }
    const int k = c.p_iters;
    e.assign(n, 0.0);
    const double beta = std::sqrt(dotv(rp, rp));
    if (beta == 0.0) return;
    std::vector<std::vector<double>> V(k + 1, std::vector<double>(n)), Z(k);
    std::vector<double> H((size_t)(k + 1) * k, 0.0), cs(k), sn(k), g(k + 1, 0.0), w(n);
    for (int32_t i = 0; i < n; ++i) V[0][i] = rp[i] / beta;
    g[0] = beta;
    int done = 0;
    for (int j = 0; j < k; ++j) {
        vcycle(c, 0, V[j], Z[j]);
        csr_mv(L, Z[j], w);
        for (int i = 0; i <= j; ++i) {
            const double h = dotv(w, V[i]);
            H[(size_t)i * k + j] = h;
            for (int32_t t = 0; t < n; ++t) w[t] -= h * V[i][t];
        }
        const double hn = std::sqrt(dotv(w, w));
        H[(size_t)(j + 1) * k + j] = hn;
        if (hn > 0.0)
            for (int32_t t = 0; t < n; ++t) V[j + 1][t] = w[t] / hn;
        for (int i = 0; i < j; ++i) {
            const double a = H[(size_t)i * k + j], b2 = H[(size_t)(i + 1) * k + j];
            H[(size_t)i * k + j] = cs[i] * a + sn[i] * b2;
            H[(size_t)(i + 1) * k + j] = -sn[i] * a + cs[i] * b2;
        }
        const double a = H[(size_t)j * k + j], b2 = H[(size_t)(j + 1) * k + j];
        const double den = std::hypot(a, b2);
        cs[j] = a / den;
        sn[j] = b2 / den;
        H[(size_t)j * k + j] = den;
        g[j + 1] = -sn[j] * g[j];
        g[j] = cs[j] * g[j];
        done = j + 1;
        if (hn == 0.0) break;
    }
    std::vector<double> y(done);
    for (int i = done - 1; i >= 0; --i) {
        double s = g[i];
        for (int t = i + 1; t < done; ++t) s -= H[(size_t)i * k + t] * y[t];
        y[i] = s / H[(size_t)i * k + i];
    }
    for (int i = 0; i < done; ++i)
        for (int32_t t = 0; t < n; ++t) e[t] += y[i] * Z[i][t];
}

}  // namespace

extern "C" {

/* Builds the CPR preconditioner of the decoupled matrix Jdec: the pressure
 * matrix, the multigrid hierarchy and the block ILU(0).  NULL if a factor is
 * singular. */
orc_cpr* orc_cpr_create(orc_model* m, const double* Jdec, int32_t p_iters, int32_t nu, double cf) {
    orc_cpr* c = new orc_cpr();
    c->m = m;
    c->p_iters = p_iters;
    c->nu = nu;
    c->cf = cf;
    const int32_t n = m->n;
    const size_t nnzb = (size_t)m->row_ptr[n];
    c->A.assign(Jdec, Jdec + nnzb * 64);
    c->LU.resize(nnzb * 64);
    c->Dinv.resize((size_t)n * 64);
    if (orc_bilu0(m, Jdec, c->LU.data(), c->Dinv.data()) != 0) {
        delete c;
        return nullptr;
    }
    /* level 0: the pressure entries of the blocks */
    Level L0;
    L0.nx = m->g.nx;
    L0.ny = m->g.ny;
    L0.nz = m->g.nz;
    L0.n = n;
    L0.rp.assign(m->row_ptr.begin(), m->row_ptr.end());
    L0.ci.assign(m->col_idx.begin(), m->col_idx.end());
    L0.val.resize(nnzb);
    for (size_t b = 0; b < nnzb; ++b) L0.val[b] = Jdec[b * 64];
    c->lv.push_back(L0);
    while (true) {
        Level& L = c->lv.back();
        if (L.n <= ORC_CPR_COARSEST || (L.nx == 1 && L.ny == 1 && L.nz == 1)) break;
        Level C;
        C.nx = (L.nx + 1) / 2;
        C.ny = (L.ny + 1) / 2;
        C.nz = (L.nz + 1) / 2;
        C.n = C.nx * C.ny * C.nz;
        L.agg.resize(L.n);
        for (int32_t i = 0; i < L.n; ++i) {
            const int32_t ix = i % L.nx, iy = (i / L.nx) % L.ny, iz = i / (L.nx * L.ny);
            L.agg[i] = ix / 2 + C.nx * (iy / 2 + C.ny * (iz / 2));
        }
        /* Galerkin product: every fine entry a_ij adds to (agg(i), agg(j)) */
        std::vector<std::map<int32_t, double>> rows(C.n);
        for (int32_t i = 0; i < L.n; ++i)
            for (int32_t k = L.rp[i]; k < L.rp[i + 1]; ++k) rows[L.agg[i]][L.agg[L.ci[k]]] += L.val[k];
        C.rp.assign(C.n + 1, 0);
        for (int32_t I = 0; I < C.n; ++I) {
            for (const auto& kv : rows[I]) {
                C.ci.push_back(kv.first);
                C.val.push_back(kv.second);
            }
            C.rp[I + 1] = (int32_t)C.ci.size();
        }
        c->lv.push_back(std::move(C));
    }
    if (!coarse_factor(*c)) {
        delete c;
        return nullptr;
    }
    return c;
}

void orc_cpr_destroy(orc_cpr* c) { delete c; }

int32_t orc_cpr_nlevels(const orc_cpr* c) { return (int32_t)c->lv.size(); }

/* dims[3] and cell count of level l */
int32_t orc_cpr_level_dims(const orc_cpr* c, int32_t l, int32_t* dims) {
    const Level& L = c->lv[l];
    dims[0] = L.nx;
    dims[1] = L.ny;
    dims[2] = L.nz;
    return L.n;
}

/* level l's matrix as a dense n_l x n_l row-major array (small levels only) */
void orc_cpr_level_dense(const orc_cpr* c, int32_t l, double* out) {
    const Level& L = c->lv[l];
    std::fill(out, out + (size_t)L.n * L.n, 0.0);
    for (int32_t i = 0; i < L.n; ++i)
        for (int32_t k = L.rp[i]; k < L.rp[i + 1]; ++k) out[(size_t)i * L.n + L.ci[k]] = L.val[k];
}

/* one red-black Gauss-Seidel sweep on level l, colour `first` first (x in/out) */
void orc_cpr_smooth(const orc_cpr* c, int32_t l, const double* b, double* x, int32_t first) {
    const Level& L = c->lv[l];
    std::vector<double> bb(b, b + L.n), xx(x, x + L.n);
    rbgs(L, bb, xx, first);
    std::copy(xx.begin(), xx.end(), x);
}

/* x = one V-cycle from level 0 applied to b */
void orc_cpr_vcycle(const orc_cpr* c, const double* b, double* x) {
    std::vector<double> bb(b, b + c->lv[0].n), xx;
    vcycle(*c, 0, bb, xx);
    std::copy(xx.begin(), xx.end(), x);
}

/* e = the stage-1 pressure solve applied to rp [N] */
void orc_cpr_pressure(const orc_cpr* c, const double* rp, double* e) {
    std::vector<double> bb(rp, rp + c->lv[0].n), ee;
    pressure_solve(*c, bb, ee);
    std::copy(ee.begin(), ee.end(), e);
}

/* z = CPR r (both [N][8]) */
void orc_cpr_apply(const orc_cpr* c, const double* r, double* z) {
    orc_model* m = c->m;
    const int32_t n = m->n;
    const size_t N = (size_t)n * 8;
    std::vector<double> rp(n), ep;
    for (int32_t i = 0; i < n; ++i) rp[i] = r[(size_t)i * 8];
    pressure_solve(*c, rp, ep);
    std::vector<double> z1(N, 0.0), az1(N), r2(N), z2(N);
    for (int32_t i = 0; i < n; ++i) z1[(size_t)i * 8] = ep[i];
    orc_spmv(m, c->A.data(), z1.data(), az1.data());
    for (size_t k = 0; k < N; ++k) r2[k] = r[k] - az1[k];
    orc_bilu0_apply(m, c->LU.data(), c->Dinv.data(), r2.data(), z2.data());
    for (size_t k = 0; k < N; ++k) z[k] = z1[k] + z2[k];
}

/* Flexible GMRES(restart) with the CPR preconditioner on Jdec x = b, x0 = 0,
 * modified Gram-Schmidt; x += Z y with Z the preconditioned basis vectors.
 * Stops when ||b - A x|| <= rtol ||b|| (true residual at every restart and at
 * exit).  Returns 0, -4 (singular factor) or -6 (no convergence). */
int orc_fgmres_cpr(orc_model* m, const double* Jdec, const double* b, double* x, int32_t restart,
                   int32_t max_restarts, double rtol, int32_t p_iters, int32_t nu, double cf, orc_solve_info* info) {
    orc_cpr* c = orc_cpr_create(m, Jdec, p_iters, nu, cf);
    if (!c) return -4;
    const size_t N = (size_t)m->n * 8;
    std::vector<double> bb(b, b + N), r(N), w(N), tmp(N);
    std::fill(x, x + N, 0.0);
    const double bnorm = std::sqrt(dotv(bb, bb));
    orc_solve_info inf;
    std::memset(&inf, 0, sizeof(inf));
    int status = -6;
    if (bnorm == 0.0) {
        orc_cpr_destroy(c);
        if (info) *info = inf;
        return 0;
    }
    const int mr = restart;
    std::vector<std::vector<double>> V(mr + 1, std::vector<double>(N)), Z(mr, std::vector<double>(N));
    std::vector<double> H((size_t)(mr + 1) * mr), cs(mr), sn(mr), g(mr + 1);
    for (int cyc = 0; cyc < max_restarts; ++cyc) {
        orc_spmv(m, Jdec, x, tmp.data());
        for (size_t k = 0; k < N; ++k) r[k] = bb[k] - tmp[k];
        const double beta = std::sqrt(dotv(r, r));
        inf.relres_true = beta / bnorm;
        if (beta <= rtol * bnorm) { status = 0; break; }
        inf.restarts = cyc;
        for (size_t k = 0; k < N; ++k) V[0][k] = r[k] / beta;
        std::fill(g.begin(), g.end(), 0.0);
        g[0] = beta;
        int done = 0;
        for (int j = 0; j < mr; ++j) {
            orc_cpr_apply(c, V[j].data(), Z[j].data());
            orc_spmv(m, Jdec, Z[j].data(), w.data());
            for (int i = 0; i <= j; ++i) {
                const double h = dotv(w, V[i]);
                H[(size_t)i * mr + j] = h;
                for (size_t k = 0; k < N; ++k) w[k] -= h * V[i][k];
            }
            const double hn = std::sqrt(dotv(w, w));
            H[(size_t)(j + 1) * mr + j] = hn;
            if (hn > 0.0)
                for (size_t k = 0; k < N; ++k) V[j + 1][k] = w[k] / hn;
            for (int i = 0; i < j; ++i) {
                const double a = H[(size_t)i * mr + j], b2 = H[(size_t)(i + 1) * mr + j];
                H[(size_t)i * mr + j] = cs[i] * a + sn[i] * b2;
                H[(size_t)(i + 1) * mr + j] = -sn[i] * a + cs[i] * b2;
            }
            const double a = H[(size_t)j * mr + j], b2 = H[(size_t)(j + 1) * mr + j];
            const double den = std::hypot(a, b2);
            cs[j] = a / den;
            sn[j] = b2 / den;
            H[(size_t)j * mr + j] = den;
            H[(size_t)(j + 1) * mr + j] = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            inf.iters++;
            done = j + 1;
            inf.relres_est = std::fabs(g[j + 1]) / bnorm;
            if (std::fabs(g[j + 1]) <= rtol * bnorm || hn == 0.0) break;
        }
        std::vector<double> y(done);
        for (int i = done - 1; i >= 0; --i) {
            double s = g[i];
            for (int t = i + 1; t < done; ++t) s -= H[(size_t)i * mr + t] * y[t];
            y[i] = s / H[(size_t)i * mr + i];
        }
        for (int i = 0; i < done; ++i)
            for (size_t k = 0; k < N; ++k) x[k] += y[i] * Z[i][k];
    }
    if (status != 0) {
        orc_spmv(m, Jdec, x, tmp.data());
        double s = 0.0;
        for (size_t k = 0; k < N; ++k) s += (bb[k] - tmp[k]) * (bb[k] - tmp[k]);
        inf.relres_true = std::sqrt(s) / bnorm;
        if (inf.relres_true <= rtol) status = 0;
    }
    orc_cpr_destroy(c);
    if (info) *info = inf;
    return status;
}

}  // extern "C"
