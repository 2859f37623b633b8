/* CPU oracle: decoupling, block ILU(0), GMRES, Newton update and time loop.
 *
 * TEST INFRASTRUCTURE ONLY.  Plain serial FP64.
 */
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "model.h"

using namespace orc;

namespace {

/* dense 8x8 inverse by Gauss-Jordan with partial pivoting; false if singular */
bool inv8(const double* A, double* Ainv) {
    double a[8][16];
    for (int r = 0; r < 8; ++r)
        for (int c = 0; c < 8; ++c) {
            a[r][c] = A[r * 8 + c];
            a[r][8 + c] = (r == c) ? 1.0 : 0.0;
        }
    for (int k = 0; k < 8; ++k) {
        int piv = k;
        for (int r = k + 1; r < 8; ++r)
            if (std::fabs(a[r][k]) > std::fabs(a[piv][k])) piv = r;
        if (!(std::fabs(a[piv][k]) > 0.0)) return false;
        if (piv != k)
            for (int c = 0; c < 16; ++c) std::swap(a[k][c], a[piv][c]);
        double d = a[k][k];
        for (int c = 0; c < 16; ++c) a[k][c] /= d;
        for (int r = 0; r < 8; ++r) {
            if (r == k) continue;
            double fct = a[r][k];
            if (fct == 0.0) continue;
            for (int c = 0; c < 16; ++c) a[r][c] -= fct * a[k][c];
        }
    }
    for (int r = 0; r < 8; ++r)
        for (int c = 0; c < 8; ++c) Ainv[r * 8 + c] = a[r][8 + c];
    return true;
}

/* C = A * B (8x8) */
void mul8(const double* A, const double* B, double* C) {
    for (int r = 0; r < 8; ++r)
        for (int c = 0; c < 8; ++c) {
            double s = 0.0;
            for (int k = 0; k < 8; ++k) s += A[r * 8 + k] * B[k * 8 + c];
            C[r * 8 + c] = s;
        }
}

void matvec8(const double* A, const double* x, double* y) {
    for (int r = 0; r < 8; ++r) {
        double s = 0.0;
        for (int k = 0; k < 8; ++k) s += A[r * 8 + k] * x[k];
        y[r] = s;
    }
}

double dot(const std::vector<double>& a, const std::vector<double>& b) {
    double s = 0.0;
    for (size_t i = 0; i < a.size(); ++i) s += a[i] * b[i];
    return s;
}
double nrm2(const std::vector<double>& a) { return std::sqrt(dot(a, a)); }

}  // namespace

extern "C" {

/* Decoupling (Section 3.2): C_L = blockdiag(J_ii^-1) applied through
 * Gauss-Jordan elimination with partial pivoting on the block row
 * [J_ii | J_i,neighbours | F_i]; row exchanges give the dynamic equation
 * alignment.  Afterwards the diagonal block is the identity. */
int orc_decouple(orc_model* m, double* J, double* F, int32_t* bad_cell) {
    const int32_t n = m->n;
    if (bad_cell) *bad_cell = -1;
    for (int32_t i = 0; i < n; ++i) {
        int32_t b0 = m->row_ptr[i], b1 = m->row_ptr[i + 1];
        int32_t nb = b1 - b0;
        int32_t dp = m->diag_pos[i];
        int ncol = 8 * nb + 1;
        std::vector<double> a((size_t)8 * ncol);
        /* augmented matrix: diagonal block first, then the other blocks in
         * column order, then the residual */
        auto col_of_block = [&](int32_t b) {
            if (b == dp) return 0;
            int pos = 1;
            for (int32_t bb = b0; bb < b; ++bb)
                if (bb != dp) ++pos;
            return pos;
        };
        double cmax[8] = {0, 0, 0, 0, 0, 0, 0, 0};  /* column maxima of J_ii */
        for (int32_t b = b0; b < b1; ++b) {
            int cb = col_of_block(b);
            for (int r = 0; r < 8; ++r)
                for (int c = 0; c < 8; ++c) {
                    double v = J[(size_t)b * 64 + r * 8 + c];
                    a[(size_t)r * ncol + cb * 8 + c] = v;
                    if (b == dp) cmax[c] = std::max(cmax[c], std::fabs(v));
                }
        }
        for (int r = 0; r < 8; ++r) a[(size_t)r * ncol + ncol - 1] = F[(size_t)i * 8 + r];
        for (int k = 0; k < 8; ++k) {
            int piv = k;
            for (int r = k + 1; r < 8; ++r)
                if (std::fabs(a[(size_t)r * ncol + k]) > std::fabs(a[(size_t)piv * ncol + k])) piv = r;
            double pv = a[(size_t)piv * ncol + k];
            /* singular: the pivot is negligible against its own column of J_ii */
            if (!(std::fabs(pv) > 1e-14 * cmax[k]) || !std::isfinite(pv)) {
                if (bad_cell) *bad_cell = i;
                return -4;
            }
            if (piv != k)
                for (int c = 0; c < ncol; ++c) std::swap(a[(size_t)k * ncol + c], a[(size_t)piv * ncol + c]);
            for (int c = 0; c < ncol; ++c) a[(size_t)k * ncol + c] /= pv;
            for (int r = 0; r < 8; ++r) {
                if (r == k) continue;
                double fct = a[(size_t)r * ncol + k];
                if (fct == 0.0) continue;
                for (int c = 0; c < ncol; ++c) a[(size_t)r * ncol + c] -= fct * a[(size_t)k * ncol + c];
            }
        }
        for (int32_t b = b0; b < b1; ++b) {
            int cb = col_of_block(b);
            for (int r = 0; r < 8; ++r)
                for (int c = 0; c < 8; ++c)
                    J[(size_t)b * 64 + r * 8 + c] = (b == dp) ? (r == c ? 1.0 : 0.0)
                                                              : a[(size_t)r * ncol + cb * 8 + c];
        }
        for (int r = 0; r < 8; ++r) F[(size_t)i * 8 + r] = a[(size_t)r * ncol + ncol - 1];
    }
    return 0;
}

/* y = J x for a block CSR matrix (all stored blocks, including the diagonal) */
void orc_spmv(orc_model* m, const double* J, const double* x, double* y) {
    for (int32_t i = 0; i < m->n; ++i) {
        double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        for (int32_t b = m->row_ptr[i]; b < m->row_ptr[i + 1]; ++b) {
            double t[8];
            matvec8(J + (size_t)b * 64, x + (size_t)m->col_idx[b] * 8, t);
            for (int r = 0; r < 8; ++r) acc[r] += t[r];
        }
        for (int r = 0; r < 8; ++r) y[(size_t)i * 8 + r] = acc[r];
    }
}

/* Block ILU(0) in natural cell order (row-wise IKJ elimination restricted to
 * the sparsity pattern of the matrix).  LU holds the factors in the matrix's
 * block CSR layout (strictly lower blocks: L_ik; diagonal and upper: U);
 * Dinv[i] = U_ii^-1. */
int orc_bilu0(orc_model* m, const double* A, double* LU, double* Dinv) {
    const int32_t n = m->n;
    std::memcpy(LU, A, sizeof(double) * (size_t)m->row_ptr[n] * 64);
    double tmp[64];
    for (int32_t i = 0; i < n; ++i) {
        for (int32_t bk = m->row_ptr[i]; bk < m->row_ptr[i + 1]; ++bk) {
            int32_t k = m->col_idx[bk];
            if (k >= i) break;
            /* L_ik = LU_ik * U_kk^-1 */
            mul8(LU + (size_t)bk * 64, Dinv + (size_t)k * 64, tmp);
            std::memcpy(LU + (size_t)bk * 64, tmp, sizeof(tmp));
            /* LU_ij -= L_ik U_kj for j > k in both row i and row k */
            for (int32_t bj = bk + 1; bj < m->row_ptr[i + 1]; ++bj) {
                int32_t j = m->col_idx[bj];
                int32_t bkj = block_of(*m, k, j);
                if (bkj < 0) continue;
                double prod[64];
                mul8(LU + (size_t)bk * 64, LU + (size_t)bkj * 64, prod);
                for (int t = 0; t < 64; ++t) LU[(size_t)bj * 64 + t] -= prod[t];
            }
        }
        if (!inv8(LU + (size_t)m->diag_pos[i] * 64, Dinv + (size_t)i * 64)) return -4;
    }
    return 0;
}

/* z = (LU)^-1 r: forward (I + L) y = r, backward U z = y */
void orc_bilu0_apply(orc_model* m, const double* LU, const double* Dinv, const double* r, double* z) {
    const int32_t n = m->n;
    std::vector<double> y((size_t)n * 8);
    for (int32_t i = 0; i < n; ++i) {
        double acc[8];
        for (int e = 0; e < 8; ++e) acc[e] = r[(size_t)i * 8 + e];
        for (int32_t b = m->row_ptr[i]; b < m->row_ptr[i + 1]; ++b) {
            int32_t k = m->col_idx[b];
            if (k >= i) break;
            double t[8];
            matvec8(LU + (size_t)b * 64, y.data() + (size_t)k * 8, t);
            for (int e = 0; e < 8; ++e) acc[e] -= t[e];
        }
        for (int e = 0; e < 8; ++e) y[(size_t)i * 8 + e] = acc[e];
    }
    for (int32_t i = n - 1; i >= 0; --i) {
        double acc[8];
        for (int e = 0; e < 8; ++e) acc[e] = y[(size_t)i * 8 + e];
        for (int32_t b = m->row_ptr[i]; b < m->row_ptr[i + 1]; ++b) {
            int32_t j = m->col_idx[b];
            if (j <= i) continue;
            double t[8];
            matvec8(LU + (size_t)b * 64, z + (size_t)j * 8, t);
            for (int e = 0; e < 8; ++e) acc[e] -= t[e];
        }
        matvec8(Dinv + (size_t)i * 64, acc, z + (size_t)i * 8);
    }
}

}  // extern "C"

namespace {

/* The well rows eliminated from a decoupled system: the operator becomes
 * x -> A x - sum_w Bt_w (C_w . x) / D_w, with Bt = the decoupled B (rows
 * scaled by the inverse diagonal blocks like the rest of the block row). */
struct Border {
    const double *Bt, *C, *D;   /* [ncp][8], [ncp][8], [ncw] */
};

void apply_op(orc_model* m, const double* A, const Border* bd, const double* x, double* y) {
    orc_spmv(m, A, x, y);
    if (!bd) return;
    for (const orc_cwell& W : m->cw) {
        double s = 0.0;
        for (int32_t k = 0; k < W.np; ++k) {
            const int32_t i = m->perfs[W.p0 + k].cell;
            for (int v = 0; v < 8; ++v) s += bd->C[(size_t)(W.c0 + k) * 8 + v] * x[(size_t)i * 8 + v];
        }
        s /= bd->D[&W - m->cw.data()];
        for (int32_t k = 0; k < W.np; ++k) {
            const int32_t i = m->perfs[W.p0 + k].cell;
            for (int e = 0; e < 8; ++e) y[(size_t)i * 8 + e] -= bd->Bt[(size_t)(W.c0 + k) * 8 + e] * s;
        }
    }
}

/* Right-preconditioned restarted GMRES(m) with modified Gram-Schmidt and
 * Givens rotations, x0 = 0, stop when ||b - Op x|| <= rtol ||b||; the true
 * residual is recomputed at every restart and at exit.  Op = A, or A with
 * the well rows eliminated; the preconditioner is block ILU(0) of A. */
int gmres_impl(orc_model* m, const double* A, const Border* bd, const double* b, double* x, int32_t restart,
               int32_t max_restarts, double rtol, orc_solve_info* info) {
    const size_t N = (size_t)m->n * 8;
    std::vector<double> LU((size_t)m->row_ptr[m->n] * 64), Dinv((size_t)m->n * 64);
    int st = orc_bilu0(m, A, LU.data(), Dinv.data());
    if (st) return st;
    std::vector<double> bb(b, b + N), r(N), w(N), z(N), tmp(N);
    std::fill(x, x + N, 0.0);
    double bnorm = nrm2(bb);
    orc_solve_info inf;
    std::memset(&inf, 0, sizeof(inf));
    if (bnorm == 0.0) {
        if (info) *info = inf;
        return 0;
    }
    std::vector<std::vector<double>> V(restart + 1, std::vector<double>(N));
    std::vector<double> H((size_t)(restart + 1) * restart), cs(restart), sn(restart), g(restart + 1);
    int status = -6;
    for (int cyc = 0; cyc < max_restarts; ++cyc) {
        apply_op(m, A, bd, x, tmp.data());
        for (size_t k = 0; k < N; ++k) r[k] = bb[k] - tmp[k];
        double beta = nrm2(r);
        inf.relres_true = beta / bnorm;
        if (beta <= rtol * bnorm) { status = 0; break; }
        inf.restarts = cyc;
        for (size_t k = 0; k < N; ++k) V[0][k] = r[k] / beta;
        std::fill(g.begin(), g.end(), 0.0);
        g[0] = beta;
        int jdone = 0;
        for (int j = 0; j < restart; ++j) {
            orc_bilu0_apply(m, LU.data(), Dinv.data(), V[j].data(), z.data());
            apply_op(m, A, bd, z.data(), w.data());
            for (int i = 0; i <= j; ++i) {
                double h = dot(w, V[i]);
                H[(size_t)i * restart + j] = h;
                for (size_t k = 0; k < N; ++k) w[k] -= h * V[i][k];
            }
            double hn = nrm2(w);
            H[(size_t)(j + 1) * restart + j] = hn;
            if (hn > 0.0)
                for (size_t k = 0; k < N; ++k) V[j + 1][k] = w[k] / hn;
            for (int i = 0; i < j; ++i) {
                double a = H[(size_t)i * restart + j], c = H[(size_t)(i + 1) * restart + j];
                H[(size_t)i * restart + j] = cs[i] * a + sn[i] * c;
                H[(size_t)(i + 1) * restart + j] = -sn[i] * a + cs[i] * c;
            }
            double a = H[(size_t)j * restart + j], c = H[(size_t)(j + 1) * restart + j];
            double den = std::hypot(a, c);
            cs[j] = a / den;
            sn[j] = c / den;
            H[(size_t)j * restart + j] = den;
            H[(size_t)(j + 1) * restart + j] = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            inf.iters++;
            jdone = j + 1;
            inf.relres_est = std::fabs(g[j + 1]) / bnorm;
            if (std::fabs(g[j + 1]) <= rtol * bnorm || hn == 0.0) break;
        }
        /* y = H^-1 g, x += M^-1 (V y) */
        std::vector<double> y(jdone);
        for (int i = jdone - 1; i >= 0; --i) {
            double s = g[i];
            for (int k = i + 1; k < jdone; ++k) s -= H[(size_t)i * restart + k] * y[k];
            y[i] = s / H[(size_t)i * restart + i];
        }
        std::fill(tmp.begin(), tmp.end(), 0.0);
        for (int i = 0; i < jdone; ++i)
            for (size_t k = 0; k < N; ++k) tmp[k] += y[i] * V[i][k];
        orc_bilu0_apply(m, LU.data(), Dinv.data(), tmp.data(), z.data());
        for (size_t k = 0; k < N; ++k) x[k] += z[k];
    }
    if (status != 0) {
        apply_op(m, A, bd, x, tmp.data());
        double s = 0.0;
        for (size_t k = 0; k < N; ++k) s += (bb[k] - tmp[k]) * (bb[k] - tmp[k]);
        inf.relres_true = std::sqrt(s) / bnorm;
        if (inf.relres_true <= rtol) status = 0;
    }
    if (info) *info = inf;
    return status;
}

}  // namespace

extern "C" {

/* Right-preconditioned restarted GMRES(m) with modified Gram-Schmidt and
 * Givens rotations, x0 = 0, stop when ||b - A x|| <= rtol ||b||; the true
 * residual is recomputed at every restart and at exit. */
int orc_gmres(orc_model* m, const double* A, const double* b, double* x, int32_t restart,
              int32_t max_restarts, double rtol, orc_solve_info* info) {
    return gmres_impl(m, A, nullptr, b, x, restart, max_restarts, rtol, info);
}

/* Right-preconditioned BiCGSTAB (van der Vorst's stabilised bi-conjugate
 * gradients; the Krylov method of the paper's experiments) with block ILU(0),
 * x0 = 0.  Each iteration applies A M^-1 twice:
 *   p = r + beta (p - omega v),  p^ = M^-1 p,  v = A p^,  alpha = rho / (r~, v),
 *   s = r - alpha v,  s^ = M^-1 s,  t = A s^,  omega = (t, s) / (t, t),
 *   x += alpha p^ + omega s^,  r = s - omega t,  rho' = (r~, r),
 *   beta' = (rho' / rho) (alpha / omega),
 * with the shadow vector r~ = the starting residual.  The iteration stops once
 * the updated residual (s at the half step, else r) satisfies
 * ||.|| <= rtol ||b||; then the true residual b - A x is formed, and if it is
 * still above the tolerance the iteration starts again from it.  A breakdown
 * -- |rho| <= 1e-12 ||r~|| ||r||, |(r~, v)| <= 1e-12 ||r~|| ||v||,
 * (t, t) = 0 (after keeping the half step x += alpha p^, whose residual is s)
 * or omega = 0 -- also starts again from the true residual, with it as the
 * new shadow vector, at most 8 times.  Returns 0, or -6 (no convergence
 * within max_iters, or a ninth breakdown). */
int orc_bicgstab(orc_model* m, const double* A, const double* b, double* x, int32_t max_iters, double rtol,
                 orc_solve_info* info) {
    const size_t N = (size_t)m->n * 8;
    std::vector<double> LU((size_t)m->row_ptr[m->n] * 64), Dinv((size_t)m->n * 64);
    int st = orc_bilu0(m, A, LU.data(), Dinv.data());
    if (st) return st;
    std::vector<double> bb(b, b + N), r(N), rs(N), p(N), v(N), s(N), t(N), ph(N), sh(N), tmp(N);
    std::fill(x, x + N, 0.0);
    const double bnorm = nrm2(bb);
    orc_solve_info inf;
    std::memset(&inf, 0, sizeof(inf));
    if (bnorm == 0.0) {
        if (info) *info = inf;
        return 0;
    }
    const double tol = rtol * bnorm;
    const double brk = 1e-12;        /* relative breakdown threshold */
    const int max_breakdowns = 8;
    int status = -6, it = 0, starts = 0, breakdowns = 0;
    while (it < max_iters) {
        orc_spmv(m, A, x, tmp.data());
        for (size_t k = 0; k < N; ++k) r[k] = bb[k] - tmp[k];
        const double rn0 = nrm2(r);
        inf.relres_true = rn0 / bnorm;
        if (rn0 <= tol) { status = 0; break; }
        inf.restarts = starts++;
        rs = r;
        std::fill(p.begin(), p.end(), 0.0);
        std::fill(v.begin(), v.end(), 0.0);
        double rho_old = 1.0, alpha = 1.0, omega = 1.0, rho = dot(rs, r), rn = rn0;
        bool converged = false, breakdown = false;
        while (it < max_iters) {
            if (!(std::fabs(rho) > brk * rn0 * rn) || !std::isfinite(rho)) { breakdown = true; break; }
            const double beta = (rho / rho_old) * (alpha / omega);
            for (size_t k = 0; k < N; ++k) p[k] = r[k] + beta * (p[k] - omega * v[k]);
            orc_bilu0_apply(m, LU.data(), Dinv.data(), p.data(), ph.data());
            orc_spmv(m, A, ph.data(), v.data());
            const double rv = dot(rs, v);
            if (!(std::fabs(rv) > brk * rn0 * nrm2(v)) || !std::isfinite(rv)) { breakdown = true; break; }
            alpha = rho / rv;
            for (size_t k = 0; k < N; ++k) s[k] = r[k] - alpha * v[k];
            ++it;
            const double sn = nrm2(s);
            inf.relres_est = sn / bnorm;
            if (sn <= tol) {
                for (size_t k = 0; k < N; ++k) x[k] += alpha * ph[k];
                converged = true;
                break;
            }
            orc_bilu0_apply(m, LU.data(), Dinv.data(), s.data(), sh.data());
            orc_spmv(m, A, sh.data(), t.data());
            const double tt = dot(t, t);
            if (!(tt > 0.0) || !std::isfinite(tt)) {
                /* s is the residual of x + alpha p^: keep that half step */
                for (size_t k = 0; k < N; ++k) x[k] += alpha * ph[k];
                breakdown = true;
                break;
            }
            omega = dot(t, s) / tt;
            for (size_t k = 0; k < N; ++k) {
                x[k] += alpha * ph[k] + omega * sh[k];
                r[k] = s[k] - omega * t[k];
            }
            rn = nrm2(r);
            inf.relres_est = rn / bnorm;
            if (rn <= tol) { converged = true; break; }
            if (omega == 0.0) { breakdown = true; break; }
            rho_old = rho;
            rho = dot(rs, r);
        }
        /* a breakdown restarts from the true residual, a bounded number of times */
        if (breakdown && ++breakdowns <= max_breakdowns) continue;
        if (!converged) break;
    }
    if (status != 0) {
        orc_spmv(m, A, x, tmp.data());
        double q = 0.0;
        for (size_t k = 0; k < N; ++k) q += (bb[k] - tmp[k]) * (bb[k] - tmp[k]);
        inf.relres_true = std::sqrt(q) / bnorm;
        if (inf.relres_true <= rtol) status = 0;
    }
    inf.iters = it;
    if (info) *info = inf;
    return status;
}

/* Convergence measure: max over cells and rows of |F| / s, with
 * s = V phi_ref rho_ref,W / dt for molar and coke rows and
 * s = V (1 - phi_ref) cp_rock (1 K) / dt for the energy row. */
double orc_scaled_norm(orc_model* m, const double* F, double dt) {
    const double V = cell_volume(*m);
    double mx = 0.0;
    for (int32_t i = 0; i < m->n; ++i) {
        double sm = V * m->poro[i] * m->fl.rho_ref[0] / dt;
        double se = V * (1.0 - m->poro[i]) * m->fl.cp_rock / dt;
        for (int e = 0; e < 8; ++e) {
            double v = std::fabs(F[(size_t)i * 8 + e]) / (e == 6 ? se : sm);
            if (!(v <= mx)) mx = v;  /* propagates NaN */
        }
    }
    return mx;
}

/* Newton update with the saturation treatment of the PER subsection (a value
 * driven negative is replaced by half of its previous value), extended to the
 * primary mole fractions and to C_c; if S_o would become negative the (S_w,
 * S_g) increments are scaled so that S_o is halved.  Before those rules every
 * increment is clipped to a per-variable limit (the paper names only the
 * saturation treatment; the limits bound a Newton step far from the root and
 * are inactive near it).  du is [N][8] (block layout). */
static const double kStepLimit[8] = {0.2 /* x |p| */, 0.2, 0.2, 0.2, 50.0 /* K */, 0.2, 0.2,
                                     1000.0 /* mol/m3 */};

int orc_update(orc_model* m, double* u, const double* du) {
    const int32_t n = m->n;
    for (int32_t i = 0; i < n; ++i) {
        double o[8], v[8];
        for (int k = 0; k < 8; ++k) {
            o[k] = u[(size_t)k * n + i];
            double d = du[(size_t)i * 8 + k];
            double lim = kStepLimit[k] * (k == 0 ? std::fabs(o[0]) : 1.0);
            if (d > lim) d = lim;
            if (d < -lim) d = -lim;
            v[k] = o[k] + d;
        }
        for (int k : {1, 2, 3}) {
            if (v[k] < 0.0) v[k] = 0.5 * o[k];
            else if (v[k] > 1.0) v[k] = 0.5 * (1.0 + o[k]);
        }
        for (int k : {5, 6})
            if (v[k] < 0.0) v[k] = 0.5 * o[k];
        double so_old = 1.0 - o[5] - o[6];
        double so_new = 1.0 - v[5] - v[6];
        if (so_new < 0.0) {
            double dsum = (v[5] - o[5]) + (v[6] - o[6]);
            double th = 0.5 * so_old / dsum;
            v[5] = o[5] + th * (v[5] - o[5]);
            v[6] = o[6] + th * (v[6] - o[6]);
        }
        if (v[7] < 0.0) v[7] = 0.5 * o[7];
        for (int k = 0; k < 8; ++k) {
            if (!std::isfinite(v[k])) return -5;
            u[(size_t)k * n + i] = v[k];
        }
    }
    return 0;
}

/* One Newton iteration.  With controlled wells the system is bordered by
 * their rows (bhp unknowns, well-modelling subsection).  First each
 * rate-controlled well's equation is solved on its own for bhp at the
 * current cells (orc_well_solve); then the bordered system is assembled and
 * its well rows eliminated:
 *   (J - B D^-1 C) du = -(F - B D^-1 R),  dbhp = -D^-1 (R + C du),
 * after decoupling J~ = C_L J, Bt = C_L B, F~ = C_L F; the reduced operator is
 * applied as J~ x - Bt D^-1 (C x) and preconditioned with block ILU(0) of J~.
 * bhp takes its whole Newton step. */
int orc_newton_step(orc_model* m, double* u, const double* u_old, double dt, double tol,
                    int32_t restart, int32_t max_restarts, double rtol, orc_newton_info* info) {
    const size_t N = (size_t)m->n * 8;
    std::vector<double> F(N), J((size_t)m->row_ptr[m->n] * 64), du(N), rhs(N);
    orc_newton_info inf;
    std::memset(&inf, 0, sizeof(inf));
    const size_t ncw = m->cw.size();
    const size_t ncp = ncw ? (size_t)(m->cw.back().c0 + m->cw.back().np) : 0;
    std::vector<double> R(ncw), D(ncw), B(ncp * 8), C(ncp * 8), Bt(ncp * 8);
    if (ncw) orc_well_solve(m, u);
    orc_assemble(m, u, u_old, dt, F.data(), J.data());
    inf.res_scaled = orc_scaled_norm(m, F.data(), dt);
    if (ncw) {
        orc_well_border(m, u, R.data(), D.data(), B.data(), C.data());
        const double rw = orc_well_scaled_norm(m, R.data(), dt);
        if (!(rw <= inf.res_scaled)) inf.res_scaled = rw;
    }
    if (!std::isfinite(inf.res_scaled)) { inf.status = -5; if (info) *info = inf; return -5; }
    if (inf.res_scaled <= tol) { inf.converged = 1; if (info) *info = inf; return 0; }
    /* Bt = J_ii^-1 B at the perforated cells, before J is decoupled */
    for (const orc_cwell& W : m->cw)
        for (int32_t k = 0; k < W.np; ++k) {
            const int32_t i = m->perfs[W.p0 + k].cell;
            double inv[64];
            if (!inv8(J.data() + (size_t)m->diag_pos[i] * 64, inv)) {
                inf.status = -4;
                if (info) *info = inf;
                return -4;
            }
            matvec8(inv, B.data() + (size_t)(W.c0 + k) * 8, Bt.data() + (size_t)(W.c0 + k) * 8);
        }
    int32_t bad;
    int st = orc_decouple(m, J.data(), F.data(), &bad);
    if (st) { inf.status = st; if (info) *info = inf; return st; }
    for (size_t k = 0; k < N; ++k) rhs[k] = -F[k];
    for (size_t w = 0; w < ncw; ++w) {
        const orc_cwell& W = m->cw[w];
        for (int32_t k = 0; k < W.np; ++k) {
            const int32_t i = m->perfs[W.p0 + k].cell;
            for (int e = 0; e < 8; ++e) rhs[(size_t)i * 8 + e] += Bt[(size_t)(W.c0 + k) * 8 + e] * R[w] / D[w];
        }
    }
    Border bd{Bt.data(), C.data(), D.data()};
    orc_solve_info si;
    st = gmres_impl(m, J.data(), ncw ? &bd : nullptr, rhs.data(), du.data(), restart, max_restarts, rtol, &si);
    inf.iters_lin = si.iters;
    inf.relres_true = si.relres_true;
    if (st) { inf.status = st; if (info) *info = inf; return st; }
    for (size_t w = 0; w < ncw; ++w) {
        orc_cwell& W = m->cw[w];
        double s = R[w];
        for (int32_t k = 0; k < W.np; ++k) {
            const int32_t i = m->perfs[W.p0 + k].cell;
            for (int v = 0; v < 8; ++v) s += C[(size_t)(W.c0 + k) * 8 + v] * du[(size_t)i * 8 + v];
        }
        W.bhp -= s / D[w];
        if (!std::isfinite(W.bhp)) { inf.status = -5; if (info) *info = inf; return -5; }
    }
    st = orc_update(m, u, du.data());
    inf.status = st;
    if (info) *info = inf;
    return st;
}

/* Implicit-Euler time loop with Newton; on a failed step the step size is
 * halved and the step retried (at most four times). */
int orc_run(orc_model* m, double* u, double dt, int32_t nsteps, double tol, int32_t max_newton,
            int32_t restart, int32_t max_restarts, double rtol, orc_step_info* steps, double* u_hist) {
    const size_t N = (size_t)m->n * 8;
    std::vector<double> u_old(N);
    if (u_hist) std::memcpy(u_hist, u, sizeof(double) * N);
    for (int32_t s = 0; s < nsteps; ++s) {
        std::memcpy(u_old.data(), u, sizeof(double) * N);
        const std::vector<orc_cwell> cw_old = m->cw;
        double dts = dt;
        int cuts = 0;
        bool ok = false;
        orc_step_info si;
        std::memset(&si, 0, sizeof(si));
        while (!ok && cuts <= 4) {
            int nit = 0, lin = 0;
            orc_well_controls(m, u);
            orc_newton_info ni;
            for (; nit < max_newton + 1; ++nit) {
                int st = orc_newton_step(m, u, u_old.data(), dts, tol, restart, max_restarts, rtol, &ni);
                lin += ni.iters_lin;
                if (st) break;
                if (ni.converged) { ok = true; break; }
            }
            si.newton_its += nit;
            si.lin_its += lin;
            si.res_final = ni.res_scaled;
            if (!ok) {
                std::memcpy(u, u_old.data(), sizeof(double) * N);
                m->cw = cw_old;
                dts *= 0.5;
                ++cuts;
            }
        }
        si.cuts = cuts;
        si.dt_used = dts;
        if (steps) steps[s] = si;
        if (!ok) return -7;
        if (u_hist) std::memcpy(u_hist + (size_t)(s + 1) * N, u, sizeof(double) * N);
    }
    return nsteps;
}

}  // extern "C"
