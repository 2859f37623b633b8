/* Forward-mode dual numbers for the oracle's analytical Jacobian.
 *
 * TEST INFRASTRUCTURE ONLY (part of the CPU oracle).
 *
 * The paper assembles Newton's system with an analytical Jacobian (abstract;
 * Section 3.1).  The oracle obtains that exact derivative by carrying, next to
 * every value, its partial derivatives with respect to the unknowns that were
 * seeded: a value of type Dual<N> is x + sum_k d[k] e_k with e_k^2 = 0.  Every
 * branch is decided on the value alone, so the derivative is the one of the
 * branch that was taken.
 */
#ifndef ISC_ORACLE_DUAL_H
#define ISC_ORACLE_DUAL_H
#include <cmath>

namespace orc {

template <int N>
struct Dual {
    double v;
    double d[N];
    Dual() : v(0.0) { for (int k = 0; k < N; ++k) d[k] = 0.0; }
    Dual(double x) : v(x) { for (int k = 0; k < N; ++k) d[k] = 0.0; }
    static Dual var(double x, int k) { Dual r(x); r.d[k] = 1.0; return r; }
};

template <int N> inline Dual<N> operator+(const Dual<N>& a, const Dual<N>& b) {
    Dual<N> r; r.v = a.v + b.v; for (int k = 0; k < N; ++k) r.d[k] = a.d[k] + b.d[k]; return r;
}
template <int N> inline Dual<N> operator-(const Dual<N>& a, const Dual<N>& b) {
    Dual<N> r; r.v = a.v - b.v; for (int k = 0; k < N; ++k) r.d[k] = a.d[k] - b.d[k]; return r;
}
template <int N> inline Dual<N> operator-(const Dual<N>& a) {
    Dual<N> r; r.v = -a.v; for (int k = 0; k < N; ++k) r.d[k] = -a.d[k]; return r;
}
template <int N> inline Dual<N> operator*(const Dual<N>& a, const Dual<N>& b) {
    Dual<N> r; r.v = a.v * b.v;
    for (int k = 0; k < N; ++k) r.d[k] = a.d[k] * b.v + a.v * b.d[k];
    return r;
}
template <int N> inline Dual<N> operator/(const Dual<N>& a, const Dual<N>& b) {
    Dual<N> r; r.v = a.v / b.v;
    for (int k = 0; k < N; ++k) r.d[k] = (a.d[k] - r.v * b.d[k]) / b.v;
    return r;
}
template <int N> inline Dual<N> operator+(const Dual<N>& a, double b) { Dual<N> r = a; r.v += b; return r; }
template <int N> inline Dual<N> operator+(double a, const Dual<N>& b) { return b + a; }
template <int N> inline Dual<N> operator-(const Dual<N>& a, double b) { Dual<N> r = a; r.v -= b; return r; }
template <int N> inline Dual<N> operator-(double a, const Dual<N>& b) { return (-b) + a; }
template <int N> inline Dual<N> operator*(const Dual<N>& a, double b) {
    Dual<N> r; r.v = a.v * b; for (int k = 0; k < N; ++k) r.d[k] = a.d[k] * b; return r;
}
template <int N> inline Dual<N> operator*(double a, const Dual<N>& b) { return b * a; }
template <int N> inline Dual<N> operator/(const Dual<N>& a, double b) {
    Dual<N> r; r.v = a.v / b; for (int k = 0; k < N; ++k) r.d[k] = a.d[k] / b; return r;
}
template <int N> inline Dual<N> operator/(double a, const Dual<N>& b) { return Dual<N>(a) / b; }

/* elementary functions: value f(x), derivative f'(x) dx */
template <int N> inline Dual<N> exp(const Dual<N>& a) {
    Dual<N> r; r.v = std::exp(a.v); for (int k = 0; k < N; ++k) r.d[k] = r.v * a.d[k]; return r;
}
template <int N> inline Dual<N> log(const Dual<N>& a) {
    Dual<N> r; r.v = std::log(a.v); for (int k = 0; k < N; ++k) r.d[k] = a.d[k] / a.v; return r;
}
template <int N> inline Dual<N> sqrt(const Dual<N>& a) {
    Dual<N> r; r.v = std::sqrt(a.v); for (int k = 0; k < N; ++k) r.d[k] = a.d[k] / (2.0 * r.v); return r;
}
/* x^c for a constant exponent c (x > 0) */
template <int N> inline Dual<N> pow(const Dual<N>& a, double c) {
    Dual<N> r; r.v = std::pow(a.v, c);
    double s = c * std::pow(a.v, c - 1.0);
    for (int k = 0; k < N; ++k) r.d[k] = s * a.d[k];
    return r;
}

inline double val(double x) { return x; }
template <int N> inline double val(const Dual<N>& a) { return a.v; }

using std::exp; using std::log; using std::sqrt; using std::pow;

}  // namespace orc
#endif
