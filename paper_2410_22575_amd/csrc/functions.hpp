// The three test functions (Sec. VII), written once over hDual<C> values.
//
// Each function struct provides
//   kTables            how many per-(point, variable) tables it uses (0 or 2)
//   tables(x, t0, t1)  the transcendental values of one input coordinate
//   eval<C>(pv, prm)   f evaluated on the CHUNK-INIT seeds of one
//                      (point, row i, chunk cs) work item
// A unary function applied to an expression whose value is an exact
// function of one coordinate (cos(2 pi x_k) in Ackley, sin/cos(x_j) in
// Fletcher-Powell) takes g, g', g'' from the per-point tables: every call of
// a point would compute the same numbers, so they are computed once per
// point and coordinate.  The hDual arithmetic itself is unchanged.
#pragma once

#include "hd.hpp"

namespace chessfad {

// One work item's view of its point, staged in LDS in structure-of-arrays
// form: coordinate k of the point lives at base[k * stride].
struct PointView {
    const double* xs;
    const double* t0;
    const double* t1;
    int stride;
    int n, i, cs;
    CF_DEV double x(int k) const { return xs[k * stride]; }
    CF_DEV double tab0(int k) const { return t0[k * stride]; }
    CF_DEV double tab1(int k) const { return t1[k * stride]; }
    template <int C>
    CF_DEV HD<double, C> y(int k) const { return seed<double, C>(x(k), k, i, cs); }
};

struct FpParams {
    const double* A;  // [n][n]
    const double* B;  // [n][n]
    const double* E;  // [n]
};

constexpr double kTwoPi = 6.283185307179586476925286766559;
constexpr double kE = 2.718281828459045235360287471352;

// sum_{k<n-1} 100 (y_{k+1} - y_k^2)^2 + (1 - y_k)^2
struct Rosenbrock {
    static constexpr int kTables = 0;
    static CF_DEV void tables(double, double&, double&) {}

    template <int C>
    static CF_DEV HD<double, C> term(const HD<double, C>& yk, const HD<double, C>& yk1) {
        HD<double, C> b = yk1 - yk * yk;
        HD<double, C> e = 1.0 - yk;
        return 100.0 * (b * b) + e * e;
    }

    template <int C>
    static CF_DEV HD<double, C> eval(const PointView& pv, const FpParams&) {
        HD<double, C> yk = pv.y<C>(0);
        HD<double, C> yk1 = pv.y<C>(1);
        HD<double, C> s = term<C>(yk, yk1);
        for (int k = 1; k + 1 < pv.n; ++k) {
            yk = yk1;
            yk1 = pv.y<C>(k + 1);
            s = s + term<C>(yk, yk1);
        }
        return s;
    }
};

// -20 exp(-0.2 sqrt(sum y^2 / n)) - exp(sum cos(2 pi y) / n) + 20 + e
struct Ackley {
    static constexpr int kTables = 2;
    // t0 = cos(2 pi x), t1 = sin(2 pi x)
    static CF_DEV void tables(double x, double& t0, double& t1) { sincos(kTwoPi * x, &t1, &t0); }

    template <int C>
    static CF_DEV HD<double, C> cos_term(const PointView& pv, int k) {
        const double c = pv.tab0(k), s = pv.tab1(k);
        return chain(kTwoPi * pv.y<C>(k), c, -s, -c);
    }

    template <int C>
    static CF_DEV HD<double, C> eval(const PointView& pv, const FpParams&) {
        HD<double, C> y = pv.y<C>(0);
        HD<double, C> ss = y * y;
        HD<double, C> cs = cos_term<C>(pv, 0);
        for (int k = 1; k < pv.n; ++k) {
            y = pv.y<C>(k);
            ss = ss + y * y;
            cs = cs + cos_term<C>(pv, k);
        }
        const double inv_n = 1.0 / pv.n;
        HD<double, C> t = inv_n * ss;
        const double rt = sqrt(t.v);
        t = chain(t, rt, 0.5 / rt, -0.25 / (rt * t.v));
        t = -0.2 * t;
        const double e1 = exp(t.v);
        t = -20.0 * chain(t, e1, e1, e1);
        HD<double, C> u = inv_n * cs;
        const double e2 = exp(u.v);
        t = t - chain(u, e2, e2, e2);
        return t + (20.0 + kE);
    }
};

// sum_m (E_m - sum_j A_mj sin y_j + B_mj cos y_j)^2
struct FletcherPowell {
    static constexpr int kTables = 2;
    // t0 = sin(x), t1 = cos(x)
    static CF_DEV void tables(double x, double& t0, double& t1) { sincos(x, &t0, &t1); }

    template <int C>
    static CF_DEV HD<double, C> inner(const PointView& pv, const FpParams& prm, int m) {
        const double* Am = prm.A + (size_t)m * pv.n;
        const double* Bm = prm.B + (size_t)m * pv.n;
        HD<double, C> y = pv.y<C>(0);
        double s = pv.tab0(0), c = pv.tab1(0);
        HD<double, C> acc = Am[0] * chain(y, s, c, -s);
        acc = acc + Bm[0] * chain(y, c, -s, -c);
        for (int j = 1; j < pv.n; ++j) {
            y = pv.y<C>(j);
            s = pv.tab0(j);
            c = pv.tab1(j);
            acc = acc + Am[j] * chain(y, s, c, -s);
            acc = acc + Bm[j] * chain(y, c, -s, -c);
        }
        return acc;
    }

    template <int C>
    static CF_DEV HD<double, C> eval(const PointView& pv, const FpParams& prm) {
        HD<double, C> r = prm.E[0] - inner<C>(pv, prm, 0);
        HD<double, C> f = r * r;
        for (int m = 1; m < pv.n; ++m) {
            r = prm.E[m] - inner<C>(pv, prm, m);
            f = f + r * r;
        }
        return f;
    }
};

}  // namespace chessfad
