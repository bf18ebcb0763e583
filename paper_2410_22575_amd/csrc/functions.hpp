// The three test functions (Sec. VII), written once over hDual<C> values and
// a precision policy P (float64, or float32 with compensated sums).
//
// Each function struct provides
//   kTables              per-(point, coordinate) transcendental tables (0 or 2)
//   tables(x, t0, t1)    those values for one coordinate, in float64
//   isl_tasks / isl_size per-point float64 "island" work: how many tasks and
//                        how many values per point
//   island(task, ...)    one task of it, in float64 (stored in float64; the
//                        hDual arithmetic rounds an island where it uses it)
//   eval<P, C>(pv, prm)  f evaluated on the CHUNK-INIT seeds of one
//                        (point, row i, chunk cs) work item
//   hvp<P, C>(pv, prm, vrow)  the same call's chunk dot
//                        sum_l h[l] v[cs + l] (CHESS-VEC), with f evaluated
//                        only on the terms whose seeds give them a
//                        second-order part (see below)
// Values that every call of a point shares - the transcendentals of single
// coordinates, Ackley's sqrt and exponentials of its two sums, the
// Fletcher-Powell residual values - are computed once per point in float64
// and enter the hDual arithmetic as the (g, g', g'') of the chain rule or as
// a value component.  The derivative components are unchanged.
#pragma once

#include "hd.hpp"
#include "trig.hpp"

namespace chessfad {

// Per-point rows of the LDS staging: a point's m entries of one array are
// contiguous, rows padded to an odd length so that the rows of different
// points start in different banks; offsets within a row are then immediates.
__host__ __device__ inline int aos_stride(int m) { return m | 1; }

// Element idx of a float64 (or, with io32, float32) output array.
CF_DEV void st_io(double* p, int64_t idx, double val, int io32) {
    if (io32)
        reinterpret_cast<float*>(p)[idx] = (float)val;
    else
        p[idx] = val;
}

// One work item's view of its point, staged in LDS: entry k of the point
// lives at base[k].
template <typename T>
struct PointView {
    const T* xs;          // coordinates (hDual precision)
    const double* t0;     // tables (float64)
    const double* t1;
    const double* isl;    // per-point island values (float64)
    int n, i, cs;
    CF_DEV T x(int k) const { return xs[k]; }
    CF_DEV T tab0(int k) const { return (T)t0[k]; }
    CF_DEV T tab1(int k) const { return (T)t1[k]; }
    CF_DEV T island(int q) const { return (T)isl[q]; }
    CF_DEV double island64(int q) const { return isl[q]; }
    template <int C>
    CF_DEV HD1<T, C> y(int k) const { return seed<T, C>(x(k), k, i, cs); }
    // y_k restricted to the W chunk components m0 .. m0 + W - 1 (slots of that
    // window outside [0, C) are never added to a sum)
    template <int W>
    CF_DEV HD1<T, W> y_at(int k, int m0) const { return seed<T, W>(x(k), k, i, cs + m0); }
};

struct FpParams {
    const double* A;    // [n][n]
    const double* B;    // [n][n]
    const double* E;    // [n]
    const float* A32;   // float32 copies (exact for the integer entries of the test problems)
    const float* B32;
    int ab32 = 0;       // 1: the float32 copies are exact, and float64 kernels may read A and B there
};

template <typename T>
CF_DEV T fp_a(const FpParams& p, size_t idx);
template <>
CF_DEV double fp_a<double>(const FpParams& p, size_t idx) { return p.A[idx]; }
template <>
CF_DEV float fp_a<float>(const FpParams& p, size_t idx) { return p.A32[idx]; }
template <typename T>
CF_DEV T fp_b(const FpParams& p, size_t idx);
template <>
CF_DEV double fp_b<double>(const FpParams& p, size_t idx) { return p.B[idx]; }
template <>
CF_DEV float fp_b<float>(const FpParams& p, size_t idx) { return p.B32[idx]; }

constexpr double kTwoPi = 6.283185307179586476925286766559;
constexpr double kE = 2.718281828459045235360287471352;

// The chunk dot of a full evaluation: sum_l h[l] v[cs + l] over columns < n.
template <class P, class F, int C>
CF_DEV double eval_dot(const PointView<typename P::T>& pv, const FpParams& prm, const typename P::T* vrow) {
    const HD<typename P::T, C> res = F::template eval<P, C>(pv, prm);
    typename P::Dot acc;
#pragma unroll
    for (int l = 0; l < C; ++l)
        if (pv.cs + l < pv.n) acc.add(res.h[l], vrow[pv.cs + l]);
    return acc.get();
}

// Second-order parts in a call (i, cs).  The row seed [k = i] is nonzero
// only on x_i, and every second-order component of an hDual operation is a
// sum of products that each hold a row-derivative factor (u_d w_g, w_d u_g,
// g'' u_d u_g) or an operand's second-order part.  So a term of f in which
// x_i does not occur has an exactly zero second-order part whatever its chunk
// seeds: it contributes value and chunk-gradient components only.  H.v reads
// the second-order part alone; `hvp` evaluates the terms that reach it -
// Rosenbrock's terms in x_i, and for Ackley the term in x_i together with the
// chunk's terms, whose gradient components pass through the outer functions'
// second derivatives - each on its CHUNK-INIT seeds, and dots their
// second-order components with v as it goes.

// sum_{k<n-1} 100 (y_{k+1} - y_k^2)^2 + (1 - y_k)^2
struct Rosenbrock {
    static constexpr int kTables = 0;
    static CF_DEV void tables(double, double&, double&) {}
    __host__ __device__ static int isl_tasks(int) { return 0; }
    __host__ __device__ static int isl_size(int) { return 0; }
    template <typename XT>
    static CF_DEV void island(int, int, const XT*, const double*, const double*, int, const FpParams&, double*) {}

    template <typename T, int C>
    static CF_DEV HD<T, C> term(const HD1<T, C>& yk, const HD1<T, C>& yk1) {
        HD<T, C> b = yk1 - sq(yk);
        HD1<T, C> e = T(1) - yk;
        return T(100) * sq(b) + sq(e);
    }

    // The terms k whose variables y_k, y_k+1 both lie outside the call's
    // chunk [cs, cs + C) have seeds with no g part, so their g and h
    // components are exact zeros; they run on HD<T, 0> (value and row
    // derivative only), in order of k with the others.  Second-order
    // component (i, cs + l) receives at most two nonzero terms.  For kernels
    // whose lanes of a wave share cs.
    template <class P, int C>
    static CF_DEV HD<typename P::T, C> eval(const PointView<typename P::T>& pv, const FpParams&) {
        using T = typename P::T;
        const int nt = pv.n - 1;                                 // terms
        const int k0 = pv.cs > 0 ? pv.cs - 1 : 0;                // first term touching the chunk
        const int k1 = pv.cs + C < nt ? pv.cs + C : nt;          // one past the last
        auto s = P::start(zero_hd<T, C>());
        for (int k = 0; k < k0; ++k) P::add_light(s, term<T, 0>(pv.template y<0>(k), pv.template y<0>(k + 1)));
        // term k = cs - 1 + p has chunk components p - 1 and p only: it runs
        // on that window of two and is added there (the other components
        // of a full-width term are exact zeros)
        static_for<C + 1>([&](auto pc) {
            constexpr int p = decltype(pc)::value;
            const int k = pv.cs - 1 + p;
            if (k >= k0 && k < k1)
                P::template add_at<p - 1>(s, term<T, 2>(pv.template y_at<2>(k, p - 1),
                                                        pv.template y_at<2>(k + 1, p - 1)));
        });
        for (int k = k1; k < nt; ++k) P::add_light(s, term<T, 0>(pv.template y<0>(k), pv.template y<0>(k + 1)));
        return P::value(s);
    }

    // H.v chunk dot of call (i, cs): the terms in x_i are k = i - 1 (on
    // x_{i-1}, x_i) and k = i (on x_i, x_{i+1}).  Each runs on the window of
    // its two variables: y_i carries the row seed, and each variable carries
    // its chunk seed when it lies in [cs, cs + C) (otherwise a zero seed, and
    // that window slot comes out zero).  A term outside 0 <= k < n - 1 gets a
    // zero row seed, so its second-order part is zero; its index is clamped.
    template <typename T, int C>
    static CF_DEV void row_terms(const PointView<T>& pv, HD<T, 2>& tm, HD<T, 2>& tp, int& km, int& kp) {
        km = pv.i > 0 ? pv.i - 1 : 0;
        kp = pv.i + 1 < pv.n ? pv.i + 1 : pv.i;
        row_terms_at<T, C>(pv.i, pv.n, pv.cs, pv.x(km), pv.x(pv.i), pv.x(kp), tm, tp);
    }
    // the same from the coordinates x_km, x_i, x_kp themselves
    template <typename T, int C>
    static CF_DEV void row_terms_at(int i, int n, int cs, T xm, T xi, T xp, HD<T, 2>& tm, HD<T, 2>& tp) {
        auto chunk_seed = [&](int k) { return (k >= cs && k < cs + C) ? T(1) : T(0); };
        {
            // term k = i - 1: window (x_{i-1}, x_i)
            HD1<T, 2> a, b;
            a.v = xm;
            a.d = T(0);
            a.g[0] = chunk_seed(i - 1);
            a.g[1] = T(0);
            b.v = xi;
            b.d = i > 0 ? T(1) : T(0);
            b.g[0] = T(0);
            b.g[1] = chunk_seed(i);
            tm = term<T, 2>(a, b);
        }
        {
            // term k = i: window (x_i, x_{i+1})
            HD1<T, 2> a, b;
            a.v = xi;
            a.d = i + 1 < n ? T(1) : T(0);
            a.g[0] = chunk_seed(i);
            a.g[1] = T(0);
            b.v = xp;
            b.d = T(0);
            b.g[0] = T(0);
            b.g[1] = chunk_seed(i + 1);
            tp = term<T, 2>(a, b);
        }
    }

    template <class P, int C>
    static CF_DEV double hvp(const PointView<typename P::T>& pv, const FpParams&, const typename P::T* vrow) {
        using T = typename P::T;
        HD<T, 2> tm, tp;
        int km, kp;
        row_terms<T, C>(pv, tm, tp, km, kp);
        typename P::Dot acc;
        acc.add(tm.h[0], vrow[km]);
        acc.add(tm.h[1], vrow[pv.i]);
        acc.add(tp.h[0], vrow[pv.i]);
        acc.add(tp.h[1], vrow[kp]);
        return acc.get();
    }

    // The call's second-order components h[l] from the same two terms (for
    // the symmetric H.v, which also needs them one by one): column i - 1
    // from term i - 1, column i from both in order of k, column i + 1 from
    // term i; every other column of the chunk is an exact zero.
    static constexpr bool kRowTerms = true;
    template <class P, int C>
    static CF_DEV void hrow(const PointView<typename P::T>& pv, const FpParams&, typename P::T (&h)[C]) {
        using T = typename P::T;
        HD<T, 2> tm, tp;
        int km, kp;
        row_terms<T, C>(pv, tm, tp, km, kp);
        const int i = pv.i, cs = pv.cs;
#pragma unroll
        for (int l = 0; l < C; ++l) {
            const int k = cs + l;
            h[l] = k == i - 1 ? tm.h[0] : k == i ? tm.h[1] + tp.h[0] : k == i + 1 ? tp.h[1] : T(0);
        }
    }
};

// -20 exp(-0.2 sqrt(sum y^2 / n)) - exp(sum cos(2 pi y) / n) + 20 + e
struct Ackley {
    static constexpr int kTables = 2;
    // t0 = cos(2 pi x), t1 = -2 pi sin(2 pi x): the value and the first
    // derivative of y -> cos(2 pi y) at x
    static CF_DEV void tables(double x, double& t0, double& t1) {
        double s;
        cf_sincos(kTwoPi * x, &s, &t0);
        t1 = -kTwoPi * s;
    }
    __host__ __device__ static int isl_tasks(int) { return 1; }
    __host__ __device__ static int isl_size(int) { return 6; }

    // float64 per-point values of the two outer functions, each composed into
    // one scalar function of its sum, with its first two derivatives there:
    //   F(s) = -20 exp(-0.2 sqrt(s / n))  at s = sum x^2
    //   G(c) = -exp(c / n)                at c = sum cos(2 pi x)
    // With r = sqrt(s / n) and E = exp(-0.2 r): F' = 2E / (n r) and
    // F'' = -E (0.2 + 1 / r) / (n r)^2; G' = G / n, G'' = G / n^2.
    template <typename XT>
    static CF_DEV void island(int, int n, const XT* xg, const double* t0, const double*, int stride,
                              const FpParams&, double* isl) {
        double ss = (double)xg[0] * (double)xg[0], cs = t0[0];
        for (int k = 1; k < n; ++k) {
            ss += (double)xg[k] * (double)xg[k];
            cs += t0[k * stride];
        }
        outer(n, ss, cs, isl, stride);
    }
    // the island values from the sums ss = sum x^2 and cs = sum cos(2 pi x)
    static CF_DEV void outer(int n, double ss, double cs, double* isl, int stride) {
        const double inv_n = 1.0 / n;
        const double rt = sqrt(inv_n * ss);
        const double e1 = exp(-0.2 * rt);
        const double inr = (1.0 / rt) * inv_n;   // 1 / (n r)
        isl[0] = -20.0 * e1;
        isl[1 * stride] = 2.0 * e1 * inr;
        isl[2 * stride] = -e1 * (0.2 + n * inr) * (inr * inr);
        const double g = -exp(inv_n * cs);
        isl[3 * stride] = g;
        isl[4 * stride] = g * inv_n;
        isl[5 * stride] = g * inv_n * inv_n;
    }

    template <typename T, int C>
    static CF_DEV HD<T, C> cos_term(const PointView<T>& pv, int k) {
        return cos_of(pv, pv.template y<C>(k), k);
    }
    // cos(2 pi y) by the chain rule of y -> cos(2 pi y): g = cos(2 pi x),
    // g' = -2 pi sin(2 pi x) (both from the point's tables), g'' = -4 pi^2 g
    template <typename T, int W>
    static CF_DEV HD<T, W> cos_of(const PointView<T>& pv, const HD1<T, W>& y, int k) {
        const T c = pv.tab0(k), c1 = pv.tab1(k);
        return chain(y, c, c1, T(-kTwoPi * kTwoPi) * c);
    }

    // As for Rosenbrock, the terms of variables outside the chunk carry no
    // chunk components, and term k = cs + m has the one chunk component m.
    // So each sum's component m is complete once its one window term is
    // added (to zero, exactly), and F's and G's chain rule is applied to it
    // right there; the sums' row-derivative components, to which every term
    // contributes, are formed first, in order of k.  The values are those of
    // the accumulated sums, and only the result's components stay live.  (The
    // sums' value components are never read: the chain takes F and G.)
    template <class P, int C>
    static CF_DEV HD<typename P::T, C> eval(const PointView<typename P::T>& pv, const FpParams&) {
        using T = typename P::T;
        T ssd = T(0), csd = T(0);
        for (int k = 0; k < pv.n; ++k) {
            const HD1<T, 0> y = pv.template y<0>(k);
            ssd += sq(y).d;
            csd += cos_term<T, 0>(pv, k).d;
        }
        // chain(a, g, g', g''): r.d = g' a.d, r.g = g' a.g, r.h = g' a.h + (g'' a.d) a.g;
        // F'' grows like 1 / |x|^3 near x = 0, so its product with the row
        // derivative (like 1 / |x|^2) is formed in float64 before it takes
        // the hDual precision
        const T f1 = pv.island(1), f2d = (T)(pv.island64(2) * (double)ssd);
        const T g1 = pv.island(4), g2d = (T)(pv.island64(5) * (double)csd);
        HD<T, C> r;
        r.v = (pv.island(0) + pv.island(3)) + T(20.0 + kE);
        r.d = f1 * ssd + g1 * csd;
        const int k0 = pv.cs, k1 = pv.cs + C < pv.n ? pv.cs + C : pv.n;
        static_for<C>([&](auto mc) {
            constexpr int m = decltype(mc)::value;
            const int k = k0 + m;
            if (k < k1) {
                const HD1<T, 1> y = pv.template y_at<1>(k, m);
                const HD<T, 1> st = sq(y), ct = cos_of(pv, y, k);
                r.g[m] = f1 * st.g[0] + g1 * ct.g[0];
                r.h[m] = (f1 * st.h[0] + f2d * st.g[0]) + (g1 * ct.h[0] + g2d * ct.g[0]);
            } else {
                r.g[m] = T(0);
                r.h[m] = T(0);
            }
        });
        return r;
    }

    // H.v chunk dot of call (i, cs).  The sums' row-derivative components
    // come from the one term in x_i, evaluated on the seed <x_i, 1, [i in
    // chunk], 0>; its second-order parts (the row seed times its own chunk
    // seed) are the sums' only ones, at slot i - cs.  The chunk's terms run on
    // seeds without the row part (<x_k, 0, 1, 0> at their slot, whose
    // second-order parts are exact zeros) and give the sums' gradient
    // components.  F's and G's chain rule then gives, per slot m,
    //   h[m] = F' S.h[m] + (F'' S.d) S.g[m] + G' C.h[m] + (G'' C.d) C.g[m]
    // with S.h, C.h nonzero only at slot i - cs: the gradient products are
    // dotted with v slot by slot, and the own slot's second-order products
    // with v_i (zero when x_i lies outside the chunk).
    template <class P, int C>
    static CF_DEV double hvp(const PointView<typename P::T>& pv, const FpParams&, const typename P::T* vrow) {
        using T = typename P::T;
        const int i = pv.i, cs = pv.cs;
        HD1<T, 1> yi;
        yi.v = pv.x(i);
        yi.d = T(1);
        yi.g[0] = (i >= cs && i < cs + C) ? T(1) : T(0);
        const HD<T, 1> si = sq(yi), ci = cos_of(pv, yi, i);
        const T f1 = pv.island(1), f2d = (T)(pv.island64(2) * (double)si.d);
        const T g1 = pv.island(4), g2d = (T)(pv.island64(5) * (double)ci.d);
        typename P::Dot acc;
        auto slot = [&](int k) {
            HD1<T, 1> y;
            y.v = pv.x(k);
            y.d = T(0);
            y.g[0] = T(1);
            const HD<T, 1> st = sq(y), ct = cos_of(pv, y, k);
            acc.add((f1 * st.h[0] + f2d * st.g[0]) + (g1 * ct.h[0] + g2d * ct.g[0]), vrow[k]);
        };
        if (cs + C <= pv.n) {
            static_for<C>([&](auto mc) { slot(cs + decltype(mc)::value); });
        } else {
            static_for<C>([&](auto mc) {
                const int k = cs + decltype(mc)::value;
                if (k < pv.n) slot(k);
            });
        }
        acc.add(f1 * si.h[0] + g1 * ci.h[0], vrow[i]);
        return acc.get();
    }

    // The call's second-order components h[m] from the same terms (for the
    // symmetric H.v): each slot's gradient products, and at slot i - cs the
    // own term's second-order products added to them.
    static constexpr bool kRowTerms = true;
    template <class P, int C>
    static CF_DEV void hrow(const PointView<typename P::T>& pv, const FpParams&, typename P::T (&h)[C]) {
        using T = typename P::T;
        const int i = pv.i, cs = pv.cs;
        HD1<T, 1> yi;
        yi.v = pv.x(i);
        yi.d = T(1);
        yi.g[0] = (i >= cs && i < cs + C) ? T(1) : T(0);
        const HD<T, 1> si = sq(yi), ci = cos_of(pv, yi, i);
        const T f1 = pv.island(1), f2d = (T)(pv.island64(2) * (double)si.d);
        const T g1 = pv.island(4), g2d = (T)(pv.island64(5) * (double)ci.d);
        const T own = f1 * si.h[0] + g1 * ci.h[0];
        static_for<C>([&](auto mc) {
            constexpr int m = decltype(mc)::value;
            const int k = cs + m;
            T hm = T(0);
            if (k < pv.n) {
                HD1<T, 1> y;
                y.v = pv.x(k);
                y.d = T(0);
                y.g[0] = T(1);
                const HD<T, 1> st = sq(y), ct = cos_of(pv, y, k);
                hm = f2d * st.g[0] + g2d * ct.g[0];
                if (k == i) hm += own;
            }
            h[m] = hm;
        });
    }
};

// sum_m (E_m - sum_j A_mj sin y_j + B_mj cos y_j)^2
struct FletcherPowell {
    static constexpr int kTables = 2;
    // t0 = sin(x), t1 = cos(x)
    static CF_DEV void tables(double x, double& t0, double& t1) { cf_sincos(x, &t0, &t1); }
    __host__ __device__ static int isl_tasks(int n) { return n; }
    __host__ __device__ static int isl_size(int n) { return n; }

    // float64 residual value r_m = E_m - sum_j A_mj sin x_j + B_mj cos x_j
    template <typename XT>
    static CF_DEV void island(int m, int n, const XT*, const double* t0, const double* t1, int stride,
                              const FpParams& prm, double* isl) {
        const double* Am = prm.A + (size_t)m * n;
        const double* Bm = prm.B + (size_t)m * n;
        double acc = Am[0] * t0[0];
        acc = acc + Bm[0] * t1[0];
        for (int j = 1; j < n; ++j) {
            acc = acc + Am[j] * t0[j * stride];
            acc = acc + Bm[j] * t1[j * stride];
        }
        isl[m * stride] = prm.E[m] - acc;
    }

    // the derivative components of inner_m = sum_j A_mj sin y_j + B_mj cos y_j;
    // its value is the per-point island
    template <typename T, int C>
    static CF_DEV HD<T, C> residual(const PointView<T>& pv, const FpParams& prm, int m) {
        const size_t row = (size_t)m * pv.n;
        HD1<T, C> y = pv.template y<C>(0);
        T s = pv.tab0(0), c = pv.tab1(0);
        HD<T, C> acc = fp_a<T>(prm, row) * chain(y, s, c, -s);
        acc = acc + fp_b<T>(prm, row) * chain(y, c, -s, -c);
        for (int j = 1; j < pv.n; ++j) {
            y = pv.template y<C>(j);
            s = pv.tab0(j);
            c = pv.tab1(j);
            acc = acc + fp_a<T>(prm, row + j) * chain(y, s, c, -s);
            acc = acc + fp_b<T>(prm, row + j) * chain(y, c, -s, -c);
        }
        HD<T, C> r = T(prm.E[m]) - acc;
        r.v = pv.island(m);
        return r;
    }

    template <class P, int C>
    static CF_DEV HD<typename P::T, C> eval(const PointView<typename P::T>& pv, const FpParams& prm) {
        using T = typename P::T;
        HD<T, C> r = residual<T, C>(pv, prm, 0);
        auto f = P::start(r * r);
        for (int m = 1; m < pv.n; ++m) {
            r = residual<T, C>(pv, prm, m);
            P::add(f, r * r);
        }
        return P::value(f);
    }

    // every residual depends on every variable: the full evaluation
    static constexpr bool kRowTerms = false;
    template <class P, int C>
    static CF_DEV double hvp(const PointView<typename P::T>& pv, const FpParams& prm, const typename P::T* vrow) {
        return eval_dot<P, FletcherPowell, C>(pv, prm, vrow);
    }
};

}  // namespace chessfad
