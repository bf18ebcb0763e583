// Register-resident hDual<C> for gfx950 kernels.
//
// An hDual with chunk size C (Sec. III.B, Sec. IV) holds 2C + 2 numbers:
//   v      the value
//   d      the derivative along the row variable x_i
//   g[l]   the derivatives along the chunk's columns x_{cs+l}, l < C
//   h[l]   the second derivatives d2/(dx_i dx_{cs+l})
// Every field is a named scalar so the whole value lives in VGPRs (4C + 4
// of them in float64); nothing is indexed dynamically.
//
// Operator rules (Sec. III.A, Fig. 1): sums act componentwise; the product
// is u0 w + w0 u on the first-order part and
//   u0 w_h + u_d w_g + w_d u_g + w0 u_h
// on the second-order part; a unary g(u) is the chain rule
//   <g, g' u_d, g' u_g, g' u_h + g'' u_d u_g>
// where g, g', g'' are scalars the caller supplies (so transcendental values
// that every call of a point shares can be computed once per point).
// HD1 below is the same number with its second-order part statically zero.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>
#include <utility>

namespace chessfad {

#define CF_DEV __device__ __forceinline__

// fn(std::integral_constant<int, I>{}) for I = 0 .. N - 1, in order: a loop
// whose index is a compile-time constant in the body
template <class Fn, int... I>
CF_DEV void static_for_impl(Fn&& fn, std::integer_sequence<int, I...>) {
    (fn(std::integral_constant<int, I>{}), ...);
}
template <int N, class Fn>
CF_DEV void static_for(Fn&& fn) {
    static_for_impl(fn, std::make_integer_sequence<int, N>{});
}

// HD<T, 0> (value and row derivative only) carries a term whose seeds have
// no component in the call's chunk: its g and h parts are exact zeros.
template <typename T, int C>
struct HD {
    T v, d;
    T g[C], h[C];
};
template <typename T>
struct HD<T, 0> {
    T v, d;
    T g[1], h[1];   // never read: every loop over the chunk has zero trips
};

template <typename T, int C>
CF_DEV HD<T, C> zero_hd() {
    HD<T, C> r;
    r.v = T(0);
    r.d = T(0);
#pragma unroll
    for (int l = 0; l < C; ++l) r.g[l] = r.h[l] = T(0);
    return r;
}

template <typename T, int C>
CF_DEV HD<T, C> operator+(const HD<T, C>& a, const HD<T, C>& b) {
    HD<T, C> r;
    r.v = a.v + b.v;
    r.d = a.d + b.d;
#pragma unroll
    for (int l = 0; l < C; ++l) {
        r.g[l] = a.g[l] + b.g[l];
        r.h[l] = a.h[l] + b.h[l];
    }
    return r;
}

template <typename T, int C>
CF_DEV HD<T, C> operator-(const HD<T, C>& a, const HD<T, C>& b) {
    HD<T, C> r;
    r.v = a.v - b.v;
    r.d = a.d - b.d;
#pragma unroll
    for (int l = 0; l < C; ++l) {
        r.g[l] = a.g[l] - b.g[l];
        r.h[l] = a.h[l] - b.h[l];
    }
    return r;
}

template <typename T, int C>
CF_DEV HD<T, C> operator*(const HD<T, C>& a, const HD<T, C>& b) {
    HD<T, C> r;
    r.v = a.v * b.v;
    r.d = a.v * b.d + b.v * a.d;
#pragma unroll
    for (int l = 0; l < C; ++l) {
        r.g[l] = a.v * b.g[l] + b.v * a.g[l];
        r.h[l] = a.v * b.h[l] + a.d * b.g[l] + b.d * a.g[l] + b.v * a.h[l];
    }
    return r;
}

// scalar x hDual scales every component
template <typename T, int C>
CF_DEV HD<T, C> operator*(T s, const HD<T, C>& a) {
    HD<T, C> r;
    r.v = s * a.v;
    r.d = s * a.d;
#pragma unroll
    for (int l = 0; l < C; ++l) {
        r.g[l] = s * a.g[l];
        r.h[l] = s * a.h[l];
    }
    return r;
}

// scalar + hDual changes only the value
template <typename T, int C>
CF_DEV HD<T, C> operator+(const HD<T, C>& a, T s) {
    HD<T, C> r = a;
    r.v = a.v + s;
    return r;
}

// scalar - hDual: value subtracts, the derivatives change sign
template <typename T, int C>
CF_DEV HD<T, C> operator-(T s, const HD<T, C>& a) {
    HD<T, C> r;
    r.v = s - a.v;
    r.d = -a.d;
#pragma unroll
    for (int l = 0; l < C; ++l) {
        r.g[l] = -a.g[l];
        r.h[l] = -a.h[l];
    }
    return r;
}

// chain rule with caller-supplied g(u0), g'(u0), g''(u0)
template <typename T, int C>
CF_DEV HD<T, C> chain(const HD<T, C>& a, T g0, T g1, T g2) {
    HD<T, C> r;
    r.v = g0;
    r.d = g1 * a.d;
    const T g2d = g2 * a.d;
#pragma unroll
    for (int l = 0; l < C; ++l) {
        r.g[l] = g1 * a.g[l];
        r.h[l] = g1 * a.h[l] + g2d * a.g[l];
    }
    return r;
}

// ------------------------------------------------------- first-order hDuals
// An hDual whose second-order part is statically zero: the CHUNK-INIT seeds
// and values that are affine in them (sums, scalings).  Its operators are the
// rules above with the products against that zero part left out; the values
// they produce are the same (a product with an exact zero adds nothing, up
// to the sign of a zero result).
template <typename T, int C>
struct HD1 {
    T v, d;
    T g[C];
};
template <typename T>
struct HD1<T, 0> {
    T v, d;
    T g[1];   // never read
};

// CHUNK-INIT for one variable: y_k = <x_k, [k = i], [k = cs + l], 0>.
template <typename T, int C>
CF_DEV HD1<T, C> seed(T xk, int k, int i, int cs) {
    HD1<T, C> y;
    y.v = xk;
    y.d = (k == i) ? T(1) : T(0);
    const int u = k - cs;
#pragma unroll
    for (int l = 0; l < C; ++l) y.g[l] = (u == l) ? T(1) : T(0);
    return y;
}

template <typename T, int C>
CF_DEV HD<T, C> widen(const HD1<T, C>& a) {
    HD<T, C> r;
    r.v = a.v;
    r.d = a.d;
#pragma unroll
    for (int l = 0; l < C; ++l) {
        r.g[l] = a.g[l];
        r.h[l] = T(0);
    }
    return r;
}

template <typename T, int C>
CF_DEV HD1<T, C> operator*(T s, const HD1<T, C>& a) {
    HD1<T, C> r;
    r.v = s * a.v;
    r.d = s * a.d;
#pragma unroll
    for (int l = 0; l < C; ++l) r.g[l] = s * a.g[l];
    return r;
}

template <typename T, int C>
CF_DEV HD1<T, C> operator-(T s, const HD1<T, C>& a) {
    HD1<T, C> r;
    r.v = s - a.v;
    r.d = -a.d;
#pragma unroll
    for (int l = 0; l < C; ++l) r.g[l] = -a.g[l];
    return r;
}

// product of two first-order hDuals: second-order part u_d w_g + w_d u_g
template <typename T, int C>
CF_DEV HD<T, C> operator*(const HD1<T, C>& a, const HD1<T, C>& b) {
    HD<T, C> r;
    r.v = a.v * b.v;
    r.d = a.v * b.d + b.v * a.d;
#pragma unroll
    for (int l = 0; l < C; ++l) {
        r.g[l] = a.v * b.g[l] + b.v * a.g[l];
        r.h[l] = a.d * b.g[l] + b.d * a.g[l];
    }
    return r;
}

// u * u for a first-order value: the product rule's pairs of equal products
// (u.v u' + u' u.v, u.d u.g + u.g u.d) are each one product with a doubled
// factor; doubling is exact, so the values are those of the two products added
template <typename T, int C>
CF_DEV HD<T, C> sq(const HD1<T, C>& a) {
    HD<T, C> r;
    const T v2 = a.v + a.v, d2 = a.d + a.d;
    r.v = a.v * a.v;
    r.d = v2 * a.d;
#pragma unroll
    for (int l = 0; l < C; ++l) {
        r.g[l] = v2 * a.g[l];
        r.h[l] = d2 * a.g[l];
    }
    return r;
}

// u * u for a full value: as above, with the second-order part
// (2 u.v) u.h + (2 u.d) u.g, the product rule's four terms paired the same way
template <typename T, int C>
CF_DEV HD<T, C> sq(const HD<T, C>& a) {
    HD<T, C> r;
    const T v2 = a.v + a.v, d2 = a.d + a.d;
    r.v = a.v * a.v;
    r.d = v2 * a.d;
#pragma unroll
    for (int l = 0; l < C; ++l) {
        r.g[l] = v2 * a.g[l];
        r.h[l] = v2 * a.h[l] + d2 * a.g[l];
    }
    return r;
}

// first-order minus full: the second-order part is the negated one of b
template <typename T, int C>
CF_DEV HD<T, C> operator-(const HD1<T, C>& a, const HD<T, C>& b) {
    HD<T, C> r;
    r.v = a.v - b.v;
    r.d = a.d - b.d;
#pragma unroll
    for (int l = 0; l < C; ++l) {
        r.g[l] = a.g[l] - b.g[l];
        r.h[l] = -b.h[l];
    }
    return r;
}

// chain rule on a first-order hDual: <g, g' u_d, g' u_g, g'' u_d u_g>
template <typename T, int C>
CF_DEV HD<T, C> chain(const HD1<T, C>& a, T g0, T g1, T g2) {
    HD<T, C> r;
    r.v = g0;
    r.d = g1 * a.d;
    const T g2d = g2 * a.d;
#pragma unroll
    for (int l = 0; l < C; ++l) {
        r.g[l] = g1 * a.g[l];
        r.h[l] = g2d * a.g[l];
    }
    return r;
}

}  // namespace chessfad

namespace chessfad {

// ---------------------------------------------------------------- precision
// Error-free transformation: Knuth's two-sum.
// The _rn intrinsics keep the compiler from contracting a neighbouring
// multiply into these additions, which would break the exact error terms.
CF_DEV void two_sum(float a, float b, float& s, float& e) {
    s = __fadd_rn(a, b);
    const float bb = __fsub_rn(s, a);
    e = __fadd_rn(__fsub_rn(a, __fsub_rn(s, bb)), __fsub_rn(b, bb));
}

// Plain float64 hDuals: accumulations are ordinary hDual sums.
struct F64 {
    using T = double;
    template <int C>
    struct Acc {
        HD<double, C> x;
    };
    template <int C>
    static CF_DEV Acc<C> start(const HD<T, C>& t) { return Acc<C>{t}; }
    template <int C>
    static CF_DEV void add(Acc<C>& a, const HD<T, C>& t) { a.x = a.x + t; }
    // a term with no component in the chunk: value and row derivative only
    template <int C>
    static CF_DEV void add_light(Acc<C>& a, const HD<T, 0>& t) {
        a.x.v += t.v;
        a.x.d += t.d;
    }
    // a term whose chunk components other than M .. M + W - 1 are exact
    // zeros, given as those W; slots outside [0, C) are skipped
    template <int M, int C, int W>
    static CF_DEV void add_at(Acc<C>& a, const HD<T, W>& t) {
        a.x.v += t.v;
        a.x.d += t.d;
#pragma unroll
        for (int w = 0; w < W; ++w)
            if (M + w >= 0 && M + w < C) {
                a.x.g[M + w] += t.g[w];
                a.x.h[M + w] += t.h[w];
            }
    }
    template <int C>
    static CF_DEV HD<T, C> value(const Acc<C>& a) { return a.x; }
    // chunk dot sum_l h[l] v[l]
    struct Dot {
        double s = 0.0;
        CF_DEV void add(T a, T b) { s += a * b; }
        CF_DEV double get() const { return s; }
    };
};

// float32 hDuals whose Hessian-chunk components are accumulated with
// two-sum compensation (a running low part per component); the chunk dot is
// float64.
struct F32C {
    using T = float;
    template <int C>
    struct Acc {
        HD<float, C> x;
        float lo[C];
    };
    template <int C>
    static CF_DEV Acc<C> start(const HD<T, C>& t) {
        Acc<C> a;
        a.x = t;
#pragma unroll
        for (int l = 0; l < C; ++l) a.lo[l] = 0.0f;
        return a;
    }
    template <int C>
    static CF_DEV void add(Acc<C>& a, const HD<T, C>& t) {
        a.x.v += t.v;
        a.x.d += t.d;
#pragma unroll
        for (int l = 0; l < C; ++l) {
            a.x.g[l] += t.g[l];
            float s, e;
            two_sum(a.x.h[l], t.h[l], s, e);
            a.x.h[l] = s;
            a.lo[l] += e;
        }
    }
    template <int C>
    static CF_DEV void add_light(Acc<C>& a, const HD<T, 0>& t) {
        a.x.v += t.v;
        a.x.d += t.d;
    }
    // A term given as its chunk components M .. M + W - 1 (the others exact
    // zeros; slots outside [0, C) are skipped), into a sum whose every
    // Hessian-chunk component receives at most two nonzero terms: a two-sum
    // pair (s, e) of two terms has s + e = a + b exactly, so value() returns
    // round(a + b) = s, which is what the rounded plain sum gives.  The low
    // part is skipped; the adds are kept apart from the terms' products, as
    // in two_sum.
    template <int M, int C, int W>
    static CF_DEV void add_at(Acc<C>& a, const HD<T, W>& t) {
        a.x.v += t.v;
        a.x.d += t.d;
#pragma unroll
        for (int w = 0; w < W; ++w)
            if (M + w >= 0 && M + w < C) {
                a.x.g[M + w] += t.g[w];
                a.x.h[M + w] = __fadd_rn(a.x.h[M + w], t.h[w]);
            }
    }
    template <int C>
    static CF_DEV HD<T, C> value(const Acc<C>& a) {
        HD<T, C> r = a.x;
#pragma unroll
        for (int l = 0; l < C; ++l) r.h[l] = a.x.h[l] + a.lo[l];
        return r;
    }
    // the chunk dot in float64: a float32 x float32 product is exact in
    // float64, so each term is exact and only the float64 sum rounds
    struct Dot {
        double s = 0.0;
        CF_DEV void add(T a, T b) { s += (double)a * (double)b; }
        CF_DEV double get() const { return s; }
    };
};

}  // namespace chessfad
