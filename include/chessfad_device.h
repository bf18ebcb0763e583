/*
 * chessfad_device.h - the hDual number type for user functions (device code).
 *
 * A user function is written once, templated on the number type, and the
 * library evaluates it on hDuals (Sec. III.A, Sec. III.B): chunked
 * forward-mode second-order AD.  Register it with chessfad_register_function
 * (chessfad.h); the library compiles it at run time together with this
 * header and runs it in its H.v / Hessian kernels.  The function must have
 * the form
 *
 *     template <class V, class Y>
 *     __device__ V chessfad_user_f(const Y& y, int n)
 *     {
 *         V s = 0.0;
 *         for (int k = 0; k + 1 < n; ++k) s += 100.0 * sq(y[k + 1] - y[k] * y[k]) + sq(1.0 - y[k]);
 *         return s;
 *     }
 *
 * where y[k] (k < n) is the k-th variable as an hDual V and the result is f.
 * Every operator below acts on all 2C + 2 components:
 *
 *   hdual<C> u  holds   v       value
 *                       d       d/dx_i          (i = the Hessian row)
 *                       g[l]    d/dx_{cs+l}     (the chunk's columns)
 *                       h[l]    d2/dx_i dx_{cs+l}
 *
 *   +, -            componentwise; a double changes only the value
 *   *               product rule: value u0 w0, first order u0 w' + w0 u',
 *                   second order u0 w_h + u_d w_g + w_d u_g + w0 u_h
 *   /               u * (1 / w), the reciprocal by the chain rule
 *   sqrt exp log sin cos tan tanh atan pow(u, p) abs sq
 *                   the chain rule g(u) = <g, g' u_d, g' u_g, g' u_h + g'' u_d u_g>
 *   < > <= >= == !=  compare values (branches follow the value, as in the
 *                   paper's scalar code; derivatives are those of the branch taken)
 *
 * abs is not differentiable at 0; there it returns the derivative of +u.
 * Division by a zero value, log of a non-positive value, sqrt of a
 * non-positive value and pow with non-positive base produce IEEE inf / NaN.
 */
#ifndef CHESSFAD_DEVICE_H
#define CHESSFAD_DEVICE_H

namespace chessfad {

#define CHESSFAD_HD __device__ __forceinline__

template <int C>
struct hdual {
    double v, d;
    double g[C], h[C];

    CHESSFAD_HD hdual() : v(0.0), d(0.0) {
        for (int l = 0; l < C; ++l) g[l] = h[l] = 0.0;
    }
    // a constant: every derivative is zero
    CHESSFAD_HD hdual(double c) : v(c), d(0.0) {
        for (int l = 0; l < C; ++l) g[l] = h[l] = 0.0;
    }
    CHESSFAD_HD hdual& operator+=(const hdual& o);
    CHESSFAD_HD hdual& operator-=(const hdual& o);
    CHESSFAD_HD hdual& operator*=(const hdual& o);
    CHESSFAD_HD hdual& operator/=(const hdual& o);
};

template <int C>
CHESSFAD_HD double value(const hdual<C>& u) { return u.v; }
CHESSFAD_HD double value(double u) { return u; }

// chain rule with g(u0), g'(u0), g''(u0)
template <int C>
CHESSFAD_HD hdual<C> apply(const hdual<C>& u, double g0, double g1, double g2) {
    hdual<C> r;
    r.v = g0;
    r.d = g1 * u.d;
    const double g2d = g2 * u.d;
    for (int l = 0; l < C; ++l) {
        r.g[l] = g1 * u.g[l];
        r.h[l] = g1 * u.h[l] + g2d * u.g[l];
    }
    return r;
}

template <int C>
CHESSFAD_HD hdual<C> operator+(const hdual<C>& a, const hdual<C>& b) {
    hdual<C> r;
    r.v = a.v + b.v;
    r.d = a.d + b.d;
    for (int l = 0; l < C; ++l) {
        r.g[l] = a.g[l] + b.g[l];
        r.h[l] = a.h[l] + b.h[l];
    }
    return r;
}
template <int C>
CHESSFAD_HD hdual<C> operator-(const hdual<C>& a) {
    hdual<C> r;
    r.v = -a.v;
    r.d = -a.d;
    for (int l = 0; l < C; ++l) {
        r.g[l] = -a.g[l];
        r.h[l] = -a.h[l];
    }
    return r;
}
template <int C>
CHESSFAD_HD hdual<C> operator-(const hdual<C>& a, const hdual<C>& b) {
    hdual<C> r;
    r.v = a.v - b.v;
    r.d = a.d - b.d;
    for (int l = 0; l < C; ++l) {
        r.g[l] = a.g[l] - b.g[l];
        r.h[l] = a.h[l] - b.h[l];
    }
    return r;
}
template <int C>
CHESSFAD_HD hdual<C> operator*(const hdual<C>& a, const hdual<C>& b) {
    hdual<C> r;
    r.v = a.v * b.v;
    r.d = a.v * b.d + b.v * a.d;
    for (int l = 0; l < C; ++l) {
        r.g[l] = a.v * b.g[l] + b.v * a.g[l];
        r.h[l] = a.v * b.h[l] + a.d * b.g[l] + b.d * a.g[l] + b.v * a.h[l];
    }
    return r;
}

// mixed with doubles: a double is a constant hDual, so only the value moves
// under + and -, and * scales every component
template <int C>
CHESSFAD_HD hdual<C> operator+(const hdual<C>& a, double s) {
    hdual<C> r = a;
    r.v = a.v + s;
    return r;
}
template <int C>
CHESSFAD_HD hdual<C> operator+(double s, const hdual<C>& a) {
    hdual<C> r = a;
    r.v = s + a.v;
    return r;
}
template <int C>
CHESSFAD_HD hdual<C> operator-(const hdual<C>& a, double s) {
    hdual<C> r = a;
    r.v = a.v - s;
    return r;
}
template <int C>
CHESSFAD_HD hdual<C> operator-(double s, const hdual<C>& a) {
    hdual<C> r = -a;
    r.v = s - a.v;
    return r;
}
template <int C>
CHESSFAD_HD hdual<C> operator*(double s, const hdual<C>& a) {
    hdual<C> r;
    r.v = s * a.v;
    r.d = s * a.d;
    for (int l = 0; l < C; ++l) {
        r.g[l] = s * a.g[l];
        r.h[l] = s * a.h[l];
    }
    return r;
}
template <int C>
CHESSFAD_HD hdual<C> operator*(const hdual<C>& a, double s) { return s * a; }

// 1 / w: g = 1/w0, g' = -1/w0^2, g'' = 2/w0^3
template <int C>
CHESSFAD_HD hdual<C> recip(const hdual<C>& w) {
    const double r = 1.0 / w.v;
    return apply(w, r, -r * r, 2.0 * r * r * r);
}
template <int C>
CHESSFAD_HD hdual<C> operator/(const hdual<C>& a, const hdual<C>& b) { return a * recip(b); }
template <int C>
CHESSFAD_HD hdual<C> operator/(const hdual<C>& a, double s) { return (1.0 / s) * a; }
template <int C>
CHESSFAD_HD hdual<C> operator/(double s, const hdual<C>& b) { return s * recip(b); }

template <int C>
CHESSFAD_HD hdual<C>& hdual<C>::operator+=(const hdual<C>& o) { return *this = *this + o; }
template <int C>
CHESSFAD_HD hdual<C>& hdual<C>::operator-=(const hdual<C>& o) { return *this = *this - o; }
template <int C>
CHESSFAD_HD hdual<C>& hdual<C>::operator*=(const hdual<C>& o) { return *this = *this * o; }
template <int C>
CHESSFAD_HD hdual<C>& hdual<C>::operator/=(const hdual<C>& o) { return *this = *this / o; }

// comparisons on values
#define CHESSFAD_CMP(op)                                                                              \
    template <int C>                                                                                  \
    CHESSFAD_HD bool operator op(const hdual<C>& a, const hdual<C>& b) { return a.v op b.v; }         \
    template <int C>                                                                                  \
    CHESSFAD_HD bool operator op(const hdual<C>& a, double b) { return a.v op b; }                    \
    template <int C>                                                                                  \
    CHESSFAD_HD bool operator op(double a, const hdual<C>& b) { return a op b.v; }
CHESSFAD_CMP(<)
CHESSFAD_CMP(>)
CHESSFAD_CMP(<=)
CHESSFAD_CMP(>=)
CHESSFAD_CMP(==)
CHESSFAD_CMP(!=)
#undef CHESSFAD_CMP

// unary functions by the chain rule
template <int C>
CHESSFAD_HD hdual<C> sq(const hdual<C>& u) { return u * u; }
template <int C>
CHESSFAD_HD hdual<C> sqrt(const hdual<C>& u) {
    const double s = ::sqrt(u.v);
    return apply(u, s, 0.5 / s, -0.25 / (s * u.v));
}
template <int C>
CHESSFAD_HD hdual<C> exp(const hdual<C>& u) {
    const double e = ::exp(u.v);
    return apply(u, e, e, e);
}
template <int C>
CHESSFAD_HD hdual<C> log(const hdual<C>& u) {
    const double r = 1.0 / u.v;
    return apply(u, ::log(u.v), r, -r * r);
}
template <int C>
CHESSFAD_HD hdual<C> sin(const hdual<C>& u) {
    double s, c;
    ::sincos(u.v, &s, &c);
    return apply(u, s, c, -s);
}
template <int C>
CHESSFAD_HD hdual<C> cos(const hdual<C>& u) {
    double s, c;
    ::sincos(u.v, &s, &c);
    return apply(u, c, -s, -c);
}
template <int C>
CHESSFAD_HD hdual<C> tan(const hdual<C>& u) {
    const double t = ::tan(u.v), sec2 = 1.0 + t * t;
    return apply(u, t, sec2, 2.0 * t * sec2);
}
template <int C>
CHESSFAD_HD hdual<C> tanh(const hdual<C>& u) {
    const double t = ::tanh(u.v), s = 1.0 - t * t;
    return apply(u, t, s, -2.0 * t * s);
}
template <int C>
CHESSFAD_HD hdual<C> atan(const hdual<C>& u) {
    const double q = 1.0 / (1.0 + u.v * u.v);
    return apply(u, ::atan(u.v), q, -2.0 * u.v * q * q);
}
// u^p for a constant exponent p
template <int C>
CHESSFAD_HD hdual<C> pow(const hdual<C>& u, double p) {
    return apply(u, ::pow(u.v, p), p * ::pow(u.v, p - 1.0), p * (p - 1.0) * ::pow(u.v, p - 2.0));
}
template <int C>
CHESSFAD_HD hdual<C> abs(const hdual<C>& u) {
    return u.v < 0.0 ? -u : u;
}

}  // namespace chessfad

#endif  // CHESSFAD_DEVICE_H
