"""Brute-force Hessian with the four-component hDual (pure Python, tiny n).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Sec. III.A: an hDual <f, df/dx_i, df/dx_j, d2f/dx_i dx_j> carries one
Hessian entry through f.  The component rules for + and x and sin are the
ones the paper states; the other unary functions follow the same chain
rule, g(u) = <g(u0), g'(u0) u1, g'(u0) u2, g'(u0) u3 + g''(u0) u1 u2>, with
g, g', g'' from calculus (1/x, log, tan, tanh, atan, x^p, |x| among them);
a quotient is u * (1 / w).
INITIALIZE seeds y_k = <a_k, [k = i], [k = j], 0> and HESSIAN calls f once
per (i, j), n^2 calls in all.  This is independent of the closed forms and
of the chunked C code, so it pins both on small inputs.
"""
from __future__ import annotations

import math


class HD4:
    __slots__ = ("v",)

    def __init__(self, v0, v1=0.0, v2=0.0, v3=0.0):
        self.v = (float(v0), float(v1), float(v2), float(v3))

    # sum rule: every component adds (Sec. III.A)
    def __add__(self, o):
        if isinstance(o, HD4):
            a, b = self.v, o.v
            return HD4(a[0] + b[0], a[1] + b[1], a[2] + b[2], a[3] + b[3])
        a = self.v
        return HD4(a[0] + o, a[1], a[2], a[3])

    __radd__ = __add__

    def __neg__(self):
        a = self.v
        return HD4(-a[0], -a[1], -a[2], -a[3])

    def __sub__(self, o):
        return self + (-o)

    def __rsub__(self, o):
        return (-self) + o

    # product rule, first and second order (Sec. III.A)
    def __mul__(self, o):
        if isinstance(o, HD4):
            u, w = self.v, o.v
            return HD4(u[0] * w[0],
                       u[0] * w[1] + w[0] * u[1],
                       u[0] * w[2] + w[0] * u[2],
                       u[0] * w[3] + u[1] * w[2] + u[2] * w[1] + u[3] * w[0])
        a = self.v
        return HD4(o * a[0], o * a[1], o * a[2], o * a[3])

    __rmul__ = __mul__

    # quotient: u * (1 / w), the reciprocal by the chain rule
    def __truediv__(self, o):
        if isinstance(o, HD4):
            return self * HDMath.recip(o)
        return self * (1.0 / o)

    def __rtruediv__(self, o):
        return o * HDMath.recip(self)

    # comparisons follow the value
    def __lt__(self, o):
        return self.v[0] < (o.v[0] if isinstance(o, HD4) else o)

    def __gt__(self, o):
        return self.v[0] > (o.v[0] if isinstance(o, HD4) else o)


def _unary(u, g, g1, g2):
    a = u.v
    return HD4(g, g1 * a[1], g1 * a[2], g1 * a[3] + g2 * a[1] * a[2])


class HDMath:
    """sin/cos/exp/sqrt on HD4 through the chain rule."""

    @staticmethod
    def sin(u):
        x = u.v[0]
        return _unary(u, math.sin(x), math.cos(x), -math.sin(x))

    @staticmethod
    def cos(u):
        x = u.v[0]
        return _unary(u, math.cos(x), -math.sin(x), -math.cos(x))

    @staticmethod
    def exp(u):
        e = math.exp(u.v[0])
        return _unary(u, e, e, e)

    @staticmethod
    def sqrt(u):
        s = math.sqrt(u.v[0])
        return _unary(u, s, 0.5 / s, -0.25 / (s * u.v[0]))

    @staticmethod
    def recip(u):
        x = u.v[0]
        return _unary(u, 1.0 / x, -1.0 / (x * x), 2.0 / (x * x * x))

    @staticmethod
    def log(u):
        x = u.v[0]
        return _unary(u, math.log(x), 1.0 / x, -1.0 / (x * x))

    @staticmethod
    def tan(u):
        t = math.tan(u.v[0])
        return _unary(u, t, 1.0 + t * t, 2.0 * t * (1.0 + t * t))

    @staticmethod
    def tanh(u):
        t = math.tanh(u.v[0])
        return _unary(u, t, 1.0 - t * t, -2.0 * t * (1.0 - t * t))

    @staticmethod
    def atan(u):
        x = u.v[0]
        q = 1.0 / (1.0 + x * x)
        return _unary(u, math.atan(x), q, -2.0 * x * q * q)

    @staticmethod
    def pow(u, p):
        x = u.v[0]
        return _unary(u, x ** p, p * x ** (p - 1.0), p * (p - 1.0) * x ** (p - 2.0))

    @staticmethod
    def abs(u):
        return -u if u.v[0] < 0.0 else u


class FloatMath:
    sin = staticmethod(math.sin)
    cos = staticmethod(math.cos)
    exp = staticmethod(math.exp)
    sqrt = staticmethod(math.sqrt)
    log = staticmethod(math.log)
    tan = staticmethod(math.tan)
    tanh = staticmethod(math.tanh)
    atan = staticmethod(math.atan)
    pow = staticmethod(lambda x, p: x ** p)
    abs = staticmethod(abs)


# ------------------------------------------------ functions, generic in the number type
def rosenbrock(y, M, params=None):
    s = 0.0
    for k in range(len(y) - 1):
        t = y[k + 1] - y[k] * y[k]
        u = 1.0 - y[k]
        s = s + 100.0 * (t * t) + u * u
    return s


def ackley(y, M, params=None):
    n = len(y)
    ss = 0.0
    cs = 0.0
    for k in range(n):
        ss = ss + y[k] * y[k]
        cs = cs + M.cos((2.0 * math.pi) * y[k])
    rho = M.sqrt(ss * (1.0 / n))
    return (-20.0) * M.exp((-0.2) * rho) - M.exp(cs * (1.0 / n)) + 20.0 + math.e


def fletcher_powell(y, M, params):
    A, B, E = params
    n = len(y)
    s = 0.0
    for m in range(n):
        inner = 0.0
        for j in range(n):
            inner = inner + float(A[m][j]) * M.sin(y[j]) + float(B[m][j]) * M.cos(y[j])
        r = float(E[m]) - inner
        s = s + r * r
    return s


FUNCS = (rosenbrock, ackley, fletcher_powell)


def initialize(a, i, j):
    """INITIALIZE: y_k = <a_k, [k = i], [k = j], 0>."""
    return [HD4(a[k], 1.0 if k == i else 0.0, 1.0 if k == j else 0.0, 0.0) for k in range(len(a))]


def hessian(func, a, params=None):
    """HESSIAN: one f call per (i, j); H[i][j] is the fourth component.
    func is one of the three test functions' ids or a callable f(y, M, params)."""
    f = FUNCS[func] if isinstance(func, int) else func
    n = len(a)
    H = [[0.0] * n for _ in range(n)]
    for i in range(n):
        for j in range(n):
            H[i][j] = f(initialize(a, i, j), HDMath, params).v[3]
    return H


def value_and_gradient(func, a, params=None):
    """f and the gradient from the first-order components of the same calls."""
    f = FUNCS[func]
    n = len(a)
    g = [0.0] * n
    val = None
    for i in range(n):
        r = f(initialize(a, i, i), HDMath, params)
        val = r.v[0]
        g[i] = r.v[1]
    return val, g


def value(func, a, params=None):
    return FUNCS[func]([float(t) for t in a], FloatMath, params)
