"""Facts the mixed-precision kernels rely on, checked on the CPU.

Rosenbrock's and Ackley's sums over k give each second-order component
(i, j) at most two (Rosenbrock) or one (Ackley) nonzero term; the other
terms are exact zeros.  A two-sum compensated float32 sum of such a sequence
returns exactly the plain float32 sum: after the second nonzero term the pair
(s, e) has s + e = a + b exactly, so rounding s + e gives round(a + b) = s.
The kernels therefore skip the low part there (the result is the same bits)
and keep the compensation where many terms are nonzero.
"""
import math

import numpy as np
import pytest

from oracle import hyperdual as hd

f32 = np.float32


def _two_sum(a, b):
    s = f32(a + b)
    bb = f32(s - a)
    e = f32(f32(a - f32(s - bb)) + f32(b - bb))
    return s, e


def _compensated(terms):
    hi, lo = f32(0), f32(0)
    for t in terms:
        hi, e = _two_sum(hi, t)
        lo = f32(lo + e)
    return f32(hi + lo)


def _plain(terms):
    s = f32(0)
    for t in terms:
        s = f32(s + t)
    return s


def test_two_sum_is_error_free():
    rng = np.random.default_rng(5)
    a = (rng.standard_normal(20000) * 10.0 ** rng.integers(-8, 8, 20000)).astype(f32)
    b = (rng.standard_normal(20000) * 10.0 ** rng.integers(-8, 8, 20000)).astype(f32)
    for x, y in zip(a, b):
        s, e = _two_sum(x, y)
        assert float(s) + float(e) == float(x) + float(y)   # exact in float64 for float32 inputs


@pytest.mark.parametrize("nonzero", [1, 2])
def test_compensated_sum_of_at_most_two_terms_is_the_plain_sum(nonzero):
    rng = np.random.default_rng(11 + nonzero)
    for _ in range(5000):
        terms = [f32(0.0)] * 16
        for pos in rng.choice(16, nonzero, replace=False):
            terms[pos] = f32(rng.standard_normal() * 10.0 ** rng.integers(-6, 6))
        assert _compensated(terms) == _plain(terms)
    # with three nonzero terms the two can differ: the low part then matters
    diff = 0
    for _ in range(5000):
        t = [f32(rng.standard_normal() * 10.0 ** rng.integers(-6, 6)) for _ in range(3)]
        diff += _compensated(t) != _plain(t)
    assert diff > 0


def _second_order_terms(func, n, i, j, a):
    """Second-order component (i, j) of every summand of f, by hyper-dual
    evaluation of the summands one at a time."""
    y = hd.initialize(a, i, j)
    M = hd.HDMath
    if func == 0:
        out = []
        for k in range(n - 1):
            t = y[k + 1] - y[k] * y[k]
            u = 1.0 - y[k]
            out.append((100.0 * (t * t) + u * u).v[3])
        return out
    return [(y[k] * y[k]).v[3] for k in range(n)] + [M.cos((2.0 * math.pi) * y[k]).v[3] for k in range(n)]


@pytest.mark.parametrize("func,most", [(0, 2), (1, 1)])
def test_sparse_second_order_terms(func, most):
    n = 9
    a = np.random.default_rng(3 + func).uniform(-2, 2, n)
    for i in range(n):
        for j in range(n):
            terms = _second_order_terms(func, n, i, j, a)
            if func == 0:
                assert sum(t != 0.0 for t in terms) <= most
            else:
                # each of Ackley's two sums separately
                assert sum(t != 0.0 for t in terms[:n]) <= most
                assert sum(t != 0.0 for t in terms[n:]) <= most
