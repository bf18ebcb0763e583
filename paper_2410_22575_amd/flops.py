"""Operation-count model of the chunked method (Sec. V), per Hessian-vector product.

Scalar operations per hDual<c> operation, counted the way the operator
rules are written (Sec. V, Fig. 1):
  hDual + hDual        2c + 2 additions
  hDual x hDual        6c + 3 multiplications and 4c + 1 additions
                       (Sec. V states 4c additions; the product rule as
                       written has c + 1 in the first-order part and 3c in
                       the second-order part)
  double x hDual       2c + 2 multiplications
  double +/- hDual     1 addition (only the value changes; the rest is a copy
                       or a sign change)
  unary g(hDual)       4c + 2 (c + 1 first-order multiplications, one for
                       g'' u_1, then a multiply and a multiply-add per
                       second-order component); the scalar values g, g', g''
                       are per-point work and not counted
  chunk dot with v     2c
One f call per (row, chunk): n * ceil(n / c) calls per point (CHUNK-HESS,
CHESS-VEC).  The symmetric forms (SCHUNK-HESS, SC-HESS-VEC) evaluate only
the chunks from a row's own chunk onwards, n (n / c + 1) / 2 calls when c
divides n (Sec. V), and each call right of the own chunk adds a mirror update
(another 2c).  The per-call totals below follow the operation sequence of the
three functions as the kernels evaluate them.
"""
from __future__ import annotations

ROSENBROCK, ACKLEY, FLETCHER_POWELL = 0, 1, 2


def calls_per_point(n: int, c: int) -> int:
    return n * ((n + c - 1) // c)


def calls_per_point_sym(n: int, c: int) -> int:
    nc = (n + c - 1) // c
    return sum(nc - i // c for i in range(n))


def flops_per_call(func: int, n: int, c: int) -> int:
    hadd = 2 * c + 2
    hmul = 10 * c + 4
    scal = 2 * c + 2
    unary = 4 * c + 2
    dot = 2 * c
    if func == ROSENBROCK:
        # per term: y^2, sub, square, 100x, 1-y, square, add, accumulate
        per_term = 3 * hmul + 3 * hadd + scal + 1
        return (n - 1) * per_term - hadd + dot
    if func == ACKLEY:
        # per k: y^2, accumulate, 2 pi x, cos, accumulate; then 4 scalings,
        # sqrt, 2 exp, one subtraction and the constant 20 + e
        per_k = hmul + hadd + scal + unary + hadd
        return n * per_k - 2 * hadd + 4 * scal + 3 * unary + hadd + 1 + dot
    if func == FLETCHER_POWELL:
        # 2n unary (sin, cos of each y_j); per residual m: 2n scalings and
        # 2n - 1 additions, E_m - inner, square; n - 1 accumulations
        per_m = 2 * n * scal + (2 * n - 1) * hadd + 1 + hmul
        return 2 * n * unary + n * per_m + (n - 1) * hadd + dot
    raise ValueError(func)


def flops_per_hvp(func: int, n: int, c: int) -> int:
    return calls_per_point(n, c) * flops_per_call(func, n, c)


def flops_per_hvp_sym(func: int, n: int, c: int) -> int:
    calls = calls_per_point_sym(n, c)
    return calls * flops_per_call(func, n, c) + (calls - n) * 2 * c


def contraction_flops_per_hvp(func: int, n: int, c: int) -> int:
    """The part of Fletcher-Powell's count that is the dense [A B] . [sin y; cos y]
    contraction over hDual components (M = n, K = 2n, N = 2c + 2 per call)."""
    if func != FLETCHER_POWELL:
        return 0
    return calls_per_point(n, c) * n * (2 * n * (2 * c + 2) + (2 * n - 1) * (2 * c + 2))
