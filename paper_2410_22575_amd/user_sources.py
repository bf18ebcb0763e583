"""The three test functions written as user functions: f once, templated on
the number type, over the hDual of include/chessfad_device.h (the paper's
library surface, Sec. I and Sec. IV), for chessfad_register_function.

The library runs such a function on its generic kernel (every hDual
operation of f evaluated in every call), so these measure the general method
beside the built-in, hand-specialised evaluations.  Fletcher-Powell's
constants have no argument slot in a user function: its source carries A, B
and E for one parameter set as constant arrays.
"""
from __future__ import annotations

import numpy as np

ROSENBROCK_HIP = """
template <class V, class Y> __device__ V chessfad_user_f(const Y& y, int n) {
    V s = 0.0;
    for (int k = 0; k + 1 < n; ++k) s += 100.0 * sq(y[k + 1] - y[k] * y[k]) + sq(1.0 - y[k]);
    return s;
}
"""

ACKLEY_HIP = """
template <class V, class Y> __device__ V chessfad_user_f(const Y& y, int n) {
    V ss = 0.0, cs = 0.0;
    for (int k = 0; k < n; ++k) {
        ss += y[k] * y[k];
        cs += cos(6.283185307179586 * y[k]);
    }
    return -20.0 * exp(-0.2 * sqrt(ss / (double)n)) - exp(cs / (double)n) + 20.0 + 2.718281828459045;
}
"""


def _array(name: str, values) -> str:
    body = ", ".join(repr(float(v)) for v in np.asarray(values, dtype=np.float64).ravel())
    return f"__device__ const double {name}[] = {{{body}}};\n"


def fletcher_powell_hip(A: np.ndarray, B: np.ndarray, E: np.ndarray) -> str:
    """Fletcher-Powell for the parameter set (A, B, E), n = len(E):
    f = sum_m (E_m - sum_j A_mj sin y_j + B_mj cos y_j)^2."""
    n = len(E)
    src = _array("kA", A) + _array("kB", B) + _array("kE", E)
    src += f"""
template <class V, class Y> __device__ V chessfad_user_f(const Y& y, int n) {{
    // n is {n}: the constants are [{n}][{n}]
    V f = 0.0;
    for (int m = 0; m < {n}; ++m) {{
        V inner = 0.0;
        for (int j = 0; j < {n}; ++j) inner += kA[m * {n} + j] * sin(y[j]) + kB[m * {n} + j] * cos(y[j]);
        f += sq(kE[m] - inner);
    }}
    return f;
}}
"""
    return src
