"""User functions for the GPU tests: the package's Rosenbrock and Ackley
sources, and a function over every operator written twice - HIP source for
chessfad_register_function (over chessfad_device.h's hDual) and Python over
the oracle's number types (oracle.hyperdual), so the oracle computes its
Hessian independently."""
from paper_2410_22575_amd.user_sources import ACKLEY_HIP, ROSENBROCK_HIP  # noqa: F401

# every operator of chessfad_device.h, and a branch on a value (n >= 6)
MIXED_OPS_HIP = """
template <class V, class Y> __device__ V chessfad_user_f(const Y& y, int n) {
    V s = 0.0;
    for (int k = 0; k < n; ++k) s += exp(y[k]) / (1.0 + y[k] * y[k]);
    s += log(1.0 + sq(y[0] * y[1]));
    s += sqrt(2.0 + sin(y[2]) * cos(y[3]));
    s += pow(1.5 + tanh(y[4]), 2.5);
    s += abs(y[5] - 0.3) * y[0];
    s += atan(y[1] * y[5]) - y[2] / (2.0 + y[3] * y[3]) + tan(0.3 * y[4]);
    if (y[0] > 0.0)
        s += y[0] * y[1] * y[2];
    else
        s -= y[3] * y[4];
    return s;
}
"""


def mixed_ops_py(y, M, params=None):
    s = 0.0
    for k in range(len(y)):
        s = s + M.exp(y[k]) / (1.0 + y[k] * y[k])
    t = y[0] * y[1]
    s = s + M.log(1.0 + t * t)
    s = s + M.sqrt(2.0 + M.sin(y[2]) * M.cos(y[3]))
    s = s + M.pow(1.5 + M.tanh(y[4]), 2.5)
    s = s + M.abs(y[5] - 0.3) * y[0]
    s = s + M.atan(y[1] * y[5]) - y[2] / (2.0 + y[3] * y[3]) + M.tan(0.3 * y[4])
    if y[0] > 0.0:
        s = s + y[0] * y[1] * y[2]
    else:
        s = s - y[3] * y[4]
    return s

