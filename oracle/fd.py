"""Central finite differences (float64), used only to pin the closed forms.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Gradient:  g_j ~ (f(x + h e_j) - f(x - h e_j)) / (2h)
Hessian:   H[:, j] ~ (grad(x + h e_j) - grad(x - h e_j)) / (2h)
with h = 6e-6 * max(1, |x_j|) (truncation error O(h^2), rounding O(u/h)).
"""
from __future__ import annotations

import numpy as np


def _step(xj):
    return 6e-6 * max(1.0, abs(xj))


def fd_gradient(fun, x):
    x = np.asarray(x, np.float64)
    g = np.empty_like(x)
    for j in range(x.size):
        h = _step(x[j])
        xp, xm = x.copy(), x.copy()
        xp[j] += h
        xm[j] -= h
        g[j] = (float(fun(xp)) - float(fun(xm))) / (xp[j] - xm[j])
    return g


def fd_hessian(grad, x):
    x = np.asarray(x, np.float64)
    n = x.size
    H = np.empty((n, n))
    for j in range(n):
        h = _step(x[j])
        xp, xm = x.copy(), x.copy()
        xp[j] += h
        xm[j] -= h
        H[:, j] = (np.asarray(grad(xp)).ravel() - np.asarray(grad(xm)).ravel()) / (xp[j] - xm[j])
    return H
