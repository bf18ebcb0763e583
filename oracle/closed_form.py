"""Closed-form f, gradient, Hessian and Hessian-vector product (float64).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The paper names its three test functions (Sec. VII) but does not write them
out; the definitions used throughout are the standard ones, 0-based:

  Rosenbrock      f = sum_{k=0}^{n-2} 100 (x_{k+1} - x_k^2)^2 + (1 - x_k)^2
  Ackley          f = -20 exp(-0.2 rho) - exp(q) + 20 + e,
                  rho = sqrt(sum_k x_k^2 / n),  q = sum_k cos(2 pi x_k) / n
  Fletcher-Powell f = sum_m r_m^2,
                  r_m = E_m - sum_j (A_mj sin x_j + B_mj cos x_j),
                  E_m = sum_j (A_mj sin alpha_j + B_mj cos alpha_j)

The chunked method of Sec. III.B evaluates f on hDuals and reads row i of
the Hessian out of the second-order components (Sec. IV); the result it
reaches is exactly the analytic Hessian H(x) and r = H(x) v (Sec. III.C),
so these hand-derived formulas are the oracle.  Derivations:

  Rosenbrock: H is tridiagonal,
      H_kk     = [k <= n-2] (1200 x_k^2 - 400 x_{k+1} + 2) + [k >= 1] 200
      H_k,k+1  = H_k+1,k = -400 x_k
  Ackley: with g = exp(-0.2 rho), s = sin(2 pi x), c = cos(2 pi x),
      H = 4 g [ I/(n rho) - x x^T (1/(n^2 rho^3) + 0.2/(n^2 rho^2)) ]
          - exp(q) [ (4 pi^2/n^2) s s^T - (4 pi^2/n) diag(c) ]
  Fletcher-Powell: with J_mk = -A_mk cos x_k + B_mk sin x_k  (= dr_m/dx_k)
      and D_mk = A_mk sin x_k + B_mk cos x_k  (= d2 r_m / dx_k^2),
      H = 2 (J^T J + diag(D^T r)),   H v = 2 (J^T (J v) + (D^T r) * v)

All functions take x of shape [npts, n] (or [n]) and work point by point.
"""
from __future__ import annotations

import numpy as np

ROSENBROCK, ACKLEY, FLETCHER_POWELL = 0, 1, 2


def _2d(x):
    x = np.asarray(x, dtype=np.float64)
    return x[None, :] if x.ndim == 1 else x


def fp_offsets(A, B, alpha):
    """E_m = sum_j A_mj sin(alpha_j) + B_mj cos(alpha_j): the offsets that
    make x = alpha a zero of every Fletcher-Powell residual."""
    A = np.asarray(A, np.float64)
    B = np.asarray(B, np.float64)
    alpha = np.asarray(alpha, np.float64)
    return A @ np.sin(alpha) + B @ np.cos(alpha)


# --------------------------------------------------------------------- f
def f_rosenbrock(x):
    x = _2d(x)
    return np.sum(100.0 * (x[:, 1:] - x[:, :-1] ** 2) ** 2 + (1.0 - x[:, :-1]) ** 2, axis=1)


def f_ackley(x):
    x = _2d(x)
    n = x.shape[1]
    rho = np.sqrt(np.sum(x * x, axis=1) / n)
    q = np.sum(np.cos(2.0 * np.pi * x), axis=1) / n
    return -20.0 * np.exp(-0.2 * rho) - np.exp(q) + 20.0 + np.e


def fp_residuals(x, A, B, E):
    x = _2d(x)
    return E[None, :] - (np.sin(x) @ A.T + np.cos(x) @ B.T)


def f_fletcher_powell(x, A, B, E):
    r = fp_residuals(x, A, B, E)
    return np.sum(r * r, axis=1)


# -------------------------------------------------------------- gradient
def grad_rosenbrock(x):
    x = _2d(x)
    g = np.zeros_like(x)
    t = x[:, 1:] - x[:, :-1] ** 2
    g[:, :-1] += -400.0 * x[:, :-1] * t - 2.0 * (1.0 - x[:, :-1])
    g[:, 1:] += 200.0 * t
    return g


def grad_ackley(x):
    x = _2d(x)
    n = x.shape[1]
    rho = np.sqrt(np.sum(x * x, axis=1) / n)[:, None]
    q = (np.sum(np.cos(2.0 * np.pi * x), axis=1) / n)[:, None]
    return (4.0 * np.exp(-0.2 * rho) * x / (n * rho)
            + np.exp(q) * 2.0 * np.pi * np.sin(2.0 * np.pi * x) / n)


def _fp_J_D(x, A, B):
    """J[p, m, k] = dr_m/dx_k and D[p, m, k] = d2 r_m/dx_k^2 at each point."""
    s = np.sin(x)[:, None, :]
    c = np.cos(x)[:, None, :]
    J = -A[None] * c + B[None] * s
    D = A[None] * s + B[None] * c
    return J, D


def grad_fletcher_powell(x, A, B, E):
    x = _2d(x)
    r = fp_residuals(x, A, B, E)
    J, _ = _fp_J_D(x, A, B)
    return 2.0 * np.einsum("pm,pmk->pk", r, J)


# --------------------------------------------------------------- Hessian
def hess_rosenbrock(x):
    x = _2d(x)
    npts, n = x.shape
    H = np.zeros((npts, n, n))
    k = np.arange(n)
    diag = np.zeros((npts, n))
    diag[:, :-1] += 1200.0 * x[:, :-1] ** 2 - 400.0 * x[:, 1:] + 2.0
    diag[:, 1:] += 200.0
    H[:, k, k] = diag
    H[:, k[:-1], k[:-1] + 1] = -400.0 * x[:, :-1]
    H[:, k[:-1] + 1, k[:-1]] = -400.0 * x[:, :-1]
    return H


def hess_ackley(x):
    x = _2d(x)
    npts, n = x.shape
    rho = np.sqrt(np.sum(x * x, axis=1) / n)
    q = np.sum(np.cos(2.0 * np.pi * x), axis=1) / n
    g = np.exp(-0.2 * rho)
    s = np.sin(2.0 * np.pi * x)
    c = np.cos(2.0 * np.pi * x)
    eye = np.eye(n)[None]
    xx = x[:, :, None] * x[:, None, :]
    ss = s[:, :, None] * s[:, None, :]
    a = (4.0 * g / (n * rho))[:, None, None]
    b = (4.0 * g * (1.0 / (n * n * rho ** 3) + 0.2 / (n * n * rho ** 2)))[:, None, None]
    eq = np.exp(q)[:, None, None]
    w = 4.0 * np.pi ** 2
    cdiag = c[:, :, None] * eye
    return a * eye - b * xx - eq * ((w / (n * n)) * ss - (w / n) * cdiag)


def hess_fletcher_powell(x, A, B, E):
    x = _2d(x)
    r = fp_residuals(x, A, B, E)
    J, D = _fp_J_D(x, A, B)
    H = 2.0 * np.einsum("pmk,pmj->pkj", J, J)
    d = 2.0 * np.einsum("pm,pmk->pk", r, D)
    k = np.arange(x.shape[1])
    H[:, k, k] += d
    return H


# ----------------------------------------------------- Hessian . vector
def hvp_rosenbrock(x, v):
    """Tridiagonal matvec, O(n) per point."""
    x = _2d(x)
    v = _2d(v)
    diag = np.zeros_like(x)
    diag[:, :-1] += 1200.0 * x[:, :-1] ** 2 - 400.0 * x[:, 1:] + 2.0
    diag[:, 1:] += 200.0
    off = -400.0 * x[:, :-1]
    r = diag * v
    r[:, :-1] += off * v[:, 1:]
    r[:, 1:] += off * v[:, :-1]
    return r


def hvp_ackley(x, v):
    """O(n) per point through x.v and s.v (no Hessian is formed)."""
    x = _2d(x)
    v = _2d(v)
    n = x.shape[1]
    rho = np.sqrt(np.sum(x * x, axis=1) / n)
    q = np.sum(np.cos(2.0 * np.pi * x), axis=1) / n
    g = np.exp(-0.2 * rho)
    s = np.sin(2.0 * np.pi * x)
    c = np.cos(2.0 * np.pi * x)
    a = (4.0 * g / (n * rho))[:, None]
    b = (4.0 * g * (1.0 / (n * n * rho ** 3) + 0.2 / (n * n * rho ** 2)))[:, None]
    eq = np.exp(q)[:, None]
    w = 4.0 * np.pi ** 2
    xv = np.sum(x * v, axis=1)[:, None]
    sv = np.sum(s * v, axis=1)[:, None]
    return a * v - b * x * xv - eq * ((w / (n * n)) * s * sv - (w / n) * c * v)


def hvp_fletcher_powell(x, A, B, E, v, block=4096):
    """2 (J^T (J v) + (D^T r) * v), O(n^2) per point, in blocks of points."""
    x = _2d(x)
    v = _2d(v)
    out = np.empty_like(x)
    for p0 in range(0, x.shape[0], block):
        xb, vb = x[p0:p0 + block], v[p0:p0 + block]
        r = fp_residuals(xb, A, B, E)
        J, D = _fp_J_D(xb, A, B)
        Jv = np.einsum("pmk,pk->pm", J, vb)
        out[p0:p0 + block] = 2.0 * (np.einsum("pmk,pm->pk", J, Jv)
                                    + np.einsum("pm,pmk->pk", r, D) * vb)
    return out


# ------------------------------------------------------------ dispatch
def f(func, x, A=None, B=None, E=None):
    if func == ROSENBROCK:
        return f_rosenbrock(x)
    if func == ACKLEY:
        return f_ackley(x)
    return f_fletcher_powell(x, A, B, E)


def grad(func, x, A=None, B=None, E=None):
    if func == ROSENBROCK:
        return grad_rosenbrock(x)
    if func == ACKLEY:
        return grad_ackley(x)
    return grad_fletcher_powell(x, A, B, E)


def hessian(func, x, A=None, B=None, E=None):
    if func == ROSENBROCK:
        return hess_rosenbrock(x)
    if func == ACKLEY:
        return hess_ackley(x)
    return hess_fletcher_powell(x, A, B, E)


def hvp(func, x, v, A=None, B=None, E=None):
    if func == ROSENBROCK:
        return hvp_rosenbrock(x, v)
    if func == ACKLEY:
        return hvp_ackley(x, v)
    return hvp_fletcher_powell(x, A, B, E, v)
