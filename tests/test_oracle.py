"""Pins for the CPU oracle (no GPU).

Each check ties the oracle to something other than itself: hand-derived
special values (tests/golden), a brute-force AD built from the paper's
four-component hDual rules, central finite differences, invariants that the
mathematics fixes, and the paper's operation-count formulas.
"""
import math
import os

import numpy as np
import pytest

from oracle import closed_form as cf
from oracle import chunked, fd, hyperdual
from paper_2410_22575_amd import flops, inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
R, A, FP = 0, 1, 2


def _fp(n, seed=3):
    rng = inputs.rng_for(100 + seed)
    Am, Bm, alpha = inputs.fp_params(n, rng)
    return Am, Bm, alpha, cf.fp_offsets(Am, Bm, alpha)


def _point(func, n, seed=0):
    rng = np.random.default_rng(seed)
    if func == R:
        return rng.uniform(-2, 2, n)
    if func == A:
        return rng.uniform(-5, 5, n)
    raise ValueError


# ------------------------------------------------------------- golden values
def _read_rosenbrock_golden():
    out = {}
    with open(os.path.join(GOLDEN, "rosenbrock_at_minimizer.txt")) as fh:
        lines = [ln.split() for ln in fh if ln.strip() and not ln.startswith("#")]
    k = 0
    while k < len(lines):
        n = int(lines[k][1])
        out[n] = np.array([[float(t) for t in row] for row in lines[k + 1:k + 1 + n]])
        k += 1 + n
    return out


@pytest.mark.parametrize("n", [2, 4])
def test_rosenbrock_minimizer_golden(n):
    H_gold = _read_rosenbrock_golden()[n]
    x = np.ones(n)
    assert cf.f_rosenbrock(x)[0] == 0.0
    assert np.all(cf.grad_rosenbrock(x) == 0.0)
    np.testing.assert_array_equal(cf.hess_rosenbrock(x)[0], H_gold)
    np.testing.assert_array_equal(np.array(hyperdual.hessian(R, list(x))), H_gold)
    for c in (1, 2, 3):
        np.testing.assert_array_equal(chunked.hessian(R, x, c)[0], H_gold)


def test_ackley_special_values_golden():
    with open(os.path.join(GOLDEN, "ackley_special_values.txt")) as fh:
        rows = [ln.split() for ln in fh if ln.strip() and not ln.startswith("#")]
    for _, n, xv, fv in rows:
        x = np.full(int(n), float(xv))
        assert abs(cf.f_ackley(x)[0] - float(fv)) <= 4e-15
        assert abs(hyperdual.value(A, x) - float(fv)) <= 4e-15


def test_fp_zero_at_alpha():
    Am, Bm, alpha, E = _fp(6)
    assert abs(cf.f_fletcher_powell(alpha, Am, Bm, E)[0]) < 1e-18 * 1e4
    assert np.abs(cf.grad_fletcher_powell(alpha, Am, Bm, E)).max() < 1e-9
    # at a zero of every residual H = 2 J^T J: symmetric positive semidefinite
    H = cf.hess_fletcher_powell(alpha, Am, Bm, E)[0]
    assert np.abs(H - H.T).max() <= 1e-13 * np.abs(H).max()
    assert np.linalg.eigvalsh(H).min() >= -1e-10 * np.abs(H).max()


# ------------------------------------------------------- brute-force hyper-duals
def test_hd4_rules_on_known_functions():
    # x0 * x1: H = [[0, 1], [1, 0]]
    f = lambda y, M, p=None: y[0] * y[1]
    for i in range(2):
        for j in range(2):
            y = hyperdual.initialize([0.7, -1.3], i, j)
            assert f(y, hyperdual.HDMath).v[3] == (1.0 if i != j else 0.0)
    # sin(x0 x1): d2/dx0dx1 = cos(u) - x0 x1 sin(u), u = x0 x1
    a = [0.4, 1.1]
    u = a[0] * a[1]
    y = hyperdual.initialize(a, 0, 1)
    r = hyperdual.HDMath.sin(y[0] * y[1])
    assert abs(r.v[3] - (math.cos(u) - u * math.sin(u))) < 1e-15
    assert abs(r.v[1] - a[1] * math.cos(u)) < 1e-15
    assert abs(r.v[2] - a[0] * math.cos(u)) < 1e-15
    # exp, sqrt, cos on one variable: second derivatives e^x, -x^{-3/2}/4, -cos x
    x = 0.9
    y = hyperdual.initialize([x], 0, 0)
    assert abs(hyperdual.HDMath.exp(y[0]).v[3] - math.exp(x)) < 1e-15
    assert abs(hyperdual.HDMath.sqrt(y[0]).v[3] + 0.25 * x ** -1.5) < 1e-15
    assert abs(hyperdual.HDMath.cos(y[0]).v[3] + math.cos(x)) < 1e-15


@pytest.mark.parametrize("func", [R, A, FP])
@pytest.mark.parametrize("n", [2, 3, 5])
def test_closed_form_vs_bruteforce(func, n):
    params = None
    if func == FP:
        Am, Bm, alpha, E = _fp(n)
        x = alpha + np.random.default_rng(n).uniform(-0.1, 0.1, n)
        params = (Am, Bm, E)
        H = cf.hess_fletcher_powell(x, Am, Bm, E)[0]
        g = cf.grad_fletcher_powell(x, Am, Bm, E)[0]
        fv = cf.f_fletcher_powell(x, Am, Bm, E)[0]
    else:
        x = _point(func, n, seed=n)
        H = cf.hessian(func, x)[0]
        g = cf.grad(func, x)[0]
        fv = cf.f(func, x)[0]
    Hb = np.array(hyperdual.hessian(func, list(x), params))
    fb, gb = hyperdual.value_and_gradient(func, list(x), params)
    scale = np.abs(H).max()
    assert np.abs(H - Hb).max() <= 1e-13 * scale
    assert np.abs(g - np.array(gb)).max() <= 1e-13 * max(1.0, np.abs(g).max())
    assert abs(fv - fb) <= 1e-13 * max(1.0, abs(fv))


@pytest.mark.parametrize("func", [R, A, FP])
def test_closed_form_vs_finite_differences(func):
    n = 7
    if func == FP:
        Am, Bm, alpha, E = _fp(n)
        x = alpha + np.random.default_rng(1).uniform(-0.1, 0.1, n)
        fun = lambda z: cf.f_fletcher_powell(z, Am, Bm, E)[0]
        gra = lambda z: cf.grad_fletcher_powell(z, Am, Bm, E)[0]
        H = cf.hess_fletcher_powell(x, Am, Bm, E)[0]
    else:
        x = _point(func, n, seed=11)
        fun = lambda z: cf.f(func, z)[0]
        gra = lambda z: cf.grad(func, z)[0]
        H = cf.hessian(func, x)[0]
    g = gra(x)
    assert np.abs(fd.fd_gradient(fun, x) - g).max() <= 1e-6 * max(1.0, np.abs(g).max())
    assert np.abs(fd.fd_hessian(gra, x) - H).max() <= 1e-7 * np.abs(H).max()


# --------------------------------------------------------------- invariants
@pytest.mark.parametrize("func", [R, A, FP])
def test_hvp_equals_hessian_times_v(func):
    n, npts = 9, 50
    w = inputs.make_workload(func, n, npts, inputs.rng_for(7))
    E = cf.fp_offsets(w.A, w.B, w.alpha) if func == FP else None
    H = cf.hessian(func, w.x, w.A, w.B, E)
    r = cf.hvp(func, w.x, w.v, w.A, w.B, E)
    ref = np.einsum("pij,pj->pi", H, w.v)
    assert np.abs(r - ref).max() <= 1e-13 * np.abs(H).max() * np.abs(w.v).max()
    assert np.abs(H - H.transpose(0, 2, 1)).max() <= 1e-13 * np.abs(H).max()


def test_rosenbrock_is_tridiagonal():
    x = np.random.default_rng(2).uniform(-2, 2, (20, 10))
    H = cf.hess_rosenbrock(x)
    i, j = np.indices((10, 10))
    assert np.all(H[:, np.abs(i - j) > 1] == 0.0)
    assert np.all(H[:, np.abs(i - j) == 1] != 0.0)


def test_ackley_equal_coordinates_structure():
    # x = t 1 makes every diagonal entry equal and every off-diagonal entry equal
    for t in (0.3, -1.7, 2.2):
        H = cf.hess_ackley(np.full(6, t))[0]
        d = np.diag(H)
        off = H[~np.eye(6, dtype=bool)]
        assert np.ptp(d) <= 1e-13 * np.abs(H).max()
        assert np.ptp(off) <= 1e-13 * np.abs(H).max()
        Hb = np.array(hyperdual.hessian(A, [t] * 6))
        assert np.abs(H - Hb).max() <= 1e-13 * np.abs(H).max()


def test_hd4_operator_set_against_calculus():
    # second derivatives of single-variable compositions from calculus,
    # f''(x) written out by hand, against the fourth hDual component
    M = hyperdual.HDMath
    cases = [
        (lambda y: 1.0 / y, lambda x: 2.0 / x ** 3, 0.7),
        (lambda y: M.log(y), lambda x: -1.0 / x ** 2, 1.9),
        (lambda y: M.tan(y), lambda x: 2.0 * math.tan(x) / math.cos(x) ** 2, 0.4),
        (lambda y: M.tanh(y), lambda x: -2.0 * math.tanh(x) / math.cosh(x) ** 2, -0.8),
        (lambda y: M.atan(y), lambda x: -2.0 * x / (1.0 + x * x) ** 2, 1.3),
        (lambda y: M.pow(y, 2.5), lambda x: 2.5 * 1.5 * x ** 0.5, 1.7),
        (lambda y: M.abs(y), lambda x: 0.0, -0.6),
        (lambda y: y / (1.0 + y * y), lambda x: (2 * x ** 3 - 6 * x) / (1 + x * x) ** 3, 0.9),
        (lambda y: M.exp(y) / y, lambda x: math.exp(x) * (x * x - 2 * x + 2) / x ** 3, 1.1),
    ]
    for f, d2, x in cases:
        y = hyperdual.initialize([x], 0, 0)
        got = f(y[0]).v[3]
        assert abs(got - d2(x)) <= 1e-13 * max(1.0, abs(d2(x))), (x, got, d2(x))
    # a mixed quotient: d2/dx dy (x / y) = -1 / y^2
    y = hyperdual.initialize([0.8, 1.6], 0, 1)
    assert abs((y[0] / y[1]).v[3] + 1.0 / 1.6 ** 2) <= 1e-15
    # first derivative of |x| follows the sign of the value
    y = hyperdual.initialize([-0.6], 0, 0)
    assert M.abs(y[0]).v[1] == -1.0


# ------------------------------------------------------ the chunked C method
@pytest.mark.parametrize("func", [R, A, FP])
@pytest.mark.parametrize("n,c", [(2, 1), (2, 2), (5, 2), (5, 3), (8, 4), (16, 4), (16, 16), (13, 4), (7, 16)])
def test_chunked_c_matches_closed_form(func, n, c):
    w = inputs.make_workload(func, n, 12, inputs.rng_for(20 + n))
    E = cf.fp_offsets(w.A, w.B, w.alpha) if func == FP else None
    H = chunked.hessian(func, w.x, c, w.A, w.B, E)
    Hs = cf.hessian(func, w.x, w.A, w.B, E)
    r = chunked.hvp(func, w.x, w.v, c, w.A, w.B, E)
    rs = cf.hvp(func, w.x, w.v, w.A, w.B, E)
    for p in range(w.npts):
        scale = np.abs(Hs[p]).max()
        assert np.abs(H[p] - Hs[p]).max() <= 1e-13 * scale
        assert np.abs(r[p] - rs[p]).max() <= 1e-13 * scale * np.abs(w.v[p]).max()
    fv, g = chunked.value_grad(func, w.x[0], c, w.A, w.B, E)
    assert abs(fv - cf.f(func, w.x[0], w.A, w.B, E)[0]) <= 1e-13 * max(1.0, abs(fv))
    gs = cf.grad(func, w.x[0], w.A, w.B, E)[0]
    assert np.abs(g - gs).max() <= 1e-13 * max(1.0, np.abs(gs).max())


@pytest.mark.parametrize("func", [R, A, FP])
def test_chunked_c_chunk_invariance(func):
    # every Hessian entry is produced by the same per-component expression
    # whatever the chunk size, so H does not depend on it at all
    n = 12
    w = inputs.make_workload(func, n, 4, inputs.rng_for(31))
    E = cf.fp_offsets(w.A, w.B, w.alpha) if func == FP else None
    H1 = chunked.hessian(func, w.x, 1, w.A, w.B, E)
    for c in (2, 3, 4, 5, 12, 16):
        np.testing.assert_array_equal(chunked.hessian(func, w.x, c, w.A, w.B, E), H1)


def test_chunked_c_threads_agree():
    w = inputs.make_workload(R, 8, 64, inputs.rng_for(5))
    np.testing.assert_array_equal(chunked.hvp(R, w.x, w.v, 4, nthreads=1),
                                  chunked.hvp(R, w.x, w.v, 4, nthreads=4))


# ----------------------------- symmetric variants (Sec. III.B, Sec. V, Sec. VI)
@pytest.mark.parametrize("func", [R, A, FP])
@pytest.mark.parametrize("n,c", [(2, 1), (2, 2), (5, 2), (5, 3), (8, 4), (16, 4), (16, 16), (13, 4), (7, 16),
                                 (12, 1)])
def test_symmetric_chunked_matches_closed_form(func, n, c):
    w = inputs.make_workload(func, n, 8, inputs.rng_for(50 + n))
    E = cf.fp_offsets(w.A, w.B, w.alpha) if func == FP else None
    Hs = cf.hessian(func, w.x, w.A, w.B, E)
    H = chunked.hessian(func, w.x, c, w.A, w.B, E, sym=True)      # starts as NaN: every entry written
    r = chunked.hvp(func, w.x, w.v, c, w.A, w.B, E, sym=True)
    rs = cf.hvp(func, w.x, w.v, w.A, w.B, E)
    for p in range(w.npts):
        scale = np.abs(Hs[p]).max()
        assert np.abs(H[p] - Hs[p]).max() <= 1e-13 * scale
        assert np.abs(r[p] - rs[p]).max() <= 1e-13 * scale * np.abs(w.v[p]).max()


@pytest.mark.parametrize("func", [R, A, FP])
def test_symmetric_hessian_structure(func):
    # entries a row evaluates itself are the CHUNK-HESS entries bit for bit;
    # entries left of the row's own chunk are exact copies of their mirrors
    n, c = 11, 3
    w = inputs.make_workload(func, n, 3, inputs.rng_for(52))
    E = cf.fp_offsets(w.A, w.B, w.alpha) if func == FP else None
    Hf = chunked.hessian(func, w.x, c, w.A, w.B, E)
    Hy = chunked.hessian(func, w.x, c, w.A, w.B, E, sym=True)
    for i in range(n):
        own = (i // c) * c
        np.testing.assert_array_equal(Hy[:, i, own:], Hf[:, i, own:])
        np.testing.assert_array_equal(Hy[:, i, :own], Hy[:, :own, i])


@pytest.mark.parametrize("func", [R, A, FP])
def test_symmetric_hvp_of_unit_vectors_gives_columns(func):
    # v = e_k picks column k of H: the symmetric product then returns the
    # column assembled from row k's own evaluations and the mirrors of the
    # rows before it, which must equal row k of the full CHUNK-HESS
    n, c = 9, 2
    w = inputs.make_workload(func, n, 1, inputs.rng_for(53))
    E = cf.fp_offsets(w.A, w.B, w.alpha) if func == FP else None
    Hf = chunked.hessian(func, w.x, c, w.A, w.B, E)[0]
    scale = np.abs(Hf).max()
    for k in range(n):
        e = np.zeros((1, n))
        e[0, k] = 1.0
        col = chunked.hvp(func, w.x, e, c, w.A, w.B, E, sym=True)[0]
        assert np.abs(col - Hf[:, k]).max() <= 1e-14 * scale


def test_symmetric_call_count_formula():
    # Sec. V: n (n / c + 1) / 2 evaluated chunks when c divides n; c = 1 gives
    # n (n + 1) / 2 and c = n gives n
    w = inputs.make_workload(R, 16, 1, inputs.rng_for(54))
    for c in (1, 2, 4, 8, 16):
        calls = chunked.count_hvp(R, w.x[0], w.v[0], c, sym=True)[2]
        assert calls == 16 * (16 // c + 1) // 2 == flops.calls_per_point_sym(16, c)
    assert chunked.count_hvp(R, w.x[0], w.v[0], 1, sym=True)[2] == 16 * 17 // 2
    assert chunked.count_hvp(R, w.x[0], w.v[0], 16, sym=True)[2] == 16
    # ragged: every row evaluates its own chunk and the ones after it
    w = inputs.make_workload(R, 7, 1, inputs.rng_for(55))
    assert chunked.count_hvp(R, w.x[0], w.v[0], 3, sym=True)[2] == 3 * 3 + 3 * 2 + 1 * 1


def test_symmetric_multiplication_count_formula():
    # Sec. V: n (n / c + 1) / 2 calls with M hDual products each cost
    # (3/2) n (2n + 2c + n/c + 1) M multiplications (Rosenbrock, c | n); the
    # other multiplications are the 100 x (.) scalings, the own chunk dot of
    # every call and the mirror update of every call right of the own chunk
    for n, c in ((8, 2), (8, 4), (16, 4), (16, 8)):
        w = inputs.make_workload(R, n, 1, inputs.rng_for(56))
        _, muls, calls = chunked.count_hvp(R, w.x[0], w.v[0], c, sym=True)
        M = 3 * (n - 1)
        scalings = (n - 1) * (2 * c + 2)
        assert muls == calls * (M * (6 * c + 3) + scalings + c) + (calls - n) * c
        assert 2 * calls * M * (6 * c + 3) == 3 * n * (2 * n + 2 * c + n // c + 1) * M


@pytest.mark.parametrize("func", [R, A, FP])
@pytest.mark.parametrize("n,c", [(8, 2), (16, 4), (12, 3)])
def test_symmetric_model_flops_match_executed_counts(func, n, c):
    w = inputs.make_workload(func, n, 1, inputs.rng_for(57))
    E = cf.fp_offsets(w.A, w.B, w.alpha) if func == FP else None
    adds, muls, _ = chunked.count_hvp(func, w.x[0], w.v[0], c, w.A, w.B, E, sym=True)
    assert adds + muls == flops.flops_per_hvp_sym(func, n, c)


# ------------------------------------------------- operation counts (Sec. V)
@pytest.mark.parametrize("c", [1, 2, 4, 8, 16])
def test_operator_counts(c):
    assert chunked.count_op(0, c) == (2 * c + 2, 0)           # hDual + hDual
    assert chunked.count_op(1, c) == (4 * c + 1, 6 * c + 3)   # hDual x hDual
    assert chunked.count_op(2, c) == (0, 2 * c + 2)           # double x hDual
    assert sum(chunked.count_op(3, c)) == 4 * c + 2           # unary


@pytest.mark.parametrize("func", [R, A, FP])
@pytest.mark.parametrize("n,c", [(4, 1), (8, 2), (8, 4), (16, 4), (16, 16), (12, 3)])
def test_model_flops_match_executed_counts(func, n, c):
    w = inputs.make_workload(func, n, 1, inputs.rng_for(40))
    E = cf.fp_offsets(w.A, w.B, w.alpha) if func == FP else None
    adds, muls, calls = chunked.count_hvp(func, w.x[0], w.v[0], c, w.A, w.B, E)
    assert calls == flops.calls_per_point(n, c) == n * math.ceil(n / c)
    assert adds + muls == flops.flops_per_hvp(func, n, c)


def test_chunk_hess_multiplication_count_formula():
    # Sec. V: n^2/c calls with M hDual products each cost (6 + 3/c) n^2 M
    # multiplications (Rosenbrock: 3 products per term, n divisible by c); the
    # other multiplications are the 100 x (.) scalings and the chunk dot
    for n, c in ((8, 2), (8, 4), (16, 8)):
        w = inputs.make_workload(R, n, 1, inputs.rng_for(41))
        _, muls, calls = chunked.count_hvp(R, w.x[0], w.v[0], c)
        M = 3 * (n - 1)                          # hDual products per call
        scalings = (n - 1) * (2 * c + 2)         # 100 x (.) per term
        dot = c                                  # chunk dot multiplications
        assert muls == calls * (M * (6 * c + 3) + scalings + dot)
        assert calls * M * (6 * c + 3) == (6 + 3 / c) * n * n * M


def test_survey_reference_counts_n16():
    # per-HVP model at n = 16 used for the roofline figures
    table = {R: [226048, 185984, 165952, 155936, 150928],
             A: [139520, 113280, 100160, 93600, 90320],
             FP: [1158656, 878336, 738176, 668096, 633056]}
    for func, vals in table.items():
        assert [flops.flops_per_hvp(func, 16, c) for c in (1, 2, 4, 8, 16)] == vals
