"""Mixed-precision path (float32 hDuals, compensated sums, float64 islands)
against the float64 oracle, through the C ABI.

Bar: the same normwise relative errors as the float64 tests,
    e_hvp = max|r - r*| / (max|H*| max|v|),  e_H = max|H - H*| / max|H*|,
must stay below the per-function gates of tests/gates.py (four times the
measured maxima, which are 1.7e-7 - 2.6e-7: the inputs are rounded to
float32 and each Hessian entry goes through a few dozen float32 operations
before the compensated sums).  The measured maxima are printed.
"""
import numpy as np
import pytest
import torch

from oracle import closed_form as cf
from gates import TOL32
from paper_2410_22575_amd import inputs

pytestmark = pytest.mark.gpu

R, A, FP = 0, 1, 2


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _setup(gpu_lib, w):
    if w.func == FP:
        gpu_lib.chessfad_fp_set_params(_dev(w.A), _dev(w.B), _dev(w.alpha))
        return cf.fp_offsets(w.A, w.B, w.alpha)
    return None


@pytest.mark.parametrize("func", [R, A, FP])
@pytest.mark.parametrize("n,chunks", [(5, (1, 2, 4)), (16, (1, 4, 16)), (40, (2, 8)), (64, (4, 16))])
def test_mixed_against_oracle(gpu_lib, func, n, chunks):
    npts = 257
    w = inputs.make_workload(func, n, npts, inputs.rng_for(7000 + 10 * func + n))
    E = _setup(gpu_lib, w)
    x, v = _dev(w.x), _dev(w.v)
    H_ref = cf.hessian(func, w.x, w.A, w.B, E)
    hmax = np.abs(H_ref).max(axis=(1, 2))
    r_ref = cf.hvp(func, w.x, w.v, w.A, w.B, E)
    for c in chunks:
        print(f"[case] mixed func={func} n={n} chunk={c}", flush=True)
        r = gpu_lib.chessfad_hvp_mixed(func, x, v, chunk=c).cpu().numpy()
        e_r = (np.abs(r - r_ref).max(axis=1) / (hmax * np.abs(w.v).max(axis=1))).max()
        H = gpu_lib.chessfad_hessian_mixed(func, x, chunk=c).cpu().numpy()
        e_H = (np.abs(H - H_ref).max(axis=(1, 2)) / hmax).max()
        print(f"  max rel err: hvp {e_r:.3e}  hessian {e_H:.3e}", flush=True)
        assert e_r <= TOL32[func] and e_H <= TOL32[func]
        assert e_r > 0.0  # it really is a float32 computation


@pytest.mark.parametrize("func", [R, A])
def test_mixed_mappings(gpu_lib, func):
    """The L0 / L1 mappings of chessfad_hvp_mixed compute the sums L2 does, in
    the same order (float32 rounding may differ where the compiler contracts
    multiply-adds differently); each stays within the mixed gate of the oracle."""
    prev = gpu_lib.chessfad_set_option(gpu_lib.CHESSFAD_OPT_MAPPING, 2)
    try:
        for n, npts in ((5, 70), (16, 300), (33, 9)):
            w = inputs.make_workload(func, n, npts, inputs.rng_for(7300 + 10 * func + n))
            x, v = _dev(w.x), _dev(w.v)
            H_ref = cf.hessian(func, w.x, w.A, w.B, None)
            hmax = np.abs(H_ref).max(axis=(1, 2))
            r_ref = cf.hvp(func, w.x, w.v, w.A, w.B, None)
            scale = hmax * np.abs(w.v).max(axis=1)
            for c in (1, 4, 16):
                if c > n:
                    continue
                gpu_lib.chessfad_set_option(gpu_lib.CHESSFAD_OPT_MAPPING, 2)
                r2 = gpu_lib.chessfad_hvp_mixed(func, x, v, chunk=c).cpu().numpy()
                for level in (1, 0):
                    print(f"[case] mixed mapping L{level} func={func} n={n} C={c}", flush=True)
                    gpu_lib.chessfad_set_option(gpu_lib.CHESSFAD_OPT_MAPPING, level)
                    r = gpu_lib.chessfad_hvp_mixed(func, x, v, chunk=c).cpu().numpy()
                    assert (np.abs(r - r2).max(axis=1) / scale).max() <= 1e-6
                    assert (np.abs(r - r_ref).max(axis=1) / scale).max() <= TOL32[func]
    finally:
        gpu_lib.chessfad_set_option(gpu_lib.CHESSFAD_OPT_MAPPING, prev)


@pytest.mark.parametrize("func", [R, A, FP])
def test_mixed_full_size_sampled(gpu_lib, func):
    n, npts = 16, 1 << 20
    w = inputs.make_workload(func, n, npts, inputs.rng_for(1))
    E = _setup(gpu_lib, w)
    r = gpu_lib.chessfad_hvp_mixed(func, _dev(w.x), _dev(w.v), chunk=4).cpu().numpy()
    assert np.all(np.isfinite(r))
    idx = np.sort(np.random.default_rng(9).choice(npts, 2048, replace=False))
    H = cf.hessian(func, w.x[idx], w.A, w.B, E)
    ref = np.einsum("pij,pj->pi", H, w.v[idx])
    e = np.abs(r[idx] - ref).max(axis=1) / (np.abs(H).max(axis=(1, 2)) * np.abs(w.v[idx]).max(axis=1))
    print(f"  full size func={func}: max rel err {e.max():.3e}", flush=True)
    assert e.max() <= TOL32[func]


def test_mixed_rosenbrock_structure(gpu_lib):
    # exact zeros survive in float32 too; at x = 1 every entry is an integer
    # well inside float32's exact range
    n = 11
    w = inputs.make_workload(R, n, 32, inputs.rng_for(7100))
    H = gpu_lib.chessfad_hessian_mixed(R, _dev(w.x), chunk=4).cpu().numpy()
    i, j = np.indices((n, n))
    assert np.all(H[:, np.abs(i - j) > 1] == 0.0)
    ones = torch.ones(2, n, dtype=torch.float64, device="cuda")
    np.testing.assert_array_equal(gpu_lib.chessfad_hessian_mixed(R, ones, chunk=2).cpu().numpy(),
                                  cf.hess_rosenbrock(np.ones((2, n))))


def test_mixed_argument_checks(gpu_lib):
    x = torch.zeros(3, 8, dtype=torch.float64, device="cuda")
    with pytest.raises(gpu_lib.ChessfadError) as ei:
        gpu_lib.chessfad_hvp_mixed(R, x, x.clone(), chunk=3)
    assert ei.value.code == -3
    empty = torch.zeros(0, 8, dtype=torch.float64, device="cuda")
    assert gpu_lib.chessfad_hvp_mixed(A, empty, empty).shape == (0, 8)


@pytest.mark.parametrize("n", [65, 130, 256, 512])
def test_mixed_fletcher_powell_large_n(gpu_lib, n):
    """Fletcher-Powell above 16 variables in mixed precision: the row-block
    kernel with float32 contraction tiles, blocked compensated sums and
    several variable passes from n = 129 on (n = 512 is the large-n
    workload's shape), H.v and Hessians element by element on a few points."""
    npts = 8 if n <= 256 else 4
    w = inputs.make_workload(FP, n, npts, inputs.rng_for(7400 + n))
    E = _setup(gpu_lib, w)
    x, v = _dev(w.x), _dev(w.v)
    H_ref = cf.hessian(FP, w.x, w.A, w.B, E)
    hmax = np.abs(H_ref).max(axis=(1, 2))
    r_ref = cf.hvp(FP, w.x, w.v, w.A, w.B, E)
    for c in (4, 16):
        print(f"[case] mixed fp n={n} chunk={c} npts={npts}", flush=True)
        r = gpu_lib.chessfad_hvp_mixed(FP, x, v, chunk=c).cpu().numpy()
        e_r = (np.abs(r - r_ref).max(axis=1) / (hmax * np.abs(w.v).max(axis=1))).max()
        H = gpu_lib.chessfad_hessian_mixed(FP, x, chunk=c).cpu().numpy()
        e_H = (np.abs(H - H_ref).max(axis=(1, 2)) / hmax).max()
        print(f"  max rel err: hvp {e_r:.3e}  hessian {e_H:.3e}", flush=True)
        assert e_r <= TOL32[FP] and e_H <= TOL32[FP]
        assert e_r > 0.0


@pytest.mark.parametrize("scale", [1.0, 1e-3, 1e-6, 1e-9])
@pytest.mark.parametrize("n", [5, 16, 64])
def test_mixed_ackley_near_zero(gpu_lib, n, scale):
    """Ackley where sqrt(sum x^2 / n) -> 0: F' grows like 1 / |x| and F'' like
    1 / |x|^3, the reason its outer functions are float64 islands.  Points
    x ~ U[-1e-3, 1e-3] * scale; the float64 path to 1e-12 and the mixed path to
    the mixed gate normwise, and entry by entry on the entries of at least 1e-3 of the
    largest (the diagnostic of the oracle's error metric)."""
    npts = 64
    rng = inputs.rng_for(7500 + n)
    x = rng.uniform(-1e-3, 1e-3, size=(npts, n)) * scale
    vv = rng.standard_normal(size=(npts, n))
    H_ref = cf.hessian(A, x)
    hmax = np.abs(H_ref).max(axis=(1, 2))
    r_ref = cf.hvp(A, x, vv)
    xd, vd = _dev(x), _dev(vv)
    big = np.abs(H_ref) >= 1e-3 * hmax[:, None, None]
    for name, fn, fh, tol in (("f64", gpu_lib.chessfad_hvp, gpu_lib.chessfad_hessian, 1e-12),
                              ("mixed", gpu_lib.chessfad_hvp_mixed, gpu_lib.chessfad_hessian_mixed, TOL32[A])):
        for c in (1, max(c for c in (1, 2, 4, 8, 16) if c <= n)):
            print(f"[case] ackley near zero n={n} scale={scale} {name} chunk={c}", flush=True)
            r = fn(A, xd, vd, chunk=c).cpu().numpy()
            H = fh(A, xd, chunk=c).cpu().numpy()
            assert np.all(np.isfinite(r)) and np.all(np.isfinite(H))
            e_r = (np.abs(r - r_ref).max(axis=1) / (hmax * np.abs(vv).max(axis=1))).max()
            e_H = (np.abs(H - H_ref).max(axis=(1, 2)) / hmax).max()
            e_el = (np.abs(H - H_ref)[big] / np.abs(H_ref)[big]).max()
            print(f"  max rel err: hvp {e_r:.3e}  hessian {e_H:.3e}  entrywise {e_el:.3e}", flush=True)
            assert e_r <= tol and e_H <= tol
            assert e_el <= (1e-10 if name == "f64" else 1e-3)
