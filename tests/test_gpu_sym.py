"""Symmetric forms (SCHUNK-HESS, SC-HESS-VEC) through the C ABI against the
float64 oracle.

Bars: the float64 path within 1e-12 of the oracle's SC-HESS-VEC /
SCHUNK-HESS and of the closed form, in the normwise errors of the other
parity tests; the mixed path within the per-function mixed gates
of tests/gates.py.  Exact properties: a symmetric
Hessian's mirrored entries (right of a row's own chunk) equal their
images bit for bit, and its own-chunk entries equal the full form's (same
per-component arithmetic) up to the last bits of the Fletcher-Powell
MFMA sum order.
"""
import numpy as np
import pytest
import torch

from gates import TOL32

from oracle import chunked
from oracle import closed_form as cf
from paper_2410_22575_amd import inputs

from test_gpu_parity import FUNC_PATHS, fp_path

pytestmark = pytest.mark.gpu

R, A, FP = 0, 1, 2
CHUNKS = (1, 2, 4, 8, 16)


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _setup(lib, w):
    if w.func != FP:
        return None
    lib.chessfad_fp_set_params(_dev(w.A), _dev(w.B), _dev(w.alpha))
    return cf.fp_offsets(w.A, w.B, w.alpha)


def _errs(w, E, r, H=None):
    Hs = cf.hessian(w.func, w.x, w.A, w.B, E)
    hmax = np.abs(Hs).max(axis=(1, 2))
    rs = np.einsum("pij,pj->pi", Hs, w.v)
    er = (np.abs(r - rs).max(axis=1) / (hmax * np.abs(w.v).max(axis=1))).max()
    eh = None if H is None else (np.abs(H - Hs).max(axis=(1, 2)) / hmax).max()
    return er, eh


@pytest.mark.parametrize("func,mfma", FUNC_PATHS)
@pytest.mark.parametrize("n", [2, 5, 13, 16, 24])
def test_symmetric_small(gpu_lib, func, mfma, n):
    npts = 203  # several workgroups and a ragged last one
    w = inputs.make_workload(func, n, npts, inputs.rng_for(6000 + 10 * func + n))
    E = _setup(gpu_lib, w)
    x, v = _dev(w.x), _dev(w.v)
    with fp_path(gpu_lib, mfma):
        for c in CHUNKS:
            if c > n:
                continue
            print(f"[case] sym func={func} mfma={mfma} n={n} C={c}", flush=True)
            r = gpu_lib.chessfad_hvp_sym(func, x, v, chunk=c).cpu().numpy()
            H = gpu_lib.chessfad_hessian_sym(func, x, chunk=c).cpu().numpy()
            er, eh = _errs(w, E, r, H)
            assert er <= 1e-12 and eh <= 1e-12, (c, er, eh)
            # the oracle's own symmetric form on a few points
            ro = chunked.hvp(func, w.x[:7], w.v[:7], c, w.A, w.B, E, sym=True)
            Ho = chunked.hessian(func, w.x[:7], c, w.A, w.B, E, sym=True)
            scale = np.abs(Ho).max()
            assert np.abs(r[:7] - ro).max() <= 1e-12 * scale * np.abs(w.v[:7]).max()
            assert np.abs(H[:7] - Ho).max() <= 1e-12 * scale
            # mirrored entries are exact copies of the evaluated ones
            for i in range(n):
                own = (i // c) * c
                np.testing.assert_array_equal(H[:, i, :own], H[:, :own, i])


@pytest.mark.parametrize("func,mfma", FUNC_PATHS)
def test_symmetric_agrees_with_full_form(gpu_lib, func, mfma):
    n, npts = 16, 500
    w = inputs.make_workload(func, n, npts, inputs.rng_for(6100 + func))
    _setup(gpu_lib, w)
    x, v = _dev(w.x), _dev(w.v)
    with fp_path(gpu_lib, mfma):
        for c in (1, 4, 16):
            Hf = gpu_lib.chessfad_hessian(func, x, chunk=c).cpu().numpy()
            Hy = gpu_lib.chessfad_hessian_sym(func, x, chunk=c).cpu().numpy()
            scale = np.abs(Hf).max()
            for i in range(n):
                own = (i // c) * c
                assert np.abs(Hy[:, i, own:] - Hf[:, i, own:]).max() <= 1e-14 * scale
            rf = gpu_lib.chessfad_hvp(func, x, v, chunk=c).cpu().numpy()
            ry = gpu_lib.chessfad_hvp_sym(func, x, v, chunk=c).cpu().numpy()
            assert np.abs(ry - rf).max() <= 1e-13 * scale * np.abs(w.v).max()


@pytest.mark.parametrize("n,npts", [(17, 11), (33, 9), (64, 7), (100, 5)])
def test_fp_symmetric_per_call_kernel(gpu_lib, n, npts):
    """Fletcher-Powell n > 16: the per-call kernel's symmetric form (block
    pairs kb >= ib in passes, mirrors summed per column) against the oracle's
    SC-HESS-VEC and SCHUNK-HESS at every point, every chunk size; mirrored
    entries are exact copies; the own-chunk entries and the counted calls
    equal the full form's (same products in the same order; the own part
    is summed in another place)."""
    w = inputs.make_workload(FP, n, npts, inputs.rng_for(6600 + n))
    E = _setup(gpu_lib, w)
    x, v = _dev(w.x), _dev(w.v)
    for c in CHUNKS:
        print(f"[case] fp sym per-call n={n} npts={npts} C={c}", flush=True)
        r = gpu_lib.chessfad_hvp_sym(FP, x, v, chunk=c).cpu().numpy()
        H = gpu_lib.chessfad_hessian_sym(FP, x, chunk=c).cpu().numpy()
        ro = chunked.hvp(FP, w.x, w.v, c, w.A, w.B, E, sym=True, nthreads=4)
        Ho = chunked.hessian(FP, w.x, c, w.A, w.B, E, sym=True, nthreads=4)
        scale = np.abs(Ho).max(axis=(1, 2))
        er = (np.abs(r - ro).max(axis=1) / (scale * np.abs(w.v).max(axis=1))).max()
        eh = (np.abs(H - Ho).max(axis=(1, 2)) / scale).max()
        assert er <= 1e-12 and eh <= 1e-12, (c, er, eh)
        for i in range(n):
            own = (i // c) * c
            np.testing.assert_array_equal(H[:, i, :own], H[:, :own, i])
        Hf = gpu_lib.chessfad_hessian(FP, x, chunk=c).cpu().numpy()
        for i in range(n):
            own = (i // c) * c
            assert np.abs(H[:, i, own:] - Hf[:, i, own:]).max() <= 1e-14 * scale.max()


@pytest.mark.parametrize("n", [40, 200])
def test_fp_symmetric_mixed_and_many_points(gpu_lib, n):
    """Several points per workgroup (2^12 points) and the mixed policy of the
    symmetric per-call kernel, against the closed form on sampled points."""
    npts = 1 << 12 if n == 40 else 1100
    w = inputs.make_workload(FP, n, npts, inputs.rng_for(6700 + n))
    E = _setup(gpu_lib, w)
    x, v = _dev(w.x), _dev(w.v)
    idx = np.random.default_rng(n).choice(npts, 6, replace=False)
    idx[0] = npts - 1   # the last, ragged workgroup
    Hs = cf.hessian(FP, w.x[idx], w.A, w.B, E)
    hmax = np.abs(Hs).max(axis=(1, 2))
    rs = np.einsum("pij,pj->pi", Hs, w.v[idx])
    for c in (2, 8, 16):
        for prec, tol in ((0, 1e-12), (1, TOL32[FP])):
            fn = gpu_lib.chessfad_hvp_sym
            r = fn(FP, x, v, chunk=c, precision=prec).cpu().numpy()[idx]
            er = (np.abs(r - rs).max(axis=1) / (hmax * np.abs(w.v[idx]).max(axis=1))).max()
            print(f"[case] fp sym n={n} C={c} precision={prec}: err {er:.2e}", flush=True)
            assert er <= tol, (c, prec, er)
            if prec == 1:
                assert er > 1e-12   # float32 arithmetic really ran


@pytest.mark.parametrize("func", [R, A, FP])
@pytest.mark.parametrize("n", [16, 40])
def test_symmetric_mixed_precision(gpu_lib, func, n):
    npts = 257
    w = inputs.make_workload(func, n, npts, inputs.rng_for(6200 + 10 * func + n))
    E = _setup(gpu_lib, w)
    x, v = _dev(w.x), _dev(w.v)
    worst = 0.0
    for c in (1, 4, 8):
        r = gpu_lib.chessfad_hvp_sym(func, x, v, chunk=c, precision=1).cpu().numpy()
        H = gpu_lib.chessfad_hessian_sym(func, x, chunk=c, precision=1).cpu().numpy()
        er, eh = _errs(w, E, r, H)
        worst = max(worst, er, eh)
        assert er <= TOL32[func] and eh <= TOL32[func], (c, er, eh)
    print(f"  mixed sym func={func} n={n} worst {worst:.3e}", flush=True)
    assert worst > 1e-12  # float32 arithmetic really ran


@pytest.mark.parametrize("func", [R, A, FP])
def test_symmetric_larger_n_and_default_chunk(gpu_lib, func):
    for n, npts in ((64, 40), (128, 6), (256, 2), (512, 2)):
        if func != FP and n > 256:
            continue
        w = inputs.make_workload(func, n, npts, inputs.rng_for(6300 + 10 * func + n))
        E = _setup(gpu_lib, w)
        r = gpu_lib.chessfad_hvp_sym(func, _dev(w.x), _dev(w.v)).cpu().numpy()   # chunk = 0
        er, _ = _errs(w, E, r)
        print(f"  sym n={n} default chunk: err {er:.2e}", flush=True)
        assert er <= 1e-12


def test_symmetric_full_size_sampled(gpu_lib):
    """The n = 16, 2^20-point workload of the throughput measurement, checked
    on sampled points against the oracle's SC-HESS-VEC."""
    n, npts = 16, 1 << 20
    idx = np.random.default_rng(11).choice(npts, 64, replace=False)
    for func in (R, A, FP):
        w = inputs.make_workload(func, n, npts, inputs.rng_for(2 + func))
        E = _setup(gpu_lib, w)
        for c in (2, 4):
            r = gpu_lib.chessfad_hvp_sym(func, _dev(w.x), _dev(w.v), chunk=c).cpu().numpy()[idx]
            ro = chunked.hvp(func, w.x[idx], w.v[idx], c, w.A, w.B, E, sym=True, nthreads=4)
            scale = np.abs(cf.hessian(func, w.x[idx], w.A, w.B, E)).max(axis=(1, 2))
            err = (np.abs(r - ro).max(axis=1) / (scale * np.abs(w.v[idx]).max(axis=1))).max()
            assert err <= 1e-12, (func, c, err)


def test_symmetric_edge_cases(gpu_lib):
    # one point; empty input; a single-variable Ackley
    w = inputs.make_workload(A, 9, 1, inputs.rng_for(6400))
    r = gpu_lib.chessfad_hvp_sym(A, _dev(w.x), _dev(w.v), chunk=2).cpu().numpy()
    assert _errs(w, None, r)[0] <= 1e-12
    empty = torch.empty((0, 8), dtype=torch.float64, device="cuda")
    assert gpu_lib.chessfad_hvp_sym(R, empty, empty).shape == (0, 8)
    w = inputs.make_workload(A, 1, 5, inputs.rng_for(6401))
    H = gpu_lib.chessfad_hessian_sym(A, _dev(w.x), chunk=1).cpu().numpy()
    assert _errs(w, None, np.einsum("pij,pj->pi", H, w.v), H)[1] <= 1e-12


def test_autotune_sym_records_default(gpu_lib):
    for func in (R, A):
        c, ms = gpu_lib.chessfad_autotune_sym(func, 20, 0, npts=2048)
        assert c in (1, 2, 4, 8, 16) and ms > 0
        w = inputs.make_workload(func, 20, 33, inputs.rng_for(6500 + func))
        r = gpu_lib.chessfad_hvp_sym(func, _dev(w.x), _dev(w.v)).cpu().numpy()
        rc = gpu_lib.chessfad_hvp_sym(func, _dev(w.x), _dev(w.v), chunk=c).cpu().numpy()
        np.testing.assert_array_equal(r, rc)
