"""User functions (chessfad_register_function): f written once over the
hDual type of chessfad_device.h, compiled at run time, run by chessfad_hvp
and chessfad_hessian.  Bars as the other float64 parity tests (1e-12 normwise):
against the closed forms for Rosenbrock and Ackley written as user code,
and against the oracle's four-component brute force for a function that uses
every operator."""
import numpy as np
import pytest
import torch

from oracle import closed_form as cf
from oracle import hyperdual
from paper_2410_22575_amd import inputs

import user_functions as uf

pytestmark = pytest.mark.gpu

R, A = 0, 1
TOL = 1e-12


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _check(gpu_lib, fid, x, v, H_ref, chunks):
    n = x.shape[1]
    hmax = np.abs(H_ref).max(axis=(1, 2))
    r_ref = np.einsum("pij,pj->pi", H_ref, v)
    for c in chunks:
        if c > n:
            continue
        print(f"[case] user func={fid} n={n} C={c}", flush=True)
        H = gpu_lib.chessfad_hessian(fid, _dev(x), chunk=c).cpu().numpy()
        r = gpu_lib.chessfad_hvp(fid, _dev(x), _dev(v), chunk=c).cpu().numpy()
        assert np.max(np.abs(H - H_ref).max(axis=(1, 2)) / hmax) <= TOL, c
        e = np.abs(r - r_ref).max(axis=1) / (hmax * np.abs(v).max(axis=1))
        assert np.max(e) <= TOL, c


@pytest.fixture(scope="module")
def user_ids(gpu_lib):
    ids = {name: gpu_lib.chessfad_register_function(src)
           for name, src in (("rosenbrock", uf.ROSENBROCK_HIP), ("ackley", uf.ACKLEY_HIP),
                             ("mixed", uf.MIXED_OPS_HIP))}
    yield ids
    for fid in ids.values():
        gpu_lib.chessfad_release_function(fid)


@pytest.mark.parametrize("n", [2, 7, 16, 33])
def test_user_rosenbrock_against_closed_form(gpu_lib, user_ids, n):
    w = inputs.make_workload(R, n, 61, inputs.rng_for(9600 + n))
    _check(gpu_lib, user_ids["rosenbrock"], w.x, w.v, cf.hessian(R, w.x), (1, 2, 4, 8, 16))
    # and against the built-in kernel
    fid = user_ids["rosenbrock"]
    r_user = gpu_lib.chessfad_hvp(fid, _dev(w.x), _dev(w.v), chunk=min(4, n)).cpu().numpy()
    r_lib = gpu_lib.chessfad_hvp(R, _dev(w.x), _dev(w.v), chunk=min(4, n)).cpu().numpy()
    scale = np.abs(r_lib).max() + 1e-300
    assert np.abs(r_user - r_lib).max() <= 1e-13 * scale


@pytest.mark.parametrize("n", [3, 16, 40])
def test_user_ackley_against_closed_form(gpu_lib, user_ids, n):
    w = inputs.make_workload(A, n, 45, inputs.rng_for(9700 + n))
    _check(gpu_lib, user_ids["ackley"], w.x, w.v, cf.hessian(A, w.x), (1, 4, 16))


@pytest.mark.parametrize("n", [6, 9])
def test_user_operator_set_against_bruteforce(gpu_lib, user_ids, n):
    rng = np.random.default_rng(9800 + n)
    x = rng.uniform(-1.0, 1.0, (12, n))
    x[:6, 0] = np.abs(x[:6, 0])      # both sides of the branch on y[0]
    x[6:, 0] = -np.abs(x[6:, 0])
    v = rng.standard_normal((12, n))
    H_ref = np.array([hyperdual.hessian(uf.mixed_ops_py, list(p)) for p in x])
    _check(gpu_lib, user_ids["mixed"], x, v, H_ref, (1, 2, 4, 8))


def test_user_edge_cases(gpu_lib, user_ids):
    fid = user_ids["rosenbrock"]
    empty = torch.empty((0, 5), dtype=torch.float64, device="cuda")
    assert gpu_lib.chessfad_hvp(fid, empty, empty).shape == (0, 5)
    w = inputs.make_workload(R, 5, 1, inputs.rng_for(9900))
    r = gpu_lib.chessfad_hvp(fid, _dev(w.x), _dev(w.v)).cpu().numpy()       # chunk 0
    H = cf.hessian(R, w.x)
    assert np.abs(r - np.einsum("pij,pj->pi", H, w.v)).max() <= TOL * np.abs(H).max() * np.abs(w.v).max()
    with pytest.raises(gpu_lib.ChessfadError) as ei:
        gpu_lib.chessfad_hvp_mixed(fid, _dev(w.x), _dev(w.v))
    assert ei.value.code == -1


@pytest.mark.parametrize("n", [3, 16])
def test_user_fletcher_powell_against_closed_form(gpu_lib, n):
    """Fletcher-Powell written once over the generic hDual, its parameter set
    as constants in the source (the package's user_sources), every chunk."""
    from paper_2410_22575_amd import user_sources

    w = inputs.make_workload(2, n, 33, inputs.rng_for(9650 + n))
    E = cf.fp_offsets(w.A, w.B, w.alpha)
    fid = gpu_lib.chessfad_register_function(user_sources.fletcher_powell_hip(w.A, w.B, E))
    try:
        _check(gpu_lib, fid, w.x, w.v, cf.hessian(2, w.x, w.A, w.B, E), (1, 2, 4, 8, 16))
    finally:
        gpu_lib.chessfad_release_function(fid)
