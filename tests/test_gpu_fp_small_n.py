"""Fletcher-Powell at n <= 16 on its two MFMA-assisted engines, at every n
from 1 to 16, both precisions, H.v, H.v with gradient and value, and
Hessians, against the float64 oracle; point counts that leave a pass (4
points), a wave (16 points) and a workgroup (64 points) partly filled, and a
single point.
  CHESSFAD_OPT_FP_MFMA = 1: the per-call kernel (the default), every chunk
    size <= n (ragged last chunks included);
  CHESSFAD_OPT_FP_MFMA = 3: the closed-form point tile (chunk-independent).
Bars as in the other GPU tests: normwise relative error <= 1e-12 (float64)
and the Fletcher-Powell mixed gate of tests/gates.py (the measured mixed
errors are printed).
"""
import numpy as np
import pytest
import torch

from oracle import closed_form as cf
from gates import TOL32 as TOL32_FP
from gates import TOL64
from paper_2410_22575_amd import inputs

pytestmark = pytest.mark.gpu

FP = 2
TOL32 = TOL32_FP[FP]
CHUNKS = (1, 2, 4, 8, 16)


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("engine", [1, 3])
@pytest.mark.parametrize("n", list(range(1, 17)))
def test_every_n(gpu_lib, engine, n):
    prev = gpu_lib.chessfad_set_option(gpu_lib.CHESSFAD_OPT_FP_MFMA, engine)
    try:
        _every_n(gpu_lib, engine, n)
    finally:
        gpu_lib.chessfad_set_option(gpu_lib.CHESSFAD_OPT_FP_MFMA, prev)


def _every_n(gpu_lib, engine, n):
    chunks = [c for c in CHUNKS if c <= n] if engine == 1 else [1 if n < 16 else 16]
    for npts in (1, 17, 70):
        w = inputs.make_workload(FP, n, npts, inputs.rng_for(9100 + 100 * n + npts))
        gpu_lib.chessfad_fp_set_params(_dev(w.A), _dev(w.B), _dev(w.alpha))
        E = cf.fp_offsets(w.A, w.B, w.alpha)
        H_ref = cf.hessian(FP, w.x, w.A, w.B, E)
        hmax = np.abs(H_ref).max(axis=(1, 2))
        vmax = np.abs(w.v).max(axis=1)
        r_ref = cf.hvp(FP, w.x, w.v, w.A, w.B, E)
        g_ref = cf.grad(FP, w.x, w.A, w.B, E)
        f_ref = cf.f(FP, w.x, w.A, w.B, E)
        x, v = _dev(w.x), _dev(w.v)
        for chunk in chunks:
            print(f"[case] engine={engine} n={n} npts={npts} chunk={chunk}", flush=True)
            for fn, fh, tol in ((gpu_lib.chessfad_hvp, gpu_lib.chessfad_hessian, TOL64),
                                (gpu_lib.chessfad_hvp_mixed, gpu_lib.chessfad_hessian_mixed, TOL32)):
                r = fn(FP, x, v, chunk=chunk).cpu().numpy()
                e_r = (np.abs(r - r_ref).max(axis=1) / (hmax * vmax)).max()
                H = fh(FP, x, chunk=chunk).cpu().numpy()
                e_H = (np.abs(H - H_ref).max(axis=(1, 2)) / hmax).max()
                if tol == TOL32:
                    print(f"  max rel err: hvp {e_r:.3e}  hessian {e_H:.3e}", flush=True)
                assert e_r <= tol and e_H <= tol, (n, npts, chunk)
            out, g, f = gpu_lib.chessfad_hvp_grad(FP, x, v, chunk=chunk)
            gscale = np.maximum(1.0, np.abs(g_ref).max(axis=1))
            assert (np.abs(g.cpu().numpy() - g_ref).max(axis=1) / gscale).max() <= TOL64, (n, npts, chunk)
            assert (np.abs(f.cpu().numpy() - f_ref) / np.maximum(1.0, np.abs(f_ref))).max() <= TOL64, (n, npts)
            assert (np.abs(out.cpu().numpy() - r_ref).max(axis=1) / (hmax * vmax)).max() <= TOL64, (n, npts)


def test_per_call_hessian_entries_chunk_invariant(gpu_lib):
    """In the per-call kernel an entry (i, k) is the same sum over m of the
    same products J_mi J_mk (plus the own term), whatever call carries it: the
    Hessians at every chunk size agree bit for bit, float64 and mixed."""
    n, npts = 16, 200
    w = inputs.make_workload(FP, n, npts, inputs.rng_for(9190))
    gpu_lib.chessfad_fp_set_params(_dev(w.A), _dev(w.B), _dev(w.alpha))
    x = _dev(w.x)
    for fh in (gpu_lib.chessfad_hessian, gpu_lib.chessfad_hessian_mixed):
        first = fh(FP, x, chunk=1)
        for c in (2, 4, 8, 16):
            assert torch.equal(fh(FP, x, chunk=c), first), c
