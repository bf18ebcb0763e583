"""The allocation-free batched entry point (chessfad_batch_run_noalloc)
against a plan of the same instances (chessfad_batch_create + run, without
plan-time tuning), through the C ABI.

Both place the same work items on the same kernels, so the bar is ③'s
float64 bar met exactly: the outputs must agree bit for bit (and, as a
check of the inputs, both stay within the float64 oracle bar 1e-12 of the
other batch tests).  Two calls in a row, the second with fewer and smaller
instances, both precisions: the second call reuses the array the first one
filled.
"""
import numpy as np
import pytest
import torch

from oracle import closed_form as cf
from paper_2410_22575_amd import inputs

pytestmark = pytest.mark.gpu

FP = 2


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _workloads(seed, count, nmin, nmax):
    rng = inputs.rng_for(seed)
    out = []
    for _ in range(count):
        func = int(rng.integers(0, 3))
        n = max(2, int(round(nmin * (nmax / nmin) ** rng.uniform())))
        npts = int(rng.choice((1, 3)))
        out.append(inputs.make_workload(func, n, npts, rng))
    return out


def _instances(ws, precision):
    insts = []
    for w in ws:
        d = {"func_id": w.func, "x": _dev(w.x), "v": _dev(w.v), "precision": precision,
             "out": torch.full((w.npts, w.n), np.nan, dtype=torch.float64, device="cuda")}
        if w.func == FP:
            d.update(A=_dev(w.A), B=_dev(w.B), alpha=_dev(w.alpha))
        insts.append(d)
    return insts


def _oracle_err(w, out):
    E = cf.fp_offsets(w.A, w.B, w.alpha) if w.func == FP else None
    H = cf.hessian(w.func, w.x, w.A, w.B, E)
    ref = np.einsum("pij,pj->pi", H, w.v)
    scale = np.abs(H).max(axis=(1, 2)) * np.abs(w.v).max(axis=1)
    return float((np.abs(out - ref).max(axis=1) / scale).max())


@pytest.mark.parametrize("precision", [0, 1])
def test_noalloc_matches_planned_batch_twice(gpu_lib, precision):
    for call, (count, nmax) in enumerate(((60, 96), (17, 24))):
        ws = _workloads(31000 + 10 * precision + call, count, 8, nmax)
        print(f"[case] noalloc precision={precision} call={call}: {count} instances, n <= {nmax}", flush=True)
        ref = _instances(ws, precision)
        # a plan of the same instances without plan-time tuning: the same work items
        prev = gpu_lib.chessfad_set_option(gpu_lib.CHESSFAD_OPT_BATCH_TUNE, 0)
        try:
            plan = gpu_lib.chessfad_batch_create(ref)
        finally:
            gpu_lib.chessfad_set_option(gpu_lib.CHESSFAD_OPT_BATCH_TUNE, prev)
        plan.run()
        torch.cuda.synchronize()
        plan.destroy()
        got = _instances(ws, precision)
        gpu_lib.chessfad_batch_run_noalloc(got)
        for w, a, b in zip(ws, ref, got):
            ra, rb = a["out"].cpu().numpy(), b["out"].cpu().numpy()
            assert np.all(np.isfinite(rb)), (call, w.func, w.n)
            np.testing.assert_array_equal(rb, ra)
            if precision == 0:
                assert _oracle_err(w, rb) <= 1e-12, (call, w.func, w.n)


def test_noalloc_rejects_a_plan_larger_than_its_array(gpu_lib):
    # mixed Fletcher-Powell at n = 512 keeps two float32 copies of A and B
    # (2 MiB); 40 such instances need more than the 64 MiB array
    w = inputs.make_workload(FP, 512, 1, inputs.rng_for(31900))
    insts = _instances([w] * 40, 1)
    with pytest.raises(gpu_lib.ChessfadError) as e:
        gpu_lib.chessfad_batch_run_noalloc(insts)
    assert e.value.code == -8
    assert np.all(np.isnan(insts[0]["out"].cpu().numpy()))
