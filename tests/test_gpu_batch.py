"""Batched plans (persistent kernel, hipGraph replay) and the autotuner,
through the C ABI.

Bars: against the float64 oracle, 1e-12 (precision 0) and the mixed gates
of tests/gates.py (mixed) in the normwise H.v error of the other GPU tests; against single-instance calls
of the library, bit-for-bit where both run the same workgroup body
(Rosenbrock, Ackley) and 1e-13 where the single-call Fletcher-Powell
kernels sum the residuals in another order or a one-chunk row runs on the
single call's L1 kernel.
"""
import numpy as np
import pytest
import torch

from gates import TOL32, TOL32_ANY, TOL_IO32_F64

from oracle import closed_form as cf
from paper_2410_22575_amd import inputs

pytestmark = pytest.mark.gpu

R, A, FP = 0, 1, 2


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _make(workloads, precision=0, chunk=0):
    insts = []
    for w in workloads:
        d = {"func_id": w.func, "x": _dev(w.x), "v": _dev(w.v), "out": torch.full((w.npts, w.n), np.nan,
             dtype=torch.float64, device="cuda"), "precision": precision, "chunk": chunk}
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


def _workloads(seed, count, nmin, nmax, npts_choices=(1,)):
    rng = inputs.rng_for(seed)
    out = []
    for _ in range(count):
        func = int(rng.integers(0, 3))
        n = int(round(nmin * (nmax / nmin) ** rng.uniform()))
        npts = int(rng.choice(npts_choices))
        out.append(inputs.make_workload(func, max(n, 2), npts, rng))
    return out


@pytest.mark.parametrize("chunk", [0, 2, 4, 8])
def test_batch_float64_matches_oracle_and_single_calls(gpu_lib, chunk):
    ws = _workloads(9000 + chunk, 48, 8, 40, npts_choices=(1, 2, 5))
    insts = _make(ws, precision=0, chunk=chunk)
    print(f"[case] batch f64 chunk={chunk}: {len(ws)} instances", flush=True)
    plan = gpu_lib.chessfad_batch_create(insts)
    plan.run()
    torch.cuda.synchronize()
    info = plan.info()
    assert info["items"] > 0 and info["workgroups"] > 0 and info["model_flops"] > 0
    for w, d in zip(ws, insts):
        got = d["out"].cpu().numpy()
        assert np.all(np.isfinite(got))
        assert _oracle_err(w, got) <= 1e-12, (w.func, w.n, w.npts)
        # the same instance through the single-instance entry point
        c = chunk or gpu_lib.chessfad_default_chunk(w.func, w.n)
        c = min(c, 8)
        if w.func == FP:
            gpu_lib.chessfad_fp_set_params(d["A"], d["B"], d["alpha"])
        single = gpu_lib.chessfad_hvp(w.func, d["x"], d["v"], chunk=c).cpu().numpy()
        if chunk:
            one_chunk = c >= w.n  # the single call then runs its L1 kernel
            # single Fletcher-Powell calls run the per-call kernels, which sum
            # the residuals in another order than the batch's body
            if w.func == FP or one_chunk:
                scale = np.abs(single).max() + 1e-300
                assert np.abs(got - single).max() <= 1e-13 * scale
            else:
                np.testing.assert_array_equal(got, single)
    plan.destroy()


def test_batch_mixed_precision(gpu_lib):
    ws = _workloads(9100, 40, 8, 64, npts_choices=(1, 3))
    insts = _make(ws, precision=1)
    plan = gpu_lib.chessfad_batch_create(insts)
    plan.run()
    torch.cuda.synchronize()
    worst = 0.0
    for w, d in zip(ws, insts):
        e = _oracle_err(w, d["out"].cpu().numpy())
        worst = max(worst, e)
        assert e <= TOL32[w.func], (w.func, w.n)
    print(f"  mixed batch max rel err {worst:.3e}", flush=True)
    assert worst > 0.0


def test_batch_both_precisions_in_one_plan(gpu_lib):
    ws = _workloads(9200, 24, 8, 24)
    insts = _make(ws, precision=0)
    for k in range(0, len(insts), 2):
        insts[k]["precision"] = 1
    plan = gpu_lib.chessfad_batch_create(insts)
    plan.run()
    torch.cuda.synchronize()
    for k, (w, d) in enumerate(zip(ws, insts)):
        assert _oracle_err(w, d["out"].cpu().numpy()) <= (TOL32[w.func] if k % 2 == 0 else 1e-12)


def test_graph_replays_and_direct_launch(gpu_lib):
    """Replay the captured graph several times with the program's own eager
    work and synchronisations in between; every replay must reproduce the
    first bit for bit, and so must the direct (uncaptured) launch."""
    ws = _workloads(9300, 32, 8, 48, npts_choices=(1, 4))
    insts = _make(ws, precision=1)
    plan = gpu_lib.chessfad_batch_create(insts)
    plan.run()
    torch.cuda.synchronize()
    first = [d["out"].clone() for d in insts]
    scratch = torch.randn(1 << 20, device="cuda", dtype=torch.float64)
    w0 = inputs.make_workload(A, 12, 100, inputs.rng_for(9301))
    for rep in range(3):
        for d in insts:
            d["out"].fill_(np.nan)
        scratch.mul_(1.0001).add_(0.5)                                 # eager work between replays
        gpu_lib.chessfad_hvp(A, _dev(w0.x), _dev(w0.v), chunk=4)
        torch.cuda.synchronize()
        plan.run()
        torch.cuda.synchronize()
        for f, d in zip(first, insts):
            assert torch.equal(f, d["out"]), f"replay {rep}"
    prev = gpu_lib.chessfad_set_option(gpu_lib.CHESSFAD_OPT_BATCH_GRAPH, 0)
    try:
        for d in insts:
            d["out"].fill_(np.nan)
        plan.run()
        torch.cuda.synchronize()
    finally:
        gpu_lib.chessfad_set_option(gpu_lib.CHESSFAD_OPT_BATCH_GRAPH, prev)
    for f, d in zip(first, insts):
        assert torch.equal(f, d["out"])


def test_batch_log_uniform_sizes_sampled(gpu_lib):
    """The shape of the batched workload (single-point instances, n
    log-uniform in [8, 256], mixed functions) at 192 instances."""
    ws = inputs.mixed_instances(192, inputs.rng_for(4), 8, 256, npts=1)
    insts = _make(ws, precision=1)
    plan = gpu_lib.chessfad_batch_create(insts)
    plan.run()
    torch.cuda.synchronize()
    idx = np.random.default_rng(3).choice(len(ws), 48, replace=False)
    worst = max(_oracle_err(ws[k], insts[k]["out"].cpu().numpy()) for k in idx)
    print(f"  log-uniform batch max rel err {worst:.3e}", flush=True)
    assert worst <= TOL32_ANY


def test_autotune_records_default(gpu_lib):
    for func in (R, A):
        c, ms = gpu_lib.chessfad_autotune(func, 24, 0, npts=4096)
        assert c in (1, 2, 4, 8, 16) and ms > 0
        assert gpu_lib.chessfad_default_chunk(func, 24) == c
        level = gpu_lib.chessfad_default_mapping(func, 24)
        assert level in (1, 2)
        # chunk = 0 now runs the tuned chunk and mapping
        w = inputs.make_workload(func, 24, 40, inputs.rng_for(9450 + func))
        d = _make([w])[0]
        r = gpu_lib.chessfad_hvp(func, d["x"], d["v"]).cpu().numpy()
        assert _oracle_err(w, r) <= 1e-12
    w = inputs.make_workload(FP, 20, 4, inputs.rng_for(9400))
    gpu_lib.chessfad_fp_set_params(_dev(w.A), _dev(w.B), _dev(w.alpha))
    c, ms = gpu_lib.chessfad_autotune(FP, 20, 1, npts=512)
    assert c in (1, 2, 4, 8, 16) and ms > 0


def test_batch_errors_name_the_instance(gpu_lib):
    ws = _workloads(9500, 3, 8, 16)
    insts = _make(ws)
    insts[1]["chunk"] = 32   # not a compiled chunk
    with pytest.raises(gpu_lib.ChessfadError) as ei:
        gpu_lib.chessfad_batch_create(insts)
    assert ei.value.code == -3 and ei.value.bad_index == 1


@pytest.mark.parametrize("precision", [0, 1])
def test_batch_float32_io(gpu_lib, precision):
    """io_fp32: x, v and out as float32.  Against the oracle evaluated at the
    float32 inputs (widened exactly): the float64 path to its float32-I/O
    gate (the float32 rounding of the output dominates), the mixed path to
    the mixed gates; and against the same instances with float64 I/O to the
    same bars."""
    ws = _workloads(9600 + precision, 36, 8, 96, npts_choices=(1, 3))
    for w in ws:
        w.x = w.x.astype(np.float32).astype(np.float64)
        w.v = w.v.astype(np.float32).astype(np.float64)
    i64 = _make(ws, precision=precision)
    i32 = []
    for d in i64:
        e = dict(d)
        e["x"], e["v"] = d["x"].float(), d["v"].float()
        e["out"] = torch.full(d["out"].shape, np.nan, dtype=torch.float32, device="cuda")
        i32.append(e)
    print(f"[case] batch float32 io precision={precision}: {len(ws)} instances", flush=True)
    for insts in (i64, i32):
        plan = gpu_lib.chessfad_batch_create(insts)
        plan.run()
        torch.cuda.synchronize()
        plan.destroy()
    worst = 0.0
    for w, a, b in zip(ws, i64, i32):
        bar = TOL_IO32_F64 if precision == 0 else TOL32[w.func]
        got = b["out"].double().cpu().numpy()
        assert np.all(np.isfinite(got)), (w.func, w.n)
        e = _oracle_err(w, got)
        worst = max(worst, e)
        assert e <= bar, (w.func, w.n)
        ref = a["out"].cpu().numpy()
        scale = np.abs(ref).max(axis=1, keepdims=True) + 1e-300
        assert np.max(np.abs(got - ref) / scale) <= bar, (w.func, w.n)
    print(f"  float32 io max rel err {worst:.3e}", flush=True)


def test_batch_plan_time_tuning(gpu_lib):
    """chunk = 0 instances are tuned per (function, octave of n, precision) on
    the plan's own instances: one choice per group, each a configuration the
    bodies are compiled for, and the results still match the oracle."""
    ws = _workloads(9700, 60, 8, 200, npts_choices=(1, 2))
    insts = _make(ws, precision=0)
    prev = gpu_lib.chessfad_set_option(gpu_lib.CHESSFAD_OPT_BATCH_TUNE, 1)
    try:
        plan = gpu_lib.chessfad_batch_create(insts)
    finally:
        gpu_lib.chessfad_set_option(gpu_lib.CHESSFAD_OPT_BATCH_TUNE, prev)
    choices = plan.choices()
    groups = {(w.func, int(np.floor(np.log2(w.n)))) for w in ws}
    assert len(choices) == len(groups)
    for ch in choices:
        print(f"  choice {ch}", flush=True)
        assert ch["chunk"] in (1, 2, 4, 8, 16) and ch["chunk"] <= ch["n_lo"]
        assert ch["candidates"] >= 1 and ch["ms"] > 0 and ch["instances"] >= 1
        if ch["func_id"] == FP:
            assert ch["points"] in (0, 1, 4, 16) and ch["blocks"] in (0, 16)
        else:
            assert ch["mapping"] in (1, 2)
            assert ch["mapping"] == 1 or ch["chunk"] <= 8
    assert sum(ch["instances"] for ch in choices) == len(ws)
    for d in insts:
        d["out"].fill_(np.nan)
    plan.run()
    torch.cuda.synchronize()
    for w, d in zip(ws, insts):
        assert _oracle_err(w, d["out"].cpu().numpy()) <= 1e-12, (w.func, w.n)
    plan.destroy()
