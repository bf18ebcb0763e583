"""Benchmark: Hessian-vector products per second on one MI355X.

One step = one pass of the whole hot path over one batch: float64 chunked
H.v for Rosenbrock, Ackley and Fletcher-Powell, each at n = 16 over 2^20
resident points (seeded synthetic inputs), three launches through the C ABI.
`value` is the total HVPs of a step divided by the step time.

Also reported:
  roofline      the dominant kernel's paper-model flops per launch divided by
                its average launch time (HIP events around each launch inside
                the timed region), against the float64 vector peak;
  cpu_baseline  the CPU oracle's chunked method (plain C, OpenMP over points,
                all host cores) timed on a bounded sample of the same inputs.

    python bench.py [--steps K] [--warmup W] [--chunk C] [--no-cpu]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

FUNCS = (0, 1, 2)
NAMES = {0: "rosenbrock", 1: "ackley", 2: "fletcher_powell"}
N = 16
NPTS = 1 << 20
PEAK_F64_TFLOPS = 78.6   # 256 CUs x 2.4 GHz x 128 float64 flops per CU-clock (FMA = 2), vector and MFMA
METRIC = "HVPs/sec at n=16..512; FP32/batched vs FP64 plain on same GPU at stated error"

# HBM bytes per launch from rocprofv3 FETCH_SIZE (x 2.0) and WRITE_SIZE (x 1.0,
# copy-kernel calibration), keyed by the kernel as it stood when the counters
# were taken; a kernel absent here reports traffic null.
MEASURED_TRAFFIC = {
    "coarse_kernel<ackley, C=1, L1, H.v>": 4.0275e+08,
    "coarse_kernel<ackley, C=2, L1, H.v>": 4.0276e+08,
    "coarse_kernel<ackley, C=4, L1, H.v>": 4.0276e+08,
    "coarse_kernel<ackley, C=8, L1, H.v>": 4.0277e+08,
    "coarse_kernel<ackley, C=16, L1, H.v>": 4.0280e+08,
    "coarse_kernel<rosenbrock, C=1, L1, H.v>": 4.0271e+08,
    "coarse_kernel<rosenbrock, C=2, L1, H.v>": 4.0270e+08,
    "coarse_kernel<rosenbrock, C=4, L1, H.v>": 4.0271e+08,
    "coarse_kernel<rosenbrock, C=8, L1, H.v>": 4.0274e+08,
    "coarse_kernel<rosenbrock, C=16, L1, H.v>": 4.0277e+08,
    "fp_tile_kernel<NK=8, H.v>": 4.0292e+08,
}

# float64 flops the vector ALUs execute per launch (rocprofv3
# SQ_INSTS_VALU_FLOPS_FP64, which counts per wavefront, x 64 lanes; FMA = 2),
# same keying and rule as MEASURED_TRAFFIC.  The kernels execute fewer flops
# than the paper's operation model counts: first-order seeds carry no
# second-order part and the compiler folds the constant seed components.
MEASURED_VALU_FLOPS = {
    "coarse_kernel<ackley, C=1, L1, H.v>": 2.2951e+10,
    "coarse_kernel<ackley, C=2, L1, H.v>": 1.4093e+10,
    "coarse_kernel<ackley, C=4, L1, H.v>": 9.6637e+09,
    "coarse_kernel<ackley, C=8, L1, H.v>": 7.4491e+09,
    "coarse_kernel<ackley, C=16, L1, H.v>": 6.3418e+09,
    "coarse_kernel<rosenbrock, C=1, L1, H.v>": 4.5298e+09,
    "coarse_kernel<rosenbrock, C=2, L1, H.v>": 4.1272e+09,
    "coarse_kernel<rosenbrock, C=4, L1, H.v>": 3.9259e+09,
    "coarse_kernel<rosenbrock, C=8, L1, H.v>": 3.8252e+09,
    "coarse_kernel<rosenbrock, C=16, L1, H.v>": 3.7749e+09,
    "fp_tile_kernel<NK=8, H.v>": 3.8588e+09,
}

# VALU wave-instructions per launch (rocprofv3 SQ_INSTS_VALU, MFMA included),
# same keying and rule as MEASURED_TRAFFIC.  A CU issues at most one vector
# wave-instruction per clock (four SIMDs, four clocks per wave64 instruction),
# so count / (256 CUs x 2.4 GHz) is the launch's minimum issue time.
MEASURED_VALU_INSTS = {
    "coarse_kernel<ackley, C=1, L1, H.v>": 7.3374e+08,
    "coarse_kernel<ackley, C=2, L1, H.v>": 4.3988e+08,
    "coarse_kernel<ackley, C=4, L1, H.v>": 2.8888e+08,
    "coarse_kernel<ackley, C=8, L1, H.v>": 2.1339e+08,
    "coarse_kernel<ackley, C=16, L1, H.v>": 1.7564e+08,
    "coarse_kernel<rosenbrock, C=1, L1, H.v>": 1.4523e+08,
    "coarse_kernel<rosenbrock, C=2, L1, H.v>": 1.2321e+08,
    "coarse_kernel<rosenbrock, C=4, L1, H.v>": 1.1141e+08,
    "coarse_kernel<rosenbrock, C=8, L1, H.v>": 1.0774e+08,
    "coarse_kernel<rosenbrock, C=16, L1, H.v>": 1.0302e+08,
    "fp_tile_kernel<NK=8, H.v>": 9.3979e+07,
}


def kernel_key(f, c, n=N, mapping=2):
    """The kernel chessfad_hvp runs for (function, chunk, mapping) at n, as
    keyed in the measured tables: the n <= 16 Fletcher-Powell MFMA kernel,
    the L1 kernel when a row has a single chunk or L1 was chosen, else the
    L2 vector kernel."""
    if f == 2 and n <= 16:
        return f"fp_tile_kernel<NK={min(8, max(1, (2 * n + 3) // 4))}, H.v>"
    if c >= n or mapping == 1:
        return f"coarse_kernel<{NAMES[f]}, C={c}, L1, H.v>"
    return f"plain_kernel<{NAMES[f]}, C={c}, H.v>"


def fp_mfma_flops(n, c, npts):
    """MFMA flops the n <= 16 Fletcher-Powell float64 kernel executes per
    launch: per 16-point wave, NK steps of 16x16x4 for the value column, and
    per point ceil(n / 4) steps for its 16 x 16 tile J^T J; 2 x 16 x 16 x 4
    flops per step.  The chunk size does not change it."""
    nk = min(8, max(1, (2 * n + 3) // 4))
    steps = nk + 16 * ((n + 3) // 4)
    return steps * 2 * 16 * 16 * 4 * (npts / 16)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--chunk", type=int, default=0, help="0 = library default per function")
    ap.add_argument("--npts", type=int, default=NPTS)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-tune", action="store_true", help="use the default chunk instead of autotuning it")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched mixed-instance workload")
    ap.add_argument("--batch-instances", type=int, default=8192)
    ap.add_argument("--large", action="store_true",
                    help="also time n=64 (2^18 points, float64 and mixed) and n=512 (1024 points) H.v")
    ap.add_argument("--only", choices=("large", "batch"), default=None,
                    help="only run the large-n timings or the batched workload and print their JSON "
                         "(for profiling; not the benchmark line)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB (calibrates HBM byte counters)")
    return ap.parse_args()


def copy_probe(mib, reps=3):
    """A plain copy kernel of known size: each launch reads and writes
    exactly `mib` MiB, so FETCH_SIZE / WRITE_SIZE per dispatch should read
    mib * 1024 KiB each; the ratio calibrates the counters."""
    import torch

    n = mib * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_mib": mib, "reps": reps, "kib_per_launch_each_way": mib * 1024}), flush=True)


def cpu_baseline(workloads, E, chunks, budget_s):
    """Time the oracle's chunked CHESS-VEC (C, OpenMP) on a bounded sample."""
    from oracle import chunked

    chunked.build()
    threads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    # calibrate on a small sample, then size the sample to the budget
    sample = 64
    while True:
        t0 = time.perf_counter()
        for f in FUNCS:
            w = workloads[f]
            chunked.hvp(f, w.x[:sample], w.v[:sample], chunks[f], w.A, w.B, E[f], nthreads=threads)
        dt = time.perf_counter() - t0
        if dt > 0.5 or sample >= 1 << 16:
            break
        sample *= 2
    sample = int(min(NPTS, max(sample, sample * budget_s / max(dt, 1e-9))))
    t0 = time.perf_counter()
    per = {}
    for f in FUNCS:
        w = workloads[f]
        t1 = time.perf_counter()
        chunked.hvp(f, w.x[:sample], w.v[:sample], chunks[f], w.A, w.B, E[f], nthreads=threads)
        per[NAMES[f]] = sample / (time.perf_counter() - t1)
    dt = time.perf_counter() - t0
    return {"value": 3 * sample / dt, "unit": "HVP/s", "cores": threads, "kind": "oracle",
            "sample": f"first {sample} of the {NPTS} points of each function (n=16, same chunk sizes), "
                      f"oracle/chunked.c CHESS-VEC with OpenMP over points",
            "per_function": per}


def large_n(binding, inputs, cf, torch, flops):
    """n = 64 over 2^18 points (all three functions, float64 and mixed) and
    n = 512 over 1024 points (Fletcher-Powell float64 and mixed, Rosenbrock
    float64): kernel time, HVP/s, paper-model TFLOP/s and the max error on
    sampled points."""
    dev = torch.device("cuda:0")
    res = {}
    cases = [(f, 64, 1 << 18, prec) for f in FUNCS for prec in (0, 1)]
    cases += [(2, 512, 1024, 1), (2, 512, 1024, 0), (0, 512, 1024, 0)]
    for f, n, npts, prec in cases:
        w = inputs.make_workload(f, n, npts, inputs.rng_for(100 + n))
        x, v = torch.from_numpy(w.x).to(dev), torch.from_numpy(w.v).to(dev)
        E = None
        if f == 2:
            binding.chessfad_fp_set_params(*(torch.from_numpy(a).to(dev) for a in (w.A, w.B, w.alpha)))
            E = cf.fp_offsets(w.A, w.B, w.alpha)
        # autotuned chunk (and mapping) except for Fletcher-Powell at n = 512,
        # where one launch per chunk takes about a second: C = 16 there
        if f == 2 and n == 512:
            c = call_c = 16
        else:
            c, _ = binding.chessfad_autotune(f, n, prec, npts=min(npts, 1 << 16))
            call_c = 0  # the tuned chunk and, for float64 on the vector ALUs, mapping
        fn = binding.chessfad_hvp_mixed if prec else binding.chessfad_hvp
        out = fn(f, x, v, chunk=call_c)
        torch.cuda.synchronize()
        reps = 1 if n == 512 and f == 2 else 3
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn(f, x, v, out, chunk=call_c)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        idx = np.random.default_rng(2).choice(npts, min(64, npts), replace=False)
        H = cf.hessian(f, w.x[idx], w.A, w.B, E)
        ref = np.einsum("pij,pj->pi", H, w.v[idx])
        got = out.cpu().numpy()[idx]
        err = float((np.abs(got - ref).max(axis=1) / (np.abs(H).max(axis=(1, 2)) * np.abs(w.v[idx]).max(axis=1))).max())
        mf = flops.flops_per_hvp(f, n, c)
        res[f"{NAMES[f]}_n{n}_{'mixed' if prec else 'f64'}"] = {
            "npts": npts, "chunk": c,
            "mapping": "MFMA" if f == 2 else (f"L{binding.chessfad_default_mapping(f, n, prec)}" if call_c == 0
                                              else "L2"),
            "kernel_ms": ms, "hvps_per_s": npts / (ms * 1e-3),
            "model_tflops": mf * npts / (ms * 1e-3) / 1e12, "max_rel_err_sampled": err}
        print(f"  large: {NAMES[f]} n={n} {'mixed' if prec else 'f64'} {ms:.2f} ms err {err:.2e}", file=sys.stderr, flush=True)
    return res


def batched(ninst, binding, inputs, cf, torch):
    """Mixed-function batch: `ninst` single-point instances, function uniform
    over the three, n log-uniform in [8, 256], each Fletcher-Powell instance
    with its own parameters.  Times one replay of the plan's hipGraph in
    float32-mixed and in float64, and the same instances as separate
    float64 chessfad_hvp launches (kernel time only, summed)."""
    ws = inputs.mixed_instances(ninst, inputs.rng_for(4), 8, 256, npts=1)
    dev = torch.device("cuda:0")
    insts = []
    for w in ws:
        d = {"func_id": w.func, "x": torch.from_numpy(w.x).to(dev), "v": torch.from_numpy(w.v).to(dev),
             "out": torch.empty((w.npts, w.n), dtype=torch.float64, device=dev)}
        if w.func == 2:
            d.update(A=torch.from_numpy(w.A).to(dev), B=torch.from_numpy(w.B).to(dev),
                     alpha=torch.from_numpy(w.alpha).to(dev))
        insts.append(d)
    torch.cuda.synchronize()

    def timed(plan, reps=3):
        plan.run()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            plan.run()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    res = {"workload": f"{ninst} single-point instances, function uniform over Rosenbrock/Ackley/Fletcher-Powell, "
                       "n log-uniform in [8, 256], own Fletcher-Powell parameters each; chunk per (function, n) "
                       "from the autotuned table or the default"}
    outs = {}
    for prec, name in ((1, "mixed_f32"), (0, "f64")):
        for d in insts:
            d["precision"] = prec
        plan = binding.chessfad_batch_create(insts)
        ms = timed(plan)
        info = plan.info()
        res[name] = {"graph_ms": ms, "hvps_per_s": ninst / (ms * 1e-3), "model_tflops": info["model_flops"] / (ms * 1e-3) / 1e12,
                     "items": info["items"], "workgroups": info["workgroups"]}
        outs[name] = [d["out"].clone() for d in insts]
        plan.destroy()
    # the same instances one launch each (float64), kernel time only
    total = 0.0
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for d, w in zip(insts, ws):
        if w.func == 2:
            binding.chessfad_fp_set_params(d["A"], d["B"], d["alpha"])
        e0.record()
        binding.chessfad_hvp(w.func, d["x"], d["v"], d["out"], chunk=min(4, w.n))
        e1.record()
        e1.synchronize()
        total += e0.elapsed_time(e1)
    res["per_instance_f64_kernel_ms_sum"] = total
    res["speedup_mixed_batched_vs_per_instance_f64"] = total / res["mixed_f32"]["graph_ms"]
    res["speedup_mixed_batched_vs_f64_batched"] = res["f64"]["graph_ms"] / res["mixed_f32"]["graph_ms"]
    # accuracy on a sample of instances
    idx = np.random.default_rng(11).choice(ninst, min(64, ninst), replace=False)
    for name in ("mixed_f32", "f64"):
        worst = 0.0
        for k in idx:
            w = ws[k]
            E = cf.fp_offsets(w.A, w.B, w.alpha) if w.func == 2 else None
            H = cf.hessian(w.func, w.x, w.A, w.B, E)
            ref = np.einsum("pij,pj->pi", H, w.v)
            got = outs[name][k].cpu().numpy()
            worst = max(worst, float((np.abs(got - ref).max(axis=1) / (np.abs(H).max(axis=(1, 2)) * np.abs(w.v).max(axis=1))).max()))
        res[name]["max_rel_err_sampled"] = worst
    return res


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported by this build "
              f"(points shard across GPUs with no communication; see DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    if args.copy_probe:
        copy_probe(args.copy_probe)
        return

    import torch

    from paper_2410_22575_amd import binding, flops, inputs
    from oracle import closed_form as cf

    binding.load()
    if args.only == "large":
        print(json.dumps({"large_n": large_n(binding, inputs, cf, torch, flops)}), flush=True)
        return
    if args.only == "batch":
        print(json.dumps({"batched": batched(args.batch_instances, binding, inputs, cf, torch)}), flush=True)
        return
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    npts = args.npts

    # seeded synthetic inputs, resident in HBM before timing
    workloads, E, xs, vs, outs, chunks = {}, {}, {}, {}, {}, {}
    for f in FUNCS:
        w = inputs.make_workload(f, N, npts, inputs.rng_for(1))
        workloads[f] = w
        xs[f] = torch.from_numpy(w.x).to(dev)
        vs[f] = torch.from_numpy(w.v).to(dev)
        outs[f] = torch.empty_like(xs[f])
        E[f] = None
        if f == 2:
            binding.chessfad_fp_set_params(torch.from_numpy(w.A).to(dev), torch.from_numpy(w.B).to(dev),
                                           torch.from_numpy(w.alpha).to(dev))
            E[f] = cf.fp_offsets(w.A, w.B, w.alpha)
    torch.cuda.synchronize()
    # chunk per function: explicit, autotuned (outside the timed region), or default
    tuned, mchunks, schunks = {}, {}, {}
    for f in FUNCS:
        if args.chunk:
            chunks[f] = mchunks[f] = schunks[f] = args.chunk
        elif not args.no_tune:
            chunks[f], tuned[NAMES[f]] = binding.chessfad_autotune(f, N, 0, npts=npts)
            mchunks[f], _ = binding.chessfad_autotune(f, N, 1, npts=npts)
            schunks[f], _ = binding.chessfad_autotune_sym(f, N, 0, npts=npts)
        else:
            chunks[f] = mchunks[f] = binding.chessfad_default_chunk(f, N)
            schunks[f] = 0
    torch.cuda.synchronize()

    # the step passes chunk 0 unless a chunk was forced: the library then runs
    # the tuned chunk and mapping
    step_chunk = {f: (args.chunk or 0) for f in FUNCS}
    mapping = {f: (args.chunk and 2) or binding.chessfad_default_mapping(f, N) for f in FUNCS}

    def step(events=None):
        for f in FUNCS:
            if events is not None:
                events[f][0].record()
            binding.chessfad_hvp(f, xs[f], vs[f], outs[f], chunk=step_chunk[f])
            if events is not None:
                events[f][1].record()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    evs = [{f: (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for f in FUNCS}
           for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(evs[k])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    kernel_ms = {f: float(np.mean([e[f][0].elapsed_time(e[f][1]) for e in evs])) for f in FUNCS}
    ms_per_step = 1e3 * elapsed / args.steps
    value = len(FUNCS) * npts / (elapsed / args.steps)

    per_func = {}
    for f in FUNCS:
        mf = flops.flops_per_hvp(f, N, chunks[f])
        per_func[NAMES[f]] = {
            "chunk": chunks[f], "mapping": f"L{mapping[f]}" if f != 2 or N > 16 else "MFMA",
            "kernel_ms": round(kernel_ms[f], 4),
            "hvps_per_s": npts / (kernel_ms[f] * 1e-3),
            "model_tflops": mf * npts / (kernel_ms[f] * 1e-3) / 1e12,
            "model_flops_per_hvp": mf,
        }
    for f in FUNCS:
        # executed flops where known: MFMA from the tile schedule, vector
        # float64 from the counters taken for this kernel
        key = kernel_key(f, chunks[f], mapping=mapping[f])
        ex = (fp_mfma_flops(N, chunks[f], npts) if key.startswith("fp_tile") else 0.0)
        valu = MEASURED_VALU_FLOPS.get(key)
        per_func[NAMES[f]]["executed_mfma_tflops"] = ex / (kernel_ms[f] * 1e-3) / 1e12 if ex else None
        per_func[NAMES[f]]["executed_valu_f64_tflops"] = valu / (kernel_ms[f] * 1e-3) / 1e12 if valu else None
    fp_mfma = N <= 16
    dom = max(FUNCS, key=lambda f: kernel_ms[f])
    kname = kernel_key(dom, chunks[dom], mapping=mapping[dom])
    model_launch = flops.flops_per_hvp(dom, N, chunks[dom]) * npts
    t_dom = kernel_ms[dom] * 1e-3
    if kname.startswith("fp_tile"):
        # executed MFMA flops (fewer than the model counts); float64 MFMA and
        # float64 VALU work do not overlap on MI355X (one float64 datapath,
        # measured), so the kernel's vector float64 flops count against the
        # same peak when their counters are known
        bound, work, basis = "mfma", fp_mfma_flops(N, chunks[dom], npts), "executed MFMA flops (tile schedule)"
        if kname in MEASURED_VALU_FLOPS:
            work += MEASURED_VALU_FLOPS[kname]
            basis += " + executed float64 VALU flops (counters)"
    elif kname in MEASURED_VALU_FLOPS:
        bound, work, basis = "alu", MEASURED_VALU_FLOPS[kname], "executed float64 VALU flops (counters)"
    else:
        bound, work, basis = "alu", model_launch, "paper-model flops"
    if work > model_launch:
        work, basis = model_launch, "paper-model flops (below the executed count)"
    achieved = work / t_dom / 1e12
    roofline = {"bound": bound, "kernel": kname, "achieved": achieved, "peak": PEAK_F64_TFLOPS,
                "unit": "TFLOP/s", "frac": achieved / PEAK_F64_TFLOPS, "traffic": MEASURED_TRAFFIC.get(kname),
                "flops_per_launch": work, "basis": basis, "model_flops_per_launch": model_launch,
                "model_tflops": model_launch / t_dom / 1e12}
    insts = MEASURED_VALU_INSTS.get(kname)
    # share of the launch the vector issue alone would take (1.0 = issue-bound)
    roofline["valu_issue_frac"] = insts / (256 * 2.4e9) / t_dom if insts else None
    if bound == "mfma":
        roofline["measured_mfma_f64_peak"] = 72.8
        valu = MEASURED_VALU_FLOPS.get(kname)
        roofline["executed_valu_f64_tflops"] = valu / t_dom / 1e12 if valu else None

    # the Fletcher-Powell vector-ALU path, for comparison (outside the timed region)
    fp_vector_ms = None
    if fp_mfma:
        # the vector path at its own best chunk (the MFMA tile ignores the chunk)
        vec_c = min(16, N)
        prev = binding.chessfad_set_option(binding.CHESSFAD_OPT_FP_MFMA, 0)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        binding.chessfad_hvp(2, xs[2], vs[2], outs[2], chunk=vec_c)
        e0.record()
        for _ in range(3):
            binding.chessfad_hvp(2, xs[2], vs[2], outs[2], chunk=vec_c)
        e1.record()
        torch.cuda.synchronize()
        fp_vector_ms = e0.elapsed_time(e1) / 3
        binding.chessfad_set_option(binding.CHESSFAD_OPT_FP_MFMA, prev)
        binding.chessfad_hvp(2, xs[2], vs[2], outs[2], chunk=vec_c)
        torch.cuda.synchronize()

    # quick sanity check of the last outputs on a few points (oracle on CPU)
    idx = np.arange(0, npts, max(1, npts // 64))
    refs = {}
    for f in FUNCS:
        w = workloads[f]
        H = cf.hessian(f, w.x[idx], w.A, w.B, E[f])
        refs[f] = (np.einsum("pij,pj->pi", H, w.v[idx]), np.abs(H).max(axis=(1, 2)) * np.abs(w.v[idx]).max(axis=1))

    def rel_err(f, out):
        ref, scale = refs[f]
        return float((np.abs(out.cpu().numpy()[idx] - ref).max(axis=1) / scale).max())

    max_err = {NAMES[f]: rel_err(f, outs[f]) for f in FUNCS}

    # full Hessians on the same points (outside the timed region): 8 n^2
    # bytes per point written on top of the H.v path's 16 n read
    hess = {}
    for f in FUNCS:
        sub = min(npts, 1 << 19)
        Hbuf = torch.empty((sub, N, N), dtype=torch.float64, device=dev)
        binding.chessfad_hessian(f, xs[f][:sub], Hbuf, chunk=chunks[f])
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(3):
            binding.chessfad_hessian(f, xs[f][:sub], Hbuf, chunk=chunks[f])
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 3
        hess[NAMES[f]] = {"npts": sub, "kernel_ms": round(ms, 4), "hessians_per_s": sub / (ms * 1e-3),
                          "hbm_gb_per_s": sub * (8 * N * N + 8 * N) / (ms * 1e-3) / 1e9}
        del Hbuf
    torch.cuda.synchronize()

    # the mixed-precision path on the same inputs (outside the timed region)
    mixed = {}
    for f in FUNCS:
        mo = torch.empty_like(xs[f])
        mc = mchunks[f]   # the mixed path's own tuned chunk
        # chunk 0 runs the tuned chunk and mapping (as the float64 step does)
        call_c = args.chunk or 0
        binding.chessfad_hvp_mixed(f, xs[f], vs[f], mo, chunk=call_c)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(5):
            binding.chessfad_hvp_mixed(f, xs[f], vs[f], mo, chunk=call_c)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 5
        mmap = "MFMA" if f == 2 and N <= 16 else f"L{binding.chessfad_default_mapping(f, N, 1)}" if not args.chunk else "L2"
        mixed[NAMES[f]] = {"chunk": mc, "mapping": mmap, "kernel_ms": round(ms, 4), "hvps_per_s": npts / (ms * 1e-3),
                           "speedup_vs_f64": kernel_ms[f] / ms, "max_rel_err_sampled": rel_err(f, mo)}

    # the paper's three GPU mappings of H.v (Sec. VI) for the vector-ALU
    # functions, outside the timed region: L0 one lane per point, L1 per
    # row, L2 per (row, chunk) - the same sums in every case
    mappings = {}
    for f in (0, 1):
        mo = torch.empty_like(xs[f])
        res = {}
        for level in (0, 1, 2):
            prev = binding.chessfad_set_option(binding.CHESSFAD_OPT_MAPPING, level)
            try:
                binding.chessfad_hvp(f, xs[f], vs[f], mo, chunk=chunks[f])
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                for _ in range(3):
                    binding.chessfad_hvp(f, xs[f], vs[f], mo, chunk=chunks[f])
                e1.record()
                torch.cuda.synchronize()
            finally:
                binding.chessfad_set_option(binding.CHESSFAD_OPT_MAPPING, prev)
            ms = e0.elapsed_time(e1) / 3
            res[f"L{level}"] = {"kernel_ms": round(ms, 4), "hvps_per_s": npts / (ms * 1e-3)}
        mappings[NAMES[f]] = {"chunk": chunks[f], **res}

    # the same comparison across n (the shape of the paper's mapping figures):
    # Rosenbrock and Ackley, C = 4, 2^17 points per n
    sweep = {}
    for f in (0, 1):
        for nn in (4, 8, 16, 32, 64):
            w = inputs.make_workload(f, nn, 1 << 17, inputs.rng_for(300 + nn))
            xw, vw = torch.from_numpy(w.x).to(dev), torch.from_numpy(w.v).to(dev)
            mo = torch.empty_like(xw)
            row = {}
            for level in (0, 1, 2):
                prev = binding.chessfad_set_option(binding.CHESSFAD_OPT_MAPPING, level)
                try:
                    binding.chessfad_hvp(f, xw, vw, mo, chunk=4)
                    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    e0.record()
                    for _ in range(3):
                        binding.chessfad_hvp(f, xw, vw, mo, chunk=4)
                    e1.record()
                    torch.cuda.synchronize()
                finally:
                    binding.chessfad_set_option(binding.CHESSFAD_OPT_MAPPING, prev)
                row[f"L{level}_ms"] = round(e0.elapsed_time(e1) / 3, 4)
            sweep[f"{NAMES[f]}_n{nn}"] = row
        del xw, vw, mo

    # the symmetric form (SC-HESS-VEC) on the same inputs, outside the timed
    # region: fewer f calls per point, the same H.v
    sym = {}
    for f in FUNCS:
        so = torch.empty_like(xs[f])
        sc = schunks[f]
        binding.chessfad_hvp_sym(f, xs[f], vs[f], so, chunk=sc)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(5):
            binding.chessfad_hvp_sym(f, xs[f], vs[f], so, chunk=sc)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 5
        sym[NAMES[f]] = {"chunk": sc or "library default", "kernel_ms": round(ms, 4),
                         "hvps_per_s": npts / (ms * 1e-3), "speedup_vs_full_f64": kernel_ms[f] / ms,
                         "calls_per_point": flops.calls_per_point_sym(N, sc) if sc else None,
                         "max_rel_err_sampled": rel_err(f, so)}
    sym_step = sum(v["kernel_ms"] for v in sym.values())
    sym_total = {"kernel_ms_sum": round(sym_step, 4), "hvps_per_s": len(FUNCS) * npts / (sym_step * 1e-3)}

    # Sec. V's chunk-size analysis against the autotuner: the multiplication
    # count (6 + 3/c) n^2 M falls with c for the full form; the symmetric
    # form's (3/2) n (2n + 2c + n/c + 1) M is smallest near sqrt(n / 2)
    def sym_model_chunk(n):
        best, bc = None, 1
        for c in (1, 2, 4, 8, 16):
            if c <= n and (best is None or 2 * c + n / c <= best):
                best, bc = 2 * c + n / c, c
        return bc
    chunk_model = {NAMES[f]: {"full": {"model": max(c for c in (1, 2, 4, 8, 16) if c <= N), "tuned": chunks[f]},
                              "symmetric": {"model": sym_model_chunk(N), "tuned": schunks[f] or None}}
                   for f in FUNCS}

    result = {
        "metric": METRIC,
        "value": value,
        "unit": "HVP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "plain FP64 H.v: Rosenbrock, Ackley, Fletcher-Powell; n=16; "
                               f"{npts} points each; chunk per function",
                   "n": N, "npts": npts, "chunks": {NAMES[f]: chunks[f] for f in FUNCS}},
        "roofline": roofline,
        "per_function": per_func,
        "max_rel_err_sampled": max_err,
        "fp_vector_path_ms": fp_vector_ms,
        "mixed_f32": mixed,
        "hessian_f64": hess,
        "symmetric_f64": {"per_function": sym, "all_three": sym_total},
        "mappings_f64": mappings,
        "mappings_f64_by_n": {"chunk": 4, "npts": 1 << 17, "kernel_ms": sweep},
        "chunk_model_vs_tuned": chunk_model,
    }
    result["autotuned_ms"] = tuned or None
    if not args.no_batch:
        result["batched"] = batched(args.batch_instances, binding, inputs, cf, torch)
    if args.large:
        result["large_n"] = large_n(binding, inputs, cf, torch, flops)
    if not args.no_cpu:
        result["cpu_baseline"] = cpu_baseline(workloads, E, chunks, args.cpu_seconds)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
