"""Benchmark: Hessian-vector products per second on one MI355X.

One step = one pass of the whole hot path over one batch: float64 chunked
H.v for Rosenbrock, Ackley and Fletcher-Powell, each at n = 16 over 2^20
resident points (seeded synthetic inputs), three launches through the C ABI
at the autotuned chunk (and mapping) of each function.  Every launch runs the
chunked method: f is evaluated per (point, row, chunk) call on CHUNK-INIT
seeds (Fletcher-Powell on the per-call kernel, CHESSFAD_OPT_FP_MFMA = 1).
`value` is the total HVPs of a step divided by the step time.

Also reported, outside the timed region:
  roofline        the dominant kernel's executed flops per launch (rocprofv3
                  counters taken on the same kernel source; `stale` when the
                  source has changed since) divided by its average launch time
                  (HIP events on the launch stream inside the timed region);
  cpu_baseline    the CPU oracle's chunked method (plain C, OpenMP over
                  points, all host cores) on a bounded sample of the same
                  inputs, with a one-thread run and the closed-form H.v
                  beside it;
  fp_engines      Fletcher-Powell at n = 16 on every engine and chunk: the
                  per-call kernels (the method) and the closed-form J^T J
                  tile (`fp_closed_form_tile`, not the method);
  generic_method  the three functions written once as user functions over
                  the generic hDual type (every operation of f in every call);
  mixed_f32, hessian_f64, symmetric_f64, mappings_f64, batched, large_n,
  cfg1_cpu_seconds.

    python bench.py [--steps K] [--warmup W] [--chunk C] [--no-cpu] [--no-batch] [--no-large]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
FUNCS = (0, 1, 2)
NAMES = {0: "rosenbrock", 1: "ackley", 2: "fletcher_powell"}
N = 16
NPTS = 1 << 20
PEAK_F64_TFLOPS = 78.6   # 256 CUs x 2.4 GHz x 128 float64 flops per CU-clock (FMA = 2), vector and MFMA
PEAK_HBM_TBPS = 8.0      # HBM3E
VALU_ISSUE_PER_S = 256 * 2.4e9   # vector wave-instructions per second (one per CU-clock)
METRIC = "HVPs/sec at n=16..512; FP32/batched vs FP64 plain on same GPU at stated error"
LARGE_FP_NPTS = {64: 1 << 18, 512: 1024}   # points of the Fletcher-Powell large-n workloads

# ---------------------------------------------------------------- counters
# Per-launch figures from rocprofv3 --pmc runs of `bench.py --only kernels`
# and `--only kernels --kernels-n 64 / 512`
# (profiles/hvp_step_and_large_n_kernel_counters.md), keyed by kernel
# (" n=<n>" for the large-n launches).  Each entry
# holds for the sources it was taken on: "sha" is kernel_sha() of its kernel
# family then, and a run whose sources differ reports the roofline with
# "stale": true.
#   traffic     HBM bytes: FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0 (KiB, copy-kernel
#               calibration; each x 1024)
#   valu_flops  SQ_INSTS_VALU_FLOPS_FP64 x 64 lanes (FMA = 2)
#   valu_insts  SQ_INSTS_VALU wave-instructions (MFMA included)
#   mfma_flops  SQ_INSTS_VALU_MFMA_MOPS_F64 x 512
#   classes     wave-instructions per class: SQ_INSTS_VALU_{ADD,MUL,FMA}_F64,
#               _INT32, _INT64, _CVT, _TRANS_F64, SQ_INSTS_LDS, SQ_INSTS_SALU
COUNTERS = {
    'fp_call_kernel<F64, 8, 1, false, false, 16>': {'traffic': 402829888, 'valu_flops': 11995709440, 'valu_insts': 122552320, 'mfma_flops': 1073741824, 'classes': {'valu_add_f64': 524288, 'valu_mul_f64': 9175040, 'valu_fma_f64': 88866816, 'valu_int32': 2686976, 'valu_int64': 1441792, 'valu_cvt': 262144, 'valu_trans_f64': 0, 'lds': 2555904, 'salu': 8781824}, 'sha': '45479999bf7d7b68'},
    'fp_call_kernel<F64, 8, 16, false, false, 16>': {'traffic': 402834752, 'valu_flops': 11995709440, 'valu_insts': 122552320, 'mfma_flops': 1073741824, 'classes': {'valu_add_f64': 524288, 'valu_mul_f64': 9175040, 'valu_fma_f64': 88866816, 'valu_int32': 2686976, 'valu_int64': 1441792, 'valu_cvt': 262144, 'valu_trans_f64': 0, 'lds': 2555904, 'salu': 8781824}, 'sha': '45479999bf7d7b68'},
    'fp_call_kernel<F64, 8, 2, false, false, 16>': {'traffic': 402816064, 'valu_flops': 11995709440, 'valu_insts': 122552320, 'mfma_flops': 1073741824, 'classes': {'valu_add_f64': 524288, 'valu_mul_f64': 9175040, 'valu_fma_f64': 88866816, 'valu_int32': 2686976, 'valu_int64': 1441792, 'valu_cvt': 262144, 'valu_trans_f64': 0, 'lds': 2555904, 'salu': 8781824}, 'sha': '45479999bf7d7b68'},
    'fp_call_kernel<F64, 8, 4, false, false, 16>': {'traffic': 402813696, 'valu_flops': 11995709440, 'valu_insts': 122552320, 'mfma_flops': 1073741824, 'classes': {'valu_add_f64': 524288, 'valu_mul_f64': 9175040, 'valu_fma_f64': 88866816, 'valu_int32': 2686976, 'valu_int64': 1441792, 'valu_cvt': 262144, 'valu_trans_f64': 0, 'lds': 2555904, 'salu': 8781824}, 'sha': '45479999bf7d7b68'},
    'fp_call_kernel<F64, 8, 8, false, false, 16>': {'traffic': 402819136, 'valu_flops': 11995709440, 'valu_insts': 122552320, 'mfma_flops': 1073741824, 'classes': {'valu_add_f64': 524288, 'valu_mul_f64': 9175040, 'valu_fma_f64': 88866816, 'valu_int32': 2686976, 'valu_int64': 1441792, 'valu_cvt': 262144, 'valu_trans_f64': 0, 'lds': 2555904, 'salu': 8781824}, 'sha': '45479999bf7d7b68'},
    'fp_dpp_kernel<F64, 16, false, false, false> n=512': {'traffic': 38173888, 'valu_flops': 291201089536, 'valu_insts': 3469672448, 'mfma_flops': 0, 'classes': {'valu_add_f64': 10928128, 'valu_mul_f64': 75595776, 'valu_fma_f64': 2231746560, 'valu_int32': 520953856, 'valu_int64': 27066368, 'valu_cvt': 151175168, 'valu_trans_f64': 0, 'lds': 338042880, 'salu': 943480832}, 'sha': '2e3a289a8c793dc7'},
    'fp_dpp_kernel<F64, 16, false, false, false> n=64': {'traffic': 403298432, 'valu_flops': 155239579648, 'valu_insts': 2216165376, 'mfma_flops': 0, 'classes': {'valu_add_f64': 45350912, 'valu_mul_f64': 51904512, 'valu_fma_f64': 1164181504, 'valu_int32': 412876800, 'valu_int64': 123731968, 'valu_cvt': 117178368, 'valu_trans_f64': 0, 'lds': 192413696, 'salu': 677642240}, 'sha': '2e3a289a8c793dc7'},
    'fp_dpp_kernel<F64, 16, false, false, true> n=512': {'traffic': 29803520, 'valu_flops': 164213817344, 'valu_insts': 1957695488, 'mfma_flops': 0, 'classes': {'valu_add_f64': 8224768, 'valu_mul_f64': 44359680, 'valu_fma_f64': 1256628224, 'valu_int32': 282664960, 'valu_int64': 21958656, 'valu_cvt': 84000768, 'valu_trans_f64': 0, 'lds': 191954944, 'salu': 523919360}, 'sha': '2e3a289a8c793dc7'},
    'fp_dpp_kernel<F64, 16, false, false, true> n=64': {'traffic': 403293184, 'valu_flops': 124772155392, 'valu_insts': 2056388608, 'mfma_flops': 0, 'classes': {'valu_add_f64': 53477376, 'valu_mul_f64': 81526784, 'valu_fma_f64': 907280384, 'valu_int32': 452460544, 'valu_int64': 116391936, 'valu_cvt': 98304000, 'valu_trans_f64': 0, 'lds': 246677504, 'salu': 493944832}, 'sha': '2e3a289a8c793dc7'},
    'plain_kernel<F64, Ackley, 1, false, false>': {'traffic': 402784256, 'valu_flops': 18723373056, 'valu_insts': 763363328, 'mfma_flops': 0, 'classes': {'valu_add_f64': 45088768, 'valu_mul_f64': 53477376, 'valu_fma_f64': 95420416, 'valu_int32': 277872640, 'valu_int64': 20971520, 'valu_cvt': 39845888, 'valu_trans_f64': 3145728, 'lds': 91226112, 'salu': 618659840}, 'sha': 'c9b5758bb627f982'},
    'plain_kernel<F64, Ackley, 2, false, false>': {'traffic': 402777088, 'valu_flops': 9898557440, 'valu_insts': 385351680, 'mfma_flops': 0, 'classes': {'valu_add_f64': 20447232, 'valu_mul_f64': 28835840, 'valu_fma_f64': 51904512, 'valu_int32': 134217728, 'valu_int64': 12582912, 'valu_cvt': 19922944, 'valu_trans_f64': 1572864, 'lds': 41418752, 'salu': 311427072}, 'sha': 'c9b5758bb627f982'},
    'plain_kernel<F64, Ackley, 4, false, false>': {'traffic': 402775040, 'valu_flops': 5687476224, 'valu_insts': 204210176, 'mfma_flops': 0, 'classes': {'valu_add_f64': 11272192, 'valu_mul_f64': 16515072, 'valu_fma_f64': 30146560, 'valu_int32': 69206016, 'valu_int64': 6291456, 'valu_cvt': 9961472, 'valu_trans_f64': 786432, 'lds': 25952256, 'salu': 157810688}, 'sha': 'c9b5758bb627f982'},
    'plain_kernel<F64, Ackley, 8, false, false>': {'traffic': 402803712, 'valu_flops': 3984588800, 'valu_insts': 125698048, 'mfma_flops': 0, 'classes': {'valu_add_f64': 7602176, 'valu_mul_f64': 11010048, 'valu_fma_f64': 21626880, 'valu_int32': 38141952, 'valu_int64': 3538944, 'valu_cvt': 5373952, 'valu_trans_f64': 393216, 'lds': 16646144, 'salu': 85590016}, 'sha': 'c9b5758bb627f982'},
    'plain_kernel<F64, Rosenbrock, 1, false, false>': {'traffic': 402741248, 'valu_flops': 8254390272, 'valu_insts': 584056832, 'mfma_flops': 0, 'classes': {'valu_add_f64': 32505856, 'valu_mul_f64': 46137344, 'valu_fma_f64': 25165824, 'valu_int32': 247463936, 'valu_int64': 19922944, 'valu_cvt': 35651584, 'valu_trans_f64': 0, 'lds': 48234496, 'salu': 481296384}, 'sha': 'c9b5758bb627f982'},
    'plain_kernel<F64, Rosenbrock, 2, false, false>': {'traffic': 402733056, 'valu_flops': 3992977408, 'valu_insts': 295698432, 'mfma_flops': 0, 'classes': {'valu_add_f64': 12058624, 'valu_mul_f64': 25165824, 'valu_fma_f64': 12582912, 'valu_int32': 125304832, 'valu_int64': 9961472, 'valu_cvt': 17825792, 'valu_trans_f64': 0, 'lds': 19922944, 'salu': 240648192}, 'sha': 'c9b5758bb627f982'},
    'plain_kernel<F64, Rosenbrock, 4, false, false>': {'traffic': 402734080, 'valu_flops': 1929379840, 'valu_insts': 145752064, 'mfma_flops': 0, 'classes': {'valu_add_f64': 4980736, 'valu_mul_f64': 12582912, 'valu_fma_f64': 6291456, 'valu_int32': 61603840, 'valu_int64': 4980736, 'valu_cvt': 8912896, 'valu_trans_f64': 0, 'lds': 8912896, 'salu': 118226944}, 'sha': 'c9b5758bb627f982'},
    'plain_kernel<F64, Rosenbrock, 8, false, false>': {'traffic': 402728960, 'valu_flops': 956301312, 'valu_insts': 77594624, 'mfma_flops': 0, 'classes': {'valu_add_f64': 2359296, 'valu_mul_f64': 6291456, 'valu_fma_f64': 3145728, 'valu_int32': 33816576, 'valu_int64': 2883584, 'valu_cvt': 4718592, 'valu_trans_f64': 0, 'lds': 4718592, 'salu': 63176704}, 'sha': 'c9b5758bb627f982'},
    'row16_ackley_kernel<F64, 16>': {'traffic': 402787328, 'valu_flops': 3024093184, 'valu_insts': 56426496, 'mfma_flops': 0, 'classes': {'valu_add_f64': 2424832, 'valu_mul_f64': 3276800, 'valu_fma_f64': 20709376, 'valu_int32': 983040, 'valu_int64': 1048576, 'valu_cvt': 393216, 'valu_trans_f64': 131072, 'lds': 2097152, 'salu': 9109504}, 'sha': 'e90b3e505afc6dd6'},
    'row16_ackley_kernel<F64, 1>': {'traffic': 402843136, 'valu_flops': 3527409664, 'valu_insts': 78118912, 'mfma_flops': 0, 'classes': {'valu_add_f64': 10551296, 'valu_mul_f64': 3538944, 'valu_fma_f64': 20447232, 'valu_int32': 2031616, 'valu_int64': 1048576, 'valu_cvt': 393216, 'valu_trans_f64': 131072, 'lds': 2097152, 'salu': 9109504}, 'sha': 'e90b3e505afc6dd6'},
    'row16_ackley_kernel<F64, 2>': {'traffic': 402807808, 'valu_flops': 3258974208, 'valu_insts': 67239936, 'mfma_flops': 0, 'classes': {'valu_add_f64': 6356992, 'valu_mul_f64': 3538944, 'valu_fma_f64': 20447232, 'valu_int32': 1507328, 'valu_int64': 1048576, 'valu_cvt': 393216, 'valu_trans_f64': 131072, 'lds': 2097152, 'salu': 9109504}, 'sha': 'e90b3e505afc6dd6'},
    'row16_ackley_kernel<F64, 4>': {'traffic': 402797568, 'valu_flops': 3124756480, 'valu_insts': 61669376, 'mfma_flops': 0, 'classes': {'valu_add_f64': 4259840, 'valu_mul_f64': 3538944, 'valu_fma_f64': 20447232, 'valu_int32': 1179648, 'valu_int64': 1048576, 'valu_cvt': 393216, 'valu_trans_f64': 131072, 'lds': 2097152, 'salu': 9109504}, 'sha': 'e90b3e505afc6dd6'},
    'row16_ackley_kernel<F64, 8>': {'traffic': 402793216, 'valu_flops': 3057647616, 'valu_insts': 58785792, 'mfma_flops': 0, 'classes': {'valu_add_f64': 3211264, 'valu_mul_f64': 3538944, 'valu_fma_f64': 20447232, 'valu_int32': 1048576, 'valu_int64': 1048576, 'valu_cvt': 393216, 'valu_trans_f64': 131072, 'lds': 2097152, 'salu': 9109504}, 'sha': 'e90b3e505afc6dd6'},
    'row16_kernel<F64, Rosenbrock, 16>': {'traffic': 402678784, 'valu_flops': 419430400, 'valu_insts': 15466496, 'mfma_flops': 0, 'classes': {'valu_add_f64': 1048576, 'valu_mul_f64': 2359296, 'valu_fma_f64': 1572864, 'valu_int32': 524288, 'valu_int64': 1048576, 'valu_cvt': 0, 'valu_trans_f64': 0, 'lds': 0, 'salu': 2621440}, 'sha': 'e90b3e505afc6dd6'},
    'row16_kernel<F64, Rosenbrock, 1>': {'traffic': 402728256, 'valu_flops': 5284823040, 'valu_insts': 100401152, 'mfma_flops': 0, 'classes': {'valu_add_f64': 4980736, 'valu_mul_f64': 37224448, 'valu_fma_f64': 20185088, 'valu_int32': 4194304, 'valu_int64': 1048576, 'valu_cvt': 0, 'valu_trans_f64': 0, 'lds': 0, 'salu': 2621440}, 'sha': 'e90b3e505afc6dd6'},
    'row16_kernel<F64, Rosenbrock, 2>': {'traffic': 402702336, 'valu_flops': 3070230528, 'valu_insts': 70254592, 'mfma_flops': 0, 'classes': {'valu_add_f64': 3145728, 'valu_mul_f64': 23330816, 'valu_fma_f64': 10747904, 'valu_int32': 5767168, 'valu_int64': 1048576, 'valu_cvt': 0, 'valu_trans_f64': 0, 'lds': 0, 'salu': 2621440}, 'sha': 'e90b3e505afc6dd6'},
    'row16_kernel<F64, Rosenbrock, 4>': {'traffic': 402682880, 'valu_flops': 1593835520, 'valu_insts': 40894464, 'mfma_flops': 0, 'classes': {'valu_add_f64': 2097152, 'valu_mul_f64': 11796480, 'valu_fma_f64': 5505024, 'valu_int32': 3407872, 'valu_int64': 1048576, 'valu_cvt': 0, 'valu_trans_f64': 0, 'lds': 0, 'salu': 2621440}, 'sha': 'e90b3e505afc6dd6'},
    'row16_kernel<F64, Rosenbrock, 8>': {'traffic': 402682880, 'valu_flops': 855638016, 'valu_insts': 25690112, 'mfma_flops': 0, 'classes': {'valu_add_f64': 1572864, 'valu_mul_f64': 6029312, 'valu_fma_f64': 2883584, 'valu_int32': 1835008, 'valu_int64': 1048576, 'valu_cvt': 0, 'valu_trans_f64': 0, 'lds': 0, 'salu': 2621440}, 'sha': 'e90b3e505afc6dd6'},
}

# The sources each kernel family is compiled from (with the build flags and,
# for the Fletcher-Powell DPP kernels, the generator of their inline-asm blocks).
KERNEL_SOURCES = {
    "coarse_kernel": ("hd.hpp", "trig.hpp", "functions.hpp", "kernel_plain.hpp"),
    "plain_kernel": ("hd.hpp", "trig.hpp", "functions.hpp", "kernel_plain.hpp"),
    "row16_kernel": ("hd.hpp", "trig.hpp", "functions.hpp", "kernel_row16.hpp"),
    "row16_ackley_kernel": ("hd.hpp", "trig.hpp", "functions.hpp", "kernel_row16.hpp"),
    "fp_call_kernel": ("hd.hpp", "trig.hpp", "functions.hpp", "kernel_fp_mfma.hpp", "kernel_fp_call.hpp"),
    "fp_dpp_kernel": ("hd.hpp", "trig.hpp", "functions.hpp", "kernel_fp_mfma.hpp", "kernel_fp_call.hpp",
                      "kernel_fp_dpp.hpp"),
    "fp_rows_kernel": ("hd.hpp", "trig.hpp", "functions.hpp", "kernel_fp_mfma.hpp", "kernel_fp_rows.hpp"),
    "sym_kernel": ("hd.hpp", "trig.hpp", "functions.hpp", "kernel_sym.hpp"),
}


def kernel_sha(key, read=None) -> str:
    """sha256 (16 hex digits) over the sources and build flags of the kernel
    family of `key`; `read(relpath)` returns a file's bytes (default: the
    working tree)."""
    import inspect

    sys.path.insert(0, ROOT)
    from paper_2410_22575_amd import build

    read = read or (lambda rel: open(os.path.join(ROOT, rel), "rb").read())
    family = key.split("<")[0]
    h = hashlib.sha256()
    h.update(" ".join(build.FLAGS[:-6]).encode())   # the flags, without the include paths
    if family.startswith(("fp_call", "fp_dpp")):
        h.update(inspect.getsource(build.write_dpp_blocks_inc).encode())
    if family.startswith("row16"):
        h.update(inspect.getsource(build.write_dpp_ackley_row16_inc).encode())
    for f in KERNEL_SOURCES.get(family, ()):
        rel = os.path.join("paper_2410_22575_amd", "csrc", f)
        h.update(rel.encode())
        h.update(read(rel))
    return h.hexdigest()[:16]


def kernel_key(f, c, n=N, mapping=2, mixed=False, sym=False):
    """The kernel chessfad_hvp (or _mixed, or _sym) runs for (function,
    chunk, mapping) at n, named as the profiler's demangled kernel name with
    the namespace and argument list removed; COUNTERS keys add " n=<n>" for
    n != 16."""
    prec = "F32C" if mixed else "F64"
    at = "" if n == N else f" n={n}"
    if f == 2 and n <= 16:
        if sym:
            return f"fp_mfma_kernel<{prec}, {c}, {min(8, max(1, (2 * n + 3) // 4))}, false, true>" + at
        return f"fp_call_kernel<{prec}, {min(8, max(1, (2 * n + 3) // 4))}, {c}, false, false, {16 if n == 16 else 0}>" + at
    if f == 2:
        return f"fp_dpp_kernel<{prec}, {c}, false, false, {'true' if sym else 'false'}>" + at
    func = {0: "Rosenbrock", 1: "Ackley"}[f]
    if sym:
        return f"sym_kernel<{prec}, {func}, {c}, false>" + at
    if n == 16 and (c >= n or mapping == 1):
        return f"row16_ackley_kernel<{prec}, {c}>" if f == 1 else f"row16_kernel<{prec}, {func}, {c}>"
    if f == 0 and (c >= n or mapping == 1):
        return f"rosenbrock_rows_kernel<{prec}, {c}>" + at
    if c >= n or mapping == 1:
        return f"coarse_kernel<{prec}, {func}, {c}, 1>" + at
    return f"plain_kernel<{prec}, {func}, {c}, false, false>" + at


def profiler_key(name):
    """A rocprofv3 kernel name reduced to the form of kernel_key."""
    name = name.replace("chessfad::", "").strip()
    if name.startswith("void "):
        name = name[5:]
    return name.split("(")[0].strip()


def fp_value_column_mfma_flops(n, npts):
    """MFMA flops of the per-call kernel's value column: per 16-point wave,
    NK steps of 16x16x4 (2 x 16 x 16 x 4 flops each), whatever the chunk."""
    nk = min(8, max(1, (2 * n + 3) // 4))
    return nk * 2 * 16 * 16 * 4 * (npts / 16)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--chunk", type=int, default=0, help="0 = the autotuned chunk per function")
    ap.add_argument("--npts", type=int, default=NPTS)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baselines and cfg1")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-tune", action="store_true", help="use the default chunk instead of autotuning it")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched mixed-instance workload")
    ap.add_argument("--batch-instances", type=int, default=8192)
    ap.add_argument("--no-large", action="store_true", help="skip the n = 64 and n = 512 workloads")
    ap.add_argument("--only", choices=("step", "large", "sym", "batch", "fp", "kernels"), default=None,
                    help="only run one part and print its JSON (for profiling; not the benchmark line)")
    ap.add_argument("--kernels-n", type=int, default=N, choices=(N, 64, 512),
                    help="--only kernels: the n = 16 step kernels, or the Fletcher-Powell n = 64 / 512 launches "
                         "of the large-n workloads (full and symmetric H.v)")
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


class Ctx:
    """Library, inputs and helpers shared by the parts of the benchmark."""

    def __init__(self, npts):
        import torch

        from oracle import closed_form as cf
        from paper_2410_22575_amd import binding, flops, inputs

        self.torch, self.cf, self.binding, self.flops, self.inputs = torch, cf, binding, flops, inputs
        binding.load()
        self.dev = torch.device("cuda:0")
        torch.cuda.set_device(self.dev)
        self.npts = npts

    def dev_array(self, a):
        return self.torch.from_numpy(np.ascontiguousarray(a)).to(self.dev)

    def set_fp(self, w):
        self.binding.chessfad_fp_set_params(self.dev_array(w.A), self.dev_array(w.B), self.dev_array(w.alpha))
        return self.cf.fp_offsets(w.A, w.B, w.alpha)

    def time_ms(self, fn, reps=3, warm=1):
        """Average time of fn() from HIP events on the current stream."""
        torch = self.torch
        for _ in range(warm):
            fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    def hvp_err(self, w, E, out, idx=None):
        """Max over sampled points of max|r - r*| / (max|H*| max|v|)."""
        if idx is None:
            idx = np.arange(0, w.npts, max(1, w.npts // 64))
        H = self.cf.hessian(w.func, w.x[idx], w.A, w.B, E)
        ref = np.einsum("pij,pj->pi", H, w.v[idx])
        got = out.cpu().numpy()[idx] if hasattr(out, "cpu") else out[idx]
        scale = np.abs(H).max(axis=(1, 2)) * np.abs(w.v[idx]).max(axis=1)
        return float((np.abs(got - ref).max(axis=1) / scale).max())


# ------------------------------------------------------------------ parts
def fp_engines(ctx, w, E, x, v):
    """Fletcher-Powell H.v at n = 16 over all points on every engine and
    chunk size.  Engines 1 and 2 run the chunked method (one evaluation per
    call); engine 3 is the closed form 2 (J^T J + diag(D^T r)) as one MFMA tile
    per point, whose result does not depend on the chunk."""
    b = ctx.binding
    out = ctx.torch.empty_like(x)
    res = {}
    labels = {1: "per_call_dpp", 2: "per_call_mfma", 3: "fp_closed_form_tile", 0: "vector_alu"}
    for eng in (1, 2, 3, 0):
        prev = b.chessfad_set_option(b.CHESSFAD_OPT_FP_MFMA, eng)
        try:
            row = {}
            chunks = (1, 2, 4, 8, 16) if eng in (1, 2) else (16,)
            for c in chunks:
                ms = ctx.time_ms(lambda: b.chessfad_hvp(2, x, v, out, chunk=c), reps=3 if eng else 1)
                row[f"C{c}"] = {"kernel_ms": round(ms, 4), "hvps_per_s": w.npts / (ms * 1e-3),
                                "max_rel_err_sampled": ctx.hvp_err(w, E, out)}
        finally:
            b.chessfad_set_option(b.CHESSFAD_OPT_FP_MFMA, prev)
        res[labels[eng]] = row
    res["fp_closed_form_tile"]["note"] = ("closed form, not the chunked method: all second-order components of a "
                                          "point as one MFMA tile 2 (J^T J + diag(D^T r)); the chunk does not enter")
    res["vector_alu"]["note"] = "every hDual operation of f in every call on the vector ALUs (L2 mapping)"
    return res


def generic_method(ctx, ws, Es, xs, vs):
    """The three functions registered as user functions (f written once over
    the generic hDual type) and run by chessfad_hvp on the same inputs: the
    general method, with no per-function specialisation."""
    from paper_2410_22575_amd import user_sources

    b = ctx.binding
    res = {}
    for f in FUNCS:
        w = ws[f]
        if f == 0:
            src = user_sources.ROSENBROCK_HIP
        elif f == 1:
            src = user_sources.ACKLEY_HIP
        else:
            src = user_sources.fletcher_powell_hip(w.A, w.B, Es[f])
        fid = b.chessfad_register_function(src)
        try:
            out = ctx.torch.empty_like(xs[f])
            row = {}
            for c in (4, 16):
                ms = ctx.time_ms(lambda: b.chessfad_hvp(fid, xs[f], vs[f], out, chunk=c), reps=1)
                row[f"C{c}"] = {"kernel_ms": round(ms, 3), "hvps_per_s": w.npts / (ms * 1e-3),
                                "max_rel_err_sampled": ctx.hvp_err(w, Es[f], out)}
            res[NAMES[f]] = row
        finally:
            b.chessfad_release_function(fid)
    res["mapping"] = "L1 (one lane per (point, row), walking its chunks), float64, every hDual operation evaluated"
    return res


def large_n(ctx):
    """cfg3: n = 64 over 2^18 points, all three functions, float64 and mixed,
    at the autotuned chunk.  cfg5: Fletcher-Powell n = 512 over 1024 points
    (float32 MFMA contraction in the mixed path, float64), Rosenbrock n = 512
    H.v.  Kernel time, HVP/s, paper-model TFLOP/s, and the max error against
    the oracle on 64 sampled points."""
    b, torch = ctx.binding, ctx.torch
    res = {}
    cases = [(f, 64, 1 << 18, prec) for f in FUNCS for prec in (0, 1)]
    cases += [(2, 512, 1024, 1), (2, 512, 1024, 0), (0, 512, 1024, 0)]
    for f, n, npts, prec in cases:
        w = ctx.inputs.make_workload(f, n, npts, ctx.inputs.rng_for(100 + n))
        x, v = ctx.dev_array(w.x), ctx.dev_array(w.v)
        E = ctx.set_fp(w) if f == 2 else None
        # autotuned chunk (and mapping) except for Fletcher-Powell at n = 512,
        # where a launch per chunk takes several milliseconds: C = 16 there
        if f == 2 and n == 512:
            c = call_c = 16
        else:
            c, _ = b.chessfad_autotune(f, n, prec, npts=min(npts, 1 << 16))
            call_c = 0
        fn = b.chessfad_hvp_mixed if prec else b.chessfad_hvp
        out = torch.empty_like(x)
        ms = ctx.time_ms(lambda: fn(f, x, v, out, chunk=call_c), reps=3)
        idx = np.random.default_rng(2).choice(npts, min(64, npts), replace=False)
        err = ctx.hvp_err(w, E, out, idx)
        mf = ctx.flops.flops_per_hvp(f, n, c)
        name = f"{NAMES[f]}_n{n}_{'mixed' if prec else 'f64'}"
        res[name] = {"npts": npts, "chunk": c,
                     "mapping": "per-call, DPP lane broadcasts" if f == 2 else f"L{b.chessfad_default_mapping(f, n, prec)}",
                     "kernel_ms": round(ms, 4), "hvps_per_s": npts / (ms * 1e-3),
                     "paper_model_equiv_tflops": mf * npts / (ms * 1e-3) / 1e12, "max_rel_err_sampled": err}
        key = kernel_key(f, c, n=n, mixed=bool(prec))
        cnt = COUNTERS.get(key)
        if cnt:
            # counters of this launch (rocprofv3 runs of bench.py --only kernels --kernels-n n)
            algo = 24 * n * npts + (16 * n * n + 8 * n if f == 2 else 0)   # x, v, out; A, B, E once
            work = cnt["valu_flops"] + cnt["mfma_flops"]
            res[name]["counters"] = {
                "kernel": key, "hbm_bytes": cnt["traffic"], "algorithmic_bytes": algo,
                "hbm_over_algorithmic": cnt["traffic"] / algo,
                "executed_f64_tflops": work / (ms * 1e-3) / 1e12,
                "flop_frac": work / (ms * 1e-3) / 1e12 / PEAK_F64_TFLOPS,
                "valu_issue_frac": cnt["valu_insts"] / VALU_ISSUE_PER_S / (ms * 1e-3),
                "stale": cnt.get("sha") != kernel_sha(key)}
        if f == 2:
            # the row-block kernel with MFMA contraction tiles, for comparison
            prev = b.chessfad_set_option(b.CHESSFAD_OPT_FP_MFMA, 2)
            try:
                ms2 = ctx.time_ms(lambda: fn(f, x, v, out, chunk=c), reps=3)
            finally:
                b.chessfad_set_option(b.CHESSFAD_OPT_FP_MFMA, prev)
            res[name]["rows_mfma_kernel_ms"] = round(ms2, 4)
            res[name]["speedup_vs_rows_mfma"] = ms2 / ms
        print(f"  large: {name} C={c} {ms:.3f} ms err {err:.2e}", file=sys.stderr, flush=True)
    for f in FUNCS:
        a, m = res[f"{NAMES[f]}_n64_f64"], res[f"{NAMES[f]}_n64_mixed"]
        m["speedup_vs_f64"] = a["kernel_ms"] / m["kernel_ms"]
    res["fletcher_powell_n512_mixed"]["speedup_vs_f64"] = (res["fletcher_powell_n512_f64"]["kernel_ms"]
                                                           / res["fletcher_powell_n512_mixed"]["kernel_ms"])
    return res


def symmetric_large_n(ctx):
    """SC-HESS-VEC against CHESS-VEC (float64) where symmetry has calls to
    save (C < n): Rosenbrock and Ackley at n = 64 and 128 over 2^16 points,
    Fletcher-Powell at n = 64 over 2^14 points (C = 4, 8, 16) and at n = 512
    over 1024 points (C = 16)."""
    b, torch = ctx.binding, ctx.torch
    res = {}
    for f, n, npts in ((0, 64, 1 << 16), (0, 128, 1 << 16), (1, 64, 1 << 16), (1, 128, 1 << 16), (2, 64, 1 << 14),
                       (2, 512, 1024)):
        w = ctx.inputs.make_workload(f, n, npts, ctx.inputs.rng_for(700 + n))
        x, v = ctx.dev_array(w.x), ctx.dev_array(w.v)
        E = ctx.set_fp(w) if f == 2 else None
        out = torch.empty_like(x)
        for c in ((16,) if n == 512 else (4, 8, 16)):
            full = ctx.time_ms(lambda: b.chessfad_hvp(f, x, v, out, chunk=c))
            try:
                sym = ctx.time_ms(lambda: b.chessfad_hvp_sym(f, x, v, out, chunk=c))
            except b.ChessfadError as e:
                res[f"{NAMES[f]}_n{n}_C{c}"] = {"full_ms": round(full, 4), "sym": f"not run: {e}"}
                continue
            err = ctx.hvp_err(w, E, out)
            res[f"{NAMES[f]}_n{n}_C{c}"] = {
                "npts": npts, "full_ms": round(full, 4), "sym_ms": round(sym, 4), "speedup_sym_vs_full": full / sym,
                "calls_full": ctx.flops.calls_per_point(n, c), "calls_sym": ctx.flops.calls_per_point_sym(n, c),
                "max_rel_err_sampled": err}
    return res


def batched(ctx, ninst):
    """Mixed-function batch: `ninst` single-point instances, function uniform
    over the three, n log-uniform in [8, 256], each Fletcher-Powell instance
    with its own parameters.  Plans are tuned at creation (chunk and mapping,
    or points per workgroup, per function, octave of n and precision, timed
    on the instances themselves); one replay of the plan's hipGraph is
    timed for float64 and mixed hDuals, each with float64 and with float32
    I/O.  The float64 baseline: plain launches grouped per (function, n) -
    Rosenbrock and Ackley instances of one n as one launch over their points,
    each Fletcher-Powell instance (its own parameters) as its own launch -
    kernel time only, summed."""
    b, torch = ctx.binding, ctx.torch
    ws = ctx.inputs.mixed_instances(ninst, ctx.inputs.rng_for(4), 8, 256, npts=1)
    insts = []
    for w in ws:
        d = {"func_id": w.func, "x": ctx.dev_array(w.x), "v": ctx.dev_array(w.v),
             "out": torch.empty((w.npts, w.n), dtype=torch.float64, device=ctx.dev)}
        if w.func == 2:
            d.update(A=ctx.dev_array(w.A), B=ctx.dev_array(w.B), alpha=ctx.dev_array(w.alpha))
        insts.append(d)
    torch.cuda.synchronize()
    res = {"workload": f"{ninst} single-point instances, function uniform over Rosenbrock/Ackley/Fletcher-Powell, "
                       "n log-uniform in [8, 256], own Fletcher-Powell parameters each; body configuration tuned "
                       "per (function, octave of n, precision) at plan time"}
    outs = {}
    for io32 in (0, 1):
        for prec, pname in ((1, "mixed_f32"), (0, "f64")):
            run = []
            for d in insts:
                e = dict(d, precision=prec)
                if io32:
                    e["x"], e["v"] = d["x"].float(), d["v"].float()
                    e["out"] = torch.empty(d["out"].shape, dtype=torch.float32, device=ctx.dev)
                run.append(e)
            t0 = time.perf_counter()
            plan = b.chessfad_batch_create(run)
            plan_s = time.perf_counter() - t0
            ms = ctx.time_ms(plan.run)
            info = plan.info()
            name = pname + ("_io32" if io32 else "")
            res[name] = {"graph_ms": round(ms, 4), "hvps_per_s": ninst / (ms * 1e-3),
                         "paper_model_equiv_tflops": info["model_flops"] / (ms * 1e-3) / 1e12,
                         "items": info["items"], "workgroups": info["workgroups"], "plan_seconds": round(plan_s, 3),
                         "tuned": plan.choices()}
            outs[name] = [e["out"].double().clone() for e in run]
            plan.destroy()
    # the grouped float64 baseline
    groups = {}
    for k, w in enumerate(ws):
        groups.setdefault((w.func, w.n) if w.func != 2 else (2, w.n, k), []).append(k)
    total, launches = 0.0, 0
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for key, ks in groups.items():
        f = key[0]
        x = torch.cat([insts[k]["x"] for k in ks])
        v = torch.cat([insts[k]["v"] for k in ks])
        out = torch.empty_like(x)
        if f == 2:
            d = insts[ks[0]]
            b.chessfad_fp_set_params(d["A"], d["B"], d["alpha"])
        e0.record()
        b.chessfad_hvp(f, x, v, out, chunk=0)
        e1.record()
        e1.synchronize()
        total += e0.elapsed_time(e1)
        launches += 1
    res["grouped_f64_launches"] = launches
    res["grouped_f64_kernel_ms_sum"] = round(total, 3)
    for name in ("mixed_f32", "f64", "mixed_f32_io32", "f64_io32"):
        res[name]["speedup_vs_grouped_f64"] = total / res[name]["graph_ms"]
    res["speedup_mixed_batched_vs_f64_batched"] = res["f64"]["graph_ms"] / res["mixed_f32"]["graph_ms"]
    idx = np.random.default_rng(11).choice(ninst, min(64, ninst), replace=False)
    for name in outs:
        worst = 0.0
        for k in idx:
            w = ws[k]
            E = ctx.cf.fp_offsets(w.A, w.B, w.alpha) if w.func == 2 else None
            if name.endswith("_io32"):
                # the oracle at the float32 inputs
                w = ctx.inputs.Workload(**{**w.__dict__, "x": w.x.astype(np.float32).astype(np.float64),
                                           "v": w.v.astype(np.float32).astype(np.float64)})
            worst = max(worst, ctx.hvp_err(w, E, outs[name][k], np.arange(w.npts)))
        res[name]["max_rel_err_sampled"] = worst
    return res


# -------------------------------------------------------------------- CPU
def cpu_model():
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                return line.split(":", 1)[1].strip()
    except Exception:
        pass
    return None


def host_threads():
    return len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()


def cpu_baseline(ws, Es, chunks, budget_s, npts):
    """The oracle timed on the host: the C chunked method (CHESS-VEC, OpenMP
    over points) on every host thread and on one thread, each on a bounded
    sample of the benchmark's points, and the numpy closed-form H.v (the
    plain definition) on one BLAS thread."""
    from threadpoolctl import threadpool_limits

    from oracle import chunked
    from oracle import closed_form as cf

    chunked.build()
    threads = host_threads()

    def run(sample, nthreads):
        t0 = time.perf_counter()
        per = {}
        for f in FUNCS:
            w = ws[f]
            t1 = time.perf_counter()
            chunked.hvp(f, w.x[:sample], w.v[:sample], chunks[f], w.A, w.B, Es[f], nthreads=nthreads)
            per[NAMES[f]] = sample / (time.perf_counter() - t1)
        return time.perf_counter() - t0, per

    def sized(nthreads, budget):
        sample, dt = 64, 0.0
        while sample < npts:
            dt, _ = run(sample, nthreads)
            if dt > 0.3:
                break
            sample *= 2
        return int(min(npts, max(sample, sample * budget / max(dt, 1e-9))))

    sample = sized(threads, budget_s)
    dt, per = run(sample, threads)
    s1 = sized(1, budget_s / 3)
    dt1, per1 = run(s1, 1)
    # closed form, one BLAS thread, on up to 2^17 points of each function
    cs = min(npts, 1 << 17)
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        per_cf = {}
        for f in FUNCS:
            w = ws[f]
            t1 = time.perf_counter()
            cf.hvp(f, w.x[:cs], w.v[:cs], w.A, w.B, Es[f])
            per_cf[NAMES[f]] = cs / (time.perf_counter() - t1)
        dtc = time.perf_counter() - t0
    return {"value": 3 * sample / dt, "unit": "HVP/s", "cores": threads, "kind": "oracle",
            "sample": f"first {sample} of the {npts} points of each function (n=16, the step's chunk sizes), "
                      f"oracle/chunked.c CHESS-VEC with OpenMP over points on {threads} threads",
            "cpu_model": cpu_model(), "per_function": per,
            "one_thread": {"value": 3 * s1 / dt1, "unit": "HVP/s", "sample": f"first {s1} points of each function",
                           "per_function": per1},
            "closed_form_one_thread": {"value": 3 * cs / dtc, "unit": "HVP/s",
                                       "sample": f"first {cs} points of each function, numpy closed-form H.v "
                                                 "(oracle/closed_form.py), one BLAS thread",
                                       "per_function": per_cf},
            "note": "the chunked C oracle evaluates every hDual component of every call (structural zeros "
                    "included); the closed form is the plain definition"}


def cfg1_cpu_seconds():
    """cfg1: Rosenbrock, n = 8, 1024 points, x ~ U[-2, 2], v ~ N(0, 1),
    C = 4: the full Hessian and H.v of every point by the oracle's chunked
    method (CHUNK-HESS + CHESS-VEC), on one thread and on every host thread."""
    from oracle import chunked
    from paper_2410_22575_amd import inputs

    w = inputs.make_workload(0, 8, 1024, inputs.rng_for(1))
    res = {"workload": "Rosenbrock n=8, 1024 points, chunk 4, full Hessian + H.v per point (oracle/chunked.c)"}
    for label, nt in (("one_thread", 1), ("all_threads", host_threads())):
        best = None
        for _ in range(5):
            t0 = time.perf_counter()
            chunked.hessian(0, w.x, 4, nthreads=nt)
            chunked.hvp(0, w.x, w.v, 4, nthreads=nt)
            dt = time.perf_counter() - t0
            best = dt if best is None else min(best, dt)
        res[label] = {"seconds": best, "threads": nt}
    return res


# ------------------------------------------------------------------- main
def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported: the library runs one GPU "
              f"per process (points would shard across GPUs with no communication during compute)",
              file=sys.stderr)
        sys.exit(2)
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return

    ctx = Ctx(args.npts)
    b, torch, cf, flops, inputs = ctx.binding, ctx.torch, ctx.cf, ctx.flops, ctx.inputs
    if args.only == "large":
        print(json.dumps({"large_n": large_n(ctx)}), flush=True)
        return
    if args.only == "batch":
        print(json.dumps({"batched": batched(ctx, args.batch_instances)}), flush=True)
        return
    if args.only == "sym":
        print(json.dumps({"symmetric_large_n": symmetric_large_n(ctx)}), flush=True)
        return
    if args.only == "kernels" and args.kernels_n != N:
        # the large-n Fletcher-Powell launches (float64 H.v, C = 16, full and
        # symmetric form), one warm-up and one launch each
        n = args.kernels_n
        npts = LARGE_FP_NPTS[n]
        w = inputs.make_workload(2, n, npts, inputs.rng_for(100 + n))
        x, v = ctx.dev_array(w.x), ctx.dev_array(w.v)
        ctx.set_fp(w)
        out = torch.empty_like(x)
        for fn, sym in ((b.chessfad_hvp, False), (b.chessfad_hvp_sym, True)):
            for _ in range(2):
                fn(2, x, v, out, chunk=16)
            torch.cuda.synchronize()
            print(f"  kernels: {kernel_key(2, 16, n=n, sym=sym)}", file=sys.stderr, flush=True)
        return
    npts = args.npts

    # seeded synthetic inputs, resident in HBM before timing
    ws, Es, xs, vs, outs = {}, {}, {}, {}, {}
    for f in FUNCS:
        w = inputs.make_workload(f, N, npts, inputs.rng_for(1))
        ws[f] = w
        xs[f], vs[f] = ctx.dev_array(w.x), ctx.dev_array(w.v)
        outs[f] = torch.empty_like(xs[f])
        Es[f] = ctx.set_fp(w) if f == 2 else None
    torch.cuda.synchronize()
    if args.only == "fp":
        print(json.dumps({"fp_engines": fp_engines(ctx, ws[2], Es[2], xs[2], vs[2])}), flush=True)
        return
    if args.only == "kernels":
        # every kernel the step can run at n = 16 (each function, chunk and
        # vector mapping), one warm-up and one launch each: the rocprofv3
        # counter runs of COUNTERS use this
        for f in FUNCS:
            for c in (1, 2, 4, 8, 16):
                for level in ((1, 2) if f != 2 else (2,)):
                    prev = b.chessfad_set_option(b.CHESSFAD_OPT_MAPPING, level)
                    try:
                        for _ in range(2):
                            b.chessfad_hvp(f, xs[f], vs[f], outs[f], chunk=c)
                    finally:
                        b.chessfad_set_option(b.CHESSFAD_OPT_MAPPING, prev)
                torch.cuda.synchronize()
                print(f"  kernels: {NAMES[f]} C={c} {kernel_key(f, c, mapping=1)}", file=sys.stderr, flush=True)
        return

    # chunk per function: explicit, autotuned (outside the timed region), or default
    chunks, mchunks, schunks, tuned = {}, {}, {}, {}
    for f in FUNCS:
        if args.chunk:
            chunks[f] = mchunks[f] = schunks[f] = args.chunk
        elif not args.no_tune:
            chunks[f], tuned[NAMES[f]] = b.chessfad_autotune(f, N, 0, npts=npts)
            mchunks[f], _ = b.chessfad_autotune(f, N, 1, npts=npts)
            schunks[f], _ = b.chessfad_autotune_sym(f, N, 0, npts=npts)
        else:
            chunks[f] = mchunks[f] = b.chessfad_default_chunk(f, N)
            schunks[f] = 0
    torch.cuda.synchronize()
    # the step passes chunk 0 unless a chunk was forced: the library then runs
    # the tuned chunk and mapping
    step_chunk = {f: (args.chunk or 0) for f in FUNCS}
    mapping = {f: (args.chunk and 2) or b.chessfad_default_mapping(f, N) for f in FUNCS}

    def step(events=None):
        for f in FUNCS:
            if events is not None:
                events[f][0].record()
            b.chessfad_hvp(f, xs[f], vs[f], outs[f], chunk=step_chunk[f])
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
    max_err = {NAMES[f]: ctx.hvp_err(ws[f], Es[f], outs[f]) for f in FUNCS}
    if args.only == "step":
        print(json.dumps({"kernel_ms": {NAMES[f]: kernel_ms[f] for f in FUNCS}, "ms_per_step": ms_per_step,
                          "max_rel_err_sampled": max_err}), flush=True)
        return

    # ---- roofline of the dominant kernel, on the executed-flop basis
    per_func = {}
    for f in FUNCS:
        mf = flops.flops_per_hvp(f, N, chunks[f])
        key = kernel_key(f, chunks[f], mapping=mapping[f])
        cnt = COUNTERS.get(key, {})
        t = kernel_ms[f] * 1e-3
        executed = cnt.get("valu_flops", 0.0) + cnt.get("mfma_flops", 0.0) if cnt else None
        per_func[NAMES[f]] = {
            "kernel": key, "chunk": chunks[f],
            "method": ("per-call chunked evaluation (value column on MFMA, per-call product rule on the vector "
                       "ALUs with DPP lane broadcasts)" if f == 2 else
                       f"per-call chunked evaluation on the vector ALUs, L{mapping[f]} mapping"),
            "kernel_ms": round(kernel_ms[f], 4), "hvps_per_s": npts / t,
            "model_flops_per_hvp": mf, "paper_model_equiv_tflops": mf * npts / t / 1e12,
            "executed_tflops": executed / t / 1e12 if executed else None,
            "valu_issue_frac": cnt["valu_insts"] / VALU_ISSUE_PER_S / t if cnt.get("valu_insts") else None,
        }
    dom = max(FUNCS, key=lambda f: kernel_ms[f])
    kname = per_func[NAMES[dom]]["kernel"]
    t_dom = kernel_ms[dom] * 1e-3
    model_launch = flops.flops_per_hvp(dom, N, chunks[dom]) * npts
    cnt = COUNTERS.get(kname)
    algo_bytes = 24 * N * npts   # x and v read, H.v written, float64
    if cnt:
        # executed flops (the lower of the executed and the paper-model count)
        work = min(cnt.get("valu_flops", 0.0) + cnt.get("mfma_flops", 0.0), model_launch)
        flop_frac = work / t_dom / 1e12 / PEAK_F64_TFLOPS
        byte_frac = algo_bytes / t_dom / 1e12 / PEAK_HBM_TBPS
        stale = cnt.get("sha") != kernel_sha(kname)
        if byte_frac > flop_frac:
            roofline = {"bound": "hbm", "achieved": algo_bytes / t_dom / 1e9, "peak": PEAK_HBM_TBPS * 1e3,
                        "unit": "GB/s", "frac": byte_frac}
        else:
            roofline = {"bound": "alu", "achieved": work / t_dom / 1e12, "peak": PEAK_F64_TFLOPS,
                        "unit": "TFLOP/s", "frac": flop_frac}
        roofline.update({
            # HBM bytes per launch from the counters; null once the kernel's
            # sources differ from those the counters were taken on
            "traffic": None if stale else cnt.get("traffic"), "kernel": kname, "flops_per_launch": work,
            "flop_basis": "executed float64 flops (rocprofv3: VALU FLOPS_FP64 x 64" + (
                " + MFMA MOPS_F64 x 512)" if cnt.get("mfma_flops") else ")"),
            "flop_frac": flop_frac, "bytes_per_launch": algo_bytes, "byte_frac": byte_frac,
            "valu_issue_frac": per_func[NAMES[dom]]["valu_issue_frac"],
            "instruction_classes": cnt.get("classes"),
            "model_flops_per_launch": model_launch, "paper_model_equiv_tflops": model_launch / t_dom / 1e12,
            "counters_sha": cnt.get("sha"), "source_sha": kernel_sha(kname), "stale": stale})
    else:
        roofline = {"bound": "alu", "achieved": None, "peak": PEAK_F64_TFLOPS, "unit": "TFLOP/s", "frac": None,
                    "traffic": None, "kernel": kname, "note": "no counters recorded for this kernel",
                    "model_flops_per_launch": model_launch, "paper_model_equiv_tflops": model_launch / t_dom / 1e12,
                    "source_sha": kernel_sha(kname), "stale": True}

    # ---- comparisons outside the timed region
    fp_eng = fp_engines(ctx, ws[2], Es[2], xs[2], vs[2])
    gen = generic_method(ctx, ws, Es, xs, vs)

    hess = {}
    for f in FUNCS:
        sub = min(npts, 1 << 19)
        Hbuf = torch.empty((sub, N, N), dtype=torch.float64, device=ctx.dev)
        # chunk 0: the library's Hessian choice, the largest compiled chunk <= n
        ms = ctx.time_ms(lambda: b.chessfad_hessian(f, xs[f][:sub], Hbuf, chunk=0))
        hess[NAMES[f]] = {"npts": sub, "chunk": max(c for c in (1, 2, 4, 8, 16) if c <= N), "kernel_ms": round(ms, 4),
                          "hessians_per_s": sub / (ms * 1e-3),
                          "hbm_gb_per_s": sub * (8 * N * N + 8 * N) / (ms * 1e-3) / 1e9}
        del Hbuf

    mixed = {}
    for f in FUNCS:
        mo = torch.empty_like(xs[f])
        call_c = args.chunk or 0
        ms = ctx.time_ms(lambda: b.chessfad_hvp_mixed(f, xs[f], vs[f], mo, chunk=call_c), reps=5)
        mixed[NAMES[f]] = {"chunk": mchunks[f], "kernel_ms": round(ms, 4), "hvps_per_s": npts / (ms * 1e-3),
                           "speedup_vs_f64": kernel_ms[f] / ms, "max_rel_err_sampled": ctx.hvp_err(ws[f], Es[f], mo)}
    mixed_ms = sum(v["kernel_ms"] for v in mixed.values())
    mixed["all_three"] = {"kernel_ms_sum": round(mixed_ms, 4), "hvps_per_s": 3 * npts / (mixed_ms * 1e-3),
                          "speedup_vs_f64": sum(kernel_ms.values()) / mixed_ms}

    mappings = {}
    for f in (0, 1):
        mo = torch.empty_like(xs[f])
        row = {}
        for level in (0, 1, 2):
            prev = b.chessfad_set_option(b.CHESSFAD_OPT_MAPPING, level)
            try:
                ms = ctx.time_ms(lambda: b.chessfad_hvp(f, xs[f], vs[f], mo, chunk=chunks[f]))
            finally:
                b.chessfad_set_option(b.CHESSFAD_OPT_MAPPING, prev)
            row[f"L{level}"] = {"kernel_ms": round(ms, 4), "hvps_per_s": npts / (ms * 1e-3)}
        mappings[NAMES[f]] = {"chunk": chunks[f], **row}

    sym = {}
    for f in FUNCS:
        so = torch.empty_like(xs[f])
        sc = schunks[f]
        ms = ctx.time_ms(lambda: b.chessfad_hvp_sym(f, xs[f], vs[f], so, chunk=sc), reps=5)
        sym[NAMES[f]] = {"chunk": sc or "library default", "kernel_ms": round(ms, 4),
                         "hvps_per_s": npts / (ms * 1e-3), "speedup_vs_full_f64": kernel_ms[f] / ms,
                         "calls_per_point": flops.calls_per_point_sym(N, sc) if sc else None,
                         "max_rel_err_sampled": ctx.hvp_err(ws[f], Es[f], so)}
    sym_step = sum(v["kernel_ms"] for v in sym.values())

    # Sec. V's chunk-size analysis against the autotuner
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
        "config": {"workload": "plain FP64 chunked H.v (CHESS-VEC): Rosenbrock, Ackley, Fletcher-Powell; n=16; "
                               f"{npts} points each; autotuned chunk per function",
                   "n": N, "npts": npts, "chunks": {NAMES[f]: chunks[f] for f in FUNCS}},
        "roofline": roofline,
        "notes": {"paper_model_equiv_tflops": "Sec. V's count of dense hDual arithmetic per call divided by the "
                                              "time; the kernels skip the seeds' structural zeros and do not "
                                              "execute that count, so it can exceed the peak. The roofline uses "
                                              "executed flops from rocprofv3 counters."},
        "per_function": per_func,
        "max_rel_err_sampled": max_err,
        "fp_engines": fp_eng,
        "generic_method": gen,
        "mixed_f32": mixed,
        "hessian_f64": hess,
        "symmetric_f64": {"per_function": sym, "all_three": {"kernel_ms_sum": round(sym_step, 4),
                                                            "hvps_per_s": 3 * npts / (sym_step * 1e-3)}},
        "mappings_f64": mappings,
        "chunk_model_vs_tuned": chunk_model,
        "autotuned_ms": tuned or None,
    }
    if not args.no_large:
        result["large_n"] = large_n(ctx)
        result["symmetric_large_n"] = symmetric_large_n(ctx)
    if not args.no_batch:
        result["batched"] = batched(ctx, args.batch_instances)
    if not args.no_cpu:
        result["cfg1_cpu_seconds"] = cfg1_cpu_seconds()
        result["cpu_baseline"] = cpu_baseline(ws, Es, chunks, args.cpu_seconds, npts)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
