"""Host-only checks of the C ABI (no GPU): the library loads, exports every
symbol include/chessfad.h declares, and rejects bad arguments with the
documented status before touching the device."""
import ctypes
import os
import re

import pytest

from paper_2410_22575_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "chessfad.h")

OK, E_FUNC, E_N, E_CHUNK, E_NULL, E_PARAMS, E_OVERLAP, E_HIP, E_ARG = 0, -1, -2, -3, -4, -5, -6, -7, -8
R, A, FP = 0, 1, 2
FAKE = 0x100000  # never dereferenced: every call below fails its host checks first


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(chessfad_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    return binding.load()


def test_header_symbols_exported(lib):
    names = declared_functions()
    assert len(names) >= 6
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(binding.SIGNATURES), "binding signatures out of sync with the header"


def test_status_strings(lib):
    for code in (OK, E_FUNC, E_N, E_CHUNK, E_NULL, E_PARAMS, E_OVERLAP, E_HIP, E_ARG, -9):
        assert binding.strerror(code)
    assert binding.strerror(-99) == "unknown status"


def hvp(lib, func, n, npts, x=FAKE, v=FAKE * 2, out=FAKE * 4, chunk=4):
    return lib.chessfad_hvp(func, n, npts, x, v, out, chunk, None)


def hess(lib, func, n, npts, x=FAKE, H=FAKE * 4, chunk=4):
    return lib.chessfad_hessian(func, n, npts, x, H, chunk, None)


def test_bad_func(lib):
    assert hvp(lib, 3, 16, 10) == E_FUNC
    assert hvp(lib, -1, 16, 10) == E_FUNC
    assert hess(lib, 7, 16, 10) == E_FUNC


def test_bad_n(lib):
    assert hvp(lib, R, 1, 10, chunk=1) == E_N      # Rosenbrock needs two variables
    assert hvp(lib, A, 0, 10, chunk=1) == E_N
    assert hvp(lib, A, 513, 10) == E_N
    assert hess(lib, FP, -4, 10) == E_N


def test_bad_chunk(lib):
    assert hvp(lib, R, 16, 10, chunk=3) == E_CHUNK   # not compiled
    assert hvp(lib, R, 16, 10, chunk=32) == E_CHUNK
    assert hvp(lib, R, 4, 10, chunk=8) == E_CHUNK    # larger than n
    assert hvp(lib, R, 16, 10, chunk=-1) == E_CHUNK


def test_npts(lib):
    assert hvp(lib, R, 16, -1) == E_ARG
    assert hvp(lib, R, 16, 0, x=None, v=None, out=None) == OK     # empty batch is a no-op
    assert hess(lib, A, 16, 0, x=None, H=None) == OK


def test_null_pointers(lib):
    assert hvp(lib, R, 16, 10, x=None) == E_NULL
    assert hvp(lib, R, 16, 10, v=None) == E_NULL
    assert hvp(lib, R, 16, 10, out=None) == E_NULL
    assert hess(lib, A, 16, 10, H=None) == E_NULL


def test_overlap(lib):
    n, npts = 16, 10
    nbytes = 8 * n * npts
    assert hvp(lib, R, n, npts, x=FAKE, v=FAKE + 10 * nbytes, out=FAKE + nbytes - 8) == E_OVERLAP
    assert hvp(lib, A, n, npts, x=FAKE, v=FAKE + 10 * nbytes, out=FAKE + 10 * nbytes) == E_OVERLAP
    assert hess(lib, R, n, npts, x=FAKE + 8 * n * n * npts - 8, H=FAKE) == E_OVERLAP


def symhvp(lib, func, n, npts, x=FAKE, v=FAKE * 2, out=FAKE * 4, chunk=4, precision=0):
    return lib.chessfad_hvp_sym(func, n, npts, x, v, out, chunk, precision, None)


def test_symmetric_argument_checks(lib):
    assert symhvp(lib, 3, 16, 10) == E_FUNC
    assert symhvp(lib, R, 1, 10, chunk=1) == E_N
    assert symhvp(lib, R, 16, 10, chunk=3) == E_CHUNK
    assert symhvp(lib, R, 4, 10, chunk=8) == E_CHUNK
    assert symhvp(lib, R, 16, 10, precision=2) == E_ARG
    assert symhvp(lib, R, 16, -1) == E_ARG
    assert symhvp(lib, R, 16, 0, x=None, v=None, out=None) == OK
    assert symhvp(lib, A, 16, 10, v=None) == E_NULL
    nbytes = 8 * 16 * 10
    assert symhvp(lib, R, 16, 10, x=FAKE, v=FAKE + 10 * nbytes, out=FAKE + nbytes - 8) == E_OVERLAP
    assert lib.chessfad_hessian_sym(A, 16, 10, FAKE, None, 4, 0, None) == E_NULL
    assert lib.chessfad_hessian_sym(A, 16, 10, FAKE, FAKE * 4, 4, -1, None) == E_ARG
    # a point's partial sums must fit in LDS: n ceil(n / chunk) doubles
    assert symhvp(lib, R, 512, 10, chunk=1) == E_CHUNK
    assert symhvp(lib, R, 512, 10, chunk=16) == E_CHUNK
    assert symhvp(lib, A, 512, 10, chunk=0) == E_CHUNK        # no compiled chunk fits
    c, ms = ctypes.c_int(), ctypes.c_float()
    assert lib.chessfad_autotune_sym(4, 16, 0, 100, None, ctypes.byref(c), ctypes.byref(ms)) == E_FUNC
    assert lib.chessfad_autotune_sym(A, 16, 2, 100, None, None, None) == E_ARG


def test_hvp_grad_argument_checks(lib):
    n, npts = 16, 10
    nbytes = 8 * n * npts
    call = lambda grad, fval, out=FAKE * 4: lib.chessfad_hvp_grad(R, n, npts, FAKE, FAKE * 2, out, grad, fval, 4, None)
    assert call(None, None) == E_NULL
    assert call(FAKE * 4 + 8, None) == E_OVERLAP                     # grad inside out
    assert call(FAKE * 8, FAKE * 8 + nbytes - 8) == E_OVERLAP         # fval inside grad
    assert call(FAKE * 8, FAKE * 2 + 16) == E_OVERLAP                 # fval inside v
    assert lib.chessfad_hvp_grad(R, n, 0, None, None, None, None, None, 4, None) == OK
    assert lib.chessfad_hvp_grad(R, n, npts, FAKE, FAKE * 2, FAKE * 4, FAKE * 8, None, 3, None) == E_CHUNK


def test_user_function_registration_host_only(lib):
    # hipRTC compiles on the host; nothing here touches a device
    import sys
    sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
    import user_functions as uf

    fid = binding.chessfad_register_function(uf.ROSENBROCK_HIP)
    assert fid >= 16
    try:
        assert lib.chessfad_hvp(fid, 8, 10, FAKE, FAKE * 2, FAKE * 4, 3, None) == E_CHUNK
        assert lib.chessfad_hvp(fid, 0, 10, FAKE, FAKE * 2, FAKE * 4, 1, None) == E_N
        assert lib.chessfad_hvp(fid, 8, 0, None, None, None, 4, None) == OK
        assert lib.chessfad_hvp(fid, 8, 10, FAKE, None, FAKE * 4, 4, None) == E_NULL
        assert lib.chessfad_hvp_mixed(fid, 8, 10, FAKE, FAKE * 2, FAKE * 4, 4, None) == E_FUNC
        assert lib.chessfad_hvp_sym(fid, 8, 10, FAKE, FAKE * 2, FAKE * 4, 4, 0, None) == E_FUNC
        assert lib.chessfad_hvp_grad(fid, 8, 10, FAKE, FAKE * 2, FAKE * 4, FAKE * 8, None, 4, None) == E_FUNC
    finally:
        binding.chessfad_release_function(fid)
    assert lib.chessfad_release_function(fid) == E_FUNC
    assert lib.chessfad_hvp(fid, 8, 10, FAKE, FAKE * 2, FAKE * 4, 4, None) == E_FUNC
    with pytest.raises(binding.ChessfadError) as ei:
        binding.chessfad_register_function("template <class V, class Y> __device__ V chessfad_user_f(const Y& y, int n)"
                                           " { return no_such_function(y[0]); }")
    assert ei.value.code == -9 and "no_such_function" in str(ei.value)
    assert lib.chessfad_register_function(None, None) == E_NULL


def test_options(lib):
    assert lib.chessfad_set_option(99, 0) == E_ARG
    assert lib.chessfad_set_option(binding.CHESSFAD_OPT_FP_MFMA, 4) == E_ARG
    assert lib.chessfad_set_option(binding.CHESSFAD_OPT_FP_MFMA, 2) == 1   # the default is 1
    assert lib.chessfad_set_option(binding.CHESSFAD_OPT_FP_MFMA, 1) == 2
    assert lib.chessfad_set_option(binding.CHESSFAD_OPT_MAPPING, 3) == E_ARG
    assert lib.chessfad_set_option(binding.CHESSFAD_OPT_MAPPING, -1) == E_ARG
    prev = lib.chessfad_set_option(binding.CHESSFAD_OPT_MAPPING, 0)
    assert prev == 2
    assert lib.chessfad_set_option(binding.CHESSFAD_OPT_MAPPING, prev) == 0
    for bad in (-1, 2, 3, 5, 17):
        assert lib.chessfad_set_option(binding.CHESSFAD_OPT_FP_POINTS, bad) == E_ARG
    assert lib.chessfad_set_option(binding.CHESSFAD_OPT_FP_POINTS, 4) == 0   # the default is 0 (automatic)
    assert lib.chessfad_set_option(binding.CHESSFAD_OPT_FP_POINTS, 0) == 4
    for bad in (-1, 17):
        assert lib.chessfad_set_option(binding.CHESSFAD_OPT_FP_BLOCKS, bad) == E_ARG
    assert lib.chessfad_set_option(binding.CHESSFAD_OPT_FP_BLOCKS, 3) == 0   # the default is 0 (cost model)
    assert lib.chessfad_set_option(binding.CHESSFAD_OPT_FP_BLOCKS, 0) == 3


def test_default_chunk(lib):
    assert lib.chessfad_default_mapping(R, 16, 0) in (1, 2)
    assert lib.chessfad_default_mapping(A, 16, 1) in (1, 2)
    assert lib.chessfad_default_mapping(9, 16, 0) == E_FUNC
    assert lib.chessfad_default_mapping(R, 16, 2) == E_ARG
    assert lib.chessfad_default_chunk(R, 16) in (1, 2, 4, 8, 16)
    assert lib.chessfad_default_chunk(A, 1) == 1
    assert lib.chessfad_default_chunk(5, 16) == E_FUNC
    assert lib.chessfad_default_chunk(R, 1) == E_N


def test_fp_params_argument_checks(lib):
    assert lib.chessfad_fp_set_params(0, FAKE, FAKE, FAKE, None) == E_N
    assert lib.chessfad_fp_set_params(600, FAKE, FAKE, FAKE, None) == E_N
    assert lib.chessfad_fp_set_params(8, None, FAKE, FAKE, None) == E_NULL
    assert lib.chessfad_fp_release(0) == E_N


def test_binding_rejects_bad_tensors():
    import torch

    x = torch.zeros(4, 8, dtype=torch.float64)  # CPU tensor: refused before any call
    with pytest.raises(ValueError):
        binding.chessfad_hvp(R, x, x)
    with pytest.raises(ValueError):
        binding.chessfad_hessian(R, x)


def _inst(func=R, n=16, chunk=4, precision=0, npts=3, x=FAKE, v=FAKE * 2, out=FAKE * 4, A=None, B=None, alpha=None,
          io_fp32=0):
    return binding.Instance(func_id=func, n=n, chunk=chunk, precision=precision, io_fp32=io_fp32, npts=npts, x=x, v=v,
                            out=out, A=A, B=B, alpha=alpha)


def _create(lib, insts):
    arr = (binding.Instance * len(insts))(*insts)
    h, bad = ctypes.c_void_p(), ctypes.c_int(-7)
    rc = lib.chessfad_batch_create(ctypes.cast(arr, ctypes.c_void_p), len(insts), None, ctypes.byref(h),
                                   ctypes.byref(bad))
    return rc, bad.value


def test_batch_validation_before_any_device_work(lib):
    ok = _inst()
    assert _create(lib, [ok, _inst(chunk=32)]) == (E_CHUNK, 1)          # compiled chunks: 1, 2, 4, 8, 16
    assert _create(lib, [ok, _inst(n=8, chunk=16)]) == (E_CHUNK, 1)     # chunk above n
    assert _create(lib, [_inst(io_fp32=2)]) == (E_ARG, 0)
    # float32 I/O: an output overlapping its input by the float32 extent only
    assert _create(lib, [_inst(npts=4, n=16, x=FAKE, v=FAKE * 8, out=FAKE + 4 * 64 - 8, io_fp32=1)]) == (E_OVERLAP, 0)
    assert _create(lib, [_inst(func=FP, chunk=16)]) == (E_PARAMS, 0)   # Fletcher-Powell takes 16
    assert _create(lib, [_inst(func=9), ok]) == (E_FUNC, 0)
    assert _create(lib, [ok, ok, _inst(n=600)]) == (E_N, 2)
    assert _create(lib, [_inst(precision=2)]) == (E_ARG, 0)
    assert _create(lib, [_inst(npts=-1)]) == (E_ARG, 0)
    assert _create(lib, [_inst(func=FP)]) == (E_PARAMS, 0)              # Fletcher-Powell without A, B, alpha
    assert _create(lib, [_inst(x=None)]) == (E_NULL, 0)
    assert _create(lib, [_inst(out=FAKE)]) == (E_OVERLAP, 0)
    assert _create(lib, [_inst(n=8, chunk=8, func=A), _inst(n=300, chunk=1)]) == (E_CHUNK, 1)  # nc > 256
    h = ctypes.c_void_p()
    assert lib.chessfad_batch_create(None, 2, None, ctypes.byref(h), None) == E_ARG
    assert lib.chessfad_batch_run(None, None) == E_ARG
    assert lib.chessfad_batch_destroy(None) == E_ARG
    assert lib.chessfad_batch_info(None, None, None, None) == E_ARG
    assert lib.chessfad_batch_choices(None, None, 0, None) == E_ARG


def test_autotune_argument_checks(lib):
    c, ms = ctypes.c_int(), ctypes.c_float()
    assert lib.chessfad_autotune(4, 16, 0, 100, None, ctypes.byref(c), ctypes.byref(ms)) == E_FUNC
    assert lib.chessfad_autotune(R, 1, 0, 100, None, None, None) == E_N
    assert lib.chessfad_autotune(A, 16, 3, 100, None, None, None) == E_ARG
    assert lib.chessfad_autotune(A, 16, 0, 0, None, None, None) == E_ARG



def test_batch_noalloc_checks_before_any_device_work(lib):
    def run(insts):
        arr = (binding.Instance * len(insts))(*insts)
        bad = ctypes.c_int(-7)
        rc = lib.chessfad_batch_run_noalloc(ctypes.cast(arr, ctypes.c_void_p), len(insts), None, ctypes.byref(bad))
        return rc, bad.value

    ok = _inst()
    assert run([ok, _inst(chunk=32)]) == (E_CHUNK, 1)
    assert run([_inst(func=9), ok]) == (E_FUNC, 0)
    assert run([_inst(func=FP)]) == (E_PARAMS, 0)
    assert run([_inst(out=FAKE)]) == (E_OVERLAP, 0)
    assert lib.chessfad_batch_run_noalloc(None, 2, None, None) == E_ARG
    # 40 mixed Fletcher-Powell instances at n = 512 keep 80 MiB of float32
    # copies of A and B: more than the fixed array holds
    big = _inst(func=FP, n=512, chunk=16, precision=1, A=FAKE * 8, B=FAKE * 16, alpha=FAKE * 32)
    assert run([big] * 40) == (E_ARG, -1)


def test_fp_launch_shape_invariants(lib):
    """The per-call Fletcher-Powell kernel's launch shapes (n > 16), full and
    symmetric form, both precisions, every points / column-blocks option:
    at most 16 lane rows per workgroup, no more blocks than the variables
    have, LDS within 64 KiB, a nonempty grid that covers the points."""
    import itertools
    for n in list(range(17, 80)) + [100, 128, 200, 255, 256, 257, 300, 400, 511, 512]:
        nb = (n + 15) // 16
        for npts, prec in itertools.product((1, 5, 37, 1024, 1 << 18), (0, 1)):
            for points, blocks in itertools.product((0, 1, 4, 16), (0, 1, 3, 16)):
                lib.chessfad_set_option(binding.CHESSFAD_OPT_FP_POINTS, points)
                lib.chessfad_set_option(binding.CHESSFAD_OPT_FP_BLOCKS, blocks)
                s = binding.chessfad_fp_launch_shape(n, npts, prec)
                assert s["points"] >= 1 and 1 <= s["row_blocks"] <= nb and 1 <= s["column_blocks"] <= nb, (n, s)
                assert s["points"] * s["row_blocks"] * s["column_blocks"] <= 16, (n, s)
                if blocks:
                    assert s["column_blocks"] == min(blocks, nb), (n, blocks, s)
                assert 0 < s["lds_bytes"] <= 64 * 1024, (n, s)
                rounds = -(-nb // s["row_blocks"])
                assert 1 <= s["split"] <= rounds, (n, s)
                assert s["grid"] == -(-npts // s["points"]) * s["split"], (n, npts, s)
            lib.chessfad_set_option(binding.CHESSFAD_OPT_FP_POINTS, 0)
            lib.chessfad_set_option(binding.CHESSFAD_OPT_FP_BLOCKS, 0)
            s = binding.chessfad_fp_launch_shape(n, npts, prec, sym=True)
            assert s["points"] >= 1 and 1 <= s["row_blocks"] <= nb and 1 <= s["column_blocks"] <= nb, (n, s)
            assert s["points"] * s["row_blocks"] * s["column_blocks"] <= 16, (n, s)
            assert 0 < s["lds_bytes"] <= 64 * 1024 and s["split"] == 1, (n, s)
            assert s["grid"] == -(-npts // s["points"]), (n, npts, s)
    for bad_n in (16, 513):
        with pytest.raises(binding.ChessfadError):
            binding.chessfad_fp_launch_shape(bad_n, 10)
    with pytest.raises(binding.ChessfadError):
        binding.chessfad_fp_launch_shape(64, 0)
    with pytest.raises(binding.ChessfadError):
        binding.chessfad_fp_launch_shape(64, 10, precision=2)
