"""Thin ctypes binding over libchessfad.so (include/chessfad.h).

Argument marshalling only: torch CUDA tensors are passed as raw device
pointers together with the current HIP stream; every step of the method
runs in the library's kernels.  The functions carry the C names.  There is
no fallback: if the library is missing, `load()` raises.
"""
from __future__ import annotations

import ctypes
import os

import torch

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libchessfad.so")

# ABI symbols and their ctypes signatures (must match include/chessfad.h)
_i, _i64, _p, _s = ctypes.c_int, ctypes.c_int64, ctypes.c_void_p, ctypes.c_char_p
_pi, _pi64, _pd, _pf, _pp = (ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int64),
                             ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_float),
                             ctypes.POINTER(ctypes.c_void_p))


class Instance(ctypes.Structure):
    """struct chessfad_instance"""
    _fields_ = [("func_id", ctypes.c_int), ("n", ctypes.c_int), ("chunk", ctypes.c_int),
                ("precision", ctypes.c_int), ("io_fp32", ctypes.c_int), ("npts", ctypes.c_int64),
                ("x", ctypes.c_void_p), ("v", ctypes.c_void_p), ("out", ctypes.c_void_p), ("A", ctypes.c_void_p),
                ("B", ctypes.c_void_p), ("alpha", ctypes.c_void_p)]


class BatchChoice(ctypes.Structure):
    """struct chessfad_batch_choice"""
    _fields_ = [("func_id", ctypes.c_int), ("n_lo", ctypes.c_int), ("n_hi", ctypes.c_int),
                ("precision", ctypes.c_int), ("instances", ctypes.c_int), ("chunk", ctypes.c_int),
                ("mapping", ctypes.c_int), ("points", ctypes.c_int), ("blocks", ctypes.c_int),
                ("candidates", ctypes.c_int),
                ("ms", ctypes.c_float)]

class FpShape(ctypes.Structure):
    """struct chessfad_fp_shape"""
    _fields_ = [("points", ctypes.c_int), ("row_blocks", ctypes.c_int), ("column_blocks", ctypes.c_int),
                ("split", ctypes.c_int), ("grid", ctypes.c_int64),
                ("lds_bytes", ctypes.c_size_t)]

SIGNATURES = {
    "chessfad_hvp": (_i, [_i, _i, _i64, _p, _p, _p, _i, _p]),
    "chessfad_hessian": (_i, [_i, _i, _i64, _p, _p, _i, _p]),
    "chessfad_hvp_mixed": (_i, [_i, _i, _i64, _p, _p, _p, _i, _p]),
    "chessfad_hessian_mixed": (_i, [_i, _i, _i64, _p, _p, _i, _p]),
    "chessfad_fp_set_params": (_i, [_i, _p, _p, _p, _p]),
    "chessfad_fp_release": (_i, [_i]),
    "chessfad_strerror": (_s, [_i]),
    "chessfad_default_chunk": (_i, [_i, _i]),
    "chessfad_default_mapping": (_i, [_i, _i, _i]),
    "chessfad_fp_launch_shape": (_i, [_i, _i64, _i, _i, _p]),
    "chessfad_register_function": (_i, [_s, _pi]),
    "chessfad_release_function": (_i, [_i]),
    "chessfad_set_option": (_i, [_i, _i]),
    "chessfad_batch_create": (_i, [_p, _i, _p, _pp, _pi]),
    "chessfad_batch_run": (_i, [_p, _p]),
    "chessfad_batch_destroy": (_i, [_p]),
    "chessfad_batch_info": (_i, [_p, _pi64, _pi, _pd]),
    "chessfad_batch_run_noalloc": (_i, [_p, _i, _p, _pi]),
    "chessfad_batch_choices": (_i, [_p, _p, _i, _pi]),
    "chessfad_autotune": (_i, [_i, _i, _i, _i64, _p, _pi, _pf]),
    "chessfad_hvp_sym": (_i, [_i, _i, _i64, _p, _p, _p, _i, _i, _p]),
    "chessfad_hvp_grad": (_i, [_i, _i, _i64, _p, _p, _p, _p, _p, _i, _p]),
    "chessfad_hessian_sym": (_i, [_i, _i, _i64, _p, _p, _i, _i, _p]),
    "chessfad_autotune_sym": (_i, [_i, _i, _i, _i64, _p, _pi, _pf]),
}

CHESSFAD_OPT_FP_MFMA = 1
CHESSFAD_OPT_BATCH_GRAPH = 2
CHESSFAD_OPT_MAPPING = 3
CHESSFAD_OPT_FP_POINTS = 4
CHESSFAD_OPT_BATCH_TUNE = 5
CHESSFAD_OPT_FP_BLOCKS = 6

_lib = None


class ChessfadError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what} failed with status {code}: {strerror(code)}")
        self.code = code


def load(path: str = LIB_PATH):
    """Load the library (once).  Raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is missing: build it with `python -m paper_2410_22575_amd.build`")
        lib = ctypes.CDLL(path)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def strerror(code: int) -> str:
    return load().chessfad_strerror(code).decode()


def _stream(stream):
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, torch.cuda.Stream):
        return stream.cuda_stream
    return int(stream)


def _check_pts(name, t, n=None):
    if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous() and t.dim() == 2):
        raise ValueError(f"{name} must be a contiguous 2-D float64 CUDA tensor")
    if n is not None and t.shape[1] != n:
        raise ValueError(f"{name} has {t.shape[1]} columns, expected {n}")


def _raise(rc, what):
    if rc != 0:
        raise ChessfadError(rc, what)


def _hvp(name, func_id, x, v, out, chunk, stream, *extra):
    _check_pts("x", x)
    npts, n = x.shape
    _check_pts("v", v, n)
    if out is None:
        out = torch.empty_like(x)
    _check_pts("out", out, n)
    rc = getattr(load(), name)(func_id, n, npts, x.data_ptr(), v.data_ptr(), out.data_ptr(), chunk, *extra,
                               _stream(stream))
    _raise(rc, name)
    return out


def _hessian(name, func_id, x, out, chunk, stream, *extra):
    _check_pts("x", x)
    npts, n = x.shape
    if out is None:
        out = torch.empty((npts, n, n), dtype=torch.float64, device=x.device)
    if not (out.is_cuda and out.dtype == torch.float64 and out.is_contiguous() and tuple(out.shape) == (npts, n, n)):
        raise ValueError("out must be a contiguous float64 CUDA tensor of shape [npts, n, n]")
    rc = getattr(load(), name)(func_id, n, npts, x.data_ptr(), out.data_ptr(), chunk, *extra, _stream(stream))
    _raise(rc, name)
    return out


def chessfad_hvp(func_id: int, x: torch.Tensor, v: torch.Tensor, out: torch.Tensor | None = None,
                 chunk: int = 0, stream=None) -> torch.Tensor:
    """out[p] = H(x[p]) v[p] (float64 hDual arithmetic)."""
    return _hvp("chessfad_hvp", func_id, x, v, out, chunk, stream)


def chessfad_hessian(func_id: int, x: torch.Tensor, out: torch.Tensor | None = None, chunk: int = 0,
                     stream=None) -> torch.Tensor:
    """out[p] = H(x[p]) as [npts, n, n] (float64 hDual arithmetic)."""
    return _hessian("chessfad_hessian", func_id, x, out, chunk, stream)


def chessfad_hvp_mixed(func_id: int, x: torch.Tensor, v: torch.Tensor, out: torch.Tensor | None = None,
                       chunk: int = 0, stream=None) -> torch.Tensor:
    """H.v with float32 hDuals, compensated sums and float64 islands."""
    return _hvp("chessfad_hvp_mixed", func_id, x, v, out, chunk, stream)


def chessfad_hessian_mixed(func_id: int, x: torch.Tensor, out: torch.Tensor | None = None, chunk: int = 0,
                           stream=None) -> torch.Tensor:
    """Hessians with float32 hDuals, compensated sums and float64 islands."""
    return _hessian("chessfad_hessian_mixed", func_id, x, out, chunk, stream)


def chessfad_hvp_grad(func_id: int, x: torch.Tensor, v: torch.Tensor, chunk: int = 0, want_f: bool = True,
                      stream=None):
    """(H.v, gradient, f or None) from the same calls (float64)."""
    _check_pts("x", x)
    npts, n = x.shape
    _check_pts("v", v, n)
    out, grad = torch.empty_like(x), torch.empty_like(x)
    fval = torch.empty(npts, dtype=torch.float64, device=x.device) if want_f else None
    rc = load().chessfad_hvp_grad(func_id, n, npts, x.data_ptr(), v.data_ptr(), out.data_ptr(), grad.data_ptr(),
                                  fval.data_ptr() if want_f else None, chunk, _stream(stream))
    _raise(rc, "chessfad_hvp_grad")
    return out, grad, fval


def chessfad_hvp_sym(func_id: int, x: torch.Tensor, v: torch.Tensor, out: torch.Tensor | None = None,
                     chunk: int = 0, precision: int = 0, stream=None) -> torch.Tensor:
    """SC-HESS-VEC: H.v evaluating only the chunks from each row's own chunk on."""
    return _hvp("chessfad_hvp_sym", func_id, x, v, out, chunk, stream, precision)


def chessfad_hessian_sym(func_id: int, x: torch.Tensor, out: torch.Tensor | None = None, chunk: int = 0,
                         precision: int = 0, stream=None) -> torch.Tensor:
    """SCHUNK-HESS: Hessians with the entries left of each row's own chunk mirrored."""
    return _hessian("chessfad_hessian_sym", func_id, x, out, chunk, stream, precision)


def chessfad_fp_set_params(A: torch.Tensor, B: torch.Tensor, alpha: torch.Tensor, stream=None) -> None:
    """Register Fletcher-Powell (A, B, alpha) for n = alpha.numel()."""
    n = alpha.numel()
    for name, t, shape in (("A", A, (n, n)), ("B", B, (n, n)), ("alpha", alpha, (n,))):
        if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous() and tuple(t.shape) == shape):
            raise ValueError(f"{name} must be a contiguous float64 CUDA tensor of shape {shape}")
    rc = load().chessfad_fp_set_params(n, A.data_ptr(), B.data_ptr(), alpha.data_ptr(), _stream(stream))
    _raise(rc, "chessfad_fp_set_params")


def chessfad_fp_release(n: int) -> None:
    _raise(load().chessfad_fp_release(n), "chessfad_fp_release")


def chessfad_register_function(source: str) -> int:
    """Compile a user function (chessfad_device.h) and return its func_id."""
    fid = ctypes.c_int(-1)
    rc = load().chessfad_register_function(source.encode(), ctypes.byref(fid))
    _raise(rc, "chessfad_register_function")
    return fid.value


def chessfad_release_function(func_id: int) -> None:
    _raise(load().chessfad_release_function(func_id), "chessfad_release_function")


def chessfad_default_mapping(func_id: int, n: int, precision: int = 0) -> int:
    return load().chessfad_default_mapping(func_id, n, precision)


def chessfad_fp_launch_shape(n: int, npts: int, precision: int = 0, sym: bool = False) -> dict:
    """The launch shape of the per-call Fletcher-Powell kernel for n > 16 (host only)."""
    out = FpShape()
    _raise(load().chessfad_fp_launch_shape(n, npts, precision, int(sym), ctypes.byref(out)),
           "chessfad_fp_launch_shape")
    return {f: getattr(out, f) for f, _ in FpShape._fields_}


def chessfad_default_chunk(func_id: int, n: int) -> int:
    rc = load().chessfad_default_chunk(func_id, n)
    if rc < 0:
        raise ChessfadError(rc, "chessfad_default_chunk")
    return rc


def chessfad_set_option(option: int, value: int) -> int:
    """Set a process-wide option; returns the previous value."""
    rc = load().chessfad_set_option(option, value)
    if rc < 0:
        raise ChessfadError(rc, "chessfad_set_option")
    return rc


def _ptr(t):
    return t.data_ptr() if t is not None else None


class BatchPlan:
    """A chessfad_batch plan.  Holds references to every tensor it reads or
    writes so they stay alive as long as the plan."""

    def __init__(self, handle, keep):
        self._h = handle
        self._keep = keep

    def run(self, stream=None):
        _raise(load().chessfad_batch_run(self._h, _stream(stream)), "chessfad_batch_run")

    def info(self):
        items, wg, fl = ctypes.c_int64(), ctypes.c_int(), ctypes.c_double()
        _raise(load().chessfad_batch_info(self._h, ctypes.byref(items), ctypes.byref(wg), ctypes.byref(fl)),
               "chessfad_batch_info")
        return {"items": items.value, "workgroups": wg.value, "model_flops": fl.value}

    def choices(self):
        """The plan-time tuner's choices, one dict per (function, octave of n,
        precision) group."""
        count = ctypes.c_int()
        _raise(load().chessfad_batch_choices(self._h, None, 0, ctypes.byref(count)), "chessfad_batch_choices")
        arr = (BatchChoice * max(1, count.value))()
        _raise(load().chessfad_batch_choices(self._h, ctypes.cast(arr, ctypes.c_void_p), count.value,
                                             ctypes.byref(count)), "chessfad_batch_choices")
        return [{f: getattr(arr[k], f) for f, _ in BatchChoice._fields_} for k in range(count.value)]

    def destroy(self):
        if self._h:
            load().chessfad_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def _instances(instances):
    """ctypes array of chessfad_instance, and the tensors it points into."""
    arr = (Instance * max(1, len(instances)))()
    keep = []
    for k, d in enumerate(instances):
        x, v, out = d["x"], d["v"], d["out"]
        # x, v, out: all float64, or all float32 (the instance's io_fp32)
        io32 = x.dtype == torch.float32
        dt = torch.float32 if io32 else torch.float64
        for name, t in (("x", x), ("v", v), ("out", out)):
            if not (t.is_cuda and t.dtype == dt and t.dim() == 2 and t.is_contiguous()):
                raise ValueError(f"instance {k}: {name} must be a contiguous [npts, n] {dt} CUDA tensor")
        npts, n = x.shape
        if v.shape != x.shape or out.shape != x.shape:
            raise ValueError(f"instance {k}: x, v and out must have the same shape")
        A, B, alpha = d.get("A"), d.get("B"), d.get("alpha")
        for name, t in (("A", A), ("B", B), ("alpha", alpha)):
            if t is not None and not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
                raise ValueError(f"instance {k}: {name} must be a contiguous float64 CUDA tensor")
        arr[k] = Instance(d["func_id"], n, d.get("chunk", 0), d.get("precision", 0), int(io32), npts, _ptr(x),
                          _ptr(v), _ptr(out), _ptr(A), _ptr(B), _ptr(alpha))
        keep += [t for t in (x, v, out, A, B, alpha) if t is not None]
    return arr, keep


def chessfad_batch_create(instances, stream=None) -> BatchPlan:
    """instances: list of dicts with func_id, x, v, out (CUDA tensors
    [npts, n], all float64 or all float32), optional chunk (0), precision
    (0 or 1) and, for
    Fletcher-Powell, A, B, alpha (float64 CUDA tensors)."""
    arr, keep = _instances(instances)
    h = ctypes.c_void_p()
    bad = ctypes.c_int(-1)
    rc = load().chessfad_batch_create(ctypes.cast(arr, ctypes.c_void_p), len(instances), _stream(stream),
                                      ctypes.byref(h), ctypes.byref(bad))
    if rc != 0:
        err = ChessfadError(rc, f"chessfad_batch_create (instance {bad.value})")
        err.bad_index = bad.value
        raise err
    return BatchPlan(h, keep)


def chessfad_batch_run_noalloc(instances, stream=None) -> None:
    """Plan and run the instances (as chessfad_batch_create) in the library's
    fixed device array, without allocating device memory; returns when the
    stream has finished the work."""
    arr, keep = _instances(instances)
    bad = ctypes.c_int(-1)
    rc = load().chessfad_batch_run_noalloc(ctypes.cast(arr, ctypes.c_void_p), len(instances), _stream(stream),
                                           ctypes.byref(bad))
    if rc != 0:
        err = ChessfadError(rc, f"chessfad_batch_run_noalloc (instance {bad.value})")
        err.bad_index = bad.value
        raise err
    del keep


def chessfad_autotune(func_id: int, n: int, precision: int = 0, npts: int = 1 << 16, stream=None):
    """Time every compiled chunk and record the fastest; returns (chunk, ms)."""
    c, ms = ctypes.c_int(), ctypes.c_float()
    _raise(load().chessfad_autotune(func_id, n, precision, npts, _stream(stream), ctypes.byref(c), ctypes.byref(ms)),
           "chessfad_autotune")
    return c.value, ms.value


def chessfad_autotune_sym(func_id: int, n: int, precision: int = 0, npts: int = 1 << 16, stream=None):
    """The same search for the symmetric H.v; returns (chunk, ms)."""
    c, ms = ctypes.c_int(), ctypes.c_float()
    _raise(load().chessfad_autotune_sym(func_id, n, precision, npts, _stream(stream), ctypes.byref(c),
                                        ctypes.byref(ms)), "chessfad_autotune_sym")
    return c.value, ms.value
