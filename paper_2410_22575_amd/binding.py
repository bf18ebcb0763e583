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
SIGNATURES = {
    "chessfad_hvp": (_i, [_i, _i, _i64, _p, _p, _p, _i, _p]),
    "chessfad_hessian": (_i, [_i, _i, _i64, _p, _p, _i, _p]),
    "chessfad_hvp_mixed": (_i, [_i, _i, _i64, _p, _p, _p, _i, _p]),
    "chessfad_hessian_mixed": (_i, [_i, _i, _i64, _p, _p, _i, _p]),
    "chessfad_fp_set_params": (_i, [_i, _p, _p, _p, _p]),
    "chessfad_fp_release": (_i, [_i]),
    "chessfad_strerror": (_s, [_i]),
    "chessfad_default_chunk": (_i, [_i, _i]),
    "chessfad_set_option": (_i, [_i, _i]),
}

CHESSFAD_OPT_FP_MFMA = 1

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


def _hvp(name, func_id, x, v, out, chunk, stream):
    _check_pts("x", x)
    npts, n = x.shape
    _check_pts("v", v, n)
    if out is None:
        out = torch.empty_like(x)
    _check_pts("out", out, n)
    rc = getattr(load(), name)(func_id, n, npts, x.data_ptr(), v.data_ptr(), out.data_ptr(), chunk,
                               _stream(stream))
    _raise(rc, name)
    return out


def _hessian(name, func_id, x, out, chunk, stream):
    _check_pts("x", x)
    npts, n = x.shape
    if out is None:
        out = torch.empty((npts, n, n), dtype=torch.float64, device=x.device)
    if not (out.is_cuda and out.dtype == torch.float64 and out.is_contiguous() and tuple(out.shape) == (npts, n, n)):
        raise ValueError("out must be a contiguous float64 CUDA tensor of shape [npts, n, n]")
    rc = getattr(load(), name)(func_id, n, npts, x.data_ptr(), out.data_ptr(), chunk, _stream(stream))
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
