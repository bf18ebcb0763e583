"""MI355X-native chunked forward-mode Hessian and Hessian-vector products.

The compute path is the HIP library `libchessfad.so` (built from csrc/ for
gfx950) behind a C ABI declared in include/chessfad.h; `binding` marshals
torch device tensors into those calls.  Importing this package does not load
the library; the first call does, and fails loudly if it is missing.
"""
from .inputs import ROSENBROCK, ACKLEY, FLETCHER_POWELL, FUNC_NAMES  # noqa: F401

__all__ = ["ROSENBROCK", "ACKLEY", "FLETCHER_POWELL", "FUNC_NAMES"]
