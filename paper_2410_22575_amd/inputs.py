"""Seeded synthetic inputs for the three test functions.

This module only draws random numbers; it holds none of the method's
arithmetic (the Fletcher-Powell offsets E are derived from alpha by the
library and, separately, by the oracle).  Both the tests and the benchmark
take their inputs from here so the GPU path and the CPU oracle see the same
bytes.

Recipe (one numpy Generator per workload, seeded 241022575 + workload id):
  * Fletcher-Powell: A then B, integers drawn uniformly from [-100, 100]
    inclusive (n x n, stored as float64); then alpha ~ U[-pi, pi] (n);
    then X = alpha + U[-0.1, 0.1] per point.
  * Rosenbrock: X ~ U[-2, 2].   Ackley: X ~ U[-5, 5].
  * V ~ N(0, 1), drawn after X.
The three functions are the ones the paper evaluates on (Sec. VII); their
domains and parameter ranges follow the usual benchmark definitions.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Optional

import numpy as np

SEED_BASE = 241022575

ROSENBROCK = 0
ACKLEY = 1
FLETCHER_POWELL = 2
FUNC_NAMES = {ROSENBROCK: "rosenbrock", ACKLEY: "ackley", FLETCHER_POWELL: "fletcher_powell"}


@dataclass
class Workload:
    func: int
    n: int
    x: np.ndarray                       # [npts, n] float64, row-major
    v: np.ndarray                       # [npts, n] float64
    A: Optional[np.ndarray] = None      # [n, n] float64 (Fletcher-Powell only)
    B: Optional[np.ndarray] = None      # [n, n] float64
    alpha: Optional[np.ndarray] = None  # [n] float64

    @property
    def npts(self) -> int:
        return self.x.shape[0]


def rng_for(workload_id: int) -> np.random.Generator:
    return np.random.default_rng(SEED_BASE + workload_id)


def fp_params(n: int, rng: np.random.Generator):
    """Draw (A, B, alpha) for one Fletcher-Powell instance, in that order."""
    A = rng.integers(-100, 101, size=(n, n)).astype(np.float64)
    B = rng.integers(-100, 101, size=(n, n)).astype(np.float64)
    alpha = rng.uniform(-np.pi, np.pi, size=n)
    return A, B, alpha


def make_workload(func: int, n: int, npts: int, rng: np.random.Generator) -> Workload:
    """Draw one function instance and `npts` points (x, v) for it."""
    if func == FLETCHER_POWELL:
        A, B, alpha = fp_params(n, rng)
        x = alpha[None, :] + rng.uniform(-0.1, 0.1, size=(npts, n))
        v = rng.standard_normal(size=(npts, n))
        return Workload(func, n, np.ascontiguousarray(x), np.ascontiguousarray(v), A, B, alpha)
    if func == ROSENBROCK:
        x = rng.uniform(-2.0, 2.0, size=(npts, n))
    elif func == ACKLEY:
        x = rng.uniform(-5.0, 5.0, size=(npts, n))
    else:
        raise ValueError(f"unknown function id {func}")
    v = rng.standard_normal(size=(npts, n))
    return Workload(func, n, np.ascontiguousarray(x), np.ascontiguousarray(v))


def mixed_instances(ninst: int, rng: np.random.Generator, nmin: int = 8, nmax: int = 256,
                    npts: int = 1):
    """Batched workload: `ninst` instances, function uniform over the three,
    n = round(nmin * (nmax/nmin)**u) with u ~ U[0, 1] (log-uniform), each
    with its own Fletcher-Powell parameters and `npts` points."""
    out = []
    for _ in range(ninst):
        func = int(rng.integers(0, 3))
        u = rng.uniform(0.0, 1.0)
        n = int(round(nmin * (nmax / nmin) ** u))
        out.append(make_workload(func, n, npts, rng))
    return out
