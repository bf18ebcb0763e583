"""The kernels' sin/cos routine (csrc/trig.hpp), built for the host and
checked against the C library's sin and cos (Python's math module).

The routine reduces x by k pi/2 with a two-part pi/2 and evaluates the Taylor
series of sin and cos on |r| <= pi/4; beyond |x| = 65536 it calls the library.
Pinned here: at most 2 ulp from the library wherever the value is not tiny,
an absolute error within 2.5e-16 everywhere, sin x = x to 2 ulp for small x,
cos 0 = 1 and sin 0 = 0 exactly, and the quadrant signs at every multiple of
pi/4 up to 64 quarter turns.
"""
import math
import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2410_22575_amd", "csrc")
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


@pytest.fixture(scope="module")
def trig_exe(tmp_path_factory):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not found")
    exe = str(tmp_path_factory.mktemp("trig") / "trig_host_check")
    src = os.path.join(ROOT, "tests", "trig_host_check.cpp")
    subprocess.run([HIPCC, "-x", "hip", "--cuda-host-only", "-O2", "-std=c++17", "-I", CSRC, src, "-o", exe],
                   check=True, capture_output=True)
    return exe


def _run(exe, xs):
    inp = "".join(float(x).hex() + "\n" for x in xs)
    out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout.split("\n")
    sc = [line.split() for line in out if line]
    return (np.array([float.fromhex(a) for a, _ in sc]), np.array([float.fromhex(b) for _, b in sc]))


def _args():
    rng = np.random.default_rng(20241029)
    return np.concatenate([
        rng.uniform(-4.0, 4.0, 20000),              # Fletcher-Powell's x = alpha + U[-0.1, 0.1]
        2.0 * math.pi * rng.uniform(-5.0, 5.0, 20000),   # Ackley's 2 pi x
        rng.uniform(-65536.0, 65536.0, 20000),      # the whole fast range
        rng.uniform(-1e-3, 1e-3, 5000),
        np.ldexp(rng.uniform(0.5, 1.0, 2000), rng.integers(-60, -10, 2000)),
        [65535.99999999999, 65536.0, 65536.00000000001, -65536.00000000001, 1e6, -3e9, 1e15, 0.0],
    ])


def test_against_library(trig_exe):
    xs = _args()
    s, c = _run(trig_exe, xs)
    rs = np.array([math.sin(x) for x in xs])
    rc = np.array([math.cos(x) for x in xs])
    assert np.max(np.abs(s - rs)) <= 2.5e-16
    assert np.max(np.abs(c - rc)) <= 2.5e-16
    for got, ref in ((s, rs), (c, rc)):
        big = np.abs(ref) >= 2.0 ** -10
        ulp = np.array([math.ulp(v) for v in ref[big]])
        assert np.max(np.abs(got[big] - ref[big]) / ulp) <= 2.0


def test_small_arguments(trig_exe):
    xs = np.ldexp(np.linspace(0.5, 1.0, 64), -30)
    s, c = _run(trig_exe, np.concatenate([xs, -xs, [0.0]]))
    ref = np.concatenate([xs, -xs, [0.0]])
    assert np.all(np.abs(s - ref) <= 2 * np.array([math.ulp(v) for v in ref]))
    assert s[-1] == 0.0 and c[-1] == 1.0
    assert np.all(c[:-1] == 1.0)


def test_quadrants(trig_exe):
    k = np.arange(-64, 65)
    xs = k * (math.pi / 4)
    s, c = _run(trig_exe, xs)
    # signs of sin and cos at k pi/4 (the values on the axes are tiny, not zero)
    q = np.mod(k, 8)
    want_s = np.array([0, 1, 1, 1, 0, -1, -1, -1])[q]
    want_c = np.array([1, 1, 0, -1, -1, -1, 0, 1])[q]
    assert np.all(np.sign(np.round(s, 12)) == want_s)
    assert np.all(np.sign(np.round(c, 12)) == want_c)
