"""The kernels' own FP64 arithmetic helpers, built for the host from the same
source.

* The logarithm (artanh reduction, written without contraction so the host
  evaluates exactly what the device does) against numpy's log in extended
  precision: within one unit in the last place over the temperature range,
  error-norm magnitudes, the whole positive normal range, subnormals and the
  neighbourhoods of 1 and sqrt(2), and the IEEE special values.
* The division by a launch constant (the system size n in the error norms'
  mean): bit-identical to the IEEE quotient x / n for every n the kernels
  take wherever the quotient is a normal number (sums of squares of all
  magnitudes), and for 0, inf and NaN; a subnormal quotient is within one
  unit of its last place."""
import ctypes
import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2312_02836_amd", "csrc")
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


@pytest.fixture(scope="module")
def hostlib(tmp_path_factory):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    out = str(tmp_path_factory.mktemp("bnlog") / "libbnlog.so")
    subprocess.run([HIPCC, "--offload-arch=gfx950", "-O2", "-fPIC", "-shared", "-I", CSRC,
                    os.path.join(HERE, "native", "bn_log_host.hip"), "-o", out],
                   check=True, capture_output=True)
    return ctypes.CDLL(out)


@pytest.fixture(scope="module")
def bn_log(hostlib):
    lib = hostlib

    def f(x):
        x = np.ascontiguousarray(x, dtype=np.float64)
        y = np.empty_like(x)
        lib.bn_log_host(x.ctypes.data_as(ctypes.c_void_p), y.ctypes.data_as(ctypes.c_void_p),
                        ctypes.c_long(x.size))
        return y
    return f


def _ulps(y, x):
    ref = np.log(x.astype(np.longdouble))
    return np.abs((y.astype(np.longdouble) - ref) / np.spacing(np.abs(ref.astype(np.float64))))


@pytest.mark.skipif(np.finfo(np.longdouble).nmant < 60, reason="needs extended long double")
def test_within_one_ulp(bn_log):
    rng = np.random.default_rng(0)
    cases = {
        "temperature": rng.uniform(0.5, 10.0, 200_000),
        "norms": 10.0 ** rng.uniform(-20, 20, 200_000),
        "near_one": 1.0 + rng.uniform(-1e-3, 1e-3, 100_000),
        "near_sqrt2": np.sqrt(2.0) * (1.0 + rng.uniform(-1e-6, 1e-6, 50_000)),
        "subnormal": rng.uniform(1e-3, 1.0, 20_000) * 2.2e-308,
        "positive_normals": np.frombuffer(
            rng.integers(0x0010000000000000, 0x7fefffffffffffff, 200_000, dtype=np.int64).tobytes(),
            dtype=np.float64),
    }
    for name, x in cases.items():
        e = _ulps(bn_log(x), x)
        assert e.max() < 1.0, (name, float(e.max()))


def test_exact_points_and_specials(bn_log):
    x = np.array([1.0, 2.0, 0.5, 2.0 ** -1074, 0.0, -0.0, -1.0, np.inf, -np.inf, np.nan])
    y = bn_log(x)
    assert y[0] == 0.0
    assert y[1] == np.log(2.0) and y[2] == -np.log(2.0)
    assert y[3] == np.log(2.0 ** -1074)
    assert y[4] == -np.inf and y[5] == -np.inf
    assert np.isnan(y[6]) and np.isnan(y[8]) and np.isnan(y[9])
    assert y[7] == np.inf


def test_div_by_launch_constant_is_the_ieee_quotient(hostlib):
    rng = np.random.default_rng(1)
    lib = hostlib
    lib.bn_div_by_host.argtypes = [ctypes.c_void_p, ctypes.c_double, ctypes.c_void_p, ctypes.c_long]
    # sums of squares of scaled components: every magnitude from the
    # smallest normal to the largest finite value, plus exact small integers
    x = np.concatenate([10.0 ** rng.uniform(-307, 308, 60_000),
                        rng.uniform(0.0, 1.0, 20_000) * 64.0,
                        np.arange(0.0, 4097.0),
                        [0.0, np.finfo(np.float64).max, np.finfo(np.float64).tiny]])
    for n in range(1, 130):
        y = np.empty_like(x)
        lib.bn_div_by_host(x.ctypes.data, float(n), y.ctypes.data, x.size)
        ref = x / float(n)
        normal = ref >= np.finfo(np.float64).tiny
        assert np.array_equal(y[normal], ref[normal]), (n, x[normal & (y != ref)][:5])
        assert np.all(np.abs(y - ref)[~normal] <= 2.0 ** -1074), n
    special = np.array([np.inf, np.nan, -0.0])
    y = np.empty_like(special)
    lib.bn_div_by_host(special.ctypes.data, 14.0, y.ctypes.data, special.size)
    assert y[0] == np.inf and np.isnan(y[1]) and y[2] == 0.0
