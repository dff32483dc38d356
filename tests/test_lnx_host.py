"""The solver's logarithm (argument reduction and the atanh series), built for
the host from the same header the kernels include, against the C library's
log: within 3 ulp over the whole double range, exact at powers of two and at
1, and the C library's values at 0, negative, infinite and NaN arguments."""
import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


@pytest.fixture(scope="module")
def lnx(tmp_path_factory):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not found")
    d = tmp_path_factory.mktemp("lnx")
    exe = str(d / "lnx_check")
    subprocess.run([HIPCC, "-x", "hip", "--cuda-host-only", "-O2", "-ffp-contract=off",
                    os.path.join(HERE, "lnx_check.cpp"), "-o", exe],
                   check=True, capture_output=True)

    def run(x):
        x = np.ascontiguousarray(x, dtype=np.float64)
        fi, fo = str(d / "in.bin"), str(d / "out.bin")
        x.tofile(fi)
        subprocess.run([exe, fi, fo], check=True)
        return np.fromfile(fo, dtype=np.float64)
    return run


def _ulps(a, b):
    return np.abs(a - b) / np.spacing(np.abs(b))


def test_lnx_within_3_ulp(lnx):
    rng = np.random.default_rng(7)
    parts = [
        np.ldexp(rng.uniform(0.5, 1.0, 200_000), rng.integers(-1074, 1025, 200_000)),
        rng.uniform(0.25, 4.0, 200_000),                  # densities and their ratios
        1.0 + rng.uniform(-1e-6, 1e-6, 100_000),          # near the zero of ln
        rng.uniform(0.7071, 1.4143, 100_000),             # the reduced range itself
    ]
    x = np.concatenate(parts)
    x = x[np.isfinite(x) & (x > 0) & (x != 1.0)]
    got, ref = lnx(x), np.log(x)
    err = _ulps(got, ref)
    assert err.max() <= 3.0, (x[err.argmax()], err.max())


def test_lnx_exact_points_and_specials(lnx):
    e = np.arange(-1074, 1024)
    x = np.ldexp(1.0, e)
    np.testing.assert_array_equal(lnx(x), np.log(x))       # powers of two
    sp = np.array([1.0, 0.0, -0.0, -1.0, np.inf, -np.inf, np.nan])
    with np.errstate(divide="ignore", invalid="ignore"):
        want = np.log(sp)
    np.testing.assert_array_equal(lnx(sp), want)
