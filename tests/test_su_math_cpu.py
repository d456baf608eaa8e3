"""The secondary-uncertainty draw's logarithm, cosine of 2 pi u and
exponential (paper_1308_2572_amd/csrc/su_math.h), built for the host and
compared with the C library over the arguments the draw gives: every step is
an IEEE operation, so the host build computes what the device computes.

Bounds: the logarithm within 2.5 ulp, the cosine within 2 ulp wherever
|cos| >= 2^-10 and within 1.5 2^-53 absolutely, the exponential within
1.5 ulp (and exact at its ends: overflow to infinity, underflow to zero,
subnormal results within one unit of the least subnormal).  A draw's loss
then differs from the oracle's by a few parts in 10^15, far inside the
1e-9 of the year loss that the GPU tests allow."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("sumath") / "su_math_driver")
    subprocess.check_call(["/opt/rocm/bin/hipcc", "--offload-arch=gfx950", "-O2", "-std=c++17", "-ffp-contract=off",
                           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_1308_2572_amd", "csrc"),
                           os.path.join(ROOT, "tests", "su_math_driver.hip"), "-o", exe],
                          stderr=subprocess.DEVNULL)
    return exe


def test_errors_against_the_c_library(driver):
    out = subprocess.run([driver, "2000000"], capture_output=True, text=True, check=True).stdout
    err = {k: float(v) for k, v in (line.split() for line in out.strip().splitlines())}
    assert err["log"] <= 2.5, err
    assert err["cos"] <= 2.0, err
    assert err["cos_abs"] <= 1.5, err
    assert err["exp"] <= 1.5, err
    assert err["exp_edges"] <= 1.0, err
