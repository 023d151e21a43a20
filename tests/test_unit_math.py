"""The FP64 logarithm and sine/cosine of pi x the device uses for its
uniforms (csrc/unit_math.hpp), checked on the host over every possible input
u = (2k+1) 2^-24, k < 2^23, against long-double references: within 2 ulp; and
e^{-y} - 1 of the KD scheme's diffusive phases on a dense sample of [0, 45].
The functions are IEEE operations only (no library calls but frexp and rint,
both exact), so the host computes the device's values bit for bit."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2004_04071_amd", "csrc")


def test_log_and_sincospi_of_every_uniform_within_two_ulp(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "unit_math_check")
    subprocess.run([hipcc, "-x", "hip", "--offload-arch=gfx950", "-O2", "-ffp-contract=off",
                    "-I", CSRC, os.path.join(ROOT, "tests", "unit_math_check.cpp"), "-o", exe],
                   check=True, capture_output=True)
    out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout.split()
    max_log, max_sin, max_cos, max_log_abs, max_em = (float(x) for x in out)
    print("max ulp: log %.3f sin %.3f cos %.3f expm1(-y) %.3f" % (max_log, max_sin, max_cos,
                                                                 max_em))
    assert max_log <= 2.0 and max_sin <= 2.0 and max_cos <= 2.0 and max_em <= 2.0
    assert max_log_abs <= 4e-15
