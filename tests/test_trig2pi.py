"""Accuracy of the FP64 step direction sin(2 pi u), cos(2 pi u) used by the FP64 walk kernels
(wos_device.hpp, sincos2pi), checked on the host against long-double sin/cos over 2 * 10^6
uniforms and every quarter-turn boundary."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "native", "trig2pi_check.hip")


def _hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    return None


def test_sincos2pi_is_within_a_few_ulps(tmp_path):
    hipcc = _hipcc()
    if hipcc is None:
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "trig2pi_check")
    subprocess.run([hipcc, "-O2", "-std=c++17", "--offload-arch=gfx950", "-x", "hip", SRC, "-o", exe],
                   check=True, capture_output=True, timeout=300)
    out = subprocess.run([exe, "2000000"], check=True, capture_output=True, text=True, timeout=120).stdout.split()
    es, ec, us, uc = map(float, out)
    print(f"sincos2pi: max abs error sin {es:.2e}, cos {ec:.2e}; max ulps {us:.2f}, {uc:.2f}")
    assert es <= 2.0 ** -52 and ec <= 2.0 ** -52
    assert us <= 4.0 and uc <= 4.0
