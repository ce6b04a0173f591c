"""The HIP build keeps packed FP32 instructions out of the device code.

build.py passes -target-feature -packed-fp32-ops to hipcc.  The host pass
warns that it does not know the feature; the device pass for gfx950 honours
it.  A two-line float2 kernel shows both: compiled for the device with the
library's flags it has no packed FP32 multiply-add, without them it has one
(so the check can fail)."""
import os
import re
import subprocess

import pytest

from paper_1307_2036_amd import build as B

PROBE = r"""
#include <hip/hip_runtime.h>
__global__ void probe(float2 *a, const float2 *b, float s) {
  int i = threadIdx.x;
  float2 x = a[i], y = b[i];
  x.x = x.x * s + y.x;
  x.y = x.y * s + y.y;
  a[i] = x;
}
"""
PACKED = re.compile(r"\bv_pk_(fma|mul|add)_f32\b")


def device_asm(tmp_path, flags):
    src = tmp_path / "probe.hip"
    src.write_text(PROBE)
    out = tmp_path / "probe.s"
    cmd = [B.HIPCC, f"--offload-arch={B.ARCH}", "-O3", "--cuda-device-only", "-S", "-o", str(out),
           str(src)] + flags
    subprocess.run(cmd, check=True, capture_output=True, timeout=300)
    return out.read_text()


@pytest.mark.skipif(not os.path.exists(B.HIPCC), reason="hipcc not installed")
def test_packed_fp32_feature_is_honoured_on_the_device(tmp_path):
    cmd = B.command("x.so")
    i = cmd.index("-target-feature")
    flags = cmd[i - 1:i + 3]
    assert flags == ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
    assert not PACKED.search(device_asm(tmp_path, flags))
    assert PACKED.search(device_asm(tmp_path, []))
