"""AddressSanitizer and UBSan builds of the host code, run on the CPU.

* The FP64 oracle (oracle/ell_oracle.c) with a driver that calls every
  exported function on small grids (tests/sanitize/oracle_driver.c).
* The host half of the C ABI (descriptor validation, schedules, tuning keys,
  invalid arguments, creation failing cleanly without a GPU) with
  tests/sanitize/abi_driver.c.  The library is compiled with the sanitizers on
  the host side only (its device code is built unoptimised and never runs
  here); the driver and the link step use clang with the same sanitizers.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")
ROCM = "/opt/rocm"
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", OMP_NUM_THREADS="2")


def run(cmd, **kw):
    return subprocess.run(cmd, capture_output=True, text=True, **kw)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not installed")
def test_oracle_under_asan_ubsan(tmp_path):
    exe = tmp_path / "oracle_driver"
    r = run(["gcc", "-O1", "-g", "-fopenmp", "-std=c99", "-ffp-contract=off",
             "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer",
             os.path.join(SAN, "oracle_driver.c"), "-lm", "-o", str(exe)], timeout=300)
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(ENV, ASAN_OPTIONS="detect_leaks=1")
    r = run([str(exe)], timeout=300, env=env)
    assert r.returncode == 0 and "oracle-ok" in r.stdout, (r.stdout[-2000:], r.stderr[-4000:])


@pytest.mark.skipif(not os.path.exists(os.path.join(ROCM, "bin", "hipcc")), reason="ROCm not installed")
def test_c_abi_host_side_under_asan_ubsan(tmp_path):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present: grid creation would succeed there")
    obj = tmp_path / "ell.o"
    san_host = []
    for flag in ("-fsanitize=address", "-fsanitize=undefined", "-fno-omit-frame-pointer"):
        san_host += ["-Xarch_host", flag]
    r = run([os.path.join(ROCM, "bin", "hipcc"), "-x", "hip", "--offload-arch=gfx950", "-c",
             os.path.join(ROOT, "paper_1307_2036_amd", "csrc", "ell.hip"),
             "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_1307_2036_amd", "csrc"),
             "-O1", "-g", "-fPIC", "-Xarch_device", "-O0", "-Xarch_device", "-g0"] + san_host +
            ["-o", str(obj)], timeout=900)
    assert r.returncode == 0, r.stderr[-3000:]
    clang = os.path.join(ROCM, "llvm", "bin", "clang")
    drv = tmp_path / "abi_driver.o"
    r = run([clang, "-c", "-O1", "-g", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"),
             "-I", os.path.join(ROCM, "include"), "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
             os.path.join(SAN, "abi_driver.c"), "-o", str(drv)], timeout=300)
    assert r.returncode == 0, r.stderr[-3000:]
    exe = tmp_path / "abi_driver"
    r = run([clang + "++", "-fsanitize=address,undefined", str(drv), str(obj), "-L", os.path.join(ROCM, "lib"),
             "-lamdhip64", "-Wl,-rpath," + os.path.join(ROCM, "lib"), "-o", str(exe)], timeout=300)
    assert r.returncode == 0, r.stderr[-3000:]
    r = run([str(exe)], timeout=300, env=ENV)
    assert r.returncode == 0 and "abi-ok" in r.stdout, (r.stdout[-2000:], r.stderr[-4000:])
