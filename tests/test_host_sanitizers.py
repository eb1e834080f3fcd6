"""Host code under AddressSanitizer (with LeakSanitizer) and UndefinedBehaviorSanitizer, on the CPU.

Two drivers under tests/sanitize/ are compiled with the sanitizers and run:
  - oracle_main.c calls every exported function of the FP64 oracle (oracle/oracle.c), with its OpenMP loops, on
    small lattices with odd and even Ns;
  - sitetab_main.cpp builds every site-local s-operator table of the library (csrc/sitetab.cpp, host code) for
    every supported Ns.
A sanitizer report (out-of-bounds access, use after free, leak, undefined arithmetic) fails the test; so does a
failed check inside a driver.  GPU code is not instrumented: the library's device kernels are covered by the
parity tests and by the bounds reasoning of each launcher, not by a sanitizer."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1",
           OMP_NUM_THREADS="4")
REPORTS = ("ERROR: AddressSanitizer", "ERROR: LeakSanitizer", "runtime error:")

# sanitizer flags of the host compilers (gcc for the oracle; the HIP compiler's host pass for the library source)
GCC_SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"]
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=undefined"]


def _run(exe):
    r = subprocess.run([exe], env=ENV, capture_output=True, text=True, timeout=300)
    out = r.stdout + r.stderr
    print(out[-3000:])
    assert r.returncode == 0, out[-3000:]
    assert not any(k in out for k in REPORTS), out[-3000:]
    return out


def test_oracle_under_sanitizers(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not found")
    exe = str(tmp_path / "oracle_san")
    cmd = ["gcc", "-std=c11", "-O1", "-g", "-fopenmp", "-fno-omit-frame-pointer"] + GCC_SAN + [
        "-o", exe, os.path.join(SAN, "oracle_main.c"), os.path.join(ROOT, "oracle", "oracle.c"), "-lm"]
    subprocess.run(cmd, check=True, timeout=300)
    assert "0 failure(s)" in _run(exe)


def test_site_tables_under_sanitizers(tmp_path):
    hip = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    if not os.path.exists(hip):
        pytest.skip("hipcc not found")
    exe = str(tmp_path / "sitetab_san")
    csrc = os.path.join(ROOT, "paper_1710_09621_amd", "csrc")
    cmd = [hip, "-x", "hip", "--offload-arch=gfx950", "--cuda-host-only", "-std=c++17", "-O1", "-g",
           "-fno-omit-frame-pointer"] + HOST_SAN + [
        "-I", csrc, "-I", os.path.join(ROOT, "include"), "-o", exe, os.path.join(SAN, "sitetab_main.cpp"),
        os.path.join(csrc, "sitetab.cpp")]
    subprocess.run(cmd, check=True, timeout=300)
    assert "0 failure(s)" in _run(exe)
