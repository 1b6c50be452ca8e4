"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

Builds, with g++/gcc and -fsanitize=address,undefined (no recovery), two
host-only programs from the repository's sources:
  * the planner and the C ABI layer (plan.cpp, api.cpp) linked with
    stand-ins for the device launchers (tests/hostcheck/device_stubs.cpp) and
    the HIP runtime, driven by tests/hostcheck/planner_check.cpp;
  * the C oracle (oracle/oracle.c) driven by tests/hostcheck/oracle_check.c.
Each must run to completion with no sanitizer report.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2405_08470_amd", "csrc")
HERE = os.path.join(ROOT, "tests", "hostcheck")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


def _need(tool):
    if shutil.which(tool) is None:
        pytest.skip(f"{tool} not available")


def _run(cmd, **kw):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout[-4000:]}"
    return r.stdout


def test_planner_and_abi_under_sanitizers(tmp_path):
    _need("g++")
    if not os.path.exists(os.path.join(ROCM, "lib", "libamdhip64.so")):
        pytest.skip("HIP runtime library not found")
    exe = str(tmp_path / "planner_check")
    _run(["g++", "-std=c++17", *SAN, "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"), "-I", CSRC,
          "-I", os.path.join(ROCM, "include"),
          os.path.join(CSRC, "plan.cpp"), os.path.join(CSRC, "api.cpp"),
          os.path.join(HERE, "device_stubs.cpp"), os.path.join(HERE, "planner_check.cpp"),
          "-L", os.path.join(ROCM, "lib"), "-lamdhip64", "-Wl,-rpath," + os.path.join(ROCM, "lib"),
          "-pthread", "-o", exe])
    out = _run([exe], env=dict(ENV, HIP_VISIBLE_DEVICES=""), timeout=600)
    assert "planner checks passed" in out


def test_oracle_under_sanitizers(tmp_path):
    _need("gcc")
    exe = str(tmp_path / "oracle_check")
    _run(["gcc", "-std=c11", *SAN, "-fopenmp", os.path.join(ROOT, "oracle", "oracle.c"),
          os.path.join(HERE, "oracle_check.c"), "-o", exe])
    out = _run([exe], env=ENV, timeout=300)
    assert "oracle checks passed" in out
