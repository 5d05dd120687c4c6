"""The C ABI library's host code under AddressSanitizer and
UndefinedBehaviorSanitizer, on the CPU.

tests/sanitize/host_abi_driver.cpp includes capi.cpp (and so nd_plan.h) in
its own translation unit and runs the host geometry, the validation of every
option, the nested-dissection plan for several partitions and panel widths,
and the autotuner cache's reader.  It is built host-only with the sanitizers
(each -fsanitize after -Xarch_host) and linked with the library's GPU objects
as built, which it never launches.  Any sanitizer report or failed check
fails the test.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2103_08513_amd", "csrc")
BUILD = os.path.join(CSRC, "_build")
ROCM = "/opt/rocm"


def _tools():
    hipcc = shutil.which("hipcc") or os.path.join(ROCM, "bin", "hipcc")
    clang = os.path.join(ROCM, "llvm", "bin", "clang++")
    if not (os.path.exists(hipcc) and os.path.exists(clang)):
        pytest.skip("ROCm compilers not found")
    return hipcc, clang


def test_host_abi_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    hipcc, clang = _tools()
    from paper_2103_08513_amd import build as B
    gpu_objs = [os.path.join(BUILD, s + ".o") for s in B.SOURCES if s.endswith(".hip")]
    if not all(os.path.exists(o) for o in gpu_objs):
        pytest.skip("the library's objects are not built (paper_2103_08513_amd.build.build())")
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
    common = ["-x", "hip", "--offload-arch=gfx950", "--offload-host-only", "-std=c++17", "-O1", "-g"]
    objs = []
    for src, name in ((os.path.join(HERE, "sanitize", "host_abi_driver.cpp"), "driver.o"),
                      (os.path.join(CSRC, "nd_plan.cpp"), "nd_plan.o")):
        obj = str(tmp_path / name)
        subprocess.run([hipcc] + common + san + ["-c", src, "-o", obj], check=True, capture_output=True)
        objs.append(obj)
    exe = str(tmp_path / "host_abi")
    subprocess.run([clang, "-fsanitize=address,undefined", "-o", exe] + objs + gpu_objs +
                   ["-L" + os.path.join(ROCM, "lib"), "-lamdhip64", "-Wl,-rpath," + os.path.join(ROCM, "lib")],
                   check=True, capture_output=True)
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=0:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    r = subprocess.run([exe, str(tmp_path / "tune_cache.txt")], capture_output=True, text=True, env=env,
                       timeout=600)
    out = r.stdout + r.stderr
    print(out[-4000:])
    assert r.returncode == 0, out[-4000:]
    assert "AddressSanitizer" not in out and "runtime error" not in out
    assert "host ABI checks: 0 failures" in out
