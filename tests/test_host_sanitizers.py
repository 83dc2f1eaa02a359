"""The library's host C++ under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

The host sources are compiled with g++ -fsanitize=address,undefined and linked, with the
kernel objects of the regular build, into a driver (tests/sanitize/host_driver.cpp) that
exercises meshes, the three space families at every order, quadrature-data sizes and
the refusal paths without touching a GPU.  Any sanitizer report fails the test.
"""
import glob
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_1911_09220_amd")
BUILD = os.path.join(PKG, "_build")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def test_host_code_under_asan_and_ubsan(tmp_path):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    hip_objs = sorted(glob.glob(os.path.join(BUILD, "*.hip.o")))
    if not hip_objs:
        pytest.skip("kernel objects not built (run __graft_entry__.build())")
    flags = ["-O1", "-g", "-std=c++17", "-fPIC", "-fno-omit-frame-pointer",
             "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
             "-D__HIP_PLATFORM_AMD__", f"-I{ROCM}/include", f"-I{ROOT}/include",
             f"-I{PKG}/csrc"]
    objs = []
    srcs = sorted(glob.glob(os.path.join(PKG, "csrc", "*.cpp"))) + \
        [os.path.join(ROOT, "tests", "sanitize", "host_driver.cpp")]
    for src in srcs:
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        subprocess.run(["g++", *flags, "-c", src, "-o", obj], check=True, capture_output=True)
        objs.append(obj)
    exe = str(tmp_path / "host_driver")
    subprocess.run(["g++", "-fsanitize=address,undefined", "-o", exe, *objs, *hip_objs,
                    f"-L{ROCM}/lib", "-lamdhip64", f"-Wl,-rpath,{ROCM}/lib"],
                   check=True, capture_output=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    res = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    out = res.stdout + res.stderr
    assert res.returncode == 0, out[-4000:]
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert "host driver ok" in out
