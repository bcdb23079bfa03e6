"""The C-ABI's host code (api.cpp, tune.cpp) built with AddressSanitizer and
UndefinedBehaviorSanitizer for the host only, linked with the ordinary kernel
objects, and driven through every entry point's host-side validation by a C
program (no GPU needed: each call is refused before any HIP call, or touches
no device)."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_1406_0559_amd")
LLVM = "/opt/rocm/lib/llvm/bin"
HIPCC = "/opt/rocm/bin/hipcc"
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]


@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(os.path.join(LLVM, "clang"))),
                    reason="needs the ROCm toolchain")
def test_abi_host_code_under_asan_and_ubsan(tmp_path):
    import sys
    sys.path.insert(0, ROOT)
    from paper_1406_0559_amd import build as B
    kernels = [os.path.join(B.BUILD, n) for n in ("shoot.o", "maps.o", "convolve.o")]
    if not all(os.path.exists(k) for k in kernels):
        B.build()
    objs = []
    for src in ("api.cpp", "tune.cpp"):
        obj = str(tmp_path / (src + ".san.o"))
        cmd = [HIPCC, *B.COMMON, *B.DEVICE, *SAN, f'-DRL_KERNEL_ID="{B.kernel_id()}"', "-g", "-O1",
               "-c", os.path.join(B.CSRC, src), "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr
        objs.append(obj)
    drv = str(tmp_path / "abi_sanitize.o")
    r = subprocess.run([os.path.join(LLVM, "clang"), "-std=c11", "-g", "-O1", "-fsanitize=address,undefined",
                        "-fno-sanitize-recover=all", "-D__HIP_PLATFORM_AMD__", "-I", "/opt/rocm/include",
                        "-I", os.path.join(ROOT, "include"), "-c",
                        os.path.join(ROOT, "tests", "native", "abi_sanitize.c"), "-o", drv],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    exe = str(tmp_path / "abi_sanitize")
    r = subprocess.run([os.path.join(LLVM, "clang++"), "-fsanitize=address,undefined", drv, *objs, *kernels,
                        "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib", "-o", exe],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
    assert "abi sanitizer run ok" in r.stdout
