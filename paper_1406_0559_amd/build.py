"""Builds the raylens HIP library (libraylens.so) for gfx950, in-tree.

hipcc compiles the kernels and the C-ABI layer; nothing is JIT-compiled at run
time. Flags:
  -ffp-contract=off      every a*b+c written in the source stays a multiply and
                         an add unless it is an explicit fma builtin, so the FP64
                         path keeps the sequential evaluation order exactly;
  -packed-fp32-ops off   no packed FP32 instructions are generated.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libraylens.so")
BUILD = os.path.join(HERE, "_build")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
COMMON = ["-O3", "-std=c++17", "-fPIC", "-ffp-contract=off", "-Wall",
          "-I", INCLUDE, "-I", CSRC]
DEVICE = ["-x", "hip", f"--offload-arch={ARCH}",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
SOURCES = [("shoot.hip", True), ("maps.hip", True), ("convolve.hip", True), ("api.cpp", True),
           ("tune.cpp", True)]


def kernel_id():
    """First 12 hex digits of the sha256 over the shoot kernel's sources
    (shoot.hip, then internal.h): tuning caches name the build they are for."""
    import hashlib
    h = hashlib.sha256()
    for name in ("shoot.hip", "internal.h"):
        with open(os.path.join(CSRC, name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:12]


def _compile(src, device, verbose):
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *COMMON, *(DEVICE if device else []), f'-DRL_KERNEL_ID="{kernel_id()}"',
           "-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    noise = "packed-fp32-ops"
    err = "\n".join(l for l in r.stderr.splitlines() if noise not in l)
    if r.returncode != 0:
        raise RuntimeError(f"compiling {src} failed:\n{err}")
    if err.strip() and verbose:
        print(err)
    return obj


PROBE = os.path.join(HERE, "issue_probe")


def build_probe(verbose=False):
    """The FP32 issue-rate microbenchmark (csrc/issue_probe.hip), a standalone
    program that measures the VALU ceiling the shoot kernel is compared with."""
    tmp = PROBE + ".tmp"
    cmd = [HIPCC, "-O3", "-std=c++17", *DEVICE[2:], f"--offload-arch={ARCH}",
           os.path.join(CSRC, "issue_probe.hip"), "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compiling issue_probe.hip failed:\n{r.stderr}")
    os.replace(tmp, PROBE)
    return PROBE


def build(verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(lambda s: _compile(s[0], s[1], verbose), SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", f"--offload-arch={ARCH}", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    build_probe(verbose)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-q" not in sys.argv))
