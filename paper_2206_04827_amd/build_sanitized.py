"""Host sanitizer build of libcylspec: the planner and the C ABI (plan.cpp,
capi.cpp) compiled by g++ with AddressSanitizer and UndefinedBehaviorSanitizer,
linked with the regular build's device objects (_build/*.o of the HIP
sources, not instrumented).  For CPU tests of the host code: argument checks,
the host-only ADI parameter query and the error paths that free partly built
handles.  Device code is never built with a sanitizer here.

Run after build.py (it needs _build/*.o); writes _build/libcylspec_san.so.
"""

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(BUILD, "libcylspec_san.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")

HOST = ["plan.cpp", "capi.cpp"]
DEVICE_OBJS = ["transforms.o", "adi.o", "adjoint.o", "boundary.o", "disk.o", "peaks.o", "scratch.o"]
SAN = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-fno-sanitize-recover=undefined"]


def runtime_preload():
    """The sanitizer runtimes a non-instrumented Python must preload."""
    libs = []
    for name in ("libasan.so", "libubsan.so"):
        path = subprocess.run(["g++", "-print-file-name=" + name], capture_output=True, text=True).stdout.strip()
        libs.append(path)
    return ":".join(libs)


def build(verbose=False):
    objs = []
    for d in DEVICE_OBJS:
        p = os.path.join(BUILD, d)
        if not os.path.exists(p):
            raise RuntimeError("%s is missing: run paper_2206_04827_amd/build.py first" % p)
    srcs = [os.path.join(CSRC, s) for s in HOST]
    deps = srcs + [os.path.join(CSRC, h) for h in ("plan.hpp", "kernels.hpp")] + \
        [os.path.join(ROOT, "include", "cylspec.h")] + [os.path.join(BUILD, d) for d in DEVICE_OBJS]
    if os.path.exists(LIB) and os.path.getmtime(LIB) >= max(os.path.getmtime(p) for p in deps):
        return LIB
    for src in srcs:
        obj = os.path.join(BUILD, os.path.splitext(os.path.basename(src))[0] + "_san.o")
        cmd = ["g++", "-std=c++17", "-O1", "-g", "-fPIC", "-pthread", "-D__HIP_PLATFORM_AMD__",
               "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROCM, "include"), "-c", src, "-o", obj] + SAN
        r = subprocess.run(cmd, capture_output=True, text=True)
        if verbose or r.returncode:
            print(" ".join(cmd))
            print(r.stdout + r.stderr)
        if r.returncode:
            raise RuntimeError("sanitizer compilation of %s failed" % src)
        objs.append(obj)
    cmd = ["g++", "-shared", "-o", LIB + ".tmp"] + objs + [os.path.join(BUILD, d) for d in DEVICE_OBJS] + \
        ["-L", os.path.join(ROCM, "lib"), "-lamdhip64", "-pthread", "-Wl,-rpath," + os.path.join(ROCM, "lib")] + SAN
    r = subprocess.run(cmd, capture_output=True, text=True)
    if verbose or r.returncode:
        print(" ".join(cmd))
        print(r.stdout + r.stderr)
    if r.returncode:
        raise RuntimeError("sanitizer link failed")
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
