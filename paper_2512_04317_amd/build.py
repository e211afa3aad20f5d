"""Build libmxfft.so (HIP for gfx950) in-tree with hipcc.

build() compiles every source and links the library.  build(incremental=True)
recompiles only sources newer than their objects (objects in _build/)."""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OBJ = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libmxfft.so")

SOURCES = ["mxfft_kernels.hip", "mxfft_fast.hip", "fast_e4m3.hip", "fast_e5m2.hip", "fast_fp32.hip",
           "fast_e4m3_128.hip", "fast_e5m2_128.hip", "fast_e4m3_256.hip", "fast_e5m2_256.hip",
           "fast_e4m3_1024.hip", "fast_e5m2_1024.hip", "fast_16_128.hip", "fast_16_256.hip", "fast_16_1024.hip",
           "fast_e2m3.hip", "fast_e3m2.hip", "fast_e2m3_128.hip", "fast_e3m2_128.hip", "fast_e2m3_256.hip",
           "fast_e3m2_256.hip", "fast_e2m3_1024.hip", "fast_e3m2_1024.hip",
           "fast_fp16.hip", "fast_bf16.hip", "mxfft_host.cpp", "mxfft_tune.cpp", "mxfft_batch.cpp",
           "mxfft_serve.cpp", "mxfft_static.hip", "fast_wide_256.hip", "fast_wide_512.hip", "fast_wide_1024.hip"]
HEADERS = ["mx_device.hpp", "mxfft_internal.hpp", "mxfft_fast.hpp"]

HIPCC_FLAGS = [
    "-O3", "--offload-arch=gfx950", "-std=c++17", "-fPIC",
    # packed FP32 instructions stay off (hipcc's host pass warns; harmless)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # FP32 subnormals are kept: the MX decode and ldexp rely on IEEE behaviour
    "-fno-gpu-flush-denormals-to-zero",
    "-Wall", "-Wno-unused-command-line-argument",
]


def hipcc():
    c = os.environ.get("HIPCC")
    if c:
        return c
    return "/opt/rocm/bin/hipcc" if os.path.exists("/opt/rocm/bin/hipcc") else "hipcc"


def _compile(src, verbose):
    obj = os.path.join(OBJ, src + ".o")
    cmd = [hipcc()] + HIPCC_FLAGS + ["-I" + os.path.join(ROOT, "include"), "-I" + CSRC, "-c",
                                     os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd, cwd=CSRC)
    return obj


def build(verbose=False, incremental=False):
    os.makedirs(OBJ, exist_ok=True)
    newest_hdr = max(os.path.getmtime(os.path.join(p, h)) for p, h in
                     [(CSRC, h) for h in HEADERS] + [(os.path.join(ROOT, "include"), "mxfft.h")])
    todo = []
    for s in SOURCES:
        obj = os.path.join(OBJ, s + ".o")
        if (not incremental or not os.path.exists(obj)
                or os.path.getmtime(obj) < max(os.path.getmtime(os.path.join(CSRC, s)), newest_hdr)):
            todo.append(s)
    with ThreadPoolExecutor(min(len(SOURCES), os.cpu_count() or 4, 16)) as ex:
        list(ex.map(lambda s: _compile(s, verbose), todo))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc(), "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp] + \
          [os.path.join(OBJ, s + ".o") for s in SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd, cwd=CSRC)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True, incremental="--incremental" in sys.argv))
    sys.exit(0)
