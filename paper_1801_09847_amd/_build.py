"""Build step of the HIP library: compiles csrc/*.hip for gfx950 into libicp.so
next to this file (in-tree, so the built object travels with the sources)."""
from __future__ import annotations

import concurrent.futures
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libicp.so")
BUILD = os.path.join(HERE, "_build")
SOURCES = ["icp_kernels.hip", "icp_build.hip", "icp_api.hip", "icp_server.hip", "icp_posegraph.hip",
           "icp_ransac.hip", "icp_ceilings.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # exact float32 / float64 expressions: no contraction into FMA
    "-ffp-contract=off",
    # no packed FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument",
]


# Host-side AddressSanitizer + UndefinedBehaviorSanitizer (CPU test runs only:
# the device code is built as usual; every -fsanitize applies to the host
# compilation alone).
SANITIZE_HOST = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                 "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]
SANITIZE_LINK = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                 "-Xarch_host", "-shared-libsan"]
ASAN_RUNTIME = "/opt/rocm/llvm/lib/clang/22/lib/linux/libclang_rt.asan-x86_64.so"


def build(verbose: bool = False, jobs: int | None = None, sanitize: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    cmds, objs = [], []
    extra = SANITIZE_HOST if sanitize else []
    for src in SOURCES:
        obj = os.path.join(BUILD, src.replace(".hip", ".o"))
        cmds.append([HIPCC, *FLAGS, *extra, "-I", os.path.join(HERE, "..", "include"), "-c",
                     os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    # one hipcc per translation unit, a few at a time (each takes several GB
    # of memory at -O3 on the largest sources)
    jobs = jobs or max(1, min(len(cmds), (os.cpu_count() or 2) // 2, 4))

    def run(cmd):
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)

    with concurrent.futures.ThreadPoolExecutor(max_workers=jobs) as ex:
        for f in [ex.submit(run, c) for c in cmds]:
            f.result()
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs,
           *(SANITIZE_LINK if sanitize else ["-Wl,-z,defs"])]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv, sanitize="--sanitize" in sys.argv)
    print(LIB)
