"""Build the HIP library libsilhouette.so in-tree for gfx950 (hipcc).

Every HIP source is compiled with packed-FP32 instruction selection disabled
(-target-feature -packed-fp32-ops).
"""

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libsilhouette.so")
SOURCES = ["main_batched.hip", "main_f32.hip", "main_bf16.hip", "main_fp8.hip", "main_assign.hip",
           "api.hip", "stats.hip", "finalize.hip", "main.hip", "backward.hip", "batched.hip",
           "stream.hip", "mahalanobis.hip", "noalloc.hip", "screen.hip",
           "main_screen.hip"]
ARCH = os.environ.get("SIL_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    return os.path.join(rocm, "bin", "hipcc")


def build(verbose: bool = False, extra=()) -> str:
    objs = []
    os.makedirs(os.path.join(HERE, "_build"), exist_ok=True)
    common = [hipcc(), f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
              "-I", os.path.join(ROOT, "include"), "-Wall", *extra]
    cmds = []
    for src in SOURCES:
        obj = os.path.join(HERE, "_build", src.replace(".hip", ".o"))
        # the fused kernels never see NaN inputs (the statistics pass reports them and the
        # result is replaced by NaN), so min/max need no NaN canonicalisation there
        extra_src = ["-fno-honor-nans"] if src.startswith("main_") else []
        cmds.append(common + extra_src + ["-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    jobs = max(1, min(len(cmds), int(os.environ.get("MAX_JOBS", os.cpu_count() or 1))))
    procs = []
    for cmd in cmds:
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append(subprocess.Popen(cmd))
        if len(procs) >= jobs:
            if procs.pop(0).wait() != 0:
                raise RuntimeError("hipcc failed")
    for pr in procs:
        if pr.wait() != 0:
            raise RuntimeError("hipcc failed")
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", OUT + ".tmp", *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(OUT + ".tmp", OUT)
    return OUT


# Sources whose host code carries the library's own logic (argument checks, workspace layout,
# plans, the stream and batched schedulers); the fused-kernel sources are mostly device code.
ASAN_HOST_SOURCES = [s for s in SOURCES if not s.startswith("main_")]
ASAN_DIR = os.path.join(HERE, "_build_asan")
ASAN_OUT = os.path.join(ASAN_DIR, "libsilhouette_asan.so")


def asan_runtime() -> str:
    """The compiler's shared AddressSanitizer runtime (preloaded into an uninstrumented Python)."""
    out = subprocess.run([hipcc(), "-print-file-name=libclang_rt.asan-x86_64.so"], check=True,
                         capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(out) or not os.path.exists(out):
        raise RuntimeError("no AddressSanitizer runtime next to hipcc")
    return out


def build_asan(verbose: bool = False) -> str:
    """The library with its host code built under AddressSanitizer (device code unchanged): the
    sources in ASAN_HOST_SOURCES are recompiled with the sanitizer on the host side only, and
    linked with the regular objects of the fused-kernel sources (run build() first).  Load it with
    the runtime from asan_runtime() preloaded and SIL_LIBRARY pointing at it."""
    os.makedirs(ASAN_DIR, exist_ok=True)
    common = [hipcc(), f"--offload-arch={ARCH}", "-O1", "-g", "-std=c++17", "-fPIC",
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
              "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer",
              "-I", os.path.join(ROOT, "include")]
    objs, procs = [], []
    for src in SOURCES:
        if src in ASAN_HOST_SOURCES:
            obj = os.path.join(ASAN_DIR, src.replace(".hip", ".o"))
            cmd = common + ["-c", os.path.join(CSRC, src), "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            procs.append(subprocess.Popen(cmd))
        else:
            obj = os.path.join(HERE, "_build", src.replace(".hip", ".o"))
            if not os.path.exists(obj):
                raise RuntimeError(f"{obj} is missing: run build() first")
        objs.append(obj)
    if any(pr.wait() != 0 for pr in procs):
        raise RuntimeError("hipcc failed")
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-Xarch_host", "-fsanitize=address",
           "-o", ASAN_OUT, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return ASAN_OUT


if __name__ == "__main__":
    if "--asan" in sys.argv:
        print(build_asan(verbose="-v" in sys.argv))
    else:
        print(build(verbose="-v" in sys.argv))
