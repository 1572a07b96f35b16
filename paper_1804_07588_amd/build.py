"""Build the HIP library libfdlbm.so in-tree for gfx950 with hipcc, and the
counter-calibration copy kernel libfdlbm_calib.so (measurement aid only)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libfdlbm.so")
CALIB_LIB = os.path.join(HERE, "libfdlbm_calib.so")
CALIB_SRC = os.path.join(CSRC, "calib_copy.hip")
SOURCES = [os.path.join(CSRC, f) for f in
           ("kern_f32_d3q19.hip", "kern_f64_d3q19.hip", "kern_f32_d2q9.hip", "kern_f64_d2q9.hip",
            "kern_f16_d3q19.hip", "kern_bf16_d3q19.hip", "kern_f16_d2q9.hip", "kern_bf16_d2q9.hip",
            "unet_kernels.hip", "fdlbm_api.cpp", "unet_api.cpp")]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-result", "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def build(verbose: bool = False, jobs: int | None = None) -> str:
    """Compile every source for gfx950 (in parallel) and link libfdlbm.so."""
    calib = subprocess.Popen([HIPCC, *FLAGS, "-shared", "-o", CALIB_LIB + ".tmp", CALIB_SRC],
                             stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True)
    objs, procs = [], []
    jobs = jobs or min(len(SOURCES), max(1, min(os.cpu_count() or 1, 16)))
    pending = list(SOURCES)
    while pending or procs:
        while pending and len(procs) < jobs:
            src = pending.pop(0)
            obj = os.path.join(CSRC, os.path.basename(src) + ".o")
            cmd = [HIPCC, *FLAGS, "-c", src, "-o", obj]
            if src.endswith(".cpp"):
                cmd[1:1] = ["-x", "hip"]
            if verbose:
                print(" ".join(cmd), flush=True)
            procs.append((src, obj, subprocess.Popen(cmd, stdout=subprocess.PIPE,
                                                     stderr=subprocess.PIPE, text=True)))
        src, obj, pr = procs.pop(0)
        _, err = pr.communicate()
        if pr.returncode != 0:
            sys.stderr.write(err)
            for _, _, other in procs:
                other.kill()
            raise RuntimeError(f"hipcc failed on {src}")
        objs.append(obj)
    tmp = LIB + ".tmp"
    subprocess.run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs],
                   check=True)
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
    _, err = calib.communicate()
    if calib.returncode != 0:
        sys.stderr.write(err)
        raise RuntimeError(f"hipcc failed on {CALIB_SRC}")
    os.replace(CALIB_LIB + ".tmp", CALIB_LIB)
    return LIB


# host code under AddressSanitizer and UndefinedBehaviorSanitizer (device code
# unchanged): the C ABI's argument checks, geometry and stencil-class
# pre-processing and layout run instrumented on the CPU; load it by naming it
# in FDLBM_LIB in a process that preloads clang's ASan runtime
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer",
            "-Xarch_host", "-g"]
SAN_LIB = os.path.join(ROOT, "_build", "hostsan", "libfdlbm.so")


def build_host_sanitized(jobs: int | None = None) -> str:
    """libfdlbm.so with sanitized host code, out of tree (_build/hostsan)."""
    out_dir = os.path.dirname(SAN_LIB)
    os.makedirs(out_dir, exist_ok=True)
    jobs = jobs or min(len(SOURCES), max(1, min(os.cpu_count() or 1, 16)))
    objs, procs, pending = [], [], list(SOURCES)
    while pending or procs:
        while pending and len(procs) < jobs:
            src = pending.pop(0)
            obj = os.path.join(out_dir, os.path.basename(src) + ".o")
            cmd = [HIPCC, *FLAGS, *HOST_SAN, "-c", src, "-o", obj]
            if src.endswith(".cpp"):
                cmd[1:1] = ["-x", "hip"]
            procs.append((src, obj, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE,
                                                     text=True)))
        src, obj, pr = procs.pop(0)
        _, err = pr.communicate()
        if pr.returncode != 0:
            sys.stderr.write(err)
            for _, _, other in procs:
                other.kill()
            raise RuntimeError(f"hipcc failed on {src}")
        objs.append(obj)
    subprocess.run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *HOST_SAN, "-shared-libsan", "-o",
                    SAN_LIB + ".tmp", *objs], check=True)
    os.replace(SAN_LIB + ".tmp", SAN_LIB)
    for o in objs:
        os.remove(o)
    return SAN_LIB


if __name__ == "__main__":
    print(build(verbose=True))
