"""The CPU suite under AddressSanitizer and UndefinedBehaviorSanitizer (host
code only; nothing here touches a device).

Run A: the oracle built by gcc with -fsanitize=address,undefined
(oracle/liboracle_san.so, named in FDLBM_ORACLE_LIB) in a process that
preloads gcc's libasan: the whole `-m "not gpu"` suite.

Run B: libfdlbm.so with its host code built by hipcc under ASan and UBSan
(_build/hostsan/libfdlbm.so, named in FDLBM_LIB; device code unchanged) in a
process that preloads clang's ASan runtime: the C-ABI tests, which run the
argument checks, the geometry and stencil-class pre-processing, the slot
order and workspace layout of every workload at every storage precision, and
the U-Net's host set-up.

UBSan is built with -fno-sanitize-recover: the first finding aborts the run.

    python tests/run_sanitized.py [--no-build] [--record FILE]
"""
from __future__ import annotations

import argparse
import glob
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def clang_asan_runtime() -> str:
    libs = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not libs:
        raise SystemExit("clang's ASan runtime was not found under /opt/rocm/llvm")
    return libs[-1]


def run(label: str, env_extra: dict, args: list[str]) -> tuple[int, str]:
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", **env_extra)
    cmd = [sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", *args]
    t0 = time.time()
    p = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True)
    out = p.stdout + p.stderr
    findings = [ln for ln in out.splitlines() if "AddressSanitizer" in ln or "runtime error:" in ln]
    tail = [ln for ln in out.splitlines() if " passed" in ln or " failed" in ln or " error" in ln][-1:]
    summary = (f"{label}: rc={p.returncode} in {time.time() - t0:.0f} s; "
               f"{tail[0].strip('= ') if tail else 'no pytest summary'}; sanitizer findings: {len(findings)}")
    print(summary, flush=True)
    for ln in findings[:20]:
        print("  " + ln, flush=True)
    if p.returncode and not findings:
        print(out[-4000:], flush=True)
    return p.returncode, summary


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--no-build", action="store_true", help="use the sanitized builds already present")
    ap.add_argument("--record", default=None, help="also write the summary lines to this file")
    a = ap.parse_args()
    sys.path.insert(0, ROOT)
    from oracle import oracle
    from paper_1804_07588_amd import build
    if not a.no_build:
        print("building the sanitized oracle and the host-sanitized library", flush=True)
        oracle.build(force=True)
        oracle.build(force=True, sanitize=True)
        build.build_host_sanitized()
    gcc_asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True,
                              text=True, check=True).stdout.strip()
    rc_a, sa = run("A  oracle (gcc ASan+UBSan), CPU suite",
                   {"LD_PRELOAD": gcc_asan, "FDLBM_ORACLE_LIB": oracle.SAN_PATH},
                   ["tests", "-m", "not gpu", "-x"])
    rc_b, sb = run("B  libfdlbm host code (clang ASan+UBSan), C-ABI tests",
                   {"LD_PRELOAD": clang_asan_runtime(), "FDLBM_LIB": build.SAN_LIB},
                   ["tests/test_abi.py", "-m", "not gpu", "-x"])
    if a.record:
        with open(a.record, "w") as f:
            f.write("CPU suite under AddressSanitizer + UndefinedBehaviorSanitizer\n")
            f.write("command: python tests/run_sanitized.py --record " + a.record + "\n")
            f.write(sa + "\n" + sb + "\n")
    return 1 if (rc_a or rc_b) else 0


if __name__ == "__main__":
    sys.exit(main())
