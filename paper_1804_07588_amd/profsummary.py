"""Summaries of rocprofv3 runs of bench.py (measurement aid, not part of the
time step).

Reads the rocpd databases of three runs made under one directory:

  <dir>/kt     rocprofv3 --kernel-trace --stats ... -- python3 bench.py ...
  <dir>/fetch  rocprofv3 --pmc FETCH_SIZE ...       -- python3 bench.py ... --calib-copy-mib M
  <dir>/write  rocprofv3 --pmc WRITE_SIZE ...       -- python3 bench.py ... --calib-copy-mib M

and writes a text summary (per-kernel durations, counter bytes per dispatch,
calibrated HBM bytes) plus a JSON traffic record that bench.py reports as
roofline.traffic while the kernel sources still hash to the recorded value.

Calibration: the counter runs start with one plain copy of M MiB
(k_copy_words, 4-byte words, the access width of the method's kernels), which
reads and writes exactly M MiB; each counter is scaled by true bytes over the
bytes it reports for that copy.

Usage: python3 -m paper_1804_07588_amd.profsummary <dir> <out.txt> <traffic.json>
       <calib MiB> "<command of the kt run>" "<command of the counter runs>"
       [<first launch> <launches> ["<workload title>"]]
"""
from __future__ import annotations

import collections
import glob
import hashlib
import json
import os
import re
import sqlite3
import sys

HERE = os.path.dirname(os.path.abspath(__file__))


def source_hash() -> str:
    """SHA-256 over the HIP sources and headers of the lattice-Boltzmann
    kernels and their C ABI (sorted; the U-Net's and the calibration copy's
    sources do not change those kernels and are left out)."""
    h = hashlib.sha256()
    csrc = os.path.join(HERE, "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".h", ".hip", ".cpp")) and f != "calib_copy.hip" and not f.startswith("unet_"):
            with open(os.path.join(csrc, f), "rb") as fh:
                h.update(f.encode() + b"\0" + fh.read())
    return h.hexdigest()


def short(name: str) -> str:
    # names the trace left mangled (the 16-bit storage instantiations): the
    # kernel's identifier and its leading bool template argument, if any
    m = re.match(r"_ZN5fdlbm(\d+)", name)
    if m:
        n = int(m.group(1))
        ident = name[m.end():m.end() + n]
        rest = name[m.end() + n:]
        flag = {"ILb1E": "<true, ...>", "ILb0E": "<false, ...>"}.get(rest[:5], "<...>")
        return ident + flag
    name = re.sub(r"\(.*", "", name)
    name = name.replace("fdlbm::", "").replace("at::native::", "").strip()
    return name[5:] if name.startswith("void ") else name


def _db(d: str) -> str:
    found = sorted(glob.glob(os.path.join(d, "**", "*_results.db"), recursive=True))
    if not found:
        raise FileNotFoundError(f"no rocpd database under {d}")
    return found[0]


def kernel_stats(d: str, skip: int = 0, take: int = 0) -> dict:
    """Per kernel: launch count and durations.  With take > 0 only launches
    skip .. skip + take - 1 of each kernel, in start order (a kernel with
    fewer launches keeps all of them)."""
    c = sqlite3.connect(_db(d)).cursor()
    runs = collections.defaultdict(list)
    for name, s, e in c.execute("select name, start, end from kernels order by start"):
        runs[short(name)].append((e - s) / 1e3)
    agg = {}
    for k, v in runs.items():
        agg[k] = v[skip:skip + take] if take > 0 and len(v) >= skip + take else v
    return {k: dict(calls=len(v), avg_us=sum(v) / len(v), min_us=min(v), max_us=max(v),
                    total_ms=sum(v) / 1e3) for k, v in agg.items()}


def counters(d: str, counter: str) -> dict:
    c = sqlite3.connect(_db(d)).cursor()
    agg = collections.defaultdict(list)
    for name, cn, v in c.execute("select name, counter_name, counter_value from pmc_events"):
        if cn == counter:
            agg[short(name)].append(v)
    return {k: sum(v) / len(v) for k, v in agg.items()}


def main(argv):
    d, out_txt, out_json, calib_mib, cmd_kt, cmd_pmc = argv[1:7]
    skip, take = (int(argv[7]), int(argv[8])) if len(argv) > 8 else (0, 0)
    title = argv[9] if len(argv) > 9 else "128^3 D3Q19, 5 species, FP32"
    calib_bytes = int(calib_mib) * 2**20
    ks = kernel_stats(os.path.join(d, "kt"), skip, take)
    fetch = counters(os.path.join(d, "fetch"), "FETCH_SIZE")   # KiB per dispatch
    write = counters(os.path.join(d, "write"), "WRITE_SIZE")
    cal_f = calib_bytes / (fetch["k_copy_words"] * 1024)
    cal_w = calib_bytes / (write["k_copy_words"] * 1024)
    lines = [f"rocprofv3 summary of the packed-bed step ({title})", "",
             "kernel trace:    " + cmd_kt, "counter passes:  " + cmd_pmc,
             "summary:         python3 -m paper_1804_07588_amd.profsummary " + " ".join(argv[1:5]) +
             " '<kernel trace command>' '<counter command>'" + (f" {skip} {take}" if take else "") +
             (f" '{title}'" if len(argv) > 9 else ""),
             "(rocprofv3 runs from the repository root after cd /tmp && export TMPDIR=/tmp)",
             (f"durations: launches {skip} .. {skip + take - 1} of each kernel, the pass of bench.py in which "
              "the kernels run one after the other (its timed pass overlaps the wall and solid kernels "
              "with the others)" if take else "durations: every launch"), "",
             f"calibration: k_copy_words over {calib_mib} MiB reads and writes {calib_bytes} B;",
             f"  FETCH_SIZE reports {fetch['k_copy_words'] * 1024:.4g} B -> factor {cal_f:.3f}",
             f"  WRITE_SIZE reports {write['k_copy_words'] * 1024:.4g} B -> factor {cal_w:.3f}", "",
             f"{'kernel':34s} {'calls':>6s} {'avg_us':>9s} {'min_us':>9s} {'max_us':>9s} "
             f"{'fetch_MB':>9s} {'write_MB':>9s} {'HBM_GB/s':>9s}"]
    traffic = {}
    for k, s in sorted(ks.items(), key=lambda kv: -kv[1]["total_ms"]):
        f = fetch.get(k)
        w = write.get(k)
        fb = f * 1024 * cal_f if f is not None else None
        wb = w * 1024 * cal_w if w is not None else None
        bw = (fb + wb) / (s["avg_us"] * 1e-6) / 1e9 if fb is not None and wb is not None else None
        lines.append(f"{k:34s} {s['calls']:6d} {s['avg_us']:9.1f} {s['min_us']:9.1f} {s['max_us']:9.1f} "
                     + (f"{fb / 1e6:9.1f} {wb / 1e6:9.1f} {bw:9.0f}" if bw is not None else ""))
        if fb is not None and wb is not None:
            traffic[k] = dict(fetch_bytes=fb, write_bytes=wb, avg_us=s["avg_us"])
    # kernel groups as bench.py times them: both launches (plain and
    # periodic-wrap node lists) of one kernel per step
    groups = collections.defaultdict(lambda: dict(fetch_bytes=0.0, write_bytes=0.0, avg_us=0.0))
    for k, t in traffic.items():
        if k.startswith("k_") and k.split("<")[0] not in ("k_copy_words", "k_observe"):
            g = groups[k.split("<")[0]]
            for f in g:
                g[f] += t[f]
    lines += ["", f"{'kernel group (per step)':34s} {'avg_us':>9s} {'fetch_MB':>9s} {'write_MB':>9s} "
              f"{'HBM_GB/s':>9s}"]
    for k, g in sorted(groups.items(), key=lambda kv: -kv[1]["avg_us"]):
        bw = (g["fetch_bytes"] + g["write_bytes"]) / (g["avg_us"] * 1e-6) / 1e9
        lines.append(f"{k:34s} {g['avg_us']:9.1f} {g['fetch_bytes'] / 1e6:9.1f} "
                     f"{g['write_bytes'] / 1e6:9.1f} {bw:9.0f}")
    traffic = dict(groups)
    lines += ["", "fetch/write MB: calibrated counter bytes per dispatch (HBM side of L2).",
              f"source sha256: {source_hash()}"]
    with open(out_txt, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    with open(out_json, "w") as fh:
        json.dump(dict(source_sha256=source_hash(), calib_mib=int(calib_mib), factors=dict(
            fetch=cal_f, write=cal_w), commands=dict(trace=cmd_kt, counters=cmd_pmc),
            kernels=traffic), fh, indent=1)
    print("\n".join(lines))


if __name__ == "__main__":
    main(sys.argv)
