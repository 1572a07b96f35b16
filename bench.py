"""Throughput of the coupled FD-LBM step on one MI355X.

Workload (default): the packed-bed configuration -- 128^3 D3Q19 lattice,
random overlapping spheres of radius 6 (SplitMix64 seed 12345) at bed
porosity 0.6, five gas species (CO, H2O, CO2, H2, N2) with water-gas-shift
chemistry on the sphere surfaces, FD heat conduction in the solid, body-force
flow with inlet/outlet planes, FP32 storage and arithmetic.  A "step" is one
full time step of the method (wall BC, streaming, moments, collision with all
corrections, solid FD, inlet/outlet).  Inputs are resident in device memory
before the timed region.

Prints ONE JSON line: MLUPS x species (gas nodes x species x steps / s / 1e6),
the fraction of the HBM roofline of the dominant kernel measured with HIP
events on the library's stream over the timed region, and the FP64 CPU oracle
timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import ctypes as ct
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, 8 TB/s
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_bed128_f32.json")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--n", type=int, default=128, help="bed edge length (nodes)")
    ap.add_argument("--precision", default="f32", choices=["f32", "f64", "f16", "bf16"],
                    help="f16/bf16: 16-bit population storage with FP32 arithmetic")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-steady-state", action="store_true",
                    help="skip the reduced learned warm-start check of the throughput run")
    ap.add_argument("--cpu-n", type=int, default=128,
                    help="edge length of the bed the CPU oracle is timed on (bounded sample)")
    ap.add_argument("--cpu-steps", type=int, default=1)
    ap.add_argument("--steady", action="store_true",
                    help="instead of the throughput run: steps and seconds from a cold start to "
                         "a steady-state residual of --tol (checked every 100 steps)")
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--log", default=None,
                    help="JSON-lines run log (observables and residual at every check of --steady)")
    ap.add_argument("--stage-tol", type=float, default=1e-5,
                    help="16-bit storage: residual at which the FP32 stage takes over")
    ap.add_argument("--max-steps", type=int, default=400000)
    ap.add_argument("--batch", action="store_true",
                    help="instead of the throughput run: a batch of packed beds of uneven size "
                         "run together to the steady-state residual --tol")
    ap.add_argument("--batch-samples", type=int, default=64)
    ap.add_argument("--batch-min", type=int, default=48)
    ap.add_argument("--batch-max", type=int, default=96)
    ap.add_argument("--batch-seed", type=int, default=2024)
    ap.add_argument("--surrogate", action="store_true",
                    help="instead of the throughput run: learned warm start -- steady states of "
                         "64^3 beds from a batched run, U-Net training on the GPU, then held-out "
                         "beds to --tol from the prediction versus from a cold start")
    ap.add_argument("--unet-bench", action="store_true",
                    help="instead of the throughput run: U-Net training iterations on synthetic "
                         "64^3 inputs (convolution throughput against the bf16 MFMA peak)")
    ap.add_argument("--sur-n", type=int, default=64, help="bed edge of the learned warm start")
    ap.add_argument("--sur-train", type=int, default=48)
    ap.add_argument("--sur-test", type=int, default=16)
    ap.add_argument("--sur-epochs", type=int, default=60)
    ap.add_argument("--sur-batch", type=int, default=4)
    ap.add_argument("--sur-lr", type=float, default=1e-3)
    ap.add_argument("--sur-seed", type=int, default=77)
    ap.add_argument("--sur-no-augment", action="store_true",
                    help="train without the bed symmetries (y/z shifts and reflections)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="run one plain device copy of this size first (counter calibration)")
    return ap.parse_args()


def alg_bytes(n_gas, n_links, n_solid, ns, Q, b):
    """Algorithmic HBM bytes of one step and their split over the kernel
    groups.  Per step every gas population is read once and written once,
    every wall link's population of each species is read and written once,
    and the solid temperature is read and written once.  The split gives
    each byte to exactly one kernel: the moments pass reads the populations
    (through the streaming taps), the collision writes them, the wall reads
    and writes the link populations, the solid its temperature.  The
    streamed copy and the moment records passed from one gas kernel to the
    other are overheads of the two-pass step, not algorithmic bytes.
    Returns (bytes per step, {kernel group: bytes per launch})."""
    per_kernel = {
        "k_moments": n_gas * Q * ns * b,       # pre-collision pops in (through the taps)
        "k_collide": n_gas * Q * ns * b,       # post-collision pops out
        "k_wall": n_links * 2 * ns * b,        # link pops in, emitted pops out
        "k_solid": n_solid * 2 * b,            # solid temperature in and out
    }
    return sum(per_kernel.values()), per_kernel


def bed(n):
    from paper_1804_07588_amd import workloads as W
    mask, nsph = W.sphere_pack_mask(n, radius=6.0, porosity=0.6, seed=12345, buffer=8)
    cfg = W.packed_bed(mask=mask)
    return cfg, W.uniform_init(cfg), nsph


def cpu_baseline(n, steps):
    """The FP64 oracle on a bed of edge n built the same way (same sphere
    radius, porosity, chemistry and flow): setup excluded, timed full time
    steps, once on every host thread the process may use (OpenMP over nodes;
    OMP_NUM_THREADS if set, else the CPU count) over 3 * steps steps, once
    on one thread over `steps` steps (the oracle's results do not depend on
    the thread count)."""
    from oracle import oracle
    oracle.build(force=not os.path.exists(oracle.LIB_PATH))
    cfg, init, _ = bed(n)
    ns = len(cfg["species"]["M"])
    threads = int(os.environ.get("OMP_NUM_THREADS", 0) or os.cpu_count() or 1)
    res = {}
    for nt, k in ((threads, 3 * steps), (1, steps)):
        used = oracle.set_threads(nt)
        sim = oracle.OracleSim(cfg, init)
        t0 = time.perf_counter()
        sim.step(k)
        dt = time.perf_counter() - t0
        o = sim.observe()
        sim.close()
        res[nt] = (o["n_gas"] * ns * k / dt / 1e6, used, k, dt, o["n_gas"])
    v, used, k, dt, ng = res[threads]
    v1, _, k1, dt1, _ = res[1]
    return dict(value=round(v, 4), unit="MLUPS*species", cores=used, kind="oracle",
                value_1thread=round(v1, 4),
                sample=f"{k} full step(s) of a {n}^3 bed of the same construction ({ng} gas nodes), "
                       f"FP64, {used} OpenMP threads, {dt:.1f} s; one thread: {k1} step(s), {dt1:.1f} s")


def calib_copy(mib):
    """One plain device copy of mib MiB (4-byte words): reads and writes
    exactly that many bytes; its byte counters calibrate the others."""
    import torch
    from paper_1804_07588_amd import build as hb
    L = ct.CDLL(hb.CALIB_LIB)
    L.fdlbm_calib_copy.argtypes = [ct.c_void_p, ct.c_void_p, ct.c_size_t, ct.c_void_p]
    words = mib * 262144
    src = torch.ones(words, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    rc = L.fdlbm_calib_copy(ct.c_void_p(src.data_ptr()), ct.c_void_p(dst.data_ptr()), words,
                            ct.c_void_p(torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    if rc != 0:
        raise RuntimeError(f"calibration copy failed ({rc})")
    del src, dst


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter record,
    or None if there is none or the library sources changed since."""
    from paper_1804_07588_amd import profsummary
    try:
        with open(TRAFFIC_FILE) as fh:
            rec = json.load(fh)
    except OSError:
        return None
    if rec.get("source_sha256") != profsummary.source_hash() or kernel not in rec.get("kernels", {}):
        return None
    k = rec["kernels"][kernel]
    return k["fetch_bytes"] + k["write_bytes"]


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the solver runs on one GPU; sharding a domain over several "
                                   "GPUs is not implemented", "n_gpus": args.gpus}))
        sys.exit(2)
    import numpy as np
    import torch
    from paper_1804_07588_amd import fdlbm

    torch.cuda.set_device(0)
    if args.batch:
        batch_run(args)
        return
    if args.surrogate:
        surrogate_run(args)
        return
    if args.unet_bench:
        unet_bench(args)
        return
    if args.calib_copy_mib:
        calib_copy(args.calib_copy_mib)
    cfg, init, nsph = bed(args.n)
    prec = {"f32": fdlbm.F32, "f64": fdlbm.F64, "f16": fdlbm.F16, "bf16": fdlbm.BF16}[args.precision]
    b = {"f32": 4, "f64": 8, "f16": 2, "bf16": 2}[args.precision]   # bytes per stored population
    sim = fdlbm.Sim(cfg, precision=prec, init=init)
    n_gas, n_wall, n_solid = sim.counts()
    kind = sim.field(fdlbm.FIELD_KIND).astype(np.int64)
    ns, Q = len(cfg["species"]["M"]), 19
    # wall links = incoming links of all wall nodes (each carries one population per species)
    n_links = int(_count_wall_links(kind, cfg))
    B_alg, kernel_alg_bytes = alg_bytes(n_gas, n_links, n_solid, ns, Q, b)

    if args.steady:
        steady(args, sim, cfg, n_gas, ns, init)
        return
    sim.step(args.warmup)
    sim.sync()
    # pass 1, for the roofline: the kernels one after the other, each timed
    # with HIP events on the stream it runs on
    sim.set_overlap(False)
    sim.set_profiling(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(args.steps)
    sim.sync()
    torch.cuda.synchronize()
    dt_serial = time.perf_counter() - t0
    times, launches = sim.kernel_times()
    sim.set_profiling(False)
    # pass 2, the throughput: the wall and solid kernels beside the others
    sim.set_overlap(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(args.steps)
    sim.sync()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    obs = sim.observe()
    if obs["bad"]:
        print(json.dumps({"error": "non-finite or negative state after the timed run"}))
        sys.exit(3)

    ms_per_step = dt * 1e3 / args.steps
    mlups_species = n_gas * ns * args.steps / dt / 1e6
    dom = max(times, key=times.get)   # dominant kernel group by event time
    achieved = kernel_alg_bytes[dom] / (times[dom] * 1e-3) / 1e9
    traffic = measured_traffic(dom) if (args.n == 128 and prec == fdlbm.F32) else None
    out = {
        "metric": "MLUPS*species (gas nodes x species x steps / s / 1e6) and % of HBM peak",
        "value": round(mlups_species, 2),
        "unit": "MLUPS*species",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == fdlbm.F64 else "f32",
        "population_storage": args.precision,
        "data": "synthetic",
        "config": {
            "workload": f"packed bed {args.n}^3 D3Q19, spheres r=6 porosity 0.6 (seed 12345), "
                        f"5 species WGS, FD solid, inlet/outlet, body force",
            "nodes": int(cfg["nx"] * cfg["ny"] * cfg["nz"]), "gas_nodes": n_gas,
            "wall_nodes": n_wall, "solid_nodes": n_solid, "wall_links": n_links,
            "spheres": nsph, "species": ns,
        },
        "step_alg_bytes": B_alg,
        "step_effective_GBs": round(B_alg * args.steps / dt / 1e9, 1),
        "step_hbm_frac": round(B_alg * args.steps / dt / 1e9 / HBM_PEAK_GBS, 4),
        "ms_per_step_serial": round(dt_serial * 1e3 / args.steps, 5),
        "kernel_ms": {k: round(v, 5) for k, v in times.items()},
        "kernel_ms_note": "per-kernel HIP-event times from a pass of the same length with the kernels "
                          "run one after the other; the timed pass (value, ms_per_step) runs the wall "
                          "and solid kernels on a second stream beside the moments and collision",
        "timed_launches": launches,
        "roofline": {
            "bound": "hbm",
            "kernel": dom,
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "alg_bytes": kernel_alg_bytes[dom],
            "traffic": traffic,
        },
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.cpu_n, args.cpu_steps)
    if not args.no_steady_state:
        sim.close()
        out["steady_state"] = steady_state_check(args)
    print(json.dumps(out), flush=True)


def steady_state_check(args):
    """The time-to-steady-state half of the metric, measured in this run with
    fewer beds: the learned warm-start pipeline (surrogate_pipeline) on 24
    beds of 64^3 (20 to train on, 4 held out) to a residual of 1e-6, about
    80 s; the full configuration (64 beds: 48 and 16) is `bench.py
    --surrogate`.  A failure is reported in the record, not raised."""
    sub = argparse.Namespace(**vars(args))
    sub.sur_n, sub.sur_train, sub.sur_test, sub.sur_epochs = 64, 20, 4, 150
    sub.sur_batch, sub.sur_lr, sub.sur_seed, sub.sur_no_augment = 4, 1e-3, 77, False
    sub.tol, sub.max_steps = 1e-6, 60000
    t0 = time.perf_counter()
    try:
        r = surrogate_pipeline(sub)
    except Exception as e:   # the throughput line is still printed
        return {"error": f"{type(e).__name__}: {e}"}
    return {
        "metric": "time to a 1e-6 steady-state residual of held-out beds: cold start / learned warm start",
        "value": r["value"], "unit": r["unit"],
        "cold": r["cold"], "warm": r["warm"], "steps_ratio": r["steps_ratio"],
        "warm_f16_then_f32": r["warm_f16_then_f32"],
        "training": {k: r["training"][k] for k in ("samples", "epochs", "seconds", "loss_first", "loss_last")},
        "data_generation": r["data_generation"],
        "config": dict(r["config"], note="24 beds measured in this run; the full configuration "
                                         "(64 beds of 64^3, 48 to train on) is bench.py --surrogate"),
        "seconds_total": round(time.perf_counter() - t0, 1),
    }


def fields_of(sim, ns):
    """Macroscopic state (rho_j, u, T at gas and wall nodes, T^s) of a run, as
    the init arrays of another run (the populations restart at equilibrium)."""
    import numpy as np
    from paper_1804_07588_amd import fdlbm
    return dict(rho=np.stack([sim.field(fdlbm.FIELD_RHO, j) for j in range(ns)]),
                u=np.stack([sim.field(fdlbm.FIELD_U, a) for a in range(3)]),
                T=sim.field(fdlbm.FIELD_T), Ts=sim.field(fdlbm.FIELD_TS))


def run_to(sim, tol, max_steps, check=100, plateau=None, label="", log=None):
    """Step until the residual (checked every `check` steps) is <= tol, or the
    step budget is spent, or (plateau = (window, factor)) the residual has not
    dropped below factor x its value `window` checks earlier.  Returns
    (steps, last residual dict).  log: a fdlbm.RunLog that records the
    observables and residual at every check."""
    sim.step(1)
    sim.residual()  # first snapshot
    steps, r, hist, last = 1, None, [], time.perf_counter()
    while steps < max_steps:
        sim.step(check)
        steps += check
        r = sim.residual()
        if log is not None:
            log.record(sim, residual=r, label=label)
        hist.append(r["max"])
        if r["max"] <= tol:
            break
        if plateau and len(hist) > plateau[0] and hist[-1] > plateau[1] * hist[-1 - plateau[0]]:
            break
        if time.perf_counter() - last > 30:
            print(f"# {label} step {steps} residual {r['max']:.3e}", file=sys.stderr, flush=True)
            last = time.perf_counter()
    return steps, r


def steady(args, sim, cfg, n_gas, ns, init):
    """Cold start (the bed filled with the inlet gas at rest) to a residual of
    args.tol, checked every 100 steps; prints one JSON line.  With 16-bit
    population storage the run goes in two stages: the 16-bit run until its
    residual reaches args.stage_tol or stops falling (the rounding floor of
    the stored populations), then an FP32 run started from its fields
    (equilibrium populations) to args.tol.  The FP32 context is built before
    the clock starts; the field hand-over is timed."""
    import torch
    from paper_1804_07588_amd import fdlbm
    two_stage = args.precision in ("f16", "bf16")
    fin = fdlbm.Sim(cfg, precision=fdlbm.F32, init=init) if two_stage else None
    log = fdlbm.RunLog(args.log, dict(run="steady", n=args.n, precision=args.precision,
                                      tol=args.tol)) if args.log else None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stages = []
    if two_stage:
        s1, r1 = run_to(sim, args.stage_tol, args.max_steps, plateau=(20, 0.9), label=args.precision,
                        log=log)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        stages.append(dict(storage=args.precision, steps=s1, seconds=round(t1 - t0, 3),
                           residual=float(r1["max"])))
        fin.init_fields(fields_of(sim, ns))
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        stages.append(dict(handover_seconds=round(t2 - t1, 3)))
        s2, r = run_to(fin, args.tol, args.max_steps - s1, label="f32", log=log)
        steps = s1 + s2
        torch.cuda.synchronize()
        stages.append(dict(storage="f32", steps=s2, seconds=round(time.perf_counter() - t2, 3),
                           residual=float(r["max"])))
        obs = fin.observe()
    else:
        steps, r = run_to(sim, args.tol, args.max_steps, label=args.precision, log=log)
        torch.cuda.synchronize()
        obs = sim.observe()
    dt = time.perf_counter() - t0
    if log is not None:
        log.close()
    print(json.dumps({
        "metric": "steps and seconds from a cold start to steady state",
        "value": round(dt, 3), "unit": "s", "steps_to_steady": steps,
        "converged": bool(r is not None and r["max"] <= args.tol), "tol": args.tol,
        "residual": {k: float(v) for k, v in r.items()} if r else None,
        "stages": stages or None,
        "n_gpus": 1, "higher_is_better": False, "data": "synthetic",
        "dtype": "f64" if args.precision == "f64" else "f32", "population_storage": args.precision,
        "config": {"workload": f"packed bed {args.n}^3 D3Q19 cold start (inlet gas at rest), "
                               f"5 species WGS", "gas_nodes": n_gas, "species": ns},
        "bad": obs["bad"], "T_max": obs["T_max"], "u_max": obs["u_max"],
    }), flush=True)


def batch_run(args):
    """A batch of packed beds of uneven size (edge uniform in [batch_min,
    batch_max], bed porosity uniform in [0.4, 0.7), radius-6 spheres, the
    water-gas-shift chemistry), cold start, advanced together by the batched
    persistent launches with autotuned launch shapes until every sample's
    residual (checked every 100 steps) is <= args.tol; converged samples are
    frozen.  Setup (geometry, contexts) is excluded from the clock; the
    autotuner's steps are inside it.  Afterwards the throughput of the batch
    is compared with the same samples stepped one context at a time."""
    import numpy as np
    import torch
    from paper_1804_07588_amd import fdlbm, workloads as W
    prec = {"f32": fdlbm.F32, "f64": fdlbm.F64, "f16": fdlbm.F16, "bf16": fdlbm.BF16}[args.precision]
    t_setup = time.perf_counter()
    cfgs = W.batch_beds(args.batch_samples, n_min=args.batch_min, n_max=args.batch_max,
                        seed=args.batch_seed)
    stream = torch.cuda.Stream()   # default priority; graph capture needs a non-default stream
    sims = []
    for k, c in enumerate(cfgs):
        sims.append(fdlbm.Sim(c, precision=prec, init=W.uniform_init(c), stream=stream))
        if (k + 1) % 8 == 0:
            print(f"# batch setup: {k + 1}/{len(cfgs)} samples", file=sys.stderr, flush=True)
    ns = len(cfgs[0]["species"]["M"])
    gas = np.array([s.counts()[0] for s in sims], dtype=np.int64)
    setup_s = time.perf_counter() - t_setup
    B = fdlbm.Batch(sims)
    S = len(sims)
    steps = np.zeros(S, dtype=np.int64)
    done = np.zeros(S, dtype=bool)
    failed = np.zeros(S, dtype=bool)
    last_r = np.full(S, np.inf)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tuned = B.autotune(5)
    B.step(1)
    for s in sims:
        s.residual()  # first snapshots
    last = time.perf_counter()
    check = 100
    while not done.all():
        B.step(check)
        newly = []
        for k, s in enumerate(sims):
            if done[k]:
                continue
            r = s.residual()
            last_r[k] = r["max"]
            if r["max"] <= args.tol:
                newly.append(k)
        for k, s in enumerate(sims):
            if done[k]:
                continue
            o = s.observe()
            steps[k] = o["step"]
            if o["bad"] and k not in newly:
                failed[k] = True   # unstable: frozen, reported, never converges
                newly.append(k)
        if newly:
            done[newly] = True
            if not done.all():
                B.set_active(~done)
        if steps[~done].max(initial=0) >= args.max_steps:
            break
        if time.perf_counter() - last > 30:
            print(f"# batch: {int(done.sum())}/{S} converged, step {int(steps.max())}",
                  file=sys.stderr, flush=True)
            last = time.perf_counter()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    conv = done & ~failed
    bad = [k for k in range(S) if failed[k]]
    work = float((gas * ns * steps).sum())
    umax = [s.observe()["u_max"] for s in sims]
    per_sample = [dict(n=c["sample"]["n"], porosity=round(c["sample"]["porosity"], 3),
                       force=float(c["flow"]["F"][0]), gas=int(gas[k]), steps=int(steps[k]),
                       converged=bool(conv[k]), u_max=round(float(umax[k]), 4),
                       residual=float(last_r[k]))
                  for k, c in enumerate(cfgs)]
    # throughput: the whole batch together versus one context at a time
    B.set_active(np.ones(S, dtype=np.uint8))
    K = 100
    B.step(K)
    torch.cuda.synchronize()
    tb = time.perf_counter()
    B.step(K)
    torch.cuda.synchronize()
    tb = time.perf_counter() - tb
    for s in sims:
        s.step(K)   # even: the batch parity is unchanged
    torch.cuda.synchronize()
    ts = time.perf_counter()
    for s in sims:
        s.step(K)
    torch.cuda.synchronize()
    ts = time.perf_counter() - ts
    per_step_work = float(gas.sum() * ns)
    mlups_b = per_step_work * K / tb / 1e6
    mlups_s = per_step_work * K / ts / 1e6
    print(json.dumps({
        "metric": "seconds for a batch of packed beds to reach steady state (cold start)",
        "value": round(elapsed, 3), "unit": "s", "higher_is_better": False, "n_gpus": 1,
        "converged": int(conv.sum()), "samples": S, "tol": args.tol, "bad_samples": bad,
        "steps_to_steady": {"min": int(steps[conv].min()) if conv.any() else None,
                            "median": int(np.median(steps[conv])) if conv.any() else None,
                            "max": int(steps[conv].max()) if conv.any() else None},
        "mlups_species_during_run": round(work / elapsed / 1e6, 1),
        "batched_mlups_species": round(mlups_b, 1), "one_at_a_time_mlups_species": round(mlups_s, 1),
        "batched_speedup": round(mlups_b / mlups_s, 3),
        "tuned_grids": tuned, "setup_seconds": round(setup_s, 1),
        "dtype": "f64" if prec == fdlbm.F64 else "f32", "population_storage": args.precision,
        "data": "synthetic",
        "config": {"workload": f"{S} packed beds, edges {args.batch_min}-{args.batch_max} "
                               f"(uniform), bed porosity 0.4-0.7, spheres r=6, 5 species WGS, "
                               f"seed {args.batch_seed}",
                   "nodes": int(sum(c["nx"] * c["ny"] * c["nz"] for c in cfgs)),
                   "gas_nodes": int(gas.sum()), "species": ns},
        "per_sample": per_sample,
    }), flush=True)


def unet_flops(R, n):
    """Multiply-adds x 2 of one training iteration over n samples: forward
    convolutions, plus the input-gradient and weight-gradient convolutions
    of the backward pass (the first layer needs no input gradient)."""
    from paper_1804_07588_amd import workloads as W
    fwd = [2 * 27 * ci * co * n * (R >> lvl) ** 3 for ci, co, lvl, _ in W.UNET_LAYERS]
    return sum(fwd) * 3 - fwd[0]


def unet_bench(args):
    """Training iterations of the warm-start U-Net (mini-batch sur_batch at
    edge sur_n, synthetic seeded inputs): time per iteration and the
    convolution work rate against the dense bf16 MFMA peak."""
    import numpy as np
    import torch
    from paper_1804_07588_amd import surrogate, workloads as W
    R, n = args.sur_n, args.sur_batch
    net = surrogate.UNet(R, n, surrogate.N_IN, 9)
    net.set_params(W.unet_init_params(seed=1))
    rng = np.random.default_rng(0)
    x = torch.as_tensor(rng.standard_normal((n, R ** 3, surrogate.N_IN)).astype(np.float32)).cuda()
    t = torch.as_tensor(rng.standard_normal((n, R ** 3, 9)).astype(np.float32)).cuda()
    w = torch.ones_like(t)
    ws = float(w.sum().item())
    for _ in range(args.warmup if args.warmup < 50 else 3):
        net.train_step(x, t, w, ws, 1e-4, want_loss=False)
    torch.cuda.synchronize()
    steps = min(args.steps, 20)
    t0 = time.perf_counter()
    for _ in range(steps):
        net.train_step(x, t, w, ws, 1e-4, want_loss=False)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    fl = unet_flops(R, n)
    print(json.dumps({
        "metric": "U-Net training iteration (forward, backward, Adam)", "value": round(dt * 1e3, 3),
        "unit": "ms", "higher_is_better": False, "n_gpus": 1, "steps": steps,
        "roofline": {"bound": "mfma", "achieved": round(fl / dt / 1e12, 2), "peak": 2500.0,
                     "unit": "TFLOP/s", "frac": round(fl / dt / 1e12 / 2500.0, 4),
                     "flops_per_iteration": fl},
        "dtype": "bf16 (MFMA, f32 accumulate)", "data": "synthetic",
        "config": {"workload": f"U-Net 32/64/160, {n} samples of {R}^3, 3 -> 9 channels",
                   "params": int(net.n_params)},
    }), flush=True)


def surrogate_run(args):
    """Learned warm start, end to end on the GPU, at the full configuration
    (the --sur-* options); prints one JSON line."""
    print(json.dumps(surrogate_pipeline(args)), flush=True)


def surrogate_pipeline(args, quiet=False):
    """(1) sur_train + sur_test packed beds of edge sur_n (porosity 0.4-0.7)
    run together from a cold start to the steady-state residual --tol (the
    steps of the held-out beds are their cold-start baseline); (2) the U-Net
    is trained on the training beds' steady mole fractions, temperature and
    velocity; (3) the held-out beds are run again, once from a cold start and
    once from the network's prediction, each as one batch, to --tol, and once
    more from the prediction with FP16 population storage to 1e-5 followed by
    FP32.  Returns the result record."""
    import numpy as np
    import torch
    from paper_1804_07588_amd import fdlbm, surrogate, warmstart, workloads as W
    S = args.sur_train + args.sur_test
    cfgs = W.batch_beds(S, n_min=args.sur_n, n_max=args.sur_n, seed=args.sur_seed)
    lg = (lambda name: None) if quiet else (lambda name: name)
    stream = torch.cuda.Stream()   # default priority
    with torch.cuda.stream(stream):
        sims = warmstart.make_sims(cfgs, fdlbm.F32, stream, log=lg("data setup"))
        gen = warmstart.run_to_steady(sims, args.tol, args.max_steps, log=lg("steady states"))
        X, T, Wt = warmstart.dataset(sims, cfgs)
        for s_ in sims:
            s_.close()
        del sims
        ok = gen["converged"]
        tr = [k for k in range(args.sur_train) if ok[k]]
        te = [k for k in range(args.sur_train, S) if ok[k]]
        norm = surrogate.Normaliser([T[k] for k in tr], [Wt[k] for k in tr])
        ns = len(cfgs[0]["species"]["M"])
        net = surrogate.UNet(args.sur_n, args.sur_batch, surrogate.N_IN, ns + 4, stream=stream)
        net.set_params(W.unet_init_params(seed=args.sur_seed))
        Tn = np.stack([norm.encode(T[k]) for k in tr])
        Wn = np.stack([Wt[k] for k in tr])
        fit = warmstart.train(net, X[tr], Tn, Wn, args.sur_epochs, args.sur_batch, args.sur_lr,
                              log=lg("training"), norm=None if args.sur_no_augment else norm, ns=ns)
        flops = unet_flops(args.sur_n, 1) * len(tr) * args.sur_epochs
        # held-out prediction error (normalised units, weighted RMS per channel)
        errs = []
        for k in te:
            y = net.forward(torch.as_tensor(X[k][None]).cuda().contiguous()).cpu().numpy()[0]
            d = (y - norm.encode(T[k])) ** 2 * Wt[k]
            errs.append(np.sqrt(d.sum(axis=0) / np.maximum(Wt[k].sum(axis=0), 1)))
        test_cfgs = [cfgs[k] for k in te]
        inits = warmstart.predict_inits(net, norm, test_cfgs)
        cold_sims = warmstart.make_sims(test_cfgs, fdlbm.F32, stream)
        cold = warmstart.run_to_steady(cold_sims, args.tol, args.max_steps, log=lg("held-out cold"))
        for s_ in cold_sims:
            s_.close()
        warm_sims = warmstart.make_sims(test_cfgs, fdlbm.F32, stream, inits=inits)
        warm = warmstart.run_to_steady(warm_sims, args.tol, args.max_steps, log=lg("held-out warm"))
        for s_ in warm_sims:
            s_.close()
        # warm start plus reduced-precision storage: FP16 populations to a
        # residual of 1e-5, then FP32 from those fields to --tol
        h_sims = warmstart.make_sims(test_cfgs, fdlbm.F16, stream, inits=inits)
        f_sims = warmstart.make_sims(test_cfgs, fdlbm.F32, stream)
        torch.cuda.synchronize()
        t_h = time.perf_counter()
        h1 = warmstart.run_to_steady(h_sims, max(args.tol, 1e-5), args.max_steps, log=lg("held-out warm f16"))
        for hs, fs in zip(h_sims, f_sims):
            fs.init_fields(fields_of(hs, ns))
        h2 = warmstart.run_to_steady(f_sims, args.tol, args.max_steps, log=lg("held-out warm f16->f32"))
        torch.cuda.synchronize()
        warm16_s = time.perf_counter() - t_h
        warm16_steps = h1["steps"] + h2["steps"]
        warm16_ok = h2["converged"]
    cs, ws = cold["steps"], warm["steps"]
    both = cold["converged"] & warm["converged"]
    return {
        "metric": "time to steady state of held-out packed beds: learned warm start vs cold start",
        "value": round(cold["seconds"] / warm["seconds"], 3), "unit": "x (cold seconds / warm seconds)",
        "higher_is_better": True, "n_gpus": 1, "tol": args.tol,
        "cold": {"seconds": round(cold["seconds"], 2), "steps_mean": float(cs[both].mean()) if both.any() else None,
                 "converged": int(cold["converged"].sum())},
        "warm": {"seconds": round(warm["seconds"], 2), "steps_mean": float(ws[both].mean()) if both.any() else None,
                 "converged": int(warm["converged"].sum())},
        "steps_ratio": float(cs[both].mean() / ws[both].mean()) if both.any() else None,
        "warm_f16_then_f32": {"seconds": round(warm16_s, 2), "steps_mean": float(warm16_steps.mean()),
                              "f16_steps_mean": float(h1["steps"].mean()),
                              "converged": int(warm16_ok.sum()),
                              "speedup_vs_cold": round(cold["seconds"] / warm16_s, 3)},
        "per_test_steps": [[int(a), int(b)] for a, b in zip(cs, ws)],
        "training": {"samples": len(tr), "epochs": args.sur_epochs, "batch": args.sur_batch,
                     "augmented": not args.sur_no_augment,
                     "seconds": round(fit["seconds"], 2), "loss_first": fit["losses"][0],
                     "loss_last": fit["losses"][-1], "params": int(net.n_params),
                     "tflops": round(flops / fit["seconds"] / 1e12, 2)},
        "test_rms_error_normalised": np.mean(errs, axis=0).round(4).tolist() if errs else None,
        "data_generation": {"samples": S, "converged": int(ok.sum()), "seconds": round(gen["seconds"], 1),
                            "steps_median": int(np.median(gen["steps"]))},
        "data": "synthetic", "dtype": "f32 (method), bf16 MFMA with f32 accumulation (network)",
        "config": {"workload": f"packed beds {args.sur_n}^3, porosity 0.4-0.7, spheres r=6, 5 species WGS, "
                               f"seed {args.sur_seed}; U-Net 32/64/160 channels",
                   "train": len(tr), "test": len(te)},
    }


def _count_wall_links(kind, cfg):
    """Number of (wall node, incoming direction) pairs: links from a gas node
    into a wall node."""
    import numpy as np
    nz, ny, nx = cfg["nz"], cfg["ny"], cfg["nx"]
    k = kind.reshape(nz, ny, nx)
    gas = (k == 0) | (k >= 3)
    wall = k == 2
    total = 0
    moving = [(a, b, c) for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1)
              if 0 < a * a + b * b + c * c <= 2]
    for cx, cy, cz in moving:
        src = np.roll(gas, shift=(cz, cy, cx), axis=(0, 1, 2))
        if cx != 0:
            # x is closed: no wrap-around
            if cx > 0:
                src[:, :, :cx] = False
            else:
                src[:, :, cx:] = False
        total += int(np.count_nonzero(wall & src))
    return total


if __name__ == "__main__":
    main()
