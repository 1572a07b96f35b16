"""Writes tests/golden/bed48_oracle_1000.npz: the FP64 oracle's state of a
48^3 packed bed (the benchmark bed's construction: spheres of radius 6,
porosity 0.6, pack seed 4848, an 8-node inlet/outlet buffer, water-gas-shift
chemistry with per-area rates, body force 1e-5) after 1000 steps from the
inlet state at rest, at 4096 gas nodes drawn with a fixed seed, with the
whole-domain observables; the solid temperature at 4096 solid and wall
nodes.  Calls only the oracle; takes about ten minutes on
eight threads.

    python tests/golden/make_bed48.py [threads]
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_1804_07588_amd import workloads as W  # noqa: E402

OUT = os.path.join(HERE, "bed48_oracle_1000.npz")
N, STEPS, SAMPLES, SEED, PACK_SEED = 48, 1000, 4096, 48, 4848


def bed48():
    mask, _ = W.sphere_pack_mask(N, radius=6.0, porosity=0.6, seed=PACK_SEED, buffer=8)
    return W.packed_bed(mask=mask)


def sample_nodes(kind: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """SAMPLES gas nodes (gas, inlet, outlet) and SAMPLES solid nodes (solid,
    wall), drawn with a fixed seed."""
    gas = np.flatnonzero((kind == 0) | (kind == 3) | (kind == 4))
    solid = np.flatnonzero((kind == 1) | (kind == 2))
    rng = np.random.default_rng(SEED)
    return (np.sort(rng.choice(gas, size=SAMPLES, replace=False)),
            np.sort(rng.choice(solid, size=SAMPLES, replace=False)))


def main():
    threads = int(sys.argv[1]) if len(sys.argv) > 1 else os.cpu_count()
    O.build(force=False)
    O.set_threads(threads)
    cfg = bed48()
    sim = O.OracleSim(cfg, W.uniform_init(cfg))
    kind = sim.field(O.OF_KIND).astype(np.int64)
    nodes, snodes = sample_nodes(kind)
    t0 = time.time()
    for k in range(STEPS // 100):
        sim.step(100)
        print(f"step {(k + 1) * 100} ({time.time() - t0:.0f} s)", flush=True)
    ns = len(cfg["species"]["M"])
    out = dict(nodes=nodes, solid_nodes=snodes, steps=np.array(STEPS))
    for j in range(ns):
        out[f"rho{j}"] = sim.field(O.OF_RHO, j)[nodes]
    for a in range(3):
        out[f"u{a}"] = sim.field(O.OF_U, a)[nodes]
    out["T"] = sim.field(O.OF_T)[nodes]
    out["Ts"] = sim.field(O.OF_TS)[snodes]
    obs = sim.observe()
    out["mass"] = np.asarray(obs["mass"])
    for key in ("e_gas", "e_solid", "moles_reacted", "heat_released", "work_body", "u_max",
                "T_min", "T_max"):
        out["obs_" + key] = np.array(obs[key])
    # field scales for the relative bounds (whole domain)
    for j in range(ns):
        out[f"scale_rho{j}"] = np.array(np.abs(sim.field(O.OF_RHO, j)).max())
    out["scale_u"] = np.array(max(np.abs(sim.field(O.OF_U, a)).max() for a in range(3)))
    np.savez_compressed(OUT, **out)
    print("wrote", OUT, flush=True)


if __name__ == "__main__":
    main()
