"""Seeded random cases against the FP64 oracle: each seed draws a lattice,
a geometry (random porous 2-D channel or sphere pack, with or without
inlet/outlet, periodic or closed axes), one to six species with masses from
1 to 22, a subset of the correction terms, species or common Prandtl
numbers, the solid scheme (forward Euler or Crank-Nicolson) and coupling
(flux-matched or Eq.(48)), the rate law's constants and options (per node or
per area, lattice or flux-scaled source), the wall position (on the node or
half-way), a second surface reaction and a body force, runs a few dozen
FP64 steps from a perturbed state on both sides and compares every field to
the FP64 bounds of test_parity_gpu.py.  The draws stay in ranges where the
method is stable; a case whose oracle run turns non-physical is reported and
skipped, not compared."""
import numpy as np
import pytest

from oracle import oracle as of
from paper_1804_07588_amd import workloads as W

pytestmark = pytest.mark.gpu

T0 = 1.0 / 3.0
TOL64, TOL64_U = 1e-12, 1e-11
MASSES = (1.0, 2.0, 4.0, 9.0, 14.0, 22.0)


@pytest.fixture(scope="module")
def fd():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1804_07588_amd import fdlbm
    fdlbm.lib()
    return fdlbm


def random_case(seed: int) -> tuple[dict, dict, int]:
    rng = np.random.default_rng(1000 + seed)
    lattice = int(rng.choice([2, 3]))
    ns = int(rng.integers(1, 7))
    if lattice == 2:
        nx, ny = int(rng.integers(20, 40)), int(rng.integers(16, 28))
        mask = (rng.random((1, ny, nx)) < rng.uniform(0.1, 0.3)).astype(np.uint8)
        mask[:, :2, :] = 1
        mask[:, -2:, :] = 1
        cfg = W.channel_c1(nx=nx, ny=ny, wall=2)
        cfg["mask"] = W.fill_closed_pores(mask, periodic=(1, 0, 1))
        steps = 60
    else:
        n = int(rng.integers(12, 18))
        m, _ = W.sphere_pack_mask(n, radius=float(rng.uniform(2.0, 3.2)), porosity=float(rng.uniform(0.55, 0.7)),
                                  seed=int(rng.integers(1, 10 ** 6)), buffer=4)
        cfg = W.packed_bed(mask=m)
        if rng.random() < 0.5:
            cfg["inout"] = 0
            cfg["periodic"] = (1, 1, 1)
        steps = 25
    M = [1.0] + sorted(float(x) for x in rng.choice(MASSES[1:], size=ns - 1, replace=True))
    X = list(rng.dirichlet(np.ones(ns)) * 0.8 + 0.2 / ns)
    sp = cfg["species"]
    sp.update(M=M, mu0=[float(rng.uniform(0.02, 0.05)) * np.sqrt(m) for m in M],
              Djk0=[[0.0 if j == k else 0.05 * np.sqrt(0.5 * (1 / M[j] + 1 / M[k])) for k in range(ns)]
                    for j in range(ns)],
              Pr=float(rng.choice([0.71, 1.0])), flags=int(rng.integers(0, 16)))
    sp.pop("names", None)
    sp.pop("Pr_j", None)
    if rng.random() < 0.3:
        sp["Pr_j"] = [float(x) for x in rng.uniform(0.6, 1.2, ns)]
    D = lattice
    so = cfg["solid"]
    if rng.random() < 0.3:
        so.update(scheme=1, alpha_s=float(rng.uniform(0.1, 1.5)), coupling=0)
    else:
        so.update(scheme=0, alpha_s=float(rng.uniform(0.01, 0.9 / (2 * D))),
                  coupling=int(rng.random() < 0.3))
    rx = cfg["reaction"]
    nu = [0.0] * ns
    order = [0.0] * ns
    if ns >= 2:
        nu[0], nu[1], order[0] = -1.0, 1.0, 1.0
    rx.update(nu=nu, order=order, k0=float(10 ** rng.uniform(-4, -2.3)), ea=float(rng.uniform(0, 5)),
              dH=float(rng.uniform(-0.4, 0.0)), rate_area=bool(lattice == 3 and rng.random() < 0.5),
              source_flux=bool(rng.random() < 0.3), max_iter=64, tol=1e-13)
    F = [float(rng.uniform(0, 1e-5)), 0.0, 0.0]
    cfg["flow"].update(F=F, X_in=X)
    cfg["init"].update(X=X)
    init = W.perturbed_init(cfg, 77 + seed, amp_rho=0.01, amp_u=0.004, amp_T=0.005)
    rx["halfway"] = bool(rng.random() < 0.3)   # drawn after the rest: the earlier draws stay as they were
    if ns >= 3 and rng.random() < 0.6:
        # a second surface reaction consuming the first one's product
        nu2, ord2 = [0.0] * ns, [0.0] * ns
        nu2[1], nu2[2], ord2[1] = -1.0, 1.0, 1.0
        rx["more"] = [dict(nu=nu2, order=ord2, k0=float(10 ** rng.uniform(-4, -2.3)), ea=float(rng.uniform(0, 5)),
                           T_ref=rx["T_ref"], dH=float(rng.uniform(-0.4, 0.2)))]
    return cfg, init, steps


def rel(a, b):
    s = np.abs(b).max()
    return np.abs(a - b).max() / (s if s > 0 else 1.0)


@pytest.mark.parametrize("seed", range(24))
def test_random_case_fp64(fd, seed):
    cfg, init, steps = random_case(seed)
    ns, D = len(cfg["species"]["M"]), cfg["lattice"]
    desc = (f"lattice {D}, {cfg['nx']}x{cfg['ny']}x{cfg['nz']}, inout {cfg['inout']}, ns {ns}, "
            f"M {cfg['species']['M']}, flags {cfg['species']['flags']}, solid {cfg['solid'].get('scheme', 0)}"
            f"/{cfg['solid'].get('coupling', 0)}, area {cfg['reaction']['rate_area']}, "
            f"flux {cfg['reaction']['source_flux']}, halfway {cfg['reaction']['halfway']}, "
            f"reactions {1 + len(cfg['reaction'].get('more', []))}")
    print(f"[random {seed}] {desc}", flush=True)
    o = of.OracleSim(cfg, init)
    o.step(steps)
    if o.observe()["bad"]:
        o.close()
        pytest.skip(f"the oracle's run of case {seed} turned non-physical ({desc})")
    g = fd.Sim(cfg, precision=fd.F64, init=init)
    g.step(steps)
    g.sync()
    errs = {}
    for j in range(ns):
        errs[f"rho{j}"] = rel(g.field(fd.FIELD_RHO, j), o.field(of.OF_RHO, j))
        errs[f"pop{j}"] = rel(g.field(fd.FIELD_POP, j), o.field(of.OF_POP, j))
    uo = [o.field(of.OF_U, a) for a in range(D)]
    umax = max(np.abs(x).max() for x in uo)
    for a in range(D):
        errs[f"u{a}"] = np.abs(g.field(fd.FIELD_U, a) - uo[a]).max() / max(umax, 1e-12)
    errs["T"] = rel(g.field(fd.FIELD_T), o.field(of.OF_T))
    errs["Ts"] = rel(g.field(fd.FIELD_TS), o.field(of.OF_TS))
    errs["wall_r"] = rel(g.field(fd.FIELD_WALL_R), o.field(of.OF_WALL_R))
    go, oo = g.observe(), o.observe()
    errs["moles"] = abs(go["moles_reacted"] - oo["moles_reacted"]) / max(abs(oo["moles_reacted"]), 1e-300)
    print({k: f"{v:.1e}" for k, v in errs.items()}, flush=True)
    for k, v in errs.items():
        bound = TOL64_U if k[0] == "u" else (1e-10 if k == "moles" else TOL64)
        assert v <= bound, (seed, k, v, desc)
    g.close()
    o.close()
