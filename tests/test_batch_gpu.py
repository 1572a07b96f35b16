"""Batched persistent launches versus one context at a time.

A batch runs the same per-node kernels as fdlbm_step, with the same logical
block numbering per sample, so every field and every FP64 accumulator of a
sample must be bitwise equal to that sample stepped alone with FP32 or FP64
storage (the standalone path is the one checked against the oracle in
test_parity_gpu.py), and equal to FP32 rounding over the first steps with
16-bit storage.  Samples
differ in size, porosity and parameters; the batch covers graph replays,
direct launches, frozen (inactive) samples re-joining with the other parity,
and the autotuner's tuning steps.  One sample is also compared with the
oracle directly.
"""
import numpy as np
import pytest

from paper_1804_07588_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fd():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1804_07588_amd import fdlbm
    fdlbm.lib()
    return fdlbm


def bed_cfgs():
    """Four beds of radius-3 spheres that stay free of negative densities over
    the steps run here (with rougher walls -- porosity 0.5 to 0.55 and faster
    rates -- the interpolated wall densities of the trace product species
    turn negative within tens of steps, in the oracle as on the GPU)."""
    out = []
    for (n, ny, nz, por, seed, k0, force) in [(20, 20, 20, 0.6, 1, 1e-3, 1e-5),
                                              (24, 20, 16, 0.6, 2, 2e-3, 2e-5),
                                              (16, 16, 16, 0.7, 3, 1e-3, 0.0),
                                              (28, 12, 20, 0.6, 4, 1e-3, 1e-5)]:
        mask, _ = W.sphere_pack_mask(n, radius=3.0, porosity=por, seed=seed, buffer=4, ny=ny, nz=nz)
        out.append(W.packed_bed(mask=mask, k0=k0, force=force))
    return out


def channel_cfgs():
    return [W.channel_c1(nx=64, ny=40), W.channel_c1(nx=40, ny=24, wall=3),
            W.with_changes(W.channel_c1(nx=24, ny=30), reaction=dict(k0=5e-3))]


def snapshot(fd, sim):
    out = {}
    for j in range(sim.ns):
        out[f"rho{j}"] = sim.field(fd.FIELD_RHO, j)
        out[f"pop{j}"] = sim.field(fd.FIELD_POP, j)
    for a in range(3):
        out[f"u{a}"] = sim.field(fd.FIELD_U, a)
    out["T"] = sim.field(fd.FIELD_T)
    out["Ts"] = sim.field(fd.FIELD_TS)
    o = sim.observe()
    for k in ("e_gas", "e_solid", "moles_reacted", "heat_released", "heat_boundary", "work_body", "step"):
        out["obs_" + k] = np.array([o[k]])
    out["obs_mass"] = o["mass"]
    return out


def assert_same(a, b, label, tol=0.0):
    """Bitwise equality (tol = 0), else max|a - b| <= tol * scale per field
    (scale: the lattice sound speed for velocities, max|a| otherwise)."""
    for k in a:
        assert np.all(np.isfinite(a[k])), f"{label}: {k} is not finite in the single run"

    def scale(k):
        return np.sqrt(1.0 / 3.0) if k[0] == "u" else max(np.abs(a[k]).max(), 1e-300)

    if tol == 0.0:
        bad = [k for k in a if not np.array_equal(a[k], b[k])]
    else:
        bad = [k for k in a if np.abs(a[k] - b[k]).max() > tol * scale(k)]
    worst = {k: float(np.abs(a[k] - b[k]).max() / scale(k)) for k in bad[:4]}
    assert not bad, f"{label}: differs in {bad[:6]} (relative {worst})"


def make(fd, cfgs, precision, stream=None):
    return [fd.Sim(c, precision=precision, init=W.uniform_init(c), stream=stream) for c in cfgs]


@pytest.fixture(scope="module")
def stream(fd):
    import torch
    return torch.cuda.Stream()  # default priority; graphs need a non-default stream


def variant_cfgs():
    """The beds with the half-way wall and a second surface reaction (the
    reverse water-gas shift) in every sample."""
    out = []
    for c in bed_cfgs():
        rx = c["reaction"]
        rx["halfway"] = True
        rx["more"] = [dict(nu=[-x for x in rx["nu"]], order=[0.0, 0.0, 1.0, 1.0, 0.0], k0=2e-4, ea=0.5 * rx["ea"],
                           T_ref=rx["T_ref"], dH=-rx["dH"])]
        out.append(c)
    return out


def eq48_cfgs():
    """The channels with the Eq.(48) solid coupling in every sample."""
    return [W.with_changes(c, solid=dict(coupling=1)) for c in channel_cfgs()]


def cn_cfgs():
    """The channels with Crank-Nicolson solids of different diffusivities, so
    that the samples take different numbers of Jacobi sweeps."""
    return [W.with_changes(c, solid=dict(scheme=1, alpha_s=a)) for c, a in zip(channel_cfgs(), (1.5, 0.4, 3.0))]


@pytest.mark.parametrize("lattice,prec", [(3, "F32"), (3, "F16"), (3, "BF16"), (2, "F64"), ("3v", "F32"),
                                          ("2e", "F64"), ("2c", "F64")])
def test_batch_bitwise_equals_single(fd, stream, lattice, prec):
    """lattice "3v": the beds with the half-way wall and two reactions; "2e":
    the channels with the Eq.(48) coupling; "2c": the channels with
    Crank-Nicolson solids."""
    precision = getattr(fd, prec)
    # FP32 / FP64 storage: bitwise.  16-bit storage: the batched kernels are
    # separate instantiations in which the compiler contracts a few FP32
    # operations of the collision differently (observed 5e-7 relative after
    # 10 steps); a rounding difference can later flip a 16-bit rounding of a
    # trace species, so the 16-bit runs are compared over the first 10 steps
    narrow = prec in ("F16", "BF16")
    tol = 1e-5 if narrow else 0.0
    cfgs = {3: bed_cfgs, "3v": variant_cfgs, 2: channel_cfgs, "2e": eq48_cfgs, "2c": cn_cfgs}[lattice]()
    print(f"[batch] lattice {lattice} {prec} samples {len(cfgs)}", flush=True)
    ref = make(fd, cfgs, precision)
    for r in ref:
        r.set_overlap(False)  # the reference: one stream, kernels in sequence
    bat = make(fd, cfgs, precision, stream)
    b = fd.Batch(bat)
    b.set_grid(graph_steps=4)  # the batch: wall and solid on a second stream
    # 10 steps: two graph replays and two direct launches
    b.step(10)
    for s in ref:
        s.step(10)
    for i, (r, s) in enumerate(zip(ref, bat)):
        assert_same(snapshot(fd, r), snapshot(fd, s), f"sample {i} after 10 steps", tol)
    if narrow:
        b.close()
        return
    # freeze sample 1 for 5 steps, then let it rejoin with the other parity
    flags = np.ones(len(cfgs), dtype=np.uint8)
    flags[1] = 0
    b.set_active(flags)
    b.step(5)
    for i, r in enumerate(ref):
        if i != 1:
            r.step(5)
    for i, (r, s) in enumerate(zip(ref, bat)):
        assert_same(snapshot(fd, r), snapshot(fd, s), f"sample {i} with sample 1 frozen", tol)
    b.set_active(np.ones(len(cfgs)))
    b.step(9)
    for r in ref:
        r.step(9)
    for i, (r, s) in enumerate(zip(ref, bat)):
        assert_same(snapshot(fd, r), snapshot(fd, s), f"sample {i} after rejoining", tol)
    b.close()


def test_batch_autotune_and_oracle(fd, stream, oracle_lib):
    cfgs = bed_cfgs()
    init = [W.uniform_init(c) for c in cfgs]
    bat = [fd.Sim(c, precision=fd.F32, init=i, stream=stream) for c, i in zip(cfgs, init)]
    b = fd.Batch(bat)
    grids = b.autotune(steps=2)
    print(f"[batch] tuned grids {grids}", flush=True)
    assert all(g > 0 and g % 8 == 0 for g in grids.values())
    b.step(24)
    steps = bat[0].observe()["step"]
    assert all(s.observe()["step"] == steps for s in bat)
    ref = fd.Sim(cfgs[1], precision=fd.F32, init=init[1])
    ref.step(steps)
    assert_same(snapshot(fd, ref), snapshot(fd, bat[1]), "sample 1 after autotune")
    # the batched sample against the FP64 oracle (FP32 parity bound)
    o = oracle_lib.OracleSim(cfgs[1], init[1])
    o.step(steps)
    for j in range(len(cfgs[1]["species"]["M"])):
        g = bat[1].field(fd.FIELD_RHO, j)
        r = o.field(oracle_lib.OF_RHO, j)
        assert np.abs(g - r).max() / np.abs(r).max() < 1e-5
    g, r = bat[1].field(fd.FIELD_T), o.field(oracle_lib.OF_T)
    assert np.abs(g - r).max() / np.abs(r).max() < 1e-5
    b.close()


def test_batch_rejects_mixed_members(fd):
    a = fd.Sim(W.channel_c1(), precision=fd.F64, init=W.uniform_init(W.channel_c1()))
    c = fd.Sim(W.channel_c1(), precision=fd.F32, init=W.uniform_init(W.channel_c1()))
    with pytest.raises(fd.FdlbmError):
        fd.Batch([a, c])
    with pytest.raises(fd.FdlbmError):
        fd.Batch([a, a])
    # wall positions differ
    h = W.with_changes(W.channel_c1(), reaction=dict(halfway=True))
    d = fd.Sim(h, precision=fd.F64, init=W.uniform_init(h))
    with pytest.raises(fd.FdlbmError):
        fd.Batch([a, d])
    # a member that gains a second reaction after the batch was made
    e = fd.Sim(W.channel_c1(), precision=fd.F64, init=W.uniform_init(W.channel_c1()))
    b = fd.Batch([a, e])
    import ctypes as ct
    dp = ct.POINTER(ct.c_double)
    nu, order = np.array([-1.0, 1.0]), np.array([1.0, 0.0])
    assert fd.lib().fdlbm_add_reaction(e.h, nu.ctypes.data_as(dp), order.ctypes.data_as(dp), 1e-3, 0.0,
                                       1.0 / 3.0, -0.1) == fd.OK
    with pytest.raises(fd.FdlbmError):
        b.set_active(np.ones(2, dtype=np.uint8))
    b.close()


def test_batch_of_benchmark_beds(fd, stream, oracle_lib):
    """The first six beds of the 64-bed batch benchmark (same generator and
    seed: edges 48-96, porosity 0.4-0.7, FP32), batched with graph replays
    and direct steps: bitwise the same samples stepped alone; the smallest
    one also against the oracle."""
    cfgs = W.batch_beds(6)
    print("[batch] benchmark beds", [c["sample"]["n"] for c in cfgs], flush=True)
    init = [W.uniform_init(c) for c in cfgs]
    bat = [fd.Sim(c, precision=fd.F32, init=i, stream=stream) for c, i in zip(cfgs, init)]
    b = fd.Batch(bat)
    b.set_grid(graph_steps=4)
    b.step(10)
    for k, (c, i) in enumerate(zip(cfgs, init)):
        ref = fd.Sim(c, precision=fd.F32, init=i)
        ref.set_overlap(False)
        ref.step(10)
        assert_same(snapshot(fd, ref), snapshot(fd, bat[k]), f"benchmark bed {k} (edge {c['sample']['n']})")
        ref.close()
    k = min(range(len(cfgs)), key=lambda q: cfgs[q]["sample"]["n"])
    o = oracle_lib.OracleSim(cfgs[k], init[k])
    o.step(10)
    for j in range(len(cfgs[k]["species"]["M"])):
        g, r = bat[k].field(fd.FIELD_RHO, j), o.field(oracle_lib.OF_RHO, j)
        assert np.abs(g - r).max() / np.abs(r).max() < 1e-5
    g, r = bat[k].field(fd.FIELD_T), o.field(oracle_lib.OF_T)
    assert np.abs(g - r).max() / np.abs(r).max() < 1e-5
    o.close()
    b.close()


@pytest.mark.parametrize("prec", ["F64", "F32"])
def test_batch_check_names_the_unstable_sample(fd, stream, prec):
    """fdlbm_batch_check: three channels batched, the middle one driven past
    the lattice sound speed by a body force of 0.02 per step (the blow-up of
    test_parity_gpu's unstable-step test); the check reports that sample and
    the step at which it alone, stepped on its own context, first turns
    non-physical; before that step the check is clean."""
    precision = getattr(fd, prec)
    base = W.with_changes(W.channel_c1(nx=16, ny=16, wall=2), init=dict(X=[0.7, 0.3]))
    cfgs = [W.with_changes(base, flow=dict(F=[F, 0, 0])) for F in (1e-6, 0.02, 2e-6)]
    init = W.uniform_init(base)
    ref = fd.Sim(cfgs[1], precision=precision, init=init)
    ref.step(300)
    s_bad = ref.last_step()
    ref.close()
    assert s_bad > 10, s_bad
    print(f"[batch] {prec}: sample 1 first unstable at step {s_bad}", flush=True)
    sims = [fd.Sim(c, precision=precision, init=init, stream=stream) for c in cfgs]
    b = fd.Batch(sims)
    b.set_grid(graph_steps=4)
    b.step(s_bad - 3)
    assert b.check() is None
    b.step(40)
    with pytest.raises(fd.FdlbmError) as ei:
        b.check()
    assert ei.value.code == fd.E_UNSTABLE
    assert (ei.value.sample, ei.value.step) == (1, s_bad)
    assert sims[0].last_step() == -1 and sims[2].last_step() == -1
    b.close()
