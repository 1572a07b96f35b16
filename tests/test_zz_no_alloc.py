"""The allocation-free observables entry point (fdlbm_observe_noalloc) against
fdlbm_observe, through the C ABI: two calls in a row on different contexts
sharing the GPU's static scratch array, the second with a smaller input,
each compared value by value (bitwise: the same FP64 folds in the same
order)."""
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


def _same(a, b):
    for k in a:
        if k == "mass":
            assert np.array_equal(a[k], b[k]), k
        else:
            assert a[k] == b[k], (k, a[k], b[k])


def test_observe_noalloc_matches_observe(fd):
    mask, _ = W.sphere_pack_mask(24, radius=3.0, porosity=0.6, seed=9, buffer=4)
    big = W.packed_bed(mask=mask, k0=1e-3, force=1e-5)
    small = W.with_changes(W.channel_c1(nx=16, ny=12, wall=2), init=dict(X=[0.7, 0.3]))
    print("[no-alloc] 24^3 bed (F32) then 16x12 channel (F64)", flush=True)
    a = fd.Sim(big, precision=fd.F32, init=W.perturbed_init(big, 3, amp_u=0.005))
    b = fd.Sim(small, precision=fd.F64, init=W.perturbed_init(small, 2))
    a.step(20)
    b.step(30)
    for sim in (a, b, a, b):   # alternate: each call overwrites what the previous left
        ref = sim.observe()
        got = sim.observe_noalloc()
        _same(got, ref)
        assert got["moles_reacted"] != 0.0 and got["e_gas"] > 0.0
        sim.step(5)
    a.close()
    b.close()
