"""What the trained network gains over the method without it, at a small
scale: ten 32^3 beds run cold to steady state as one batch, the U-Net trains
on eight, and the two held-out beds reach the steady-state residual in fewer
steps from its prediction than from a cold start.  The method decides
convergence either way."""
import numpy as np
import pytest

from paper_1804_07588_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-5


def test_learned_warm_start_needs_fewer_steps():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1804_07588_amd import fdlbm, surrogate, warmstart
    st = torch.cuda.Stream()
    cfgs = W.batch_beds(10, n_min=32, n_max=32, seed=77)
    with torch.cuda.stream(st):
        print("[warm] cold runs of 10 beds", flush=True)
        sims = warmstart.make_sims(cfgs, fdlbm.F32, st)
        gen = warmstart.run_to_steady(sims, TOL, 30000)
        assert gen["converged"].all(), gen["steps"]
        X, T, Wt = warmstart.dataset(sims, cfgs)
        for s in sims:
            s.close()
        norm = surrogate.Normaliser(T[:8], Wt[:8])
        net = surrogate.UNet(32, 4, surrogate.N_IN, 9, stream=st)
        net.set_params(W.unet_init_params(seed=77))
        print("[warm] training", flush=True)
        fit = warmstart.train(net, X[:8], np.stack([norm.encode(t) for t in T[:8]]), np.stack(Wt[:8]),
                              epochs=150, batch=4, lr=1e-3)
        assert fit["losses"][-1] < 0.5 * fit["losses"][0]
        inits = warmstart.predict_inits(net, norm, cfgs[8:])
        print("[warm] warm runs of the 2 held-out beds", flush=True)
        warm_sims = warmstart.make_sims(cfgs[8:], fdlbm.F32, st, inits=inits)
        warm = warmstart.run_to_steady(warm_sims, TOL, 30000)
    cold_steps, warm_steps = gen["steps"][8:], warm["steps"]
    print(f"[warm] held-out steps cold {cold_steps.tolist()} warm {warm_steps.tolist()}; "
          f"loss {fit['losses'][0]:.3f} -> {fit['losses'][-1]:.3f}", flush=True)
    assert warm["converged"].all()
    assert warm_steps.sum() < cold_steps.sum()
