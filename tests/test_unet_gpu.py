"""The U-Net's HIP kernels (bf16 MFMA convolutions, FP32 accumulation)
against the FP64 CPU oracle of the same network: forward output, loss and
every layer's parameter gradient, plus training and the parameter round
trip.  Tolerances follow bf16 rounding of activations, weights and
back-propagated gradients (8-bit mantissa, relative 4e-3 per rounding)
compounded over 11 layers: forward 2e-2 relative L2; gradients 0.1 relative
L2 per layer with a cosine above 0.995 (the deepest layer sees ten rounded
backward convolutions).  Every reduction over positions (weight and bias
gradients, the loss) adds per-block partials in a fixed order, so repeated
gradients and training runs are bitwise equal."""
import numpy as np
import pytest

from oracle import unet_oracle as U
from paper_1804_07588_amd import workloads as W

pytestmark = pytest.mark.gpu

R, NIN, NOUT = 16, 3, 9


@pytest.fixture(scope="module")
def net():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1804_07588_amd import surrogate
    return surrogate.UNet(R, 2, NIN, NOUT)


def data(seed, n=2):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((n, R ** 3, NIN)).astype(np.float32)
    t = rng.standard_normal((n, R ** 3, NOUT)).astype(np.float32)
    w = (rng.random((n, R ** 3, NOUT)) > 0.25).astype(np.float32)
    return x, t, w


def dev(a):
    import torch
    return torch.as_tensor(a).cuda().contiguous()


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def test_params_round_trip(net):
    p = W.unet_init_params(seed=2, bias_scale=0.1)
    assert p.size == net.n_params == W.unet_layout()[1]
    net.set_params(p)
    assert np.array_equal(net.params(), p)


def test_forward_matches_oracle(net):
    p = W.unet_init_params(seed=3, bias_scale=0.1)
    net.set_params(p)
    x, _, _ = data(1)
    print("[unet] forward R=16 n=2", flush=True)
    y = net.forward(dev(x)).cpu().numpy()
    ref = U.forward(p.astype(np.float64), x.reshape(2, R, R, R, NIN), W.UNET_LAYERS).numpy()
    ref = ref[..., :NOUT].reshape(2, R ** 3, NOUT)
    assert rel(y, ref) < 2e-2
    assert np.abs(y - ref).max() < 5e-2 * np.abs(ref).max()


def test_gradient_matches_oracle(net):
    p = W.unet_init_params(seed=4, bias_scale=0.1)
    net.set_params(p)
    x, t, w = data(2)
    print("[unet] gradient R=16 n=2", flush=True)
    loss, g = net.gradient(dev(x), dev(t), dev(w), float(w.sum()))
    lo, go = U.loss_and_grad(p.astype(np.float64), x.reshape(2, R, R, R, NIN), t.reshape(2, R, R, R, NOUT),
                             w.reshape(2, R, R, R, NOUT), float(w.sum()), W.UNET_LAYERS)
    assert abs(loss - lo) < 1e-2 * abs(lo)
    offs, n = W.unet_layout()
    bounds = [o for pair in offs for o in pair] + [n]
    errs = []
    for k, (a, b) in enumerate(zip(bounds[:-1], bounds[1:])):
        e = rel(g[a:b], go[a:b])
        cos = float(np.dot(g[a:b], go[a:b]) / (np.linalg.norm(g[a:b]) * np.linalg.norm(go[a:b]) + 1e-300))
        errs.append((k // 2, "w" if k % 2 == 0 else "b", round(e, 4), round(cos, 5)))
    print("[unet] per-layer gradient (layer, part, rel L2 error, cosine):", errs, flush=True)
    # the gradient of layer l passes 10 - l bf16-rounded backward convolutions
    for layer, part, e, cos in errs:
        assert e < 0.1 and cos > 0.995, (layer, part, e, cos)


def test_training_reduces_the_loss(net):
    net.set_params(W.unet_init_params(seed=5))
    x, t, w = data(3)
    xd, td, wd = dev(x), dev(t * 0.5 + x[..., :1] * 0.5), dev(w)
    ws = float(w.sum())
    l0 = net.train_step(xd, td, wd, ws, 1e-3)
    for _ in range(60):
        net.train_step(xd, td, wd, ws, 1e-3, want_loss=False)
    l1 = net.train_step(xd, td, wd, ws, 1e-3)
    print(f"[unet] loss {l0:.4f} -> {l1:.4f}", flush=True)
    assert np.isfinite(l1) and l1 < 0.7 * l0


def test_gradient_and_training_are_bitwise_reproducible(net):
    """Two gradients of the same batch, and two 5-step training runs from the
    same parameters, agree bit for bit (no atomics in any reduction)."""
    p = W.unet_init_params(seed=8, bias_scale=0.1)
    x, t, w = data(4)
    xd, td, wd = dev(x), dev(t), dev(w)
    ws = float(w.sum())
    print("[unet] reproducibility R=16 n=2", flush=True)
    net.set_params(p)
    l1, g1 = net.gradient(xd, td, wd, ws)
    l2, g2 = net.gradient(xd, td, wd, ws)
    assert l1 == l2 and np.array_equal(g1, g2)
    runs = []
    for _ in range(2):
        net.set_params(p)
        losses = [net.train_step(xd, td, wd, ws, 1e-3) for _ in range(5)]
        runs.append((losses, net.params()))
    assert runs[0][0] == runs[1][0]
    assert np.array_equal(runs[0][1], runs[1][1])
    assert not np.array_equal(runs[0][1], p)


def test_full_size_forward_and_gradient():
    """The network at the size the learned warm start uses (64^3 cubes; one
    sample, so the FP64 oracle finishes in seconds): forward output and every
    layer's gradient against the oracle, to the bounds above."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1804_07588_amd import surrogate
    R64 = 64
    big = surrogate.UNet(R64, 1, NIN, NOUT)
    p = W.unet_init_params(seed=6, bias_scale=0.1)
    big.set_params(p)
    rng = np.random.default_rng(7)
    x = rng.standard_normal((1, R64 ** 3, NIN)).astype(np.float32)
    t = rng.standard_normal((1, R64 ** 3, NOUT)).astype(np.float32)
    w = (rng.random((1, R64 ** 3, NOUT)) > 0.25).astype(np.float32)
    print("[unet] forward and gradient R=64 n=1", flush=True)
    y = big.forward(dev(x)).cpu().numpy()
    shape_in, shape_out = (1, R64, R64, R64, NIN), (1, R64, R64, R64, NOUT)
    ref = U.forward(p.astype(np.float64), x.reshape(shape_in), W.UNET_LAYERS).numpy()
    ref = ref[..., :NOUT].reshape(1, R64 ** 3, NOUT)
    assert rel(y, ref) < 2e-2
    loss, g = big.gradient(dev(x), dev(t), dev(w), float(w.sum()))
    lo, go = U.loss_and_grad(p.astype(np.float64), x.reshape(shape_in), t.reshape(shape_out),
                             w.reshape(shape_out), float(w.sum()), W.UNET_LAYERS)
    assert abs(loss - lo) < 1e-2 * abs(lo)
    offs, n = W.unet_layout()
    bounds = [o for pair in offs for o in pair] + [n]
    errs = []
    for k, (a, b) in enumerate(zip(bounds[:-1], bounds[1:])):
        e = rel(g[a:b], go[a:b])
        cos = float(np.dot(g[a:b], go[a:b]) / (np.linalg.norm(g[a:b]) * np.linalg.norm(go[a:b]) + 1e-300))
        errs.append((k // 2, "w" if k % 2 == 0 else "b", round(e, 4), round(cos, 5)))
    print("[unet] R=64 per-layer gradient (layer, part, rel L2 error, cosine):", errs, flush=True)
    for layer, part, e, cos in errs:
        assert e < 0.1 and cos > 0.995, (layer, part, e, cos)
    big.close()
