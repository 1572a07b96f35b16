"""Pins of the U-Net oracle (CPU, FP64): the convolution's weight layout and
taps against a brute-force loop, pooling and upsampling against their
definitions, a closed form with zero weights, and the autograd parameter
gradient against central finite differences on a narrow network."""
import numpy as np
import torch

from oracle import unet_oracle as U
from paper_1804_07588_amd import workloads as W

NARROW = [(4, 4, 0, 1), (4, 4, 0, 1), (4, 4, 1, 1), (4, 4, 1, 1), (4, 6, 2, 1), (6, 6, 2, 1),
          (10, 4, 1, 1), (4, 4, 1, 1), (8, 4, 0, 1), (4, 4, 0, 1), (4, 4, 0, 0)]


def test_conv_matches_brute_force():
    rng = np.random.default_rng(3)
    R, ci, co = 4, 3, 2
    x = rng.standard_normal((1, R, R, R, ci))
    p = rng.standard_normal(co * 27 * ci + co)
    y = U.conv(torch.as_tensor(x).permute(0, 4, 1, 2, 3), torch.as_tensor(p), 0, co * 27 * ci, ci, co)
    y = y.permute(0, 2, 3, 4, 1).numpy()
    Wt = p[:co * 27 * ci].reshape(co, 27, ci)
    b = p[co * 27 * ci:]
    ref = np.zeros((1, R, R, R, co))
    for z in range(R):
        for yy in range(R):
            for xx in range(R):
                for o in range(co):
                    s = b[o]
                    for tap in range(27):
                        dz, dy, dx = tap // 9 - 1, (tap // 3) % 3 - 1, tap % 3 - 1
                        zz, y2, x2 = z + dz, yy + dy, xx + dx
                        if 0 <= zz < R and 0 <= y2 < R and 0 <= x2 < R:
                            s += Wt[o, tap] @ x[0, zz, y2, x2]
                    ref[0, z, yy, xx, o] = s
    assert np.abs(y - ref).max() < 1e-12


def test_pool_and_upsample_definitions():
    x = torch.arange(2 * 4 * 4 * 4, dtype=torch.float64).reshape(1, 2, 4, 4, 4)
    p = torch.nn.functional.avg_pool3d(x, 2)
    ref = x.reshape(1, 2, 2, 2, 2, 2, 2, 2).mean(dim=(3, 5, 7))
    assert torch.allclose(p, ref)
    u = torch.nn.functional.interpolate(p, scale_factor=2, mode="nearest")
    idx = torch.arange(4) // 2
    assert torch.equal(u, p[:, :, idx][:, :, :, idx][:, :, :, :, idx])


def test_zero_weights_give_the_head_bias():
    offs, n = W.unet_layout(NARROW)
    rng = np.random.default_rng(5)
    p = np.zeros(n)
    hb = rng.standard_normal(4)
    p[offs[-1][1]:offs[-1][1] + 4] = hb
    x = rng.standard_normal((2, 8, 8, 8, 3))
    y = U.forward(p, x, NARROW, cpad=4).numpy()
    assert np.abs(y - hb).max() < 1e-15
    t = rng.standard_normal((2, 8, 8, 8, 2))
    w = (rng.random((2, 8, 8, 8, 2)) > 0.3).astype(float)
    loss, g = U.loss_and_grad(p, x, t, w, w.sum(), NARROW, cpad=4)
    # closed forms: L = sum w (b - t)^2 / W, dL/db_c = 2 sum w (b_c - t) / W
    assert abs(loss - (w * (hb[:2] - t) ** 2).sum() / w.sum()) < 1e-12
    gb = g[offs[-1][1]:offs[-1][1] + 4]
    assert np.allclose(gb[:2], 2 * (w * (hb[:2] - t)).sum(axis=(0, 1, 2, 3)) / w.sum(), atol=1e-12)
    assert np.all(gb[2:] == 0)


def test_gradient_matches_finite_differences():
    offs, n = W.unet_layout(NARROW)
    rng = np.random.default_rng(11)
    p = W.unet_init_params(seed=4, layers=NARROW, bias_scale=0.1).astype(np.float64)
    x = rng.standard_normal((1, 8, 8, 8, 3))
    t = rng.standard_normal((1, 8, 8, 8, 3))
    w = np.ones_like(t)
    _, g = U.loss_and_grad(p, x, t, w, w.sum(), NARROW, cpad=4)
    # one weight and one bias of every layer
    picks = []
    for wo, bo in offs:
        picks += [wo + int(rng.integers(bo - wo)), bo]
    h = 1e-6
    for k in picks:
        e = np.zeros(n)
        e[k] = h
        lp, _ = U.loss_and_grad(p + e, x, t, w, w.sum(), NARROW, cpad=4)
        lm, _ = U.loss_and_grad(p - e, x, t, w, w.sum(), NARROW, cpad=4)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(g[k])), (k, fd, g[k])


def test_oracle_layout_is_the_headers():
    """The oracle reads the network's channel counts from the header and
    lays the parameters out by the header's statement; the product's table
    must agree with both."""
    convs = U.header_convs()
    assert len(convs) == 11
    assert [(ci, co) for ci, co, _, _ in W.UNET_LAYERS] == convs
    offs, n = U.param_offsets(convs)
    p_offs, p_n = W.unet_layout()
    assert offs == [tuple(o) for o in p_offs] and n == p_n == 1825504
