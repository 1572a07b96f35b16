"""Oracle of the learned warm start's network (test infrastructure only).

A plain FP64 CPU implementation of the 3-D U-Net declared in
include/fdlbm_unet.h, written with PyTorch CPU primitives (conv3d, average
pooling, nearest upsampling, concatenation) and autograd for the parameter
gradient.  It shares nothing with the HIP kernels; it takes the parameter
vector in the same documented layout.  The network is an addition to the
paper's method (the paper has no learned component), so its definition is
the header's, and the pins in tests/test_unet_oracle.py check this code
against brute-force loops and finite differences.
"""
from __future__ import annotations

import os
import re

import numpy as np
import torch
import torch.nn.functional as F

torch.set_num_threads(max(1, min(8, torch.get_num_threads())))


HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include",
                      "fdlbm_unet.h")


def header_convs(path: str = HEADER) -> list:
    """(c_in, c_out) of every convolution, in the order the header's network
    description lists them ("conv a->b")."""
    with open(path) as fh:
        text = fh.read()
    desc = text[text.index("Network"):text.index("Parameters:")]
    return [(int(a), int(b)) for a, b in re.findall(r"conv (\d+)->(\d+)", desc)]


def param_offsets(layers) -> tuple[list, int]:
    """[(weight offset, bias offset)] per convolution and the parameter count,
    from the header's statement of the layout: for each convolution in order,
    its weights W[c_out][tap][c_in], then its biases [c_out]."""
    offs, p = [], 0
    for layer in layers:
        ci, co = layer[0], layer[1]
        offs.append((p, p + co * 27 * ci))
        p += co * 27 * ci + co
    return offs, p


def _w(params: torch.Tensor, off: int, ci: int, co: int) -> torch.Tensor:
    # W[co][tap][ci], tap = 9 kd + 3 kh + kw -> torch layout [co][ci][kd][kh][kw]
    return params[off:off + co * 27 * ci].reshape(co, 3, 3, 3, ci).permute(0, 4, 1, 2, 3)


def conv(x: torch.Tensor, params: torch.Tensor, w_off: int, b_off: int, ci: int, co: int) -> torch.Tensor:
    """3x3x3 cross-correlation with zero padding 1 of x [n][ci][R][R][R]."""
    return F.conv3d(x, _w(params, w_off, ci, co), params[b_off:b_off + co], padding=1)


def forward(params, x, layers, cpad: int = 32) -> torch.Tensor:
    """x: [n][R][R][R][c_in] (channels last, c_in <= cpad), float64 tensor or
    array; returns the head output [n][R][R][R][c_out of the head]."""
    p = params if isinstance(params, torch.Tensor) else torch.as_tensor(np.asarray(params, np.float64))
    xt = x if isinstance(x, torch.Tensor) else torch.as_tensor(np.asarray(x, np.float64))
    xt = xt.permute(0, 4, 1, 2, 3)
    if xt.shape[1] < cpad:
        xt = F.pad(xt, (0, 0, 0, 0, 0, 0, 0, cpad - xt.shape[1]))
    offs, _ = param_offsets(layers)

    def L(i, h):
        ci, co, _, relu = layers[i]
        y = conv(h, p, offs[i][0], offs[i][1], ci, co)
        return torch.relu(y) if relu else y

    a1 = L(1, L(0, xt))
    a3 = L(3, L(2, F.avg_pool3d(a1, 2)))
    a5 = L(5, L(4, F.avg_pool3d(a3, 2)))
    c2 = torch.cat([F.interpolate(a5, scale_factor=2, mode="nearest"), a3], dim=1)
    a7 = L(7, L(6, c2))
    c1 = torch.cat([F.interpolate(a7, scale_factor=2, mode="nearest"), a1], dim=1)
    out = L(10, L(9, L(8, c1)))
    return out.permute(0, 2, 3, 4, 1)


def loss_and_grad(params, x, t, w, wsum: float, layers, cpad: int = 32):
    """L = sum w (y - t)^2 / wsum over the first t.shape[-1] output channels
    (t, w: [n][R][R][R][n_out]) and dL/dparams (float64)."""
    p = torch.tensor(np.asarray(params, np.float64), requires_grad=True)
    y = forward(p, x, layers, cpad)
    tt = torch.as_tensor(np.asarray(t, np.float64))
    ww = torch.as_tensor(np.asarray(w, np.float64))
    nout = tt.shape[-1]
    loss = (ww * (y[..., :nout] - tt) ** 2).sum() / wsum
    loss.backward()
    return float(loss.detach()), p.grad.detach().numpy().copy()
