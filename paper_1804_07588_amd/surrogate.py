"""Python binding of the learned warm start (include/fdlbm_unet.h): argument
marshalling only, every step runs in the library's HIP kernels.  Also the
feature / target encoding between lattice fields and network channels."""
from __future__ import annotations

import ctypes as ct

import numpy as np

from . import fdlbm
from .fdlbm import FdlbmError, OK, lib

UNET_EXPORTS = ["fdlbm_unet_create", "fdlbm_unet_destroy", "fdlbm_unet_last_error",
                "fdlbm_unet_param_count", "fdlbm_unet_workspace_bytes", "fdlbm_unet_bind_workspace",
                "fdlbm_unet_set_params", "fdlbm_unet_get_params", "fdlbm_unet_forward",
                "fdlbm_unet_gradient", "fdlbm_unet_train_step"]

_bound = False


def _L():
    global _bound
    L = lib()
    if not _bound:
        vp, fp, dp = ct.c_void_p, ct.POINTER(ct.c_float), ct.POINTER(ct.c_double)
        L.fdlbm_unet_create.argtypes = [ct.c_int, ct.c_int, ct.c_int, ct.c_int, vp, ct.POINTER(vp)]
        L.fdlbm_unet_destroy.argtypes = [vp]
        L.fdlbm_unet_destroy.restype = None
        L.fdlbm_unet_last_error.argtypes = [vp]
        L.fdlbm_unet_last_error.restype = ct.c_char_p
        L.fdlbm_unet_param_count.argtypes = [vp, ct.POINTER(ct.c_size_t)]
        L.fdlbm_unet_workspace_bytes.argtypes = [vp, ct.POINTER(ct.c_size_t)]
        L.fdlbm_unet_bind_workspace.argtypes = [vp, vp, ct.c_size_t]
        L.fdlbm_unet_set_params.argtypes = [vp, fp, ct.c_size_t]
        L.fdlbm_unet_get_params.argtypes = [vp, fp, ct.c_size_t]
        L.fdlbm_unet_forward.argtypes = [vp, vp, ct.c_int, vp]
        L.fdlbm_unet_gradient.argtypes = [vp, vp, vp, vp, ct.c_int, ct.c_double, dp, fp]
        L.fdlbm_unet_train_step.argtypes = [vp, vp, vp, vp, ct.c_int, ct.c_double, ct.c_float, dp]
        _bound = True
    return L


def _p(t) -> ct.c_void_p:
    return ct.c_void_p(t.data_ptr())


class UNet:
    """The network on the current HIP device.  Tensors passed to the methods
    are torch float32 CUDA tensors, contiguous, [n][R^3][channels]."""

    def __init__(self, R: int, n_max: int, c_in: int, n_out: int, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise FdlbmError(fdlbm.E_STATE, "no HIP device available")
        L = _L()
        self.R, self.n_max, self.c_in, self.n_out = R, n_max, c_in, n_out
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = ct.c_void_p()
        rc = L.fdlbm_unet_create(R, n_max, c_in, n_out, ct.c_void_p(self.stream.cuda_stream), ct.byref(h))
        if rc != OK:
            raise FdlbmError(rc, "fdlbm_unet_create rejected the shape")
        self.h = h
        n, nb = ct.c_size_t(), ct.c_size_t()
        self._check(L.fdlbm_unet_param_count(h, ct.byref(n)))
        self._check(L.fdlbm_unet_workspace_bytes(h, ct.byref(nb)))
        self.n_params = n.value
        with torch.cuda.stream(self.stream):
            self.workspace = torch.empty(nb.value + 256, dtype=torch.uint8, device="cuda")
        aligned = (self.workspace.data_ptr() + 255) & ~255
        self._check(L.fdlbm_unet_bind_workspace(h, ct.c_void_p(aligned), nb.value))

    def _check(self, rc: int):
        if rc != OK:
            raise FdlbmError(rc, _L().fdlbm_unet_last_error(self.h).decode())

    def _shape_ok(self, t, ch):
        n = t.shape[0]
        if t.dtype.__str__() != "torch.float32" or not t.is_cuda or not t.is_contiguous() or \
                tuple(t.shape[1:]) != (self.R ** 3, ch) or not 1 <= n <= self.n_max:
            raise ValueError(f"expected a contiguous CUDA float32 tensor [n][{self.R ** 3}][{ch}]")
        return n

    def set_params(self, p: np.ndarray):
        a = np.ascontiguousarray(p, dtype=np.float32)
        self._check(_L().fdlbm_unet_set_params(self.h, a.ctypes.data_as(ct.POINTER(ct.c_float)), a.size))

    def params(self) -> np.ndarray:
        a = np.empty(self.n_params, dtype=np.float32)
        self._check(_L().fdlbm_unet_get_params(self.h, a.ctypes.data_as(ct.POINTER(ct.c_float)), a.size))
        return a

    def forward(self, x):
        import torch
        n = self._shape_ok(x, self.c_in)
        y = torch.empty((n, self.R ** 3, self.n_out), dtype=torch.float32, device=x.device)
        self._check(_L().fdlbm_unet_forward(self.h, _p(x), n, _p(y)))
        self.stream.synchronize()
        return y

    def gradient(self, x, t, w, wsum: float):
        n = self._shape_ok(x, self.c_in)
        self._shape_ok(t, self.n_out)
        self._shape_ok(w, self.n_out)
        loss = ct.c_double()
        g = np.empty(self.n_params, dtype=np.float32)
        self._check(_L().fdlbm_unet_gradient(self.h, _p(x), _p(t), _p(w), n, float(wsum), ct.byref(loss),
                                             g.ctypes.data_as(ct.POINTER(ct.c_float))))
        return loss.value, g

    def train_step(self, x, t, w, wsum: float, lr: float, want_loss: bool = True):
        n = self._shape_ok(x, self.c_in)
        loss = ct.c_double()
        self._check(_L().fdlbm_unet_train_step(self.h, _p(x), _p(t), _p(w), n, float(wsum), float(lr),
                                               ct.byref(loss) if want_loss else None))
        return loss.value if want_loss else None

    def close(self):
        if getattr(self, "h", None):
            _L().fdlbm_unet_destroy(self.h)
            self.h = None
            self.workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# encoding between a packed bed and the network's channels
# ---------------------------------------------------------------------------
# inputs: solid mask, x / (R - 1), body force / 1e-5
N_IN = 3
# outputs: mole fractions of the ns species, temperature, velocity (3)


def features(cfg: dict) -> np.ndarray:
    """Network input of a packed bed: [R^3][3] float32 (position index
    x + R (y + R z))."""
    nz, ny, nx = cfg["nz"], cfg["ny"], cfg["nx"]
    m = np.asarray(cfg["mask"], np.float32).reshape(nz, ny, nx)
    xs = np.broadcast_to(np.arange(nx, dtype=np.float32) / (nx - 1), (nz, ny, nx))
    f = np.full((nz, ny, nx), cfg["flow"]["F"][0] / 1e-5, np.float32)
    return np.stack([m, xs, f], axis=-1).reshape(-1, N_IN)


def steady_targets(sim, cfg: dict) -> tuple[np.ndarray, np.ndarray]:
    """Raw targets of a converged run: [R^3][ns + 4] (X_j, T, u) and the
    weights (1 on gas nodes for X and u; 1 everywhere for T, which holds the
    solid temperature on solid nodes)."""
    ns = len(cfg["species"]["M"])
    M = np.asarray(cfg["species"]["M"], np.float64)
    kind = sim.field(fdlbm.FIELD_KIND)
    gas = (kind == 0) | (kind >= 3)
    rho = np.stack([sim.field(fdlbm.FIELD_RHO, j) for j in range(ns)])
    C = rho / M[:, None]
    X = np.where(gas, C / np.maximum(C.sum(axis=0), 1e-300), 0.0)
    T = np.where(gas, sim.field(fdlbm.FIELD_T), sim.field(fdlbm.FIELD_TS))
    T = np.where(kind == 2, sim.field(fdlbm.FIELD_TS), T)
    u = np.stack([np.where(gas, sim.field(fdlbm.FIELD_U, a), 0.0) for a in range(3)])
    t = np.concatenate([X, T[None], u]).T.astype(np.float32)
    w = np.zeros_like(t)
    w[gas, :ns] = 1.0
    w[:, ns] = 1.0
    w[gas, ns + 1:] = 1.0
    return t, w


class Normaliser:
    """Per-channel affine map of the targets (mean and spread over the
    weighted training entries), so that every channel has unit scale."""

    def __init__(self, targets: list, weights: list):
        t = np.concatenate(targets)
        w = np.concatenate(weights)
        s = np.maximum(w.sum(axis=0), 1.0)
        self.mean = (t * w).sum(axis=0) / s
        self.std = np.sqrt(((t - self.mean) ** 2 * w).sum(axis=0) / s)
        self.std = np.where(self.std > 0, self.std, 1.0)
        on = w > 0
        self.lo = np.array([t[on[:, c], c].min() if on[:, c].any() else -np.inf for c in range(t.shape[1])])
        self.hi = np.array([t[on[:, c], c].max() if on[:, c].any() else np.inf for c in range(t.shape[1])])

    def encode(self, t):
        return ((t - self.mean) / self.std).astype(np.float32)

    def decode(self, y):
        """Physical values, clamped to the range of the training targets: an
        unseen value (e.g. a trace species' mole fraction below its inlet
        level) would put a steep, unphysical gradient into the warm start,
        and the diffusion velocity of a nearly absent species then makes its
        equilibrium negative within a step."""
        return np.clip(y * self.std + self.mean, self.lo, self.hi)


def smooth_gas(field: np.ndarray, gas: np.ndarray, shape, passes: int) -> np.ndarray:
    """`passes` sweeps of the mean over each gas node and its gas face
    neighbours (x closed, y and z periodic); other nodes keep their values.
    field: [n] or [n][c] over nodes x + nx (y + ny z)."""
    nz, ny, nx = shape
    f = field.reshape(nz, ny, nx, -1).astype(np.float64)
    g = gas.reshape(nz, ny, nx, 1).astype(np.float64)
    for _ in range(passes):
        acc, cnt = f * g, g.copy()
        for ax, per in ((0, True), (1, True), (2, False)):
            for d in (1, -1):
                fs, gs = np.roll(f * g, d, axis=ax), np.roll(g, d, axis=ax)
                if not per:
                    idx = [slice(None)] * 4
                    idx[ax] = 0 if d == 1 else -1
                    gs[tuple(idx)] = 0.0
                    fs[tuple(idx)] = 0.0
                acc += fs
                cnt += gs
        f = np.where(g > 0, acc / np.maximum(cnt, 1.0), f)
    return f.reshape(field.shape)


def warm_init(cfg: dict, pred: np.ndarray, passes: int = 4) -> dict:
    """Initial fields for fdlbm_init_fields from a decoded prediction
    [R^3][ns + 4]: mole fractions and velocity smoothed over the gas
    (`passes` neighbour-mean sweeps: the network's node-to-node noise puts
    steep gradients into trace species, whose diffusion velocities then turn
    their equilibria negative within a few steps), densities from the mole
    fractions at the inlet pressure and the predicted temperature, solid
    temperature = predicted T."""
    ns = len(cfg["species"]["M"])
    gas = np.asarray(cfg["mask"]).reshape(-1) == 0
    shape = (cfg["nz"], cfg["ny"], cfg["nx"])
    if passes:
        pred = pred.copy()
        pred[:, :ns] = smooth_gas(pred[:, :ns], gas, shape, passes)
        pred[:, ns + 1:ns + 4] = smooth_gas(pred[:, ns + 1:ns + 4], gas, shape, passes)
    M = np.asarray(cfg["species"]["M"], np.float64)
    X = np.clip(pred[:, :ns].T.astype(np.float64), 1e-6, None)
    X /= X.sum(axis=0, keepdims=True)
    T = np.clip(pred[:, ns].astype(np.float64), 0.2, 0.5)
    C = cfg["flow"]["p_in"] / T
    rho = M[:, None] * X * C[None, :]
    u = pred[:, ns + 1:ns + 4].T.astype(np.float64)
    kind_solid = np.asarray(cfg["mask"]).reshape(-1) == 1
    u[:, kind_solid] = 0.0
    return dict(rho=rho, u=u, T=T, Ts=T.copy())
