"""Driver of the learned warm start: steady states of many packed beds from
batched runs of the method, training of the U-Net on them, and runs to the
steady-state residual from a cold start or from the network's prediction.
Control flow only: every step runs in the library's kernels."""
from __future__ import annotations

import sys
import time

import numpy as np

from . import fdlbm, surrogate, workloads as W


def make_sims(cfgs, precision, stream, inits=None, log=None):
    sims = []
    for k, c in enumerate(cfgs):
        init = W.uniform_init(c) if inits is None else inits[k]
        sims.append(fdlbm.Sim(c, precision=precision, init=init, stream=stream))
        if log and (k + 1) % 8 == 0:
            print(f"# {log}: {k + 1}/{len(cfgs)} contexts", file=sys.stderr, flush=True)
    return sims


def run_to_steady(sims, tol: float, max_steps: int, check: int = 100, autotune_steps: int = 5,
                  log: str | None = None) -> dict:
    """Advance the samples together (one batch) until each one's residual,
    checked every `check` steps, is <= tol; converged or unstable samples are
    frozen.  Returns per-sample steps, convergence and instability flags,
    the last residuals, the tuned grids and the elapsed seconds (including
    the autotuner's steps, excluding nothing else)."""
    import torch
    S = len(sims)
    B = fdlbm.Batch(sims)
    steps = np.zeros(S, dtype=np.int64)
    done = np.zeros(S, dtype=bool)
    failed = np.zeros(S, dtype=bool)
    last_r = np.full(S, np.inf)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tuned = B.autotune(autotune_steps) if autotune_steps else None
    B.step(1)
    for s in sims:
        s.residual()  # first snapshots
    last = time.perf_counter()
    while not done.all():
        B.step(check)
        newly = []
        for k, s in enumerate(sims):
            if done[k]:
                continue
            r = s.residual()
            last_r[k] = r["max"]
            o = s.observe()
            steps[k] = o["step"]
            if o["bad"]:
                failed[k] = True   # unstable: frozen, reported, never converges
                newly.append(k)
            elif r["max"] <= tol:
                newly.append(k)
        if newly:
            done[newly] = True
            if not done.all():
                B.set_active(~done)
        if not done.all() and steps[~done].max() >= max_steps:
            break
        if log and time.perf_counter() - last > 30:
            print(f"# {log}: {int(done.sum())}/{S} done, step {int(steps.max())}", file=sys.stderr, flush=True)
            last = time.perf_counter()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    B.close()
    return dict(steps=steps, converged=done & ~failed, failed=failed, residual=last_r, tuned=tuned,
                seconds=elapsed)


def dataset(sims, cfgs):
    """Features and raw targets / weights of converged runs."""
    X = np.stack([surrogate.features(c) for c in cfgs])
    TW = [surrogate.steady_targets(s, c) for s, c in zip(sims, cfgs)]
    return X, [t for t, _ in TW], [w for _, w in TW]


def augment(x, t, w, R, flip_sign, rng):
    """A symmetry of the beds applied to a mini-batch on the device: periodic
    shifts along y and z (the beds are periodic there) and reflections of y
    and z, with the reflected velocity component's sign flipped.  flip_sign:
    per target channel (a, b) such that a reflected normalised value is
    a * t + b, or None for channels a reflection leaves unchanged."""
    import torch
    b = x.shape[0]
    sh = lambda a: a.view(b, R, R, R, a.shape[-1])  # [n][z][y][x][c]
    xs, ts, ws = sh(x), sh(t), sh(w)
    dz, dy = int(rng.integers(R)), int(rng.integers(R))
    xs, ts, ws = (torch.roll(a, shifts=(dz, dy), dims=(1, 2)) for a in (xs, ts, ws))
    for dim, key in ((1, "z"), (2, "y")):
        if rng.random() < 0.5:
            xs, ts, ws = (torch.flip(a, dims=(dim,)) for a in (xs, ts, ws))
            c, (a, off) = flip_sign[key]
            ts = ts.clone()
            ts[..., c] = a * ts[..., c] + off
    return (xs.reshape(x.shape).contiguous(), ts.reshape(t.shape).contiguous(),
            ws.reshape(w.shape).contiguous())


def train(net, X, T, Wt, epochs: int, batch: int, lr: float, seed: int = 0, log: str | None = None,
          norm=None, ns: int = 5) -> dict:
    """Adam on the weighted squared error of the normalised targets, in
    shuffled mini-batches; the learning rate decays as a cosine to lr/20.
    X [S][R^3][c_in], T and Wt [S][R^3][n_out] (normalised), numpy.  With
    `norm` (the targets' Normaliser) every mini-batch is a random symmetry of
    the beds (augment)."""
    import torch
    S = X.shape[0]
    R = net.R
    flip = None
    if norm is not None:
        # velocity channels ns+1 (x), ns+2 (y), ns+3 (z): reflecting y negates
        # u_y, i.e. t -> -t - 2 mean/std in normalised units
        cy, cz = ns + 2, ns + 3
        flip = {"y": (cy, (-1.0, float(-2 * norm.mean[cy] / norm.std[cy]))),
                "z": (cz, (-1.0, float(-2 * norm.mean[cz] / norm.std[cz])))}
    xd = torch.as_tensor(X).cuda()
    td = torch.as_tensor(T).cuda()
    wd = torch.as_tensor(Wt).cuda()
    rng = np.random.default_rng(seed)
    n_it = epochs * ((S + batch - 1) // batch)
    it, losses = 0, []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    last = t0
    for ep in range(epochs):
        order = rng.permutation(S)
        ep_loss = []
        for b0 in range(0, S, batch):
            idx = torch.as_tensor(order[b0:b0 + batch]).cuda()
            x, t, w = xd[idx].contiguous(), td[idx].contiguous(), wd[idx].contiguous()
            if flip is not None:
                x, t, w = augment(x, t, w, R, flip, rng)
            cur = lr * (0.05 + 0.95 * 0.5 * (1 + np.cos(np.pi * it / max(1, n_it - 1))))
            want = b0 == 0
            l = net.train_step(x, t, w, float(w.sum().item()), cur, want_loss=want)
            if want:
                ep_loss.append(l)
            it += 1
        losses.append(float(np.mean(ep_loss)))
        if log and time.perf_counter() - last > 20:
            print(f"# {log}: epoch {ep + 1}/{epochs} loss {losses[-1]:.4f}", file=sys.stderr, flush=True)
            last = time.perf_counter()
    torch.cuda.synchronize()
    return dict(seconds=time.perf_counter() - t0, losses=losses, iterations=it)


def predict_inits(net, norm, cfgs):
    """Warm-start fields of each bed from the network's prediction."""
    import torch
    out = []
    for c in cfgs:
        x = torch.as_tensor(surrogate.features(c)[None]).cuda().contiguous()
        y = net.forward(x).cpu().numpy()[0]
        out.append(surrogate.warm_init(c, norm.decode(y)))
    return out
