"""Training of the path-length MLP on the GPU with the library's own kernels.

Pairs (state, target cylinder) -> transverse path length come from the
seeded generator (truth states on layer l moved along the surface by
fit-like errors, paired with layer l + 1, and the fit starts paired with the
first layer; the path length of each pair from the RK4 simulation of that
state).  Features and targets are computed by the library
(p2r_mlp_features), and every optimisation step is the library's
p2r_mlp_train_step (forward and backward on the matrix cores, Adam).

    python -m paper_2401_14221_amd.learned --out CKPT [--tracks N] [--epochs E]
"""
from __future__ import annotations

import argparse
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_CKPT = os.path.join(HERE, "data", "mlp_p2r.ckpt")


def flat_params(p: dict) -> np.ndarray:
    """W1, b1, W2, b2, W3, b3 -> the library's flat parameter vector."""
    return np.concatenate([np.asarray(p[k], np.float32).reshape(-1) for k in ("W1", "b1", "W2", "b2", "W3", "b3")])


def split_params(flat: np.ndarray, n_in: int = 7, n_hid: int = 64) -> dict:
    sizes = [("W1", (n_hid, n_in)), ("b1", (n_hid,)), ("W2", (n_hid, n_hid)), ("b2", (n_hid,)),
             ("W3", (1, n_hid)), ("b3", (1,))]
    out, o = {}, 0
    for k, shp in sizes:
        n = int(np.prod(shp))
        out[k] = np.asarray(flat[o:o + n], np.float32).reshape(shp)
        o += n
    return out


def make_training_set(mlp, n_tracks: int, seed: int, device="cuda"):
    """Features x, targets t on the device (pairs without a straight-line path dropped)."""
    import torch
    from synth import events as ev
    d = ev.make_mlp_pairs(n_tracks, seed=seed)
    f = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float32, device=device)  # noqa: E731
    par, q, R, s = f(d["par"]), f(d["q"]), f(d["R"]), f(d["s"])
    x, t, sl = mlp.features(par, q, R, s_label=s)
    keep = sl > 0
    return x[keep].contiguous(), t[keep].contiguous(), dict(par=par[keep], q=q[keep], R=R[keep], s=s[keep], sl=sl[keep])


def train(ctx, n_tracks=500_000, epochs=30, batch=8192, lr=2e-3, seed=None, init=None, log=print,
          stream=None, max_seconds=None):
    """Train a fresh network; returns (mlp, history)."""
    import torch
    import paper_2401_14221_amd as p2r
    from synth import events as ev
    seed = ev.LEARNED_TRAIN_SEED if seed is None else seed
    params = init if init is not None else flat_params(ev.make_mlp_init(seed))
    mlp = p2r.Mlp(ctx, params)
    t0 = time.time()
    x, t, _ = make_training_set(mlp, n_tracks, seed)
    n = x.shape[0]
    log(f"[learned] {n} training pairs in {time.time() - t0:.1f}s")
    g = torch.Generator(device=x.device)
    g.manual_seed(seed)
    steps_per_epoch = n // batch
    total = steps_per_epoch * epochs
    loss = torch.zeros(1, device=x.device)
    hist = []
    k = 0
    t1 = time.time()
    for ep in range(epochs):
        perm = torch.randperm(n, device=x.device, generator=g)
        acc = torch.zeros(1, device=x.device)
        for b in range(steps_per_epoch):
            idx = perm[b * batch:(b + 1) * batch]
            xb, tb = x[idx].contiguous(), t[idx].contiguous()
            lr_k = lr * 0.5 * (1.0 + math.cos(math.pi * k / max(1, total)))     # cosine decay
            mlp.train_step(xb, tb, lr_k, loss_out=loss, stream=stream)
            acc += loss
            k += 1
        m = float(acc.item()) / max(1, steps_per_epoch)
        hist.append(m)
        log(f"[learned] epoch {ep}: mean loss {m:.4e} ({time.time() - t1:.1f}s)")
        if max_seconds and time.time() - t1 > max_seconds:
            break
    return mlp, hist


def proposal_quality(mlp, n_tracks=20_000, seed=2024):
    """Median |s0 - s*| of the trained proposal and of the straight line on fresh pairs."""
    import torch
    x, t, d = make_training_set(mlp, n_tracks, seed)
    y = mlp.forward(x)
    s0 = d["sl"] * (1.0 + torch.sinh(y.clamp(-8, 8)) / 100.0)
    e_mlp = (s0 - d["s"]).abs()
    e_line = (d["sl"] - d["s"]).abs()
    return dict(median_err_mlp=float(e_mlp.median()), median_err_line=float(e_line.median()),
                p99_err_mlp=float(torch.quantile(e_mlp, 0.99)), p99_err_line=float(torch.quantile(e_line, 0.99)),
                frac_within_1e3=float((e_mlp <= 1e-3).float().mean()), n=int(x.shape[0]))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=DEFAULT_CKPT)
    ap.add_argument("--tracks", type=int, default=500_000)
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--batch", type=int, default=8192)
    ap.add_argument("--lr", type=float, default=2e-3)
    a = ap.parse_args()
    import paper_2401_14221_amd as p2r
    ctx = p2r.Context(0)
    mlp, hist = train(ctx, a.tracks, a.epochs, a.batch, a.lr)
    os.makedirs(os.path.dirname(os.path.abspath(a.out)), exist_ok=True)
    mlp.save(a.out)
    print("[learned] quality", proposal_quality(mlp), flush=True)
    print(f"[learned] saved {a.out}", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
