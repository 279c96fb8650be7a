"""FP64 NumPy reference of the path-length MLP (test infrastructure only).

Network: x[7] -> relu(W1 x + b1)[64] -> relu(W2 h1 + b2)[64] -> W3 h2 + b3.
Loss: mean squared error, L = mean((y - t)^2).  Optimiser: Adam.
Features: the dimensionless description of a (state, cylinder) pair that
the path-length proposal consumes, and the residual target it predicts.

With ``bf16=True`` the operands that go through the matrix cores are
rounded to bfloat16 (round to nearest even) before an FP64 product: x and
W1 (layer 1), h1 and W2 (layer 2), dz2 and W2 (dh1 = W2^T dz2 in the
backward pass), dz2 and h1 (dW2 = dz2^T h1), dz1 and x (dW1 = dz1^T x).
Biases, the last layer and the bias-gradient sums stay unrounded.  This
reproduces what the matrix cores consume and leaves only the accumulation
order as a difference.
"""
from __future__ import annotations

import numpy as np

KAPPA = 2.99792458e-3
TARGET_SCALE = 100.0          # the network predicts asinh(100 * (s / s_line - 1))


def bf16_round(a):
    """Round float values to the nearest bfloat16 (ties to even), as float64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    return np.where(np.isfinite(f), out, f.astype(np.float64))


def _op(a, bf16):
    return bf16_round(a) if bf16 else np.asarray(a, dtype=np.float64)


def forward(params, x, bf16=False):
    """Returns y [B] and the cache of intermediates."""
    W1, b1, W2, b2, W3, b3 = (np.asarray(params[k], np.float64) for k in ("W1", "b1", "W2", "b2", "W3", "b3"))
    x = np.asarray(x, np.float64)
    z1 = _op(x, bf16) @ _op(W1, bf16).T + b1
    h1 = np.maximum(z1, 0.0)
    z2 = _op(h1, bf16) @ _op(W2, bf16).T + b2
    h2 = np.maximum(z2, 0.0)
    y = (h2 @ W3.T)[:, 0] + b3[0]
    return y, dict(x=x, z1=z1, h1=h1, z2=z2, h2=h2)


def loss_and_grads(params, x, t, bf16=False):
    """MSE loss and its gradients with respect to every parameter."""
    y, c = forward(params, x, bf16)
    B = y.shape[0]
    W2, W3 = np.asarray(params["W2"], np.float64), np.asarray(params["W3"], np.float64)
    d = y - np.asarray(t, np.float64)
    loss = float(np.mean(d * d))
    dy = 2.0 * d / B                                   # dL/dy
    g = {}
    g["W3"] = (dy @ c["h2"])[None, :]
    g["b3"] = np.array([dy.sum()])
    dh2 = dy[:, None] * W3[0][None, :]
    dz2 = dh2 * (c["z2"] > 0)
    g["W2"] = _op(dz2, bf16).T @ _op(c["h1"], bf16)
    g["b2"] = dz2.sum(0)
    dh1 = _op(dz2, bf16) @ _op(W2, bf16)
    dz1 = dh1 * (c["z1"] > 0)
    g["W1"] = _op(dz1, bf16).T @ _op(c["x"], bf16)
    g["b1"] = dz1.sum(0)
    return loss, g


def adam_step(params, grads, state, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (bias-corrected) on FP64 copies; returns new params/state."""
    t = state.get("t", 0) + 1
    new_p, new_s = {}, {"t": t}
    for k, p in params.items():
        m = beta1 * state.get("m_" + k, 0.0) + (1 - beta1) * grads[k]
        v = beta2 * state.get("v_" + k, 0.0) + (1 - beta2) * grads[k] ** 2
        mh = m / (1 - beta1 ** t)
        vh = v / (1 - beta2 ** t)
        new_p[k] = np.asarray(p, np.float64) - lr * mh / (np.sqrt(vh) + eps)
        new_s["m_" + k], new_s["v_" + k] = m, v
    return new_p, new_s


def features(par, q, R, bz=3.8):
    """The 7 features of a (state, target cylinder) pair and s_line.

    With r0 = |(x, y)|, the straight-line path to |xy| = R is
    s_line = (R^2 - r0^2) / (b + sqrt(b^2 + R^2 - r0^2)), b = x cos(phi) + y sin(phi);
    a = y cos(phi) - x sin(phi); omega = -q KAPPA B / pT.  Features:
      [r0/R, b/R, a/R, omega R, s_line/R, omega s_line, omega a].
    """
    par = np.asarray(par, np.float64)
    x, y, ipt, phi = par[:, 0], par[:, 1], par[:, 3], par[:, 4]
    R = np.asarray(R, np.float64)
    c, s = np.cos(phi), np.sin(phi)
    b = x * c + y * s
    a = y * c - x * s
    r0sq = x * x + y * y
    dr2 = R * R - r0sq
    sline = dr2 / (b + np.sqrt(b * b + dr2))
    w = -np.asarray(q, np.float64) * KAPPA * bz * ipt
    f = np.stack([np.sqrt(r0sq) / R, b / R, a / R, w * R, sline / R, w * sline, w * a], 1)
    return f, sline


def target(s, sline):
    """asinh(100 (s / s_line - 1)): linear near 0, logarithmic in the rare large tails."""
    return np.arcsinh(TARGET_SCALE * (np.asarray(s) / sline - 1.0))


def proposal(y, sline):
    return sline * (1.0 + np.sinh(np.asarray(y)) / TARGET_SCALE)
