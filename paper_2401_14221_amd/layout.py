"""AoSoA layouts of the fit's inputs and outputs (torch reshapes, no math).

Track record (28 floats): 6 parameters (x, y, z, 1/pT, phi, theta), 21
packed covariance values (lower triangle, row-major), charge (+-1.0).
Hit record (9 floats): x, y, z and the packed 3x3 covariance.

p2r: tracks [nb][28][W], hits [nb][L][9][W]   (block-outer)
p2z: tracks [nb][28][64], hits [L][nb][9][64] (layer-outer)
Lanes beyond n in the last block are zero-filled and ignored by the kernels.
"""
from __future__ import annotations

import torch


def n_blocks(n: int, W: int) -> int:
    return (n + W - 1) // W


def _pad_rows(x: torch.Tensor, n_pad: int) -> torch.Tensor:
    if n_pad == x.shape[0]:
        return x
    pad = torch.zeros((n_pad - x.shape[0],) + tuple(x.shape[1:]), dtype=x.dtype, device=x.device)
    return torch.cat([x, pad], 0)


def pack_tracks(par, cov, q, W: int, device=None) -> torch.Tensor:
    """(n,6), (n,21), (n,) -> [nb, 28, W] float32."""
    par = torch.as_tensor(par, dtype=torch.float32, device=device)
    cov = torch.as_tensor(cov, dtype=torch.float32, device=par.device)
    q = torch.as_tensor(q, dtype=torch.float32, device=par.device)
    n = par.shape[0]
    rec = torch.cat([par, cov, q[:, None]], 1)                      # [n, 28]
    nb = n_blocks(n, W)
    rec = _pad_rows(rec, nb * W).reshape(nb, W, 28).transpose(1, 2)  # [nb, 28, W]
    return rec.contiguous()


def unpack_tracks(t: torch.Tensor, n: int):
    """[nb, 28, W] -> par (n,6), cov (n,21), q (n,)."""
    nb, f, W = t.shape
    assert f == 28
    rec = t.transpose(1, 2).reshape(nb * W, 28)[:n]
    return rec[:, :6], rec[:, 6:27], rec[:, 27]


def pack_hits_p2r(hits, hitcov, W: int, device=None) -> torch.Tensor:
    """(n,L,3), (n,L,6) -> [nb, L, 9, W] float32."""
    h = torch.as_tensor(hits, dtype=torch.float32, device=device)
    v = torch.as_tensor(hitcov, dtype=torch.float32, device=h.device)
    n, L, _ = h.shape
    rec = torch.cat([h, v], 2)                                      # [n, L, 9]
    nb = n_blocks(n, W)
    rec = _pad_rows(rec, nb * W).reshape(nb, W, L, 9).permute(0, 2, 3, 1)
    return rec.contiguous()


def pack_hits_p2z(hits, hitcov, device=None) -> torch.Tensor:
    """(n,L,3), (n,L,6) -> [L, nb, 9, 64] float32."""
    W = 64
    h = torch.as_tensor(hits, dtype=torch.float32, device=device)
    v = torch.as_tensor(hitcov, dtype=torch.float32, device=h.device)
    n, L, _ = h.shape
    rec = torch.cat([h, v], 2)
    nb = n_blocks(n, W)
    rec = _pad_rows(rec, nb * W).reshape(nb, W, L, 9).permute(2, 0, 3, 1)
    return rec.contiguous()
