"""Element-by-element comparison of GPU fit outputs with the FP64 oracle.

Tolerances (FP32 GPU against FP64 oracle on the same FP32-rounded inputs):
  parameters: |d| <= 1e-4 max(|ref|, f), f = 1 cm for x, y, z, 1 rad for
              phi (compared modulo 2 pi), 0 for 1/pT and theta;
  chi2:       |d| <= 1e-3 max(ref, 1);
  covariance: element (i, j) passes when |d| <= 1e-3 |ref| or
              |d| / sqrt(ref_ii ref_jj) <= 1e-4.  The second form is for
              elements near zero (correlations that change sign, those along
              the surface normal), whose relative error is unbounded: the
              covariance is carried along the fitted state through
              state-dependent Jacobians, so the 1e-4 relative state
              difference allowed above moves every element by up to ~1e-4 of
              sqrt(C_ii C_jj) (measured: up to a few 1e-5).  The position diagonals
              are floored at 1e-4 of the track's largest position variance,
              because along the last surface's normal -- z after a plane, x or
              y when a cylinder's normal lies along an axis -- the variance
              itself is rounding noise);
  status:     flags bit-exact except FP64_FALLBACK (GPU only); the count of
              applied updates exact.
Covariance tolerances are multiplied by the conditioning of the final
crossing, 1 / cos(incidence) for a track that ends on a cylinder (1 for a
plane).  The path-length derivative ds*/dp = -(dg/dp) / (dg/ds) divides by
dg/ds = cos(incidence), so FP32 rounding in the transport of a track that
grazes its last cylinder is amplified by that factor; for almost every
track it is close to 1 (the largest seen, 43, belongs to a 0.56 GeV track
whose largest radius lies 0.1 mm outside its last layer).
Tracks whose reachability of a surface differs between FP32 and FP64 (the
surface grazes the track's largest radius), or whose hit chi2 falls on the
other side of a chi2 cut, are listed and excluded from the value comparison;
their number must stay below 1e-4 of the tracks.
"""
from __future__ import annotations

import numpy as np

PAR_F = np.array([1.0, 1.0, 1.0, 0.0, 1.0, 0.0])
IL = np.tril_indices(6)
ST_FP64_FALLBACK = 1 << 2
ST_NO_CROSSING = 1 << 0
ST_NEWTON_FAIL = 1 << 1
ST_CHI2_CUT = 1 << 7
NORM_TOL = 1e-4      # covariance error in units of sqrt(C_ii C_jj)


def incidence_condition(ref_par, final_surface) -> np.ndarray:
    """Per-track factor 1 / cos(incidence) at the final surface (1 for planes).

    final_surface: "cylinder", "plane", or a per-track array (0 cylinder,
    1 plane).  cos(incidence) on a cylinder is the radial component of the
    transverse direction, |x cos(phi) + y sin(phi)| / r, taken from the
    oracle's final state."""
    p = np.asarray(ref_par, np.float64)
    n = p.shape[0]
    if isinstance(final_surface, str):
        cyl = np.full(n, final_surface == "cylinder")
    else:
        cyl = np.asarray(final_surface) == 0
    r = np.hypot(p[:, 0], p[:, 1])
    with np.errstate(invalid="ignore", divide="ignore"):
        c = np.abs(p[:, 0] * np.cos(p[:, 4]) + p[:, 1] * np.sin(p[:, 4])) / r
    c = np.where(np.isfinite(c), c, 1.0)
    return np.where(cyl, 1.0 / np.clip(c, 1e-3, 1.0), 1.0)


def final_surface_of(par, offsets, surf_type, surf_val) -> np.ndarray:
    """0/1 kind of the surface each (oracle) final state lies on, for ragged
    fits: the last of the track's surfaces that the final position is on."""
    p = np.asarray(par, np.float64)
    n = p.shape[0]
    out = np.zeros(n, np.int64)
    r = np.hypot(p[:, 0], p[:, 1])
    for t in range(n):
        a, b = int(offsets[t]), int(offsets[t + 1])
        best = None
        for h in range(a, b):
            d = abs(r[t] - surf_val[h]) if surf_type[h] == 0 else abs(p[t, 2] - surf_val[h])
            if d < 1e-3:
                best = h
        if best is not None:
            out[t] = int(surf_type[best])
    return out


def compare(gpu: dict, ref: dict, max_excluded_frac: float = 1e-4, ctx: str = "",
            final_surface="cylinder") -> dict:
    """gpu/ref dicts with par (n,6), cov (n,21), chi2 (n,), status (n,) [ref: + nused].

    final_surface: "cylinder", "plane" or a per-track 0/1 array (see
    incidence_condition)."""
    gp, rp = np.asarray(gpu["par"], np.float64), np.asarray(ref["par"], np.float64)
    gc, rc = np.asarray(gpu["cov"], np.float64), np.asarray(ref["cov"], np.float64)
    gx, rx = np.asarray(gpu["chi2"], np.float64), np.asarray(ref["chi2"], np.float64)
    gs = np.asarray(gpu["status"]).astype(np.int64) & 0xFFFFFFFF
    rs = (np.asarray(ref["status"]).astype(np.int64) & 0xFFFFFFFF) | (np.asarray(ref["nused"]).astype(np.int64) << 8)
    n = gp.shape[0]
    flags_g = gs & ~np.int64(ST_FP64_FALLBACK)
    flags_r = rs
    geo = np.int64(ST_NO_CROSSING | ST_NEWTON_FAIL)
    # reachability disagreements near tangency, and chi2 within rounding of the cut
    excl = ((flags_g & geo) != (flags_r & geo)) | ((flags_g & ST_CHI2_CUT) != (flags_r & ST_CHI2_CUT))
    n_excl = int(excl.sum())
    assert n_excl <= max(1, int(max_excluded_frac * n)), f"{ctx}: {n_excl} reachability disagreements"
    keep = ~excl
    bad_status = np.nonzero(keep & (flags_g != flags_r))[0]
    assert bad_status.size == 0, f"{ctx}: status mismatch at {bad_status[:10]}: gpu {gs[bad_status[:5]]} ref {rs[bad_status[:5]]}"
    d = gp - rp
    d[:, 4] = np.angle(np.exp(1j * d[:, 4]))
    both_nan = np.isnan(gp) & np.isnan(rp)      # passed-through NaN of a rejected input
    d[both_nan] = 0.0
    tolp = 1e-4 * np.maximum(np.nan_to_num(np.abs(rp)), PAR_F)
    okp = (np.abs(d) <= tolp) | both_nan
    okp[~keep] = True
    assert okp.all(), _worst(f"{ctx}: params", d, tolp, okp)
    dx = np.abs(gx - rx)
    tolx = 1e-3 * np.maximum(rx, 1.0)
    okx = (dx <= tolx) | ~keep
    assert okx.all(), _worst(f"{ctx}: chi2", dx[:, None], tolx[:, None], okx[:, None])
    dc = np.abs(gc - rc)
    cnan = np.isnan(gc) & np.isnan(rc)
    dc[cnan] = 0.0
    diag = np.abs(rc[:, [0, 2, 5, 9, 14, 20]])
    # the position block has an exact null direction (the normal of the last
    # surface): z after a plane, or x / y when a cylinder's normal lies along an
    # axis.  Its diagonal is rounding noise, so the position diagonals used for
    # normalisation are floored at 1e-4 of the track's largest position variance
    diag[:, :3] = np.maximum(diag[:, :3], 1e-4 * diag[:, :3].max(1, keepdims=True))
    scale = np.sqrt(diag[:, IL[0]] * diag[:, IL[1]])
    cond = incidence_condition(rp, final_surface)[:, None]
    ok_rel = dc <= 1e-3 * np.abs(rc) * cond
    ok_norm = dc <= NORM_TOL * scale * cond
    okc = ok_rel | ok_norm | cnan
    okc[~keep] = True
    assert okc.all(), _worst(f"{ctx}: cov", dc, np.maximum(1e-3 * np.abs(rc), NORM_TOL * scale) * cond, okc)
    relp = np.abs(d) / np.maximum(np.abs(rp), np.maximum(PAR_F, 1e-30))
    normerr = np.where(keep[:, None], dc / np.maximum(scale, 1e-300), 0.0)
    return dict(n=n, excluded=n_excl, cov_norm_err_max=float(normerr.max()),
                cov_norm_err_p999=float(np.quantile(normerr, 0.999)), max_rel_par=relp[keep].max(0) if keep.any() else np.zeros(6),
                max_rel_chi2=float((dx / np.maximum(rx, 1.0))[keep].max()) if keep.any() else 0.0,
                cov_rel_pass=int(ok_rel[keep].sum()), cov_norm_only=int((ok_norm & ~ok_rel)[keep].sum()),
                fp64_fallbacks=int(((gs & ST_FP64_FALLBACK) != 0).sum()),
                max_incidence_condition=float(cond.max()) if n else 1.0)


def _worst(what, d, tol, ok):
    bad = np.argwhere(~ok)
    r = (np.abs(d) / np.maximum(tol, 1e-300))
    i = np.unravel_index(np.argmax(np.where(ok, 0, r)), r.shape)
    return f"{what}: {bad.shape[0]} failures; worst at {i}: |d|={np.abs(d)[i]:.3e} tol={tol[i]:.3e}"
