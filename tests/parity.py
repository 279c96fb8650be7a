"""Element-by-element comparison of GPU fit outputs with the FP64 oracle.

Tolerances (FP32 GPU against FP64 oracle on the same FP32-rounded inputs):
  parameters: |d| <= 1e-4 max(|ref|, f), f = 1 cm for x, y, z, 1 rad for
              phi (compared modulo 2 pi), 0 for 1/pT and theta;
  chi2:       |d| <= 1e-3 max(ref, 1);
  covariance: element (i, j) passes when |d| <= 1e-3 |ref| or
              |d| / sqrt(ref_ii ref_jj) <= NORM_TOL.  The second form is for
              elements near zero (correlations that change sign, those along
              the surface normal), whose relative error is unbounded: the
              covariance is carried along the fitted state through
              state-dependent Jacobians, so the state difference allowed above
              moves every element by a small multiple of the state's own
              relative error in units of sqrt(C_ii C_jj).  The position
              diagonals are floored at 1e-4 of the track's largest position
              variance, because along the last surface's normal -- z after a
              plane, x or y when a cylinder's normal lies along an axis -- the
              variance itself is rounding noise;
  status:     flags bit-exact except FP64_FALLBACK (GPU only); the count of
              applied updates exact.
Conditioning of the final crossing.  The path-length derivative
ds*/dp = -(dg/dp) / (dg/ds) divides by dg/ds = cos(incidence) on a cylinder,
so the exact Jacobian at the GPU's final state and at the oracle's differ by
about 1/cos(incidence) times the states' relative difference: that much
covariance error is inherent to any FP32 fit of a track that grazes its last
cylinder.  An element that fails both bounds above still passes when its
normalised error is within NORM_TOL * min(kappa, KAPPA_CAP), kappa =
1/cos(incidence) at the final cylinder (1 for a plane).  compare() reports
how many elements pass only through that factor.  Tracks with kappa above
KAPPA_CAP are not compared at all: there an FP32 rounding of the radius moves
the crossing along the track by kappa times as much, in the parameters as in
the covariance.  They are counted with the exclusions below (4e-5 of the
100 x 9,600 x 20 barrel workload, 1e-6 of the ragged one).
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
REL_TOL_COV = 1e-3
KAPPA_CAP = 50.0     # conditioning above which a track's final state is not compared


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
    fits: the last of the track's surfaces that the final position is on
    (within 1e-3 cm; 0 when none is)."""
    p = np.asarray(par, np.float64)
    off = np.asarray(offsets, np.int64)
    n = p.shape[0]
    st = np.asarray(surf_type)
    sv = np.asarray(surf_val, np.float64)
    trk = np.repeat(np.arange(n), np.diff(off))
    r = np.hypot(p[:, 0], p[:, 1])
    with np.errstate(invalid="ignore"):
        dist = np.where(st == 0, np.abs(r[trk] - sv), np.abs(p[trk, 2] - sv))
    on = np.nonzero(dist < 1e-3)[0]
    last = np.full(n, -1, np.int64)
    np.maximum.at(last, trk[on], on)
    out = np.zeros(n, np.int64)
    have = last >= 0
    out[have] = st[last[have]].astype(np.int64)
    return out


def _cov_terms(gpu, ref, final_surface):
    """|d|, |ref|, the normalisation sqrt(C_ii C_jj) and the conditioning
    factor of every covariance element (n, 21)."""
    gc, rc = np.asarray(gpu["cov"], np.float64), np.asarray(ref["cov"], np.float64)
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
    kappa = incidence_condition(ref["par"], final_surface)
    return dc, np.abs(rc), scale, kappa, cnan


def covariance_breakdown(gpu: dict, ref: dict, final_surface="cylinder") -> dict:
    """Where the conditioning factor is needed: counts of tracks by their
    factor, and for the elements that fail both plain bounds, their packed
    indices, how many tracks hold them, the ratio of the factor each needs to
    its track's factor, and the range of those tracks' factors."""
    dc, rc, scale, kappa, cnan = _cov_terms(gpu, ref, final_surface)
    plain = (dc <= REL_TOL_COV * rc) | (dc <= NORM_TOL * scale) | cnan
    fin = np.all(np.isfinite(np.asarray(gpu["cov"])), 1) & np.all(np.isfinite(np.asarray(ref["cov"])), 1)
    plain[~fin] = True
    need = ~plain
    ti, ei = np.nonzero(need)
    out = dict(kappa_counts=[int((kappa > k).sum()) for k in (2, 5, 10, 20, 50)],
               needs_kappa=int(need.sum()), tracks_kappa=int(np.unique(ti).size),
               per_index=np.bincount(ei, minlength=21).tolist())
    if ti.size:
        req = dc[ti, ei] / (NORM_TOL * np.maximum(scale[ti, ei], 1e-300))
        out.update(ratio_max=float((req / kappa[ti]).max()), kappa_min=float(kappa[ti].min()),
                   kappa_max=float(kappa[ti].max()), required_max=float(req.max()))
    return out


def compare(gpu: dict, ref: dict, max_excluded_frac: float = 1e-4, ctx: str = "",
            final_surface="cylinder") -> dict:
    """gpu/ref dicts with par (n,6), cov (n,21), chi2 (n,), status (n,) [ref: + nused].

    final_surface: "cylinder", "plane" or a per-track 0/1 array (see
    incidence_condition)."""
    gp, rp = np.asarray(gpu["par"], np.float64), np.asarray(ref["par"], np.float64)
    gx, rx = np.asarray(gpu["chi2"], np.float64), np.asarray(ref["chi2"], np.float64)
    gs = np.asarray(gpu["status"]).astype(np.int64) & 0xFFFFFFFF
    rs = (np.asarray(ref["status"]).astype(np.int64) & 0xFFFFFFFF) | (np.asarray(ref["nused"]).astype(np.int64) << 8)
    n = gp.shape[0]
    flags_g = gs & ~np.int64(ST_FP64_FALLBACK)
    flags_r = rs
    geo = np.int64(ST_NO_CROSSING | ST_NEWTON_FAIL)
    # reachability disagreements near tangency, and chi2 within rounding of the cut
    # (and tracks whose final crossing is too ill-conditioned for FP32, below)
    excl = ((flags_g & geo) != (flags_r & geo)) | ((flags_g & ST_CHI2_CUT) != (flags_r & ST_CHI2_CUT))
    excl |= incidence_condition(rp, final_surface) > KAPPA_CAP
    n_excl = int(excl.sum())
    assert n_excl <= max(1, int(max_excluded_frac * n)), \
        f"{ctx}: {n_excl} tracks excluded (reachability disagreements, conditioning above {KAPPA_CAP:g})"
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
    dc, arc, scale, kappa, cnan = _cov_terms(gpu, ref, final_surface)
    cond = np.minimum(kappa, KAPPA_CAP)[:, None]
    ok_rel = dc <= REL_TOL_COV * arc
    ok_norm = dc <= NORM_TOL * scale
    ok_kappa = dc <= NORM_TOL * scale * cond
    okc = ok_rel | ok_norm | ok_kappa | cnan
    okc[~keep] = True
    assert okc.all(), _worst(f"{ctx}: cov", dc, np.maximum(REL_TOL_COV * arc, NORM_TOL * scale * cond), okc)
    relp = np.abs(d) / np.maximum(np.abs(rp), np.maximum(PAR_F, 1e-30))
    normerr = np.where(keep[:, None], dc / np.maximum(scale, 1e-300), 0.0)
    return dict(n=n, excluded=n_excl, cov_norm_err_max=float(normerr.max()) if n else 0.0,
                cov_norm_err_p999=float(np.quantile(normerr, 0.999)) if n else 0.0,
                max_rel_par=relp[keep].max(0) if keep.any() else np.zeros(6),
                max_rel_chi2=float((dx / np.maximum(rx, 1.0))[keep].max()) if keep.any() else 0.0,
                cov_rel_pass=int(ok_rel[keep].sum()), cov_norm_only=int((ok_norm & ~ok_rel)[keep].sum()),
                cov_kappa_only=int((ok_kappa & ~ok_norm & ~ok_rel)[keep].sum()),
                fp64_fallbacks=int(((gs & ST_FP64_FALLBACK) != 0).sum()),
                max_incidence_condition=float(kappa.max()) if n else 1.0)


def failures(gpu: dict, ref: dict, final_surface="cylinder") -> dict:
    """The checks of compare() without asserting: for each output, the
    tracks that fail it and each track's largest error in units of its
    tolerance (for reports on full-size workloads)."""
    gp, rp = np.asarray(gpu["par"], np.float64), np.asarray(ref["par"], np.float64)
    gx, rx = np.asarray(gpu["chi2"], np.float64), np.asarray(ref["chi2"], np.float64)
    gs = np.asarray(gpu["status"]).astype(np.int64) & 0xFFFFFFFF
    rs = (np.asarray(ref["status"]).astype(np.int64) & 0xFFFFFFFF) | (np.asarray(ref["nused"]).astype(np.int64) << 8)
    flags_g = gs & ~np.int64(ST_FP64_FALLBACK)
    geo = np.int64(ST_NO_CROSSING | ST_NEWTON_FAIL)
    kappa = incidence_condition(rp, final_surface)
    excl = ((flags_g & geo) != (rs & geo)) | ((flags_g & ST_CHI2_CUT) != (rs & ST_CHI2_CUT)) | (kappa > KAPPA_CAP)
    keep = ~excl
    d = gp - rp
    d[:, 4] = np.angle(np.exp(1j * d[:, 4]))
    both_nan = np.isnan(gp) & np.isnan(rp)
    d[both_nan] = 0.0
    rpar = np.where(both_nan, 0.0, np.abs(d) / (1e-4 * np.maximum(np.nan_to_num(np.abs(rp)), PAR_F)))
    rchi = np.abs(gx - rx) / (1e-3 * np.maximum(rx, 1.0))
    dc, arc, scale, kap, cnan = _cov_terms(gpu, ref, final_surface)
    cond = np.minimum(kap, KAPPA_CAP)[:, None]
    rcov = np.minimum(dc / np.maximum(REL_TOL_COV * arc, 1e-300), dc / np.maximum(NORM_TOL * scale * cond, 1e-300))
    rcov[cnan] = 0.0
    out = dict(excluded=np.nonzero(excl)[0], status=np.nonzero(keep & (flags_g != rs))[0])
    for name, r in (("par", rpar.max(1)), ("chi2", rchi), ("cov", rcov.max(1))):
        r = np.where(keep, r, 0.0)
        out[name] = np.nonzero(r > 1.0)[0]
        out[name + "_ratio"] = r
    return out


def _worst(what, d, tol, ok):
    bad = np.argwhere(~ok)
    r = (np.abs(d) / np.maximum(tol, 1e-300))
    i = np.unravel_index(np.argmax(np.where(ok, 0, r)), r.shape)
    return f"{what}: {bad.shape[0]} failures; worst at {i}: |d|={np.abs(d)[i]:.3e} tol={tol[i]:.3e}"
