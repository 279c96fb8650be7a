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
              state-dependent Jacobians, so a state difference moves every
              element by a small multiple of the state's own relative error
              in units of sqrt(C_ii C_jj).  The position diagonals are floored
              at 1e-4 of the track's largest position variance, because along
              the last surface's normal -- z after a plane, x or y when a
              cylinder's normal lies along an axis -- the variance itself is
              rounding noise;
  status:     flags bit-exact except FP64_FALLBACK (GPU only); the count of
              applied updates exact.

Conditioning, measured per track.  Some fits amplify rounding: a track that
meets its surface at a shallow angle carries a large variance along the
surface, which one precise hit removes, so the update cancels most of the
prior covariance (thousands of times, for a track that grazes a cylinder
or a looper that meets a disk after half a turn); a fit that outliers have
wrecked.  For those no FP32 implementation can meet the bounds above, and
how far it can stay from the exact result is a property of the track,
which the oracle measures: it fits every track again as an FP32
implementation of its algorithm would (stored values, matrix algebra and
cylinder crossing rounded to FP32), once with round-to-nearest and three
times with random rounding (the CESTAC method), oracle.fit's "f32_runs".
Where those runs deviate from the exact fit by up to a fraction s of a
bound, the GPU's bound for that output kind (parameters, chi2, covariance)
of that track is max(1, SENS_FACTOR s) times the bound above, up to
SENS_CAP: a track whose FP32 runs deviate more than that is taken as
ill-posed in FP32 and excluded (and counted) like the decision differences
below.  compare() reports how many tracks had a bound widened and by how
much.

Tracks whose reachability of a surface differs between FP32 and FP64 (the
surface grazes the track's largest radius), or where a hit's chi2 falls on
the other side of a chi2 cut (the CHI2_CUT flag, or with it the number of
applied updates, differs), between the GPU and the oracle or between one
of the oracle's FP32 runs and its exact fit, are listed and excluded from
the value comparison, together with the FP32-ill-posed tracks above; their
number must stay below 1e-4 of the tracks.
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
PAR_TOL = 1e-4
CHI2_TOL = 1e-3
SENS_FACTOR = 3.0    # bound = max(1, SENS_FACTOR x the FP32 runs' largest deviation) x base bound
SENS_CAP = 100.0     # a track whose bound would widen beyond this is excluded instead (counted)


def incidence_condition(ref_par, final_surface) -> np.ndarray:
    """Per-track factor 1 / cos(incidence) at the final surface.

    final_surface: "cylinder", "plane", or a per-track array (0 cylinder,
    1 plane).  On a cylinder cos(incidence) is the radial component of the
    transverse direction, |x cos(phi) + y sin(phi)| / r (the crossing is
    solved in the transverse path); on a plane z = Z it is the z component
    of the direction, |cos(theta)|.  Taken from the oracle's final state,
    capped at 1000.  (A geometric indicator, reported beside the measured
    conditioning.)"""
    p = np.asarray(ref_par, np.float64)
    n = p.shape[0]
    if isinstance(final_surface, str):
        cyl = np.full(n, final_surface == "cylinder")
    else:
        cyl = np.asarray(final_surface) == 0
    r = np.hypot(p[:, 0], p[:, 1])
    with np.errstate(invalid="ignore", divide="ignore"):
        c = np.abs(p[:, 0] * np.cos(p[:, 4]) + p[:, 1] * np.sin(p[:, 4])) / r
        cz = np.abs(np.cos(p[:, 5]))
    c = np.where(np.isfinite(c), c, 1.0)
    cz = np.where(np.isfinite(cz), cz, 1.0)
    return 1.0 / np.clip(np.where(cyl, c, cz), 1e-3, 1.0)


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


def _flags(res, with_nused: bool) -> np.ndarray:
    """Status words as int64, FP64_FALLBACK cleared; with_nused: the oracle's
    separate update count folded into bits 8..15 like the GPU's (saturating
    at 255, as the status word's field does)."""
    s = np.asarray(res["status"]).astype(np.int64) & 0xFFFFFFFF
    if with_nused:
        s = s | (np.minimum(np.asarray(res["nused"]).astype(np.int64), 255) << 8)
    return s & ~np.int64(ST_FP64_FALLBACK)


def _cut_differs(flags_g, flags_r):
    """Tracks where a chi2 cut decided differently: the CHI2_CUT flag differs,
    or both cut hits but a different number of updates was applied (a hit
    whose chi2 lies within rounding of the cut, after which the two fits
    follow different hit sets)."""
    cut_g, cut_r = (flags_g & ST_CHI2_CUT) != 0, (flags_r & ST_CHI2_CUT) != 0
    nused_g, nused_r = (flags_g >> 8) & 0xFF, (flags_r >> 8) & 0xFF
    return (cut_g != cut_r) | ((cut_g | cut_r) & (nused_g != nused_r))


def _decisions_differ(flags_a, flags_b):
    geo = np.int64(ST_NO_CROSSING | ST_NEWTON_FAIL)
    return ((flags_a & geo) != (flags_b & geo)) | _cut_differs(flags_a, flags_b)


def _ratios(out: dict, ref: dict):
    """Per-track errors of `out` against `ref` in units of the base bounds:
    parameters (n, 6), chi2 (n,), covariance (n, 21) (the smaller of the
    relative and the normalised measure), and the covariance split
    (relative ratio, normalised ratio)."""
    gp, rp = np.asarray(out["par"], np.float64), np.asarray(ref["par"], np.float64)
    d = gp - rp
    d[:, 4] = np.angle(np.exp(1j * d[:, 4]))
    both_nan = np.isnan(gp) & np.isnan(rp)      # passed-through NaN of a rejected input
    d[both_nan] = 0.0
    rpar = np.abs(d) / (PAR_TOL * np.maximum(np.nan_to_num(np.abs(rp)), PAR_F))
    rpar[both_nan] = 0.0
    gx, rx = np.asarray(out["chi2"], np.float64), np.asarray(ref["chi2"], np.float64)
    rchi = np.abs(gx - rx) / (CHI2_TOL * np.maximum(rx, 1.0))
    gc, rc = np.asarray(out["cov"], np.float64), np.asarray(ref["cov"], np.float64)
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
    with np.errstate(invalid="ignore", divide="ignore"):
        r_rel = dc / (REL_TOL_COV * np.abs(rc))
        r_norm = dc / (NORM_TOL * scale)
    r_rel = np.where(dc == 0.0, 0.0, r_rel)
    r_norm = np.where(dc == 0.0, 0.0, r_norm)
    rcov = np.minimum(r_rel, r_norm)
    return rpar, rchi, rcov, r_rel, r_norm


def _sensitivity(ref: dict, n: int, cap: float = SENS_CAP):
    """Per-track widening of the bounds for parameters, chi2 and covariance
    from the oracle's FP32 runs (the largest deviation over them; ones when
    the oracle result has none), and the tracks where any of those runs took
    different decisions."""
    ones = np.ones(n)
    runs = ref.get("f32_runs") or ([ref["f32"]] if "f32" in ref else [])
    if not runs:
        return ones, ones, ones, np.zeros(n, bool)
    wp, wx, wc = np.zeros(n), np.zeros(n), np.zeros(n)
    decided = np.zeros(n, bool)
    for f32 in runs:
        sp, sx, sc, _, _ = _ratios(f32, ref)
        wp, wx, wc = np.fmax(wp, sp.max(1)), np.fmax(wx, sx), np.fmax(wc, sc.max(1))
        decided |= _decisions_differ(_flags(f32, True), _flags(ref, True))
    wid = lambda s: np.maximum(1.0, SENS_FACTOR * np.nan_to_num(s, nan=0.0, posinf=1e30))  # noqa: E731
    wp, wx, wc = wid(wp), wid(wx), wid(wc)
    decided |= (wp > cap) | (wx > cap) | (wc > cap)
    return np.minimum(wp, cap), np.minimum(wx, cap), np.minimum(wc, cap), decided


def compare(gpu: dict, ref: dict, max_excluded_frac: float = 1e-4, ctx: str = "",
            final_surface="cylinder", sens_cap: float = SENS_CAP) -> dict:
    """gpu/ref dicts with par (n,6), cov (n,21), chi2 (n,), status (n,) [ref: + nused, and the
    oracle's FP32 runs under "f32_runs" when it made them].

    final_surface ("cylinder", "plane" or a per-track 0/1 array) is used only
    to report the largest geometric conditioning 1/cos(incidence).  sens_cap:
    the largest widening before a track counts as ill-posed (raised only by
    tests whose inputs are ill-conditioned by construction)."""
    gp = np.asarray(gpu["par"], np.float64)
    n = gp.shape[0]
    flags_g = _flags(gpu, False)
    flags_r = _flags(ref, True)
    w_par, w_chi, w_cov, decided32 = _sensitivity(ref, n, sens_cap)
    # reachability disagreements near tangency, and chi2 within rounding of the
    # cut, between the GPU and the oracle or between one of the FP32 runs and it
    excl = _decisions_differ(flags_g, flags_r) | decided32
    n_excl = int(excl.sum())
    assert n_excl <= max(1, int(max_excluded_frac * n)), \
        f"{ctx}: {n_excl} tracks excluded (reachability or chi2-cut decisions within rounding, or FP32-ill-posed)"
    keep = ~excl
    bad_status = np.nonzero(keep & (flags_g != flags_r))[0]
    assert bad_status.size == 0, \
        f"{ctx}: status mismatch at {bad_status[:10]}: gpu {flags_g[bad_status[:5]]} ref {flags_r[bad_status[:5]]}"
    rpar, rchi, rcov, r_rel, r_norm = _ratios(gpu, ref)
    okp = (rpar <= w_par[:, None]) | ~keep[:, None]
    assert okp.all(), _worst(f"{ctx}: params", rpar / w_par[:, None], okp)
    okx = (rchi <= w_chi) | ~keep
    assert okx.all(), _worst(f"{ctx}: chi2", (rchi / w_chi)[:, None], okx[:, None])
    okc = (rcov <= w_cov[:, None]) | ~keep[:, None]
    assert okc.all(), _worst(f"{ctx}: cov", rcov / w_cov[:, None], okc)
    relp = np.abs(gp - np.asarray(ref["par"], np.float64))
    relp[:, 4] = np.abs(np.angle(np.exp(1j * relp[:, 4])))
    relp = np.nan_to_num(relp / np.maximum(np.abs(np.asarray(ref["par"], np.float64)), np.maximum(PAR_F, 1e-30)))
    gx, rx = np.asarray(gpu["chi2"], np.float64), np.asarray(ref["chi2"], np.float64)
    k = keep
    widened = (w_par > 1) | (w_chi > 1) | (w_cov > 1)
    normerr = np.where(k[:, None], r_norm * NORM_TOL, 0.0)
    return dict(n=n, excluded=n_excl,
                max_rel_par=relp[k].max(0) if k.any() else np.zeros(6),
                max_rel_chi2=float((np.abs(gx - rx) / np.maximum(rx, 1.0))[k].max()) if k.any() else 0.0,
                max_ratio=dict(par=float(rpar[k].max()) if k.any() else 0.0,
                               chi2=float(rchi[k].max()) if k.any() else 0.0,
                               cov=float(rcov[k].max()) if k.any() else 0.0),
                cov_norm_err_max=float(normerr.max()) if n else 0.0,
                cov_norm_err_p999=float(np.quantile(normerr, 0.999)) if n else 0.0,
                cov_rel_pass=int((r_rel <= 1.0)[k].sum()),
                cov_norm_only=int(((r_norm <= 1.0) & (r_rel > 1.0))[k].sum()),
                cov_widened_only=int(((rcov > 1.0) & (rcov <= w_cov[:, None]))[k].sum()),
                tracks_widened=int((widened & k).sum()),
                widest=dict(par=float(w_par[k].max()) if k.any() else 1.0,
                            chi2=float(w_chi[k].max()) if k.any() else 1.0,
                            cov=float(w_cov[k].max()) if k.any() else 1.0),
                fp64_fallbacks=int(((np.asarray(gpu["status"]).astype(np.int64) & ST_FP64_FALLBACK) != 0).sum()),
                max_incidence_condition=float(incidence_condition(ref["par"], final_surface).max()) if n else 1.0)


def failures(gpu: dict, ref: dict) -> dict:
    """The checks of compare() without asserting: for each output kind, the
    tracks that fail it, each track's largest error in units of its (widened)
    bound, and the widening itself (for reports on full-size workloads)."""
    n = len(np.asarray(gpu["chi2"]))
    flags_g, flags_r = _flags(gpu, False), _flags(ref, True)
    w_par, w_chi, w_cov, decided32 = _sensitivity(ref, n)
    excl = _decisions_differ(flags_g, flags_r) | decided32
    keep = ~excl
    rpar, rchi, rcov, _, _ = _ratios(gpu, ref)
    out = dict(excluded=np.nonzero(excl)[0], status=np.nonzero(keep & (flags_g != flags_r))[0],
               widen_par=w_par, widen_chi2=w_chi, widen_cov=w_cov)
    for name, r, w in (("par", rpar.max(1), w_par), ("chi2", rchi, w_chi), ("cov", rcov.max(1), w_cov)):
        r = np.where(keep, r, 0.0)
        out[name] = np.nonzero(r > w)[0]
        out[name + "_ratio"] = r / w
        out[name + "_raw"] = r
    return out


def _worst(what, r, ok):
    bad = np.argwhere(~ok)
    i = np.unravel_index(np.argmax(np.where(ok, 0, r)), r.shape)
    return f"{what}: {bad.shape[0]} failures; worst at {i}: error / bound = {r[i]:.3g}"
