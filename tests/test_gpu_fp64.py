"""The FP64 fits (every step in FP64 on the same FP32 inputs, results rounded
to FP32) against the FP64 oracle, and the per-output precision table of the
FP32 and FP64 fits.

Both the FP64 fit and the oracle compute the same mathematics in FP64, so
their results differ by FP64 rounding (relative ~1e-13, amplified by the
fit's conditioning) plus the FP32 rounding of the stored results (half an
ulp, 6e-8 relative) plus the FP64 Newton tolerance (1e-9 cm).  The bounds
below allow for those with a margin: parameters 1e-6 relative (1e-6 cm or
rad near zero), chi2 1e-6 relative, covariance 1e-6 relative or 1e-7 of
sqrt(C_ii C_jj).  They are 100 (parameters) to 1000 (covariance) times
tighter than the FP32 fit's bounds.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2401_14221_amd as p2r
from synth import events as ev

from .parity import compare, final_surface_of, incidence_condition
from .test_gpu_fit import run_p2r, run_p2z
from .test_gpu_ragged import CUT, run as run_ragged, upload

pytestmark = pytest.mark.gpu

PAR_F = np.array([1.0, 1.0, 1.0, 0.0, 1.0, 0.0])
IL = np.tril_indices(6)


@pytest.fixture(scope="module")
def ctx():
    c = p2r.Context(0)
    yield c
    c.close()


def errors(g, r, final_surface):
    """Per-output error measures of a GPU result against the oracle."""
    st_ok = ((np.asarray(r["status"]) & 0x3) == 0)          # reached every surface it had a hit on
    d = np.abs(np.asarray(g["par"], np.float64) - r["par"])
    d[:, 4] = np.abs(np.angle(np.exp(1j * (np.asarray(g["par"][:, 4], np.float64) - r["par"][:, 4]))))
    relp = d / np.maximum(np.abs(r["par"]), np.maximum(PAR_F, 1e-30))
    dx = np.abs(np.asarray(g["chi2"], np.float64) - r["chi2"]) / np.maximum(r["chi2"], 1.0)
    rc = np.asarray(r["cov"])
    dc = np.abs(np.asarray(g["cov"], np.float64) - rc)
    diag = np.abs(rc[:, [0, 2, 5, 9, 14, 20]])
    diag[:, :3] = np.maximum(diag[:, :3], 1e-4 * diag[:, :3].max(1, keepdims=True))
    scale = np.sqrt(diag[:, IL[0]] * diag[:, IL[1]])
    cond = incidence_condition(r["par"], final_surface)[:, None]
    # covariance: the smaller of the relative and the normalised error, per element
    relc = np.minimum(dc / np.maximum(np.abs(rc), 1e-300), dc / np.maximum(scale, 1e-300)) / cond
    return dict(par=relp[st_ok], chi2=dx[st_ok], cov=relc[st_ok])


def check_tight(g, r, final_surface, ctx_name):
    gs = np.asarray(g["status"]).astype(np.int64) & 0xFFFFFFFF
    rs = (np.asarray(r["status"]).astype(np.int64) & 0xFFFFFFFF) | (np.asarray(r["nused"]).astype(np.int64) << 8)
    assert np.array_equal(gs & ~np.int64(p2r.ST_FP64_FALLBACK), rs), f"{ctx_name}: status differs"
    e = errors(g, r, final_surface)
    worst = {k: float(v.max()) if v.size else 0.0 for k, v in e.items()}
    print(f"{ctx_name}: FP64 fit max error: params {worst['par']:.2e}, chi2 {worst['chi2']:.2e}, "
          f"cov {worst['cov']:.2e}", flush=True)
    assert worst["par"] <= 1e-6, worst
    assert worst["chi2"] <= 1e-6, worst
    # covariance: 1e-6 relative or 1e-7 normalised
    rc = np.asarray(r["cov"])
    dc = np.abs(np.asarray(g["cov"], np.float64) - rc)
    diag = np.abs(rc[:, [0, 2, 5, 9, 14, 20]])
    diag[:, :3] = np.maximum(diag[:, :3], 1e-4 * diag[:, :3].max(1, keepdims=True))
    scale = np.sqrt(diag[:, IL[0]] * diag[:, IL[1]])
    cond = incidence_condition(r["par"], final_surface)[:, None]
    ok = (dc <= 1e-6 * np.abs(rc) * cond) | (dc <= 1e-7 * scale * cond)
    assert ok.all(), f"{ctx_name}: {int((~ok).sum())} covariance elements beyond the FP64 bound"
    return e


def _table(name, e32, e64):
    lines = [f"precision table, {name} (max and 99.9th percentile of the error against the FP64 oracle)",
             f"  {'output':10s} {'FP32 max':>10s} {'FP32 p999':>10s} {'FP64 max':>10s} {'FP64 p999':>10s}"]
    labels = ["x", "y", "z", "1/pT", "phi", "theta"]
    for i, lab in enumerate(labels):
        a, b = e32["par"][:, i], e64["par"][:, i]
        lines.append(f"  {lab:10s} {a.max():10.2e} {np.quantile(a, .999):10.2e} {b.max():10.2e} {np.quantile(b, .999):10.2e}")
    for k in ("chi2", "cov"):
        a, b = e32[k].reshape(-1), e64[k].reshape(-1)
        lines.append(f"  {k:10s} {a.max():10.2e} {np.quantile(a, .999):10.2e} {b.max():10.2e} {np.quantile(b, .999):10.2e}")
    print("\n".join(lines), flush=True)


@pytest.mark.parametrize("W", [32, 64, 128, 256])
def test_fp64_p2r_matches_oracle_tightly(ctx, W):
    d = ev.make_barrel_event(ev.P2R_THROUGHPUT.with_(seed=71), n_tracks=6000)
    r = oracle.fit_event(d, "barrel")
    g64 = run_p2r(ctx, d, W, fp64=1)
    e64 = check_tight(g64, r, "cylinder", f"p2r FP64 W={W}")
    g32 = run_p2r(ctx, d, W)
    compare(g32, r, ctx="p2r FP32")
    _table(f"p2r 6000 tracks x 20 layers, W={W}", errors(g32, r, "cylinder"), e64)


def test_fp64_p2z_matches_oracle_tightly(ctx):
    d = ev.make_disk_event(ev.P2Z_THROUGHPUT.with_(seed=72), n_tracks=6000)
    r = oracle.fit_event(d, "disk")
    e64 = check_tight(run_p2z(ctx, d, fp64=1), r, "plane", "p2z FP64")
    g32 = run_p2z(ctx, d)
    _table("p2z 6000 tracks x 20 disks", errors(g32, r, "plane"), e64)


def test_fp64_ragged_matches_oracle_tightly(ctx):
    d = ev.make_ragged_event(ev.RAGGED.with_(seed=73), n_tracks=6000)
    r = oracle.fit_ragged(d, chi2_cut=CUT)
    fs = final_surface_of(r["par"], d["offsets"], d["surf_type"], d["surf_val"])
    u = upload(d)
    H = int(d["offsets"][-1])
    e64 = check_tight(run_ragged(ctx, u, H, fp64=1), r, fs, "ragged FP64")
    _table("ragged 6000 tracks", errors(run_ragged(ctx, u, H), r, fs), e64)


def test_fp64_option_errors(ctx):
    d = ev.make_barrel_event(ev.P2R_PARITY, n_tracks=64)
    with pytest.raises(p2r.P2RError):
        run_p2r(ctx, d, 64, fp64=2)
    m = p2r.Mlp(ctx)
    with pytest.raises(p2r.P2RError):
        run_p2r(ctx, d, 64, fp64=1, mlp=m.handle.value)
    assert p2r._lib.default_opts().fp64 == 0
