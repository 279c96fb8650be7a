"""GPU parity of the update in the hit's (r-phi, z) frame (opts.update_2d)
against the oracle's (pinned) 2D update."""
import numpy as np
import pytest
import torch

import oracle
import paper_2401_14221_amd as p2r
from synth import events as ev

from .parity import compare, final_surface_of
from .test_gpu_fit import run_p2r, run_p2z
from .test_gpu_fp64 import check_tight
from .test_gpu_ragged import CUT, run as run_ragged, upload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = p2r.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("W", [32, 64, 128, 256])
def test_update_2d_parity_1024x10(ctx, W):
    d = ev.make_barrel_event(ev.P2R_PARITY)
    r = oracle.fit_event(d, "barrel", update_2d=True)
    g = run_p2r(ctx, d, W, update_2d=1)
    rep = compare(g, r, ctx=f"2D W={W}")
    print(f"2D W={W}", rep, flush=True)


def test_update_2d_throughput_sample(ctx):
    d = ev.make_barrel_event(ev.P2R_THROUGHPUT.with_(seed=91), n_tracks=8000)
    r = oracle.fit_event(d, "barrel", update_2d=True)
    g = run_p2r(ctx, d, 64, update_2d=1)
    rep = compare(g, r, ctx="2D sample")
    print("2D sample", rep, flush=True)
    # chi2 per track from the 2D update is smaller: it has no radial term
    g3 = run_p2r(ctx, d, 64)
    full = ((g["status"] >> 8) & 0xFF) == 20
    assert np.mean(g["chi2"][full]) < np.mean(g3["chi2"][full])
    assert np.mean(g["chi2"][full]) / 40.0 == pytest.approx(1.0, abs=0.05)   # chi2(2) x 20 surfaces


def test_update_2d_fp64_matches_oracle_tightly(ctx):
    d = ev.make_barrel_event(ev.P2R_THROUGHPUT.with_(seed=92), n_tracks=4000)
    r = oracle.fit_event(d, "barrel", update_2d=True)
    check_tight(run_p2r(ctx, d, 64, update_2d=1, fp64=1), r, "cylinder", "p2r 2D FP64")
    with pytest.raises(p2r.P2RError):
        run_p2r(ctx, d, 128, update_2d=1, fp64=1)      # the FP64 2D fit is built for W = 64 only


def test_update_2d_leaves_planes_alone(ctx):
    d = ev.make_disk_event(ev.P2Z_THROUGHPUT.with_(seed=93), n_tracks=3000)
    a = run_p2z(ctx, d)
    b = run_p2z(ctx, d, update_2d=1)
    for k in ("par", "cov", "chi2", "status"):
        assert np.array_equal(a[k], b[k]), k


def test_update_2d_ragged(ctx):
    d = ev.make_ragged_event(ev.RAGGED.with_(seed=94), n_tracks=12000)
    r = oracle.fit_ragged(d, chi2_cut=CUT, update_2d=True)
    fs = final_surface_of(r["par"], d["offsets"], d["surf_type"], d["surf_val"])
    u = upload(d)
    H = int(d["offsets"][-1])
    s = torch.cuda.Stream()
    for use_graph in (0, 1):
        g = run_ragged(ctx, u, H, stream=s, use_graph=use_graph, update_2d=1)
        rep = compare(g, r, ctx=f"ragged 2D graph={use_graph}", final_surface=fs)
    print("ragged 2D", rep, flush=True)
    check_tight(run_ragged(ctx, u, H, update_2d=1, fp64=1), r, fs, "ragged 2D FP64")


def _correlated_hits(d, rho2_gap):
    """Every barrel hit covariance replaced by one that, in the hit frame, is
    10 cm wide along the layer and in z with correlation sqrt(1 - rho2_gap):
    the 2x2 S is then ill-conditioned (1 - rho^2 of S ~ rho2_gap)."""
    h = d["hits"]
    ok = np.isfinite(h[..., 0])
    rh = np.where(ok, np.hypot(h[..., 0], h[..., 1]), 1.0)
    c, s = np.where(ok, h[..., 0] / rh, 1.0), np.where(ok, h[..., 1] / rh, 0.0)
    su, sz = 10.0, 10.0
    rho = np.sqrt(1.0 - rho2_gap)
    vuu, vuz, vzz, vrr = su * su, rho * su * sz, sz * sz, 1e-4
    # V = vuu t t^T + vuz (t z^T + z t^T) + vzz z z^T + vrr n n^T, t = (-s, c, 0), n = (c, s, 0)
    V = np.zeros(h.shape[:-1] + (6,))
    V[..., 0] = vuu * s * s + vrr * c * c
    V[..., 1] = -vuu * s * c + vrr * c * s
    V[..., 2] = vuu * c * c + vrr * s * s
    V[..., 3] = -vuz * s
    V[..., 4] = vuz * c
    V[..., 5] = vzz
    e = dict(d)
    e["hitcov"] = np.where(ok[..., None], V, d["hitcov"]).astype(np.float32)
    return e


def _close(g, r, ctx_name):
    """Contrived ill-conditioned inputs: parameters within 1e-3 of max(|ref|, 1),
    chi2 within 1e-2 of max(ref, 1), status identical.  Here the one precisely
    measured direction has a variance of 2.5e-2 cm^2 while the FP32 transported
    covariance that enters S carries absolute errors of ~1e-6 cm^2, so the gain
    itself is only known to ~1e-4 in FP32, whatever precision the update runs in
    (the same bounds as the 3D ill-conditioned test, for the same reason)."""
    gs = np.asarray(g["status"]).astype(np.int64) & ~np.int64(p2r.ST_FP64_FALLBACK)
    rs = np.asarray(r["status"]).astype(np.int64) | (np.asarray(r["nused"]).astype(np.int64) << 8)
    assert np.array_equal(gs, rs), ctx_name
    d = np.abs(g["par"] - r["par"])
    d[:, 4] = np.abs(np.angle(np.exp(1j * (g["par"][:, 4] - r["par"][:, 4]))))
    assert (d / np.maximum(np.abs(r["par"]), 1.0)).max() < 1e-3, ctx_name
    assert (np.abs(g["chi2"] - r["chi2"]) / np.maximum(r["chi2"], 1.0)).max() < 1e-2, ctx_name


def test_update_2d_fp64_fallbacks(ctx):
    """Ill-conditioned 2x2 S (1 - rho^2 = 5e-4 < the FP32 test's 1e-3): the FP32
    test fails and the FP64 paths take over."""
    d = _correlated_hits(ev.make_barrel_event(ev.P2R_PARITY, n_tracks=512), 5e-4)
    r = oracle.fit_event(d, "barrel", update_2d=True)
    g = run_p2r(ctx, d, 64, update_2d=1)                          # mode 3: the whole update in FP64
    assert np.mean((g["status"] & p2r.ST_FP64_FALLBACK) != 0) > 0.9
    _close(g, r, "2D fallback mode 3")
    g2 = run_p2r(ctx, d, 64, update_2d=1, fp64_fallback=2)        # FP64 update on every surface
    _close(g2, r, "2D forced fp64")
    g1 = run_p2r(ctx, d, 64, update_2d=1, fp64_fallback=1)        # FP64 2x2 inverse, FP32 rest
    assert np.mean((g1["status"] & p2r.ST_FP64_FALLBACK) != 0) > 0.9
    _close(g1, r, "2D fallback mode 1")
    g0 = run_p2r(ctx, d, 64, update_2d=1, fp64_fallback=0)        # skip
    assert np.mean((g0["status"] & p2r.ST_S_NOT_PD) != 0) > 0.9
    # the FP64 fit resolves the same inputs far better
    check = run_p2r(ctx, d, 64, update_2d=1, fp64=1)
    dd = np.abs(check["par"] - r["par"]) / np.maximum(np.abs(r["par"]), 1.0)
    assert dd.max() < 1e-5


def test_update_2d_option_errors(ctx):
    d = ev.make_barrel_event(ev.P2R_PARITY, n_tracks=64)
    with pytest.raises(p2r.P2RError):
        run_p2r(ctx, d, 64, update_2d=3)
    m = p2r.Mlp(ctx)
    with pytest.raises(p2r.P2RError):
        run_p2r(ctx, d, 64, update_2d=1, mlp=m.handle.value)
