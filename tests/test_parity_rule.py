"""The element-by-element comparison rule itself: it accepts what it should
and rejects planted errors (CPU only, on oracle output)."""
import numpy as np
import pytest

import oracle
from synth import events as ev

from .parity import compare, incidence_condition, final_surface_of


@pytest.fixture(scope="module")
def fit():
    d = ev.make_barrel_event(ev.P2R_PARITY, n_tracks=200)
    return d, oracle.fit_event(d, "barrel")


def _as_gpu(r):
    st = (np.asarray(r["status"]).astype(np.int64) | (np.asarray(r["nused"]).astype(np.int64) << 8))
    return dict(par=r["par"].copy(), cov=r["cov"].copy(), chi2=r["chi2"].copy(), status=st.astype(np.uint32))


def test_incidence_condition_geometry():
    # radial motion: cos(incidence) = 1; motion at 60 degrees to the radius: 2
    par = np.array([[10.0, 0.0, 0.0, 1.0, 0.0, 1.0],
                    [0.0, 10.0, 0.0, 1.0, np.pi / 2 + np.pi / 3, 1.0],
                    [0.0, 10.0, 0.0, 1.0, 0.0, 1.0]])
    c = incidence_condition(par, "cylinder")
    assert c[0] == pytest.approx(1.0) and c[1] == pytest.approx(2.0)
    assert c[2] == pytest.approx(1e3)                  # exactly tangent: capped
    # planes z = Z: the z component of the direction, cos(theta)
    pz = par.copy()
    pz[:, 5] = [0.0, np.pi / 3, np.pi / 2]
    assert incidence_condition(pz, "plane") == pytest.approx([1.0, 2.0, 1e3])
    mixed = incidence_condition(np.vstack([par[:1], pz[1:2]]), np.array([0, 1]))
    assert mixed == pytest.approx([1.0, 2.0])


def test_final_surface_of_matches_the_surface_reached():
    par = np.array([[30.0, 40.0, 7.0, 1, 0, 1], [1.0, 1.0, -80.0, 1, 0, 1]])
    off = np.array([0, 2, 4])
    stype = np.array([0, 1, 0, 1], np.uint8)
    sval = np.array([50.0, 200.0, 3.0, -80.0])
    assert list(final_surface_of(par, off, stype, sval)) == [0, 1]


def test_identical_outputs_pass(fit):
    d, r = fit
    rep = compare(_as_gpu(r), r, ctx="self")
    assert rep["excluded"] == 0


@pytest.mark.parametrize("what", ["par", "cov", "chi2", "status"])
def test_planted_errors_are_caught(fit, what):
    d, r = fit
    g = _as_gpu(r)
    t = 17
    if what == "par":
        g["par"][t, 3] *= 1 + 3e-4                      # 1/pT off by 3e-4 relative
    elif what == "cov":
        g["cov"][t, 9] *= 1 + 5e-3                      # C(1/pT,1/pT) off by 5e-3 relative
    elif what == "chi2":
        g["chi2"][t] = r["chi2"][t] * (1 + 3e-3) + 3e-3
    else:
        g["status"][t] ^= np.uint32(1 << 6)             # a HIT_MISSING flag that the oracle did not set
    with pytest.raises(AssertionError):
        compare(g, r, ctx=f"planted {what}")


def test_chi2_cut_decisions_are_counted_exclusions(fit):
    """A track whose chi2-cut decision differs (flag, or with the flag set the
    number of applied updates) is excluded and counted; a different update
    count without any cut is a status mismatch."""
    d, r = fit
    g = _as_gpu(r)
    t = 23
    r2 = {k: (v.copy() if hasattr(v, "copy") else v) for k, v in r.items()}
    r2["status"][t] |= np.uint32(1 << 7)
    g["status"][t] |= np.uint32(1 << 7)
    g["status"][t] -= np.uint32(1 << 8)           # one update fewer on the GPU side
    g["par"][t, 0] += 1.0                          # and a different state: not compared
    rep = compare(g, r2, ctx="cut", max_excluded_frac=0.01)
    assert rep["excluded"] == 1
    g2 = _as_gpu(r)
    g2["status"][t] -= np.uint32(1 << 8)
    with pytest.raises(AssertionError, match="status mismatch"):
        compare(g2, r, ctx="no cut")


def test_fp32_runs_deviate_at_fp32_rounding_level(fit):
    """Each of the oracle's FP32 runs differs from the exact fit by about FP32
    rounding amplified by the fit: not at all (it would measure nothing) and
    not beyond the base bounds on well-conditioned tracks; the random-rounding
    runs differ from each other."""
    d, r = fit
    assert len(r["f32_runs"]) >= 2 and r["f32"] is r["f32_runs"][0]
    assert not np.array_equal(r["f32_runs"][0]["par"], r["f32_runs"][1]["par"])
    assert not np.array_equal(r["f32_runs"][1]["par"], r["f32_runs"][2]["par"])
    s = r["f32"]
    rel = np.abs(s["par"] - r["par"]) / np.maximum(np.abs(r["par"]), [1, 1, 1, 1e-30, 1, 1e-30])
    assert np.median(rel[:, [0, 1, 3, 5]]) > 1e-9              # it is a different computation
    assert np.quantile(rel[:, [0, 1, 3, 5]], 0.5) < 1e-5       # of FP32 size
    assert np.array_equal(s["nused"], r["nused"])
    # its own deviation passes the base bounds on almost every track
    from .parity import failures
    f = failures(_as_gpu(s), {k: v for k, v in r.items() if k not in ("f32", "f32_runs")})
    assert len(f["par"]) + len(f["cov"]) + len(f["chi2"]) <= 2


def _with_sensitivity(r, t, col, frac):
    """A copy of the oracle result with one FP32 run, deviating at track t in
    parameter col by frac of the base bound."""
    from .parity import PAR_F, PAR_TOL
    r2 = dict(r)
    s = {k: v.copy() for k, v in r["f32"].items()}
    s["par"] = r["par"].copy()
    s["cov"], s["chi2"] = r["cov"].copy(), r["chi2"].copy()
    s["par"][t, col] += frac * PAR_TOL * max(abs(r["par"][t, col]), PAR_F[col])
    r2["f32_runs"] = [s]
    return r2


def test_sensitivity_widens_only_that_track_and_kind(fit):
    from .parity import PAR_F, PAR_TOL, SENS_FACTOR
    d, r = fit
    t, col = 31, 3
    r2 = _with_sensitivity(r, t, col, 4.0)          # bound widened to SENS_FACTOR x 4
    step = PAR_TOL * max(abs(r["par"][t, col]), PAR_F[col])
    g = _as_gpu(r)
    g["par"][t, col] += 0.9 * SENS_FACTOR * 4.0 * step
    rep = compare(g, r2, ctx="widened")
    assert rep["tracks_widened"] == 1 and rep["widest"]["par"] == pytest.approx(SENS_FACTOR * 4.0)
    g["par"][t, col] += 0.2 * SENS_FACTOR * 4.0 * step
    with pytest.raises(AssertionError, match="params"):
        compare(g, r2, ctx="beyond widened")
    # another track keeps the base bound
    g = _as_gpu(r)
    g["par"][t + 1, col] += 3.0 * step
    with pytest.raises(AssertionError, match="params"):
        compare(g, r2, ctx="other track")
    # and the same track's covariance keeps its base bound
    g = _as_gpu(r)
    g["cov"][t, 9] *= 1 + 5e-3
    with pytest.raises(AssertionError, match="cov"):
        compare(g, r2, ctx="other kind")


def test_decisions_of_an_fp32_run_exclude_the_track(fit):
    d, r = fit
    t = 40
    r2 = dict(r)
    s = {k: v.copy() for k, v in r["f32"].items()}
    s["status"][t] |= np.uint32(1 << 7)            # a cut the exact fit did not make
    r2["f32_runs"] = [r["f32_runs"][0], s]
    g = _as_gpu(r)
    g["par"][t, 0] += 1.0
    rep = compare(g, r2, ctx="f32 decision", max_excluded_frac=0.01)
    assert rep["excluded"] == 1


def test_widening_is_capped_and_beyond_it_the_track_is_excluded(fit):
    from .parity import PAR_F, PAR_TOL, SENS_CAP, SENS_FACTOR
    d, r = fit
    t, col = 12, 0
    r2 = _with_sensitivity(r, t, col, 2 * SENS_CAP / SENS_FACTOR)   # would widen to 2 SENS_CAP
    g = _as_gpu(r)
    g["par"][t, col] += 10 * SENS_CAP * PAR_TOL * max(abs(r["par"][t, col]), PAR_F[col])
    rep = compare(g, r2, ctx="ill-posed")          # one exclusion is always allowed
    assert rep["excluded"] == 1 and rep["widest"]["par"] <= SENS_CAP
    # a second ill-posed track exceeds the 1e-4 allowance of 200 tracks
    r3 = dict(r2)
    s = {k: v.copy() for k, v in r2["f32_runs"][0].items()}
    s["par"][t + 5, col] += 2 * SENS_CAP / SENS_FACTOR * PAR_TOL * max(abs(r["par"][t + 5, col]), PAR_F[col])
    r3["f32_runs"] = [s]
    with pytest.raises(AssertionError, match="excluded"):
        compare(g, r3, ctx="two ill-posed tracks")
