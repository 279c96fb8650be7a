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
    # radial motion: cos(incidence) = 1; motion at 60 degrees to the radius: 2; along a plane: 1
    par = np.array([[10.0, 0.0, 0.0, 1.0, 0.0, 1.0],
                    [0.0, 10.0, 0.0, 1.0, np.pi / 2 + np.pi / 3, 1.0],
                    [0.0, 10.0, 0.0, 1.0, 0.0, 1.0]])
    c = incidence_condition(par, "cylinder")
    assert c[0] == pytest.approx(1.0) and c[1] == pytest.approx(2.0)
    assert c[2] == pytest.approx(1e3)                  # exactly tangent: capped
    assert np.all(incidence_condition(par, "plane") == 1.0)
    assert np.all(incidence_condition(par, np.array([0, 1, 1])) == [1.0, 1.0, 1.0])


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
