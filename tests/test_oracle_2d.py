"""Pins of the oracle's update in the hit's (r-phi, z) frame on a cylinder.

Measuring only the two coordinates along the surface is the same as a 3D
measurement whose third, radial, coordinate has an unbounded variance: the
2D update must therefore equal the (separately pinned) 3D update with the
hit covariance rotated into the hit frame and its radial variance made
huge.  And its chi2 must follow chi2(2) per barrel hit.
"""
import numpy as np
import pytest

import oracle
from synth import events as ev

IL = np.tril_indices(6)


def pack21(C):
    return C[IL]


def _case(rng, theta=1.1, ipt=0.7):
    """A state propagated onto R = 50 cm, its transported covariance, and a hit near it."""
    p0 = np.array([0.02, -0.01, 1.5, ipt, rng.uniform(-np.pi, np.pi), theta])
    A = rng.normal(size=(6, 6)) * np.array([0.1, 0.1, 0.5, 1e-2, 1e-2, 1e-2])
    C0 = A @ A.T + np.diag([1e-2, 1e-2, 1.0, 1e-4, 1e-4, 1e-4])
    pp, J, _ = oracle.propagate(p0, 1.0, 3.8, 0, 50.0)
    Cp = J @ C0 @ J.T
    Cp = 0.5 * (Cp + Cp.T)
    r = np.hypot(pp[0], pp[1])
    n = np.array([pp[0], pp[1]]) / r
    t = np.array([-n[1], n[0]])
    m = np.array([pp[0], pp[1], pp[2]])
    m[:2] += 0.013 * t + 0.004 * n       # off in r-phi and radially
    m[2] += 0.05
    B = rng.normal(size=(3, 3))
    V = B @ B.T * 1e-4 + np.diag([1e-4, 1e-4, 1e-2])
    return pp, Cp, m, V


def _v21(V):
    return np.array([V[0, 0], V[1, 0], V[1, 1], V[2, 0], V[2, 1], V[2, 2]])


def _rotation(c, s):
    """Linear map of the state into the frame turned by the hit's azimuth (x along the hit)."""
    G = np.eye(6)
    G[0, 0], G[0, 1], G[1, 0], G[1, 1] = c, s, -s, c
    return G


@pytest.mark.parametrize("seed", range(6))
def test_update_2d_equals_3d_without_radial_information(orc, seed):
    rng = np.random.default_rng(seed)
    pp, Cp, m, V = _case(rng, theta=rng.uniform(0.4, 2.7), ipt=rng.uniform(0.1, 2.0))
    st2, p2, C2, c2 = oracle.update_2d(pp, Cp.reshape(-1), m, _v21(V))
    assert st2 == 0
    # the same measurement in 3D, in the frame where the hit lies on +x: the
    # radial coordinate is x there, measured with a variance of 1e20 cm^2
    rh = np.hypot(m[0], m[1])
    c, s = m[0] / rh, m[1] / rh
    G = _rotation(c, s)
    phi_h = np.arctan2(s, c)
    pr = G @ pp
    pr[4] = pp[4] - phi_h
    Cr = G @ Cp @ G.T
    R3 = G[:3, :3]
    mr = R3 @ m
    Vr = R3 @ V @ R3.T
    Vr[0, :] = 0.0
    Vr[:, 0] = 0.0
    Vr[0, 0] = 1e20
    st3, p3r, C3r, c3 = oracle.update(pr, Cr.reshape(-1), mr, _v21(Vr))
    assert st3 == 0
    p3 = G.T @ p3r
    p3[4] = p3r[4] + phi_h
    C3 = G.T @ C3r @ G
    scale = np.sqrt(np.outer(np.diag(C3), np.diag(C3)))
    dp = np.abs(p2 - p3)
    dp[4] = abs(np.angle(np.exp(1j * (p2[4] - p3[4]))))
    assert np.all(dp <= 1e-10 * np.maximum(np.abs(p3), 1.0)), dp
    assert np.all(np.abs(C2 - C3) <= 1e-8 * scale), np.max(np.abs(C2 - C3) / scale)
    # chi2: the 3D value carries the radial term r_n^2 / (1e20 + C'_nn), negligible
    assert c2 == pytest.approx(c3, rel=1e-9, abs=1e-14)


def test_update_2d_uses_the_hit_frame(orc):
    """A hit displaced only radially (same azimuth as the state) changes nothing but chi2 = 0."""
    rng = np.random.default_rng(9)
    pp, Cp, m, V = _case(rng)
    r = np.hypot(pp[0], pp[1])
    m = np.array([pp[0] * (1 + 0.3 / r), pp[1] * (1 + 0.3 / r), pp[2]])
    st, p2, C2, c2 = oracle.update_2d(pp, Cp.reshape(-1), m, _v21(V))
    assert st == 0 and c2 == pytest.approx(0.0, abs=1e-20)
    assert np.allclose(p2, pp, rtol=0, atol=1e-12)


def test_filter_statistics_2d(orc):
    """chi2 per barrel hit follows chi2(2) with the update in the hit frame; pulls keep unit width."""
    from scipy import stats
    n = 50_000
    d = ev.make_barrel_event(ev.P2R_THROUGHPUT.with_(seed=77), n_tracks=n)
    out = oracle.fit_event(d, "barrel", layers=True, update_2d=True)
    L = len(d["surf"])
    full = out["nused"] == L
    lay = out["lay_chi2"].reshape(-1, L)[full]
    per = np.diff(lay, axis=1, prepend=0.0)
    assert per.mean() / 2 == pytest.approx(1.0, abs=0.01)
    chi = lay[:, -1] - lay[:, 0]
    assert chi.mean() / (2 * (L - 1)) == pytest.approx(1.0, abs=0.01)
    assert stats.kstest(chi, stats.chi2(2 * (L - 1)).cdf).pvalue > 1e-3
    tr = d["truth"][full, -1]
    p = out["par"][full]
    Cm = ev.unpack21(out["cov"][full])
    dd = p - tr
    dd[:, 4] = np.angle(np.exp(1j * dd[:, 4]))
    for i in (3, 4, 5):
        pull = dd[:, i] / np.sqrt(Cm[:, i, i])
        assert abs(pull.mean()) < 0.02 and abs(pull.std() - 1) < 0.03, i
