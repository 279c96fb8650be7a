"""Pins of the FP64 oracle against facts that do not come from the oracle.

Each test states what fixes the expected value: a closed form of the
geometry, an invariant of the motion, a different algebraic route to the
same estimate (information form of the Kalman update, minimisation of the
least-squares objective), an independent numerical simulation (RK4 of the
Lorentz force), brute force, or statistics of a consistent filter.
"""
import numpy as np
import pytest

import oracle
from oracle import mlp
from synth import events as ev
from synth.events import KAPPA

B = 3.8
PI = np.pi


def rstate(g, r0=(0.0, 30.0), pt=(0.5, 10.0), eta=(-1.5, 1.5)):
    r = g.uniform(*r0)
    a = g.uniform(-PI, PI)
    th = 2 * np.arctan(np.exp(-g.uniform(*eta)))
    return np.array([r * np.cos(a), r * np.sin(a), g.normal(0, 5), 1 / g.uniform(*pt),
                     g.uniform(-PI, PI), th]), (1.0 if g.random() < 0.5 else -1.0)


def rspd(g, n, scale=1.0):
    A = g.normal(size=(n, n)) * scale
    return A @ A.T + n * scale * scale * 0.1 * np.eye(n)


# ------------------------------------------------------------ straight lines
def test_line_from_origin_hits_R_on_axis(orc):
    """B = 0, start at the origin heading along +x: crosses R at (R, 0) after s = R."""
    th = 1.0
    pout, J, s = oracle.propagate([0, 0, 0, 0.5, 0.0, th], 1.0, 0.0, 0, 10.0)
    assert s == pytest.approx(10.0, abs=1e-12)
    assert pout[:3] == pytest.approx([10.0, 0.0, 10.0 / np.tan(th)], abs=1e-12)
    assert pout[4] == 0.0


def test_line_crossing_brute_force(orc):
    """B = 0: the crossing lies on the circle, on the line, and no earlier point of the line reaches R."""
    g = np.random.default_rng(1)
    for _ in range(200):
        p, q = rstate(g, r0=(0.0, 20.0))
        R = g.uniform(21.0, 100.0)
        pout, _, s = oracle.propagate(p, q, 0.0, 0, R)
        d = np.array([np.cos(p[4]), np.sin(p[4])])
        P = p[:2] + s * d
        assert np.hypot(*P) == pytest.approx(R, rel=1e-13)
        assert pout[:2] == pytest.approx(P, abs=1e-10)
        ss = np.linspace(0, s, 2001)[:-1]
        assert np.all(np.hypot(p[0] + ss * d[0], p[1] + ss * d[1]) < R)


def test_line_plane(orc):
    g = np.random.default_rng(2)
    for _ in range(100):
        p, q = rstate(g, eta=(0.5, 2.5))
        Z = 100.0
        pout, _, s = oracle.propagate(p, q, 0.0, 1, Z)
        assert pout[2] == pytest.approx(Z, abs=1e-11)
        assert s == pytest.approx((Z - p[2]) * np.tan(p[5]), rel=1e-13)
        assert pout[:2] == pytest.approx(p[:2] + s * np.array([np.cos(p[4]), np.sin(p[4])]), abs=1e-10)


def test_small_field_tends_to_line(orc):
    """As B -> 0 the helix path to the cylinder tends to the straight-line one (arc-chord ~ s^3/(24 rho^2))."""
    p = np.array([1.0, -2.0, 0.0, 1.0, 0.3, 1.2])
    s0 = oracle.path(p, 1.0, 0.0, 0, 50.0)
    for b in (1e-1, 1e-2, 1e-3):
        s = oracle.path(p, 1.0, b, 0, 50.0)
        rho = 1.0 / (KAPPA * b)
        assert abs(s - s0) < 3 * s0 ** 2 / rho + 1e-9


# ------------------------------------------------------------------ helices
def test_helix_radius_units_and_turning_sense(orc):
    """Circumradius of three helix points is pT/(0.29979 B) m; q>0 turns clockwise seen from +z."""
    for q in (1.0, -1.0):
        p = np.array([0.3, -0.2, 1.0, 1.0 / 2.0, 0.7, 1.1])
        P = [oracle.helix(p, q, B, s)[:2] for s in (0.0, 40.0, 90.0)]
        a, b, c = (np.linalg.norm(P[1] - P[2]), np.linalg.norm(P[0] - P[2]), np.linalg.norm(P[0] - P[1]))
        cross = (P[1] - P[0])[0] * (P[2] - P[1])[1] - (P[1] - P[0])[1] * (P[2] - P[1])[0]
        area = 0.5 * abs(cross)
        radius = a * b * c / (4 * area)
        assert radius == pytest.approx(2.0 / (0.299792458 * B) * 100.0, rel=1e-10)
        assert np.sign(cross) == -q


def test_helix_invariants(orc):
    """|dP/ds| = 1 in xy, dz/ds = cot(theta), dphi/ds = omega, one period returns to the start."""
    g = np.random.default_rng(3)
    for _ in range(50):
        p, q = rstate(g)
        w = -q * KAPPA * B * p[3]
        s = g.uniform(0, 200)
        h = 1e-4
        a, b = oracle.helix(p, q, B, s - h), oracle.helix(p, q, B, s + h)
        v = (b - a) / (2 * h)
        assert np.hypot(v[0], v[1]) == pytest.approx(1.0, abs=1e-7)
        assert np.arctan2(v[1], v[0]) == pytest.approx(
            np.angle(np.exp(1j * (p[4] + w * s))), abs=1e-6)
        assert v[2] == pytest.approx(1 / np.tan(p[5]), rel=1e-7)
        P = oracle.helix(p, q, B, 2 * PI / abs(w))
        assert P[:2] == pytest.approx(p[:2], abs=1e-9)
        assert P[4] - p[4] == pytest.approx(2 * PI * np.sign(w), abs=1e-12)


def test_helix_from_origin_closed_form(orc):
    """From the origin the chord to radius R subtends 2 asin(R/(2 rho)): s* = 2 rho asin(R/(2 rho))."""
    for q in (1.0, -1.0):
        for pt in (0.7, 1.0, 3.0, 10.0):
            rho = pt / (KAPPA * B)
            for R in (2.5, 30.0, 1.2 * rho):
                p = np.array([0.0, 0.0, 0.0, 1 / pt, 0.4, 1.0])
                s = oracle.path(p, q, B, 0, R)
                assert s == pytest.approx(2 * rho * np.arcsin(R / (2 * rho)), rel=1e-12)
            assert oracle.path(p, q, B, 0, 2.0 * rho * 1.0001) is None   # beyond the diameter


def test_cylinder_vs_bisection(orc):
    """The closed-form crossing equals bisection on |xy(s)| - R over the helix map (to 1e-10 cm)."""
    g = np.random.default_rng(4)
    for _ in range(200):
        p, q = rstate(g, r0=(0.0, 40.0))
        R = g.uniform(41.0, 110.0)
        s = oracle.path(p, q, B, 0, R)
        rho = 1 / (KAPPA * B * p[3])
        if s is None:
            continue
        # bracket: scan to the first sign change
        ss = np.linspace(0, 2 * PI * rho, 20001)
        r = np.array([np.hypot(*oracle.helix(p, q, B, x)[:2]) for x in ss[::50]])
        k = np.nonzero(r >= R)[0][0]
        lo, hi = ss[::50][k - 1], ss[::50][k]
        for _ in range(100):
            mid = 0.5 * (lo + hi)
            if np.hypot(*oracle.helix(p, q, B, mid)[:2]) < R:
                lo = mid
            else:
                hi = mid
        assert s == pytest.approx(0.5 * (lo + hi), abs=1e-10)


def _bisect_path(p, q, R, lo, hi):
    """Root of |xy(s)| = R in [lo, hi] by bisection over the helix map."""
    f = lambda s: np.hypot(*oracle.helix(p, q, B, s)[:2]) - R  # noqa: E731
    flo = f(lo)
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if (f(mid) < 0) == (flo < 0):
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def test_crossing_rule_backward_step_and_half_turn(orc):
    """The next crossing is the smallest s > -1 cm among the crossings within half a turn.

    A state 0.3 cm beyond the layer, moving out, is taken back to it (bisection on
    the helix gives the same s < 0); 3 cm beyond, no crossing lies within half a
    turn; a start 0.12 cm off the axis and pointing inward still crosses forward.
    """
    for q in (1.0, -1.0):
        R = 40.0
        p = np.array([R + 0.3, 0.0, 0.0, 1 / 5.0, 0.2, 1.0])
        s = oracle.path(p, q, B, 0, R)
        assert -1.0 < s < 0.0
        assert s == pytest.approx(_bisect_path(p, q, R, -1.0, 0.0), abs=1e-10)
        p3 = np.array([R + 3.0, 0.0, 0.0, 1 / 5.0, 0.2, 1.0])
        assert oracle.path(p3, q, B, 0, R) is None
        pv = np.array([0.12, 0.0, 0.0, 1 / 2.0, np.pi - 0.3, 1.0])
        s = oracle.path(pv, q, B, 0, 2.5)
        assert s > 0 and s == pytest.approx(_bisect_path(pv, q, 2.5, 0.0, 3.0), abs=1e-10)
    # planes: 0.5 cm behind is reached backwards, 2 cm behind is not a crossing
    p = np.array([1.0, 2.0, 100.5, 0.5, 0.3, 0.5])
    s = oracle.path(p, 1.0, B, 1, 100.0)
    assert s == pytest.approx(-0.5 * np.tan(0.5), rel=1e-14)
    assert oracle.path(np.array([1.0, 2.0, 105.0, 0.5, 0.3, 0.5]), 1.0, B, 1, 100.0) is None
    # a plane more than half a turn ahead (a looper spiralling along z) is not the next surface
    pt = 0.6
    half = np.pi * pt / (KAPPA * B)
    th = np.arctan2(1.0, 1.0 / (1.1 * half / 100.0))        # reaches z = 100 after 1.1 half turns
    assert oracle.path(np.array([0.0, 0.0, 0.0, 1 / pt, 0.0, th]), 1.0, B, 1, 100.0) is None
    th = np.arctan2(1.0, 1.0 / (0.9 * half / 100.0))
    assert oracle.path(np.array([0.0, 0.0, 0.0, 1 / pt, 0.0, th]), 1.0, B, 1, 100.0) == pytest.approx(0.9 * half)


def test_crossings_match_independent_rk4_simulation(orc):
    """Oracle path lengths to cylinders and planes agree with the generator's RK4 of the Lorentz force."""
    g = np.random.default_rng(5)
    n = 300
    par = np.array([rstate(g, r0=(0, 5))[0] for _ in range(n)])
    # moving outward, so the next crossing is the first forward one the simulation finds
    par[:, 4] = np.arctan2(par[:, 1], par[:, 0]) + g.uniform(-1.2, 1.2, n)
    q = np.where(g.random(n) < 0.5, -1.0, 1.0)
    R = g.uniform(10.0, 80.0, n)
    s_rk4 = ev.simulate_to_cylinder(par, q, R)
    for i in range(n):
        s = oracle.path(par[i], q[i], B, 0, R[i])
        if s is None:
            assert np.isnan(s_rk4[i])
        else:
            assert s == pytest.approx(s_rk4[i], abs=2e-5)
    # planes: the oracle's crossing point equals the simulated one
    cfg = ev.P2Z_THROUGHPUT
    d = ev.make_disk_event(cfg, n_tracks=50)
    tr = d["truth_start"]
    for i in range(50):
        for li in (0, 9, 19):
            Z = np.sign(np.cos(tr[i, 5])) * cfg.surfaces[li]
            pout, _, _ = oracle.propagate(tr[i], d["q"][i], B, 1, Z)
            assert pout[:3] == pytest.approx(d["truth"][i, li, :3], abs=2e-5)
            assert np.angle(np.exp(1j * (pout[4] - d["truth"][i, li, 4]))) == pytest.approx(0, abs=1e-6)


# ---------------------------------------------------------------- Jacobian
def _fd_jacobian(p, q, stype, v, h_rel=1e-6):
    J = np.zeros((6, 6))
    for j in range(6):
        h = h_rel * max(1.0, abs(p[j]))
        a, b = p.copy(), p.copy()
        a[j] -= h
        b[j] += h
        pa = oracle.propagate(a, q, B, stype, v)[0]
        pb = oracle.propagate(b, q, B, stype, v)[0]
        J[:, j] = (pb - pa) / (2 * h)
    return J


@pytest.mark.parametrize("stype", [0, 1])
def test_jacobian_vs_finite_differences(orc, stype):
    g = np.random.default_rng(6 + stype)
    for _ in range(100):
        p, q = rstate(g, r0=(0, 30), eta=(0.3, 2.5) if stype else (-1.5, 1.5))
        v = g.uniform(35, 100) if stype == 0 else np.sign(np.cos(p[5])) * g.uniform(30, 200)
        res = oracle.propagate(p, q, B, stype, v)
        if res is None:
            continue
        _, J, _ = res
        Jfd = _fd_jacobian(p, q, stype, v)
        scale = np.maximum(np.abs(J), 1.0)
        assert np.max(np.abs(J - Jfd) / scale) < 2e-5


def test_jacobian_invariants(orc):
    """Cylinder: n^T J_pos = 0 and J v = 0 for the flow tangent v; plane: row z of J is 0."""
    g = np.random.default_rng(8)
    for _ in range(100):
        p, q = rstate(g, r0=(0, 30))
        w = -q * KAPPA * B * p[3]
        R = g.uniform(35, 100)
        res = oracle.propagate(p, q, B, 0, R)
        if res is None:
            continue
        pout, J, _ = res
        n = np.array([pout[0], pout[1]]) / R
        assert np.max(np.abs(n @ J[:2])) < 1e-9 * np.max(np.abs(J))
        flow = np.array([np.cos(p[4]), np.sin(p[4]), 1 / np.tan(p[5]), 0.0, w, 0.0])
        assert np.max(np.abs(J @ flow)) < 1e-9 * np.max(np.abs(J))
        # rows 1/pT and theta are unit rows
        assert J[3] == pytest.approx(np.eye(6)[3])
        assert J[5] == pytest.approx(np.eye(6)[5])
    for _ in range(50):
        p, q = rstate(g, eta=(0.5, 2.5))
        pout, J, _ = oracle.propagate(p, q, B, 1, 150.0)
        assert np.all(J[2] == 0.0) or np.max(np.abs(J[2])) < 1e-12


# ----------------------------------------------------------- Kalman update
def test_update_equals_information_form(orc):
    """Posterior from the information filter (C^-1 + H^T V^-1 H) with numpy.linalg; chi2 = min of the LSQ objective."""
    g = np.random.default_rng(9)
    H = np.hstack([np.eye(3), np.zeros((3, 3))])
    for _ in range(200):
        C = rspd(g, 6)
        V = rspd(g, 3, 0.5)
        p = g.normal(size=6)
        p[5] = 1.0
        p[4] = 0.1
        m = g.normal(size=3)
        st, pu, Cu, chi2 = oracle.update(p, C, m, ev.pack21(np.pad(V, ((0, 3), (0, 3))))[:6], form=0)
        assert st == 0
        Ci, Vi = np.linalg.inv(C), np.linalg.inv(V)
        P = np.linalg.inv(Ci + H.T @ Vi @ H)
        mu = P @ (Ci @ p + H.T @ Vi @ m)
        assert pu == pytest.approx(mu, abs=1e-9)
        assert Cu == pytest.approx(P, abs=1e-9)
        obj = (mu - p) @ Ci @ (mu - p) + (m - H @ mu) @ Vi @ (m - H @ mu)
        assert chi2 == pytest.approx(obj, rel=1e-9)
        r = m - p[:3]
        assert chi2 == pytest.approx(r @ np.linalg.solve(C[:3, :3] + V, r), rel=1e-10)
        st2, pu2, Cu2, chi22 = oracle.update(p, C, m, ev.pack21(np.pad(V, ((0, 3), (0, 3))))[:6], form=1)
        assert np.max(np.abs(Cu2 - Cu)) < 1e-12 * np.max(np.abs(Cu)) * 100
        assert pu2 == pytest.approx(pu, abs=0)


def test_update_scalar_gain(orc):
    """Diagonal C and V: each position is a 1D filter, gain C/(C+V)."""
    C = np.diag([4.0, 2.0, 1.0, 1.0, 1.0, 1.0])
    V = np.array([1.0, 0.0, 2.0, 0.0, 0.0, 1.0])      # packed diag(1, 2, 1)
    p = np.array([1.0, 2.0, 3.0, 0.5, 0.2, 1.0])
    m = np.array([2.0, 0.0, 4.0])
    st, pu, Cu, chi2 = oracle.update(p, C, m, V)
    k = np.array([4 / 5, 2 / 4, 1 / 2])
    assert pu[:3] == pytest.approx(p[:3] + k * (m - p[:3]), abs=1e-14)
    assert np.diag(Cu)[:3] == pytest.approx([4 * 1 / 5, 2 * 2 / 4, 1 * 1 / 2], abs=1e-14)
    assert chi2 == pytest.approx(1 / 5 + 4 / 4 + 1 / 2, abs=1e-14)


def test_update_status(orc):
    C = np.zeros((6, 6))
    C[3:, 3:] = np.eye(3)
    p = np.array([1.0, 2.0, 3.0, 0.5, 0.2, 1.0])
    st, *_ = oracle.update(p, C, [1, 2, 3], np.zeros(6))
    assert st == oracle.ST_S_NOT_PD
    st, *_ = oracle.update(p, np.eye(6), [101, 2, 3], [1, 0, 1, 0, 0, 1], chi2_cut=30.0)
    assert st == oracle.ST_CHI2_CUT


# --------------------------------------------------------------- full fits
def _fit1(par, cov, q, hits, hitcov, radii, kind="barrel", **kw):
    return oracle.fit_layers(par[None], cov[None], np.array([q]), hits[None], hitcov[None], radii, kind, **kw)


def test_fit_rotation_and_mirror_symmetry(orc):
    d = ev.make_barrel_event(ev.P2R_PARITY, n_tracks=40)
    out = oracle.fit_event(d, "barrel")
    for al in (0.3, -2.0):
        c, s = np.cos(al), np.sin(al)
        Rm = np.array([[c, -s], [s, c]])
        par = d["par"].copy()
        par[:, :2] = par[:, :2] @ Rm.T
        par[:, 4] += al
        par[:, 4] = np.angle(np.exp(1j * par[:, 4]))
        hits = d["hits"].copy()
        hits[..., :2] = hits[..., :2] @ Rm.T
        o2 = oracle.fit_layers(par, d["cov"], d["q"], hits, d["hitcov"], d["surf"], "barrel")
        T = np.eye(6)
        T[:2, :2] = Rm
        Cexp = T @ ev.unpack21(out["cov"]) @ T.T
        assert o2["chi2"] == pytest.approx(out["chi2"], rel=1e-8)
        assert o2["par"][:, :2] == pytest.approx(out["par"][:, :2] @ Rm.T, rel=1e-9, abs=1e-8)
        assert ev.unpack21(o2["cov"]) == pytest.approx(Cexp, abs=1e-12)
    # charge conjugation + mirror y -> -y
    M = np.diag([1, -1, 1, 1, -1, 1.0])
    par = d["par"] @ M
    hits = d["hits"] * np.array([1, -1, 1.0])
    hc = d["hitcov"].copy()
    hc[..., 1] *= -1
    hc[..., 4] *= -1
    o3 = oracle.fit_layers(par, d["cov"], -d["q"], hits, hc, d["surf"], "barrel")
    assert o3["chi2"] == pytest.approx(out["chi2"], rel=1e-8)
    assert o3["par"] == pytest.approx(out["par"] @ M, abs=1e-8)
    assert ev.unpack21(o3["cov"]) == pytest.approx(M @ ev.unpack21(out["cov"]) @ M, abs=1e-12)


def test_output_covariance_structure(orc):
    """Symmetric, PSD, one null direction = surface normal; the 5 surface-local parameters are PD."""
    d = ev.make_barrel_event(ev.P2R_PARITY, n_tracks=200)
    out = oracle.fit_event(d, "barrel", layers=True)
    L = len(d["surf"])
    lp = out["lay_par"].reshape(-1, L, 6)
    lc = ev.unpack21(out["lay_cov"].reshape(-1, L, 21))
    for i in range(200):
        prev = d["par"][i]
        for li in range(L):
            if not np.isfinite(d["hits"][i, li, 0]):
                continue
            # the null direction is the normal at the propagated (pre-update) point:
            # the update moves the position only within that tangent plane
            pp = oracle.propagate(prev, d["q"][i], B, 0, d["surf"][li])[0]
            prev = lp[i, li]
            Cm = lc[i, li]
            assert np.allclose(Cm, Cm.T)
            n6 = np.zeros(6)
            n6[:2] = pp[:2] / np.hypot(*pp[:2])
            assert np.linalg.norm(Cm @ n6) < 1e-9 * np.linalg.norm(Cm)
            T = np.linalg.svd(n6[None])[2][1:].T      # 6x5 orthonormal complement of n
            np.linalg.cholesky(T.T @ Cm @ T)


def test_disk_vzz_independence(orc):
    """On planes the result does not depend on the hit's z variance (z' = Z exactly)."""
    d = ev.make_disk_event(ev.P2Z_THROUGHPUT, n_tracks=100)
    outs = []
    for vzz in (1e-6, 1e-4, 1.0):
        hc = d["hitcov"].copy()
        hc[..., 5] = vzz
        outs.append(oracle.fit_layers(d["par"], d["cov"], d["q"], d["hits"], hc, d["surf"], "disk"))
    for o in outs[1:]:
        assert o["par"] == pytest.approx(outs[0]["par"], abs=1e-9)
        assert o["cov"] == pytest.approx(outs[0]["cov"], abs=1e-12)
        assert o["chi2"] == pytest.approx(outs[0]["chi2"], rel=1e-7, abs=1e-9)


def test_fit_status_bits(orc):
    d = ev.make_barrel_event(ev.P2R_PARITY, n_tracks=4)
    par, cov, q, hits, hc = d["par"].copy(), d["cov"].copy(), d["q"], d["hits"].copy(), d["hitcov"].copy()
    par[0, 3] = 1 / 0.3          # pT 0.3: 2 rho = 53 cm, outer layers unreachable
    cov[0, 9] = 1e-14            # ... and 1/pT pinned so the hits cannot change it
    par[1, 0] = np.nan
    hits[2, 3] = np.nan
    par[3, 5] = -0.1
    o = oracle.fit_layers(par, cov, q, hits, hc, d["surf"], "barrel")
    assert o["status"][0] & oracle.ST_NO_CROSSING
    assert o["status"][1] & oracle.ST_BAD_INPUT and o["nused"][1] == 0
    assert o["status"][2] & oracle.ST_HIT_MISSING and o["nused"][2] == 9
    assert o["status"][3] & oracle.ST_BAD_INPUT
    assert np.all(o["status"] & oracle.ST_DONE)


@pytest.mark.parametrize("kind", ["barrel", "disk"])
def test_filter_statistics(orc, kind):
    """Consistency over 1e5 outlier-free tracks: unit-width pulls; chi2 per hit 3 (barrel) or 2 (disk)."""
    from scipy import stats
    n = 100_000
    if kind == "barrel":
        d = ev.make_barrel_event(ev.P2R_THROUGHPUT, n_tracks=n)
    else:
        d = ev.make_disk_event(ev.P2Z_THROUGHPUT, n_tracks=n)
    out = oracle.fit_event(d, kind, layers=True)
    L = len(d["surf"])
    full = out["nused"] == L
    assert full.mean() > 0.97
    ndf_hit = 3 if kind == "barrel" else 2
    lay = out["lay_chi2"].reshape(-1, L)[full]
    per = np.diff(lay, axis=1, prepend=0.0)
    assert per.mean() / ndf_hit == pytest.approx(1.0, abs=0.01)
    # the first surface sees the start's large position spread (0.1 cm against a
    # 2.5 cm first radius), where the linearised step is visibly inexact; from the
    # second surface on, the chi2 sum must follow chi2(ndf) exactly
    chi = lay[:, -1] - lay[:, 0]
    assert chi.mean() / (ndf_hit * (L - 1)) == pytest.approx(1.0, abs=0.01)
    ks = stats.kstest(chi, stats.chi2(ndf_hit * (L - 1)).cdf)
    assert ks.pvalue > 1e-3
    tr = d["truth"][full, -1]
    p = out["par"][full]
    Cm = ev.unpack21(out["cov"][full])
    dd = p - tr
    dd[:, 4] = np.angle(np.exp(1j * dd[:, 4]))
    pulls = {}
    if kind == "barrel":
        r = np.hypot(tr[:, 0], tr[:, 1])
        t = np.stack([-tr[:, 1] / r, tr[:, 0] / r], 1)
        vt = np.einsum("ni,nij,nj->n", t, Cm[:, :2, :2], t)
        pulls["u"] = np.einsum("ni,ni->n", dd[:, :2], t) / np.sqrt(vt)
        pulls["z"] = dd[:, 2] / np.sqrt(Cm[:, 2, 2])
    else:
        pulls["x"] = dd[:, 0] / np.sqrt(Cm[:, 0, 0])
        pulls["y"] = dd[:, 1] / np.sqrt(Cm[:, 1, 1])
    for i, k in ((3, "ipt"), (4, "phi"), (5, "theta")):
        pulls[k] = dd[:, i] / np.sqrt(Cm[:, i, i])
    for k, v in pulls.items():
        assert abs(v.mean()) < 0.02, k
        assert abs(v.std() - 1) < 0.03, k


# --------------------------------------------------------------------- MLP
def test_mlp_gradients_vs_finite_differences():
    g = np.random.default_rng(10)
    p = {k: v.astype(np.float64) for k, v in ev.make_mlp_init(7).items()}
    for k in p:
        p[k] = p[k] + 0.1 * g.normal(size=p[k].shape)
    x = g.normal(size=(32, 7))
    t = g.normal(size=32)
    loss, gr = mlp.loss_and_grads(p, x, t)
    for k in p:
        flat = p[k].reshape(-1)
        for idx in g.choice(flat.size, size=min(flat.size, 12), replace=False):
            h = 1e-6
            old = flat[idx]
            flat[idx] = old + h
            lp, _ = mlp.loss_and_grads(p, x, t)
            flat[idx] = old - h
            lm, _ = mlp.loss_and_grads(p, x, t)
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            assert gr[k].reshape(-1)[idx] == pytest.approx(fd, rel=1e-6, abs=1e-9), k


def test_mlp_adam_first_step_is_signed_lr():
    """With zero moments, Adam's first step is -lr * g / (|g| + eps)."""
    p = {"w": np.array([1.0, -2.0, 3.0])}
    gr = {"w": np.array([0.5, -1e-3, 0.0])}
    newp, st = mlp.adam_step(p, gr, {}, lr=0.01)
    assert newp["w"] == pytest.approx(p["w"] - 0.01 * gr["w"] / (np.abs(gr["w"]) + 1e-8), abs=1e-15)


def test_bf16_rounding_known_values():
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 1.0 + 2 ** -9, -3.140625, 65504.0])
    exp = np.array([1.0, 1.0, 1.0 + 4 * 2 ** -8, 1.0, -3.140625, 65536.0])
    assert mlp.bf16_round(vals) == pytest.approx(exp, abs=0)


def test_mlp_features_reduce_to_geometry():
    """s_line is the straight-line path; the proposal of a zero output is s_line."""
    g = np.random.default_rng(11)
    par = np.array([rstate(g, r0=(0, 20))[0] for _ in range(50)])
    R = g.uniform(25, 100, 50)
    f, sl = mlp.features(par, np.ones(50), R)
    for i in range(50):
        assert sl[i] == pytest.approx(oracle.path(par[i], 1.0, 0.0, 0, R[i]), rel=1e-12)
    assert mlp.proposal(np.zeros(50), sl) == pytest.approx(sl)
    assert f[:, 0] == pytest.approx(np.hypot(par[:, 0], par[:, 1]) / R)


def test_mlp_forward_hand_network():
    """A network set by hand, evaluated by hand: two hidden units pass x0 + 0.5
    and -x1 + 0.5 through ReLU, the second layer copies them, the output
    weighs them 2 and 3 and adds 0.25."""
    p = {k: np.zeros(s) for k, s in (("W1", (64, 7)), ("b1", 64), ("W2", (64, 64)), ("b2", 64),
                                      ("W3", (1, 64)), ("b3", 1))}
    p["W1"][0, 0], p["W1"][1, 1] = 1.0, -1.0
    p["b1"][:2] = 0.5
    p["W2"][0, 0] = p["W2"][1, 1] = 1.0
    p["W3"][0, :2] = [2.0, 3.0]
    p["b3"][0] = 0.25
    x = np.array([[1.0, -2.0, 3, 0, 0, 0, 0],     # h = (1.5, 2.5): y = 3 + 7.5 + 0.25
                  [-1.0, 2.0, 0, 0, 0, 0, 0],     # h = (0, 0): both clipped, y = b3
                  [0.25, 0.25, 0, 0, 0, 0, 9]])   # h = (0.75, 0.25): y = 1.5 + 0.75 + 0.25
    for bf16 in (False, True):                    # every value here is exact in bfloat16
        y, c = mlp.forward(p, x, bf16=bf16)
        assert y == pytest.approx([10.75, 0.25, 2.5], abs=0)
        assert c["h1"][0, :2] == pytest.approx([1.5, 2.5], abs=0) and not c["h1"][:, 2:].any()


def test_mlp_features_closed_forms():
    """All seven features on states whose straight-line path is known in
    closed form, and their rotation and charge symmetries."""
    R, r0, ipt, bz = 50.0, 30.0, 2.0, 3.8
    w = -2.99792458e-3 * bz * ipt                  # q = +1: omega = -q c B / pT in 1/cm (c = 0.299792458 GeV / (T m))
    cases = [
        # at the origin: s_line = R
        ([0.0, 0.0, 0.0, ipt, 0.7, 1.0], [0.0, 0.0, 0.0, w * R, 1.0, w * R, 0.0]),
        # on the x axis, moving radially: b = r0, a = 0, s_line = R - r0
        ([r0, 0.0, 0.0, ipt, 0.0, 1.0], [r0 / R, r0 / R, 0.0, w * R, (R - r0) / R, w * (R - r0), 0.0]),
        # on the x axis, moving along +y: b = 0, a = -r0, s_line = sqrt(R^2 - r0^2)
        ([r0, 0.0, 0.0, ipt, np.pi / 2, 1.0],
         [r0 / R, 0.0, -r0 / R, w * R, 40.0 / R, w * 40.0, -w * r0]),
    ]
    for par, exp in cases:
        f, sl = mlp.features(np.array([par]), np.array([1.0]), np.array([R]), bz=bz)
        assert f[0] == pytest.approx(exp, rel=1e-12, abs=1e-12)
    g = np.random.default_rng(12)
    par = np.array([rstate(g, r0=(0, 20))[0] for _ in range(40)])
    Rs = g.uniform(25, 100, 40)
    f, sl = mlp.features(par, np.ones(40), Rs)
    # rotating the state about the z axis changes no feature
    for a in (0.3, -2.0):
        rp = par.copy()
        rp[:, 0] = np.cos(a) * par[:, 0] - np.sin(a) * par[:, 1]
        rp[:, 1] = np.sin(a) * par[:, 0] + np.cos(a) * par[:, 1]
        rp[:, 4] = par[:, 4] + a
        assert mlp.features(rp, np.ones(40), Rs)[0] == pytest.approx(f, rel=1e-9, abs=1e-12)
    # the opposite charge flips exactly the curvature features (3, 5, 6)
    fm = mlp.features(par, -np.ones(40), Rs)[0]
    sign = np.array([1, 1, 1, -1, 1, -1, -1])
    assert fm == pytest.approx(f * sign, rel=1e-12, abs=1e-15)
