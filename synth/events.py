"""Seeded synthetic events: truth simulation, hits, fit starts, MLP pairs.

Units: cm, GeV, tesla, radians.  Track parameters are
(x, y, z, 1/pT, phi, theta) with the charge q = +-1 stored separately.

Truth trajectories come from a Runge-Kutta (RK4) integration of the
equation of motion of a charged particle in the field B = B z-hat,

    dr/dl = t,    dt/dl = (q * KAPPA * B / p) * (t x z-hat),

with l the 3D path length, t the unit tangent and p the momentum.  This is a
simulation of the particle, independent of the analytic helix the fit uses.
Crossings with surfaces are located inside a step by Newton iteration on the
RK4 sub-step length.  With a 2 cm transverse step the integration error is
below 1e-6 cm over a whole track, far below the 100 um hit resolution.

Random numbers come from NumPy's Philox counter-based generator keyed by
(seed, purpose), one independent stream per purpose.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

KAPPA = 2.99792458e-3     # GeV / (T cm): p[GeV] = KAPPA * B[T] * radius[cm]
B_TESLA = 3.8
STEP_CM = 2.0             # transverse RK4 step
TWO_PI = 2.0 * np.pi

# purposes of the independent random streams
_S_KINE, _S_VTX, _S_START, _S_HIT, _S_OUTL, _S_LEN, _S_MLP, _S_PAIR = range(8)

# initial-state covariance of the fit start (diagonal, per the benchmark
# configuration): x, y [cm^2], z [cm^2], 1/pT [GeV^-2], phi, theta
C0_DIAG = np.array([0.01, 0.01, 1.0, 1e-4, 1e-4, 1e-4])


def rng(seed: int, purpose: int) -> np.random.Generator:
    return np.random.Generator(np.random.Philox(key=np.array([seed, purpose], dtype=np.uint64)))


def pack21(m: np.ndarray) -> np.ndarray:
    """(..., 6, 6) symmetric -> (..., 21) lower triangle, row-major."""
    il = np.tril_indices(6)
    return m[..., il[0], il[1]]


def unpack21(v: np.ndarray) -> np.ndarray:
    """(..., 21) lower triangle row-major -> (..., 6, 6) symmetric."""
    out = np.zeros(v.shape[:-1] + (6, 6), dtype=v.dtype)
    il = np.tril_indices(6)
    out[..., il[0], il[1]] = v
    out[..., il[1], il[0]] = v
    return out


def _f32(a):
    """Surface positions as the float32 values the fit receives."""
    return tuple(float(v) for v in np.asarray(a, dtype=np.float32))


@dataclass(frozen=True)
class EventConfig:
    name: str
    kind: str                      # 'barrel' | 'disk' | 'ragged'
    n_events: int
    n_tracks: int                  # per event
    surfaces: tuple                # barrel radii or |z| of the disks [cm]
    eta: tuple = (-1.5, 1.5)       # for 'disk': range of |eta|, both signs
    pt: tuple = (0.5, 10.0)
    seed: int = 0
    hit_sigma: tuple = (0.01, 0.01, 0.1)   # x, y, z smear [cm]
    extra: dict = field(default_factory=dict, hash=False, compare=False)

    @property
    def n_total(self) -> int:
        return self.n_events * self.n_tracks

    def with_(self, **kw) -> "EventConfig":
        d = dict(self.__dict__)
        d.update(kw)
        return EventConfig(**d)


P2R_PARITY = EventConfig("p2r-parity-1x1024x10", "barrel", 1, 1024,
                         _f32(np.linspace(4.0, 100.0, 10)), seed=1000)
P2R_THROUGHPUT = EventConfig("p2r-100x9600x20", "barrel", 100, 9600,
                             _f32(np.linspace(2.5, 110.0, 20)), seed=1001)
P2Z_THROUGHPUT = EventConfig("p2z-100x8192x20", "disk", 100, 8192,
                             _f32(np.linspace(30.0, 270.0, 20)), eta=(1.7, 2.5),
                             seed=1002, hit_sigma=(0.01, 0.01, 0.0))
RAGGED = EventConfig("ragged-1M-L5..25", "ragged", 1, 1_000_000, (), eta=(-2.5, 2.5),
                     seed=1003,
                     extra=dict(barrels=_f32(np.linspace(2.5, 110.0, 25)),
                                disks=_f32(np.linspace(30.0, 270.0, 25)),
                                zmax=270.0, rmax=110.0, lmin=5, lmax=25,
                                outlier_frac=0.05, outlier_half=1.0))
LEARNED_EVAL = P2R_THROUGHPUT.with_(name="learned-eval-100x9600x20", seed=1005)
LEARNED_TRAIN_SEED = 1004

# hit covariance for disks: z is exact, a small v_zz keeps S invertible
DISK_VZZ = 1e-4


# ---------------------------------------------------------------- kinematics
def _draw_truth(cfg: EventConfig, n: int):
    g = rng(cfg.seed, _S_KINE)
    pt = g.uniform(cfg.pt[0], cfg.pt[1], n)
    if cfg.kind == "disk":
        eta = g.uniform(cfg.eta[0], cfg.eta[1], n) * np.where(g.random(n) < 0.5, -1.0, 1.0)
    else:
        eta = g.uniform(cfg.eta[0], cfg.eta[1], n)
    phi = g.uniform(-np.pi, np.pi, n)
    q = np.where(g.random(n) < 0.5, -1.0, 1.0)
    gv = rng(cfg.seed, _S_VTX)
    x = gv.normal(0.0, 0.01, n)
    y = gv.normal(0.0, 0.01, n)
    z = gv.normal(0.0, 5.0, n)
    theta = 2.0 * np.arctan(np.exp(-eta))
    return dict(x=x, y=y, z=z, pt=pt, eta=eta, phi=phi, theta=theta, q=q)


def _fit_start(cfg: EventConfig, tr: dict) -> np.ndarray:
    """Truth vertex state smeared with N(0, C0): the fit's starting point."""
    n = tr["x"].shape[0]
    g = rng(cfg.seed, _S_START)
    sig = np.sqrt(C0_DIAG)
    d = g.normal(size=(n, 6)) * sig
    par = np.stack([tr["x"], tr["y"], tr["z"], 1.0 / tr["pt"], tr["phi"], tr["theta"]], 1) + d
    par[:, 3] = np.maximum(par[:, 3], 1e-3)          # 1/pT stays positive
    par[:, 4] = _wrap(par[:, 4])
    return par


def _wrap(a):
    return a - TWO_PI * np.floor((a + np.pi) / TWO_PI)


# ------------------------------------------------------------ RK4 simulator
class _Sim:
    """Vectorised RK4 integrator in 3D path length for many particles."""

    def __init__(self, x, y, z, phi, theta, pt, q, bz=B_TESLA):
        st = np.sin(theta)
        self.s = np.stack([x, y, z, st * np.cos(phi), st * np.sin(phi), np.cos(theta)]).astype(np.float64)
        p = pt / st
        self.k = q * KAPPA * bz / p               # dt/dl = k * (t_y, -t_x, 0)
        self.sinth = st
        self.theta = theta
        self.ipt = 1.0 / pt
        self.path = np.zeros_like(x)             # transverse path travelled

    @staticmethod
    def rk4(s, k, h):
        """One classic RK4 step of length h for every particle.

        The equation of motion is linear in (r, t), so the four RK4 stages
        collapse to the fourth-order Taylor polynomial of the step map;
        it is evaluated in that form (a = k h):
          t' = (1 - a^2/2 + a^4/24) t + (a - a^3/6) J t
          r' = r + h (1 - a^2/6) t + h (a/2 - a^3/24) J t,   J t = (t_y, -t_x, 0)
        """
        a = k * h
        a2 = a * a
        c1 = 1.0 - a2 * (0.5 - a2 / 24.0)
        c2 = a * (1.0 - a2 / 6.0)
        d1 = h * (1.0 - a2 / 6.0)
        d2 = h * a * (0.5 - a2 / 24.0)
        tx, ty, tz = s[3], s[4], s[5]
        return np.stack([s[0] + d1 * tx + d2 * ty, s[1] + d1 * ty - d2 * tx, s[2] + h * tz,
                         c1 * tx + c2 * ty, c1 * ty - c2 * tx, tz])

    @classmethod
    def solve_cylinder(cls, s0, k, R, h_full):
        """Sub-step h in (0, h_full] at which |xy| reaches R (Newton)."""
        r0 = s0[0] ** 2 + s0[1] ** 2
        s1 = cls.rk4(s0, k, h_full)
        r1 = s1[0] ** 2 + s1[1] ** 2
        h = h_full * np.clip((R * R - r0) / np.maximum(r1 - r0, 1e-300), 0.0, 1.0)
        for _ in range(5):
            sh = cls.rk4(s0, k, h)
            g = sh[0] ** 2 + sh[1] ** 2 - R * R
            dg = 2.0 * (sh[0] * sh[3] + sh[1] * sh[4])
            dg = np.where(np.abs(dg) < 1e-30, 1e-30, dg)
            h = np.clip(h - g / dg, 0.0, h_full)
        return h

    @staticmethod
    def solve_plane(s0, Z):
        return (Z - s0[2]) / s0[5]


def _state_of(s, ipt, theta):
    """Truth track parameters from a simulator state (columns)."""
    return np.stack([s[0], s[1], s[2], ipt, np.arctan2(s[4], s[3]), theta], -1)


_CHUNK = 16384


def _chunked(fn, arrays, *rest):
    """Run fn over slices of the per-particle arrays and concatenate (cache-sized work)."""
    n = arrays[0].shape[0]
    if n <= _CHUNK:
        return fn(*arrays, *rest)
    parts = [fn(*[a[i:i + _CHUNK] for a in arrays], *rest) for i in range(0, n, _CHUNK)]
    return tuple(np.concatenate([p[j] for p in parts]) for j in range(len(parts[0])))


def simulate_barrels(x, y, z, phi, theta, pt, q, radii, bz=B_TESLA):
    return _chunked(_simulate_barrels, (x, y, z, phi, theta, pt, q), radii, bz)


def simulate_disks(x, y, z, phi, theta, pt, q, zabs, bz=B_TESLA):
    return _chunked(_simulate_disks, (x, y, z, phi, theta, pt, q), zabs, bz)


def _simulate_barrels(x, y, z, phi, theta, pt, q, radii, bz=B_TESLA):
    """Truth crossings of concentric cylinders, innermost first.

    Returns (pos [n,L,3], state [n,L,6], path [n,L]) with NaN where the
    particle turns back before reaching the layer (and all layers beyond).
    path is the transverse arc length from the start to the crossing.
    """
    n, L = x.shape[0], len(radii)
    radii = np.asarray(radii, dtype=np.float64)
    sim = _Sim(x, y, z, phi, theta, pt, q, bz)
    pos = np.full((n, L, 3), np.nan)
    state = np.full((n, L, 6), np.nan)
    path = np.full((n, L), np.nan)
    nxt = np.zeros(n, dtype=np.int64)
    alive = np.ones(n, dtype=bool)
    while True:
        idx = np.nonzero(alive)[0]
        if idx.size == 0:
            break
        s0 = sim.s[:, idx]
        k = sim.k[idx]
        st = sim.sinth[idx]
        h = STEP_CM / st
        s1 = _Sim.rk4(s0, k, h)
        R = radii[nxt[idx]]
        r0 = np.hypot(s0[0], s0[1])
        r1 = np.hypot(s1[0], s1[1])
        cross = r1 >= R
        turned = (~cross) & (r1 < r0)           # past its largest radius
        # accept full steps
        acc = ~cross
        sim.s[:, idx[acc]] = s1[:, acc]
        sim.path[idx[acc]] += STEP_CM
        # crossings: land exactly on the layer
        if cross.any():
            c = np.nonzero(cross)[0]
            hc = _Sim.solve_cylinder(s0[:, c], k[c], R[c], h[c])
            sc = _Sim.rk4(s0[:, c], k[c], hc)
            ic = idx[c]
            sim.s[:, ic] = sc
            sim.path[ic] += hc * st[c]
            li = nxt[ic]
            pos[ic, li] = sc[:3].T
            state[ic, li] = _state_of(sc, sim.ipt[ic], sim.theta[ic])
            path[ic, li] = sim.path[ic]
            nxt[ic] += 1
        alive[idx[turned]] = False
        alive &= nxt < L
    return pos, state, path


def simulate_to_cylinder(par, q, R, bz=B_TESLA, max_path=400.0):
    """Transverse path length from each state to its first crossing of |xy|=R.

    par: (n,6) track parameters; R: (n,) radii.  NaN when not reached.
    """
    par = np.asarray(par, dtype=np.float64)
    R = np.broadcast_to(np.asarray(R, dtype=np.float64), (par.shape[0],))
    q = np.broadcast_to(np.asarray(q, dtype=np.float64), (par.shape[0],))
    return _chunked(lambda p, qq, rr: (_simulate_to_cylinder(p, qq, rr, bz, max_path),), (par, q, R))[0]


def _simulate_to_cylinder(par, q, R, bz, max_path):
    n = par.shape[0]
    sim = _Sim(par[:, 0], par[:, 1], par[:, 2], par[:, 4], par[:, 5], 1.0 / par[:, 3], q, bz)
    out = np.full(n, np.nan)
    alive = np.ones(n, dtype=bool)
    R = np.asarray(R, dtype=np.float64)
    rstart = np.hypot(par[:, 0], par[:, 1])
    outward = R >= rstart
    while True:
        idx = np.nonzero(alive)[0]
        if idx.size == 0:
            break
        s0 = sim.s[:, idx]
        k = sim.k[idx]
        st = sim.sinth[idx]
        h = STEP_CM / st
        s1 = _Sim.rk4(s0, k, h)
        Ri = R[idx]
        r0 = np.hypot(s0[0], s0[1])
        r1 = np.hypot(s1[0], s1[1])
        cross = np.where(outward[idx], (r0 < Ri) & (r1 >= Ri), (r0 > Ri) & (r1 <= Ri))
        acc = ~cross
        sim.s[:, idx[acc]] = s1[:, acc]
        sim.path[idx[acc]] += STEP_CM
        if cross.any():
            c = np.nonzero(cross)[0]
            hc = _Sim.solve_cylinder(s0[:, c], k[c], Ri[c], h[c])
            ic = idx[c]
            out[ic] = sim.path[ic] + hc * st[c]
            alive[ic] = False
        alive[idx[acc & (sim.path[idx] > max_path)]] = False
    return out


def _simulate_disks(x, y, z, phi, theta, pt, q, zabs, bz=B_TESLA):
    """Truth crossings of the planes z = sign(cot theta) * zabs[i]."""
    n, L = x.shape[0], len(zabs)
    zabs = np.asarray(zabs, dtype=np.float64)
    sim = _Sim(x, y, z, phi, theta, pt, q, bz)
    sgn = np.sign(np.cos(theta))
    pos = np.full((n, L, 3), np.nan)
    state = np.full((n, L, 6), np.nan)
    path = np.full((n, L), np.nan)
    for li in range(L):
        Z = sgn * zabs[li]
        remaining = (Z - sim.s[2]) / sim.s[5]          # 3D length to the plane
        # march in full steps while the plane is farther than one step
        while True:
            h = STEP_CM / sim.sinth
            far = remaining > h
            if not far.any():
                break
            idx = np.nonzero(far)[0]
            sim.s[:, idx] = _Sim.rk4(sim.s[:, idx], sim.k[idx], h[idx])
            sim.path[idx] += STEP_CM
            remaining[idx] = (Z[idx] - sim.s[2, idx]) / sim.s[5, idx]
        sim.s = _Sim.rk4(sim.s, sim.k, remaining)
        sim.path += remaining * sim.sinth
        sim.s[2] = Z                                    # t_z is constant
        pos[:, li] = sim.s[:3].T
        state[:, li] = _state_of(sim.s, sim.ipt, sim.theta)
        path[:, li] = sim.path
    return pos, state, path


# -------------------------------------------------------------------- events
def _barrel_hits(cfg, pos, g):
    n, L, _ = pos.shape
    sx, sy, sz = cfg.hit_sigma
    hits = pos + g.normal(size=(n, L, 3)) * np.array([sx, sy, sz])
    V = np.zeros((n, L, 6))
    V[..., 0], V[..., 2], V[..., 5] = sx * sx, sy * sy, sz * sz
    return hits, V


def make_barrel_event(cfg: EventConfig = P2R_PARITY, n_tracks: int | None = None):
    """p2r workload: fit starts, hits on fixed-r cylinders, truth.

    Returns a dict of float64 arrays already rounded to float32 values
    (what the GPU sees), plus float64 truth:
      par [n,6], cov [n,21], q [n], hits [n,L,3], hitcov [n,L,6],
      radii [L], truth [n,L,6], truth_start [n,6], path [n,L]
    n_tracks overrides n_events*n_tracks (takes the first n of the stream).
    """
    assert cfg.kind == "barrel"
    n = cfg.n_total if n_tracks is None else n_tracks
    tr = _draw_truth(cfg, n)
    pos, state, path = simulate_barrels(tr["x"], tr["y"], tr["z"], tr["phi"], tr["theta"],
                                        tr["pt"], tr["q"], cfg.surfaces)
    hits, V = _barrel_hits(cfg, pos, rng(cfg.seed, _S_HIT))
    par = _fit_start(cfg, tr)
    return _finish(cfg, tr, par, hits, V, state, path, np.asarray(cfg.surfaces, dtype=np.float64))


def make_disk_event(cfg: EventConfig = P2Z_THROUGHPUT, n_tracks: int | None = None):
    """p2z workload on planes at z = +-surfaces (sign of eta); |z| in 'zabs'."""
    assert cfg.kind == "disk"
    n = cfg.n_total if n_tracks is None else n_tracks
    tr = _draw_truth(cfg, n)
    pos, state, path = simulate_disks(tr["x"], tr["y"], tr["z"], tr["phi"], tr["theta"],
                                      tr["pt"], tr["q"], cfg.surfaces)
    g = rng(cfg.seed, _S_HIT)
    sx, sy, _ = cfg.hit_sigma
    L = len(cfg.surfaces)
    hits = pos.copy()
    hits[..., 0] += g.normal(size=(n, L)) * sx
    hits[..., 1] += g.normal(size=(n, L)) * sy
    V = np.zeros((n, L, 6))
    V[..., 0], V[..., 2], V[..., 5] = sx * sx, sy * sy, DISK_VZZ
    par = _fit_start(cfg, tr)
    return _finish(cfg, tr, par, hits, V, state, path, np.asarray(cfg.surfaces, dtype=np.float64))


def _finish(cfg, tr, par, hits, V, state, path, surf):
    f32 = lambda a: a.astype(np.float32).astype(np.float64)  # noqa: E731
    n = par.shape[0]
    cov = np.tile(pack21(np.diag(C0_DIAG)), (n, 1))
    truth_start = np.stack([tr["x"], tr["y"], tr["z"], 1.0 / tr["pt"], tr["phi"], tr["theta"]], 1)
    return dict(par=f32(par), cov=f32(cov), q=tr["q"].copy(), hits=f32(hits), hitcov=f32(V),
                surf=f32(surf), truth=state, truth_start=truth_start, path=path,
                name=cfg.name, n_events=cfg.n_events)


# -------------------------------------------------------------------- ragged
def make_ragged_event(cfg: EventConfig = RAGGED, n_tracks: int | None = None):
    """Mixed barrel/disk tracks with per-track surface lists (CSR).

    Geometry: cylinders at extra['barrels'] (|z| <= zmax) and planes at
    +-extra['disks'] (r <= rmax).  Walking the truth trajectory, the
    surfaces are taken in the order they are crossed (outward barrels not yet
    crossed, disks on the side the particle moves to), up to L ~ U{lmin..lmax}
    per track; the walk stops early when the particle leaves the volume, or
    when it has turned by half a turn since its last surface (a looper, which
    the fit does not follow either).  A fraction of hits are outliers:
    the crossing moved uniformly within +-outlier_half cm in the surface's
    local coordinates (r-phi arc and z on cylinders, x and y on planes),
    with the hit covariance unchanged.

    Returns dict with offsets [n+1] (int64), surf_type [H] (uint8, 0 barrel
    1 disk), surf_val [H] (radius, or signed z), hits [H,3], hitcov [H,6],
    par [n,6], cov [n,21], q [n], truth [H,6], outlier [H] (bool).
    """
    ex = cfg.extra
    n = cfg.n_total if n_tracks is None else n_tracks
    tr = _draw_truth(cfg, n)
    Lwant = rng(cfg.seed, _S_LEN).integers(ex["lmin"], ex["lmax"] + 1, n)
    barrels = np.asarray(ex["barrels"], dtype=np.float64)
    disks = np.asarray(ex["disks"], dtype=np.float64)
    nb, nd = len(barrels), len(disks)
    zmax, rmax = ex["zmax"], ex["rmax"]
    sim = _Sim(tr["x"], tr["y"], tr["z"], tr["phi"], tr["theta"], tr["pt"], tr["q"])
    sgn = np.sign(np.cos(tr["theta"]))
    kb = np.zeros(n, dtype=np.int64)
    kd = np.zeros(n, dtype=np.int64)
    cnt = np.zeros(n, dtype=np.int64)
    Lmax = int(ex["lmax"])
    s_type = np.full((n, Lmax), 255, dtype=np.uint8)
    s_val = np.zeros((n, Lmax))
    s_state = np.full((n, Lmax, 6), np.nan)
    alive = np.ones(n, dtype=bool)
    last = np.zeros(n)                      # transverse path at the last recorded surface
    half_turn = np.pi * tr["pt"] / (KAPPA * B_TESLA)
    while True:
        idx = np.nonzero(alive)[0]
        if idx.size == 0:
            break
        s0 = sim.s[:, idx]
        k = sim.k[idx]
        st = sim.sinth[idx]
        h = STEP_CM / st
        s1 = _Sim.rk4(s0, k, h)
        r0 = np.hypot(s0[0], s0[1])
        r1 = np.hypot(s1[0], s1[1])
        hasb = kb[idx] < nb
        Rb = barrels[np.minimum(kb[idx], nb - 1)]
        cb = hasb & (r1 >= Rb)
        hasd = kd[idx] < nd
        Zd = sgn[idx] * disks[np.minimum(kd[idx], nd - 1)]
        hd_all = _Sim.solve_plane(s0, Zd)
        cd = hasd & (hd_all <= h) & (hd_all >= 0.0)
        hb = np.full(idx.size, np.inf)
        if cb.any():
            c = np.nonzero(cb)[0]
            hb[c] = _Sim.solve_cylinder(s0[:, c], k[c], Rb[c], h[c])
        hdd = np.where(cd, hd_all, np.inf)
        event = cb | cd
        take_b = cb & (hb <= hdd)
        take_d = cd & ~take_b
        hev = np.where(take_b, hb, hdd)
        # no event: full step
        acc = ~event
        sim.s[:, idx[acc]] = s1[:, acc]
        sim.path[idx[acc]] += STEP_CM
        # barrels past their largest radius cannot be reached any more
        kb[idx[acc & (r1 < r0)]] = nb
        if event.any():
            e = np.nonzero(event)[0]
            se = _Sim.rk4(s0[:, e], k[e], hev[e])
            ie = idx[e]
            tb = take_b[e]
            se[2, ~tb] = Zd[e][~tb]
            sim.s[:, ie] = se
            sim.path[ie] += hev[e] * st[e]
            valid = np.where(tb, np.abs(se[2]) <= zmax, np.hypot(se[0], se[1]) <= rmax)
            iv = ie[valid]
            slot = cnt[iv]
            s_type[iv, slot] = np.where(tb[valid], 0, 1)
            s_val[iv, slot] = np.where(tb[valid], Rb[e][valid], Zd[e][valid])
            s_state[iv, slot] = _state_of(se[:, valid], sim.ipt[iv], sim.theta[iv])
            cnt[iv] += 1
            last[iv] = sim.path[iv]
            kb[ie[tb]] += 1
            kd[ie[~tb]] += 1
        done = (cnt >= Lwant) | ((kb >= nb) & (kd >= nd)) | (sim.path - last > half_turn)
        done |= (np.hypot(sim.s[0], sim.s[1]) > rmax) & (np.abs(sim.s[2]) > zmax)
        alive &= ~done
    # CSR
    offsets = np.zeros(n + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(cnt)
    mask = np.arange(Lmax)[None, :] < cnt[:, None]
    surf_type = s_type[mask]
    surf_val = s_val[mask]
    truth = s_state[mask]
    H = surf_type.shape[0]
    g = rng(cfg.seed, _S_HIT)
    hits = truth[:, :3].copy()
    barrel = surf_type == 0
    sx, sy, sz = cfg.hit_sigma
    noise = g.normal(size=(H, 3))
    hits[barrel] += noise[barrel] * np.array([sx, sy, sz])
    hits[~barrel, 0] += noise[~barrel, 0] * sx
    hits[~barrel, 1] += noise[~barrel, 1] * sy
    V = np.zeros((H, 6))
    V[:, 0], V[:, 2] = sx * sx, sy * sy
    V[:, 5] = np.where(barrel, sz * sz, DISK_VZZ)
    # outliers
    go = rng(cfg.seed, _S_OUTL)
    outl = go.random(H) < ex["outlier_frac"]
    a = go.uniform(-ex["outlier_half"], ex["outlier_half"], H)
    b = go.uniform(-ex["outlier_half"], ex["outlier_half"], H)
    ob = outl & barrel
    rr = np.hypot(truth[ob, 0], truth[ob, 1])
    ang = np.arctan2(truth[ob, 1], truth[ob, 0]) + a[ob] / rr
    hits[ob, 0] = rr * np.cos(ang)
    hits[ob, 1] = rr * np.sin(ang)
    hits[ob, 2] = truth[ob, 2] + b[ob]
    od = outl & ~barrel
    hits[od, 0] = truth[od, 0] + a[od]
    hits[od, 1] = truth[od, 1] + b[od]
    hits[od, 2] = truth[od, 2]
    par = _fit_start(cfg, tr)
    f32 = lambda v: v.astype(np.float32).astype(np.float64)  # noqa: E731
    cov = np.tile(pack21(np.diag(C0_DIAG)), (n, 1))
    return dict(offsets=offsets, surf_type=surf_type, surf_val=f32(surf_val), hits=f32(hits),
                hitcov=f32(V), par=f32(par), cov=f32(cov), q=tr["q"].copy(), truth=truth,
                outlier=outl, name=cfg.name)


# ------------------------------------------------------------------ learned
def make_mlp_pairs(n_tracks: int, seed: int = LEARNED_TRAIN_SEED, cfg: EventConfig = P2R_THROUGHPUT):
    """(state, q, R) -> transverse path length pairs for the path-length MLP.

    States: the fit start (paired with the first layer), and truth states on
    layer l moved along the surface by fit-like errors (paired with layer
    l+1).  Labels: transverse path to the first crossing of the target
    cylinder, from the RK4 simulation of each paired state.  Pairs with no
    crossing are dropped.  Returns par [m,6], q [m], R [m], s [m] (float64,
    par rounded to float32 values).
    """
    c = cfg.with_(seed=seed, n_events=1, n_tracks=n_tracks)
    tr = _draw_truth(c, n_tracks)
    radii = np.asarray(c.surfaces, dtype=np.float64)
    _, state, _ = simulate_barrels(tr["x"], tr["y"], tr["z"], tr["phi"], tr["theta"], tr["pt"],
                                   tr["q"], radii)
    start = _fit_start(c, tr)
    L = radii.shape[0]
    g = rng(seed, _S_PAIR)
    pars = [start]
    Rs = [np.full(n_tracks, radii[0])]
    qs = [tr["q"]]
    for li in range(L - 1):
        st = state[:, li].copy()
        ok = np.isfinite(st[:, 0])
        st = st[ok]
        m = st.shape[0]
        r = np.hypot(st[:, 0], st[:, 1])
        ang = np.arctan2(st[:, 1], st[:, 0]) + g.normal(0.0, 0.01, m) / r
        st[:, 0], st[:, 1] = r * np.cos(ang), r * np.sin(ang)
        st[:, 2] += g.normal(0.0, 0.05, m)
        st[:, 3] *= 1.0 + g.normal(0.0, 0.01, m)
        st[:, 4] = _wrap(st[:, 4] + g.normal(0.0, 1e-3, m))
        st[:, 5] += g.normal(0.0, 1e-3, m)
        pars.append(st)
        Rs.append(np.full(m, radii[li + 1]))
        qs.append(tr["q"][ok])
    par = np.concatenate(pars).astype(np.float32).astype(np.float64)
    R = np.concatenate(Rs)
    q = np.concatenate(qs)
    s = simulate_to_cylinder(par, q, R)
    ok = np.isfinite(s)
    return dict(par=par[ok], q=q[ok], R=R[ok], s=s[ok])


def make_mlp_init(seed: int = LEARNED_TRAIN_SEED, n_in: int = 7, n_hid: int = 64):
    """Initial weights (uniform, fan-in scaled) of the n_in->n_hid->n_hid->1 MLP.

    Returns float32 arrays W1 [h,n_in], b1 [h], W2 [h,h], b2 [h], W3 [1,h], b3 [1].
    """
    g = rng(seed, _S_MLP)

    def u(shape, fan_in):
        lim = np.sqrt(6.0 / fan_in)
        return g.uniform(-lim, lim, shape).astype(np.float32)

    return dict(W1=u((n_hid, n_in), n_in), b1=np.zeros(n_hid, np.float32),
                W2=u((n_hid, n_hid), n_hid), b2=np.zeros(n_hid, np.float32),
                W3=(u((1, n_hid), n_hid) * 0.1).astype(np.float32), b3=np.zeros(1, np.float32))
