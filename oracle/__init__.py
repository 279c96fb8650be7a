"""FP64 CPU oracle of the track fit (test infrastructure only).

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg
use this package.  It wraps ``liboracle.so`` (plain C++17, built with g++
from ``oracle.cpp`` by :func:`build`) and the NumPy MLP reference in
:mod:`oracle.mlp`.  Nothing here is shared with the GPU library.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None

ST_NO_CROSSING = 1 << 0
ST_NEWTON_FAIL = 1 << 1
ST_FP64_FALLBACK = 1 << 2
ST_S_NOT_PD = 1 << 3
ST_BAD_INPUT = 1 << 4
ST_ML_REJECTED = 1 << 5
ST_HIT_MISSING = 1 << 6
ST_CHI2_CUT = 1 << 7
ST_DONE = 1 << 31
HALF_PI_F32 = float(np.float32(np.pi / 2))


def build() -> str:
    """Compile liboracle.so with g++ (-O2, no fast-math)."""
    cmd = ["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-pthread",
           os.path.join(_HERE, "oracle.cpp"), "-o", _SO + ".tmp"]
    subprocess.run(cmd, check=True)
    os.replace(_SO + ".tmp", _SO)
    return _SO


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        L = C.CDLL(_SO)
        dp = C.POINTER(C.c_double)
        L.orc_helix.argtypes = [dp, C.c_double, C.c_double, C.c_double, dp]
        L.orc_path.argtypes = [dp, C.c_double, C.c_double, C.c_int, C.c_double, dp]
        L.orc_path.restype = C.c_int
        L.orc_propagate.argtypes = [dp, C.c_double, C.c_double, C.c_int, C.c_double, dp, dp, dp]
        L.orc_propagate.restype = C.c_int
        L.orc_update.argtypes = [dp, dp, dp, dp, C.c_int, C.c_double, dp, dp, dp]
        L.orc_update.restype = C.c_uint32
        L.orc_update_2d.argtypes = [dp, dp, dp, dp, C.c_double, dp, dp, dp]
        L.orc_update_2d.restype = C.c_uint32
        L.orc_fit.argtypes = [C.c_int64] + [C.c_void_p] * 8 + [C.c_double, C.c_double, C.c_int, C.c_int, C.c_int,
                                                               C.c_int] + [C.c_void_p] * 8
        L.orc_fit.restype = None
        L.orc_disk_sign.argtypes = [C.c_double]
        L.orc_disk_sign.restype = C.c_double
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a if shape is None else a.reshape(shape)


# ------------------------------------------------------------ single track
def helix(p, q, bz, s):
    p = _f64(p, (6,))
    out = np.zeros(6)
    lib().orc_helix(_dp(p), float(q), float(bz), float(s), _dp(out))
    return out


def path(p, q, bz, stype, v):
    """Transverse path to the surface, or None when it is not reached."""
    p = _f64(p, (6,))
    s = np.zeros(1)
    ok = lib().orc_path(_dp(p), float(q), float(bz), int(stype), float(v), _dp(s))
    return float(s[0]) if ok else None


def propagate(p, q, bz, stype, v):
    """(state after, 6x6 Jacobian, path) or None when the surface is missed."""
    p = _f64(p, (6,))
    out, J, s = np.zeros(6), np.zeros(36), np.zeros(1)
    ok = lib().orc_propagate(_dp(p), float(q), float(bz), int(stype), float(v), _dp(out), _dp(J), _dp(s))
    if not ok:
        return None
    return out, J.reshape(6, 6), float(s[0])


def update(p, C6, m, V21, form=0, chi2_cut=0.0):
    """Kalman update on full matrices: (status, p+, C+ 6x6, chi2)."""
    p, C6, m, V21 = _f64(p, (6,)), _f64(C6, (36,)), _f64(m, (3,)), _f64(V21, (6,))
    po, Co, c2 = np.zeros(6), np.zeros(36), np.zeros(1)
    st = lib().orc_update(_dp(p), _dp(C6), _dp(m), _dp(V21), int(form), float(chi2_cut),
                          _dp(po), _dp(Co), _dp(c2))
    return int(st), po, Co.reshape(6, 6), float(c2[0])


def update_2d(p, C6, m, V21, chi2_cut=0.0):
    """Update in the hit's (r-phi, z) frame on a cylinder: (status, p+, C+ 6x6, chi2)."""
    p, C6, m, V21 = _f64(p, (6,)), _f64(C6, (36,)), _f64(m, (3,)), _f64(V21, (6,))
    po, Co, c2 = np.zeros(6), np.zeros(36), np.zeros(1)
    st = lib().orc_update_2d(_dp(p), _dp(C6), _dp(m), _dp(V21), float(chi2_cut), _dp(po), _dp(Co), _dp(c2))
    return int(st), po, Co.reshape(6, 6), float(c2[0])


# ------------------------------------------------------------------ batches
SENS_RUNS = 4   # conditioning-measurement runs: round to nearest + 3 random-rounding seeds


def fit(par, cov, q, offsets, stype, sval, hits, hitcov, bz=3.8, chi2_cut=0.0, form=0,
        nthreads=0, layers=False, update_2d=False, sensitivity=True, round32=0):
    """Per-track fit over CSR surface lists; returns a dict of outputs.

    update_2d: cylinders take the update in the hit's (r-phi, z) frame.
    round32 (0: the exact FP64 fit): the fit as an FP32 implementation
    computes it -- stored values, the matrix algebra and the cylinder
    crossing rounded to FP32 -- with round-to-nearest (1) or random rounding
    seeded by the value (>= 2).  sensitivity: also run SENS_RUNS such fits
    (modes 1 .. SENS_RUNS) and return their outputs as a list under
    "f32_runs" (the first also as "f32"): how far FP32 rounding moves each
    track's result, which the parity rule uses as the track's conditioning."""
    par, cov, q = _f64(par), _f64(cov), _f64(q)
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    stype = np.ascontiguousarray(stype, dtype=np.uint8)
    sval, hits, hitcov = _f64(sval), _f64(hits), _f64(hitcov)
    n = par.shape[0]
    H = int(offsets[-1])
    assert par.shape == (n, 6) and cov.shape == (n, 21) and q.shape == (n,)
    assert offsets.shape == (n + 1,) and stype.shape == (H,) and sval.shape == (H,)
    assert hits.shape == (H, 3) and hitcov.shape == (H, 6)
    out = dict(par=np.zeros((n, 6)), cov=np.zeros((n, 21)), chi2=np.zeros(n),
               nused=np.zeros(n, np.int32), status=np.zeros(n, np.uint32))
    if layers:
        out.update(lay_par=np.zeros((H, 6)), lay_cov=np.zeros((H, 21)), lay_chi2=np.zeros(H))
    vp = lambda a: a.ctypes.data_as(C.c_void_p)  # noqa: E731
    lp = [vp(out[k]) if layers else None for k in ("lay_par", "lay_cov", "lay_chi2")] if layers \
        else [None, None, None]
    lib().orc_fit(n, vp(par), vp(cov), vp(q), vp(offsets), vp(stype), vp(sval), vp(hits), vp(hitcov),
                  float(bz), float(chi2_cut), int(form), int(bool(update_2d)), int(round32), int(nthreads),
                  vp(out["par"]), vp(out["cov"]), vp(out["chi2"]), vp(out["nused"]), vp(out["status"]),
                  *lp)
    if sensitivity and not round32:
        out["f32_runs"] = [fit(par, cov, q, offsets, stype, sval, hits, hitcov, bz=bz, chi2_cut=chi2_cut,
                               form=form, nthreads=nthreads, update_2d=update_2d, sensitivity=False, round32=k)
                           for k in range(1, SENS_RUNS + 1)]
        out["f32"] = out["f32_runs"][0]
    return out


def disk_sign(theta):
    """+1 when the track moves to +z (theta below float32(pi/2)), else -1."""
    return np.where(np.asarray(theta) < HALF_PI_F32, 1.0, -1.0)


def fit_layers(par, cov, q, hits, hitcov, surf, kind, **kw):
    """Fit with the same ordered surfaces for every track.

    kind 'barrel': surf are radii; 'disk': surf are |z|, placed on the side
    given by the sign of each track's starting theta.
    """
    n, L = hits.shape[0], hits.shape[1]
    offsets = np.arange(n + 1, dtype=np.int64) * L
    surf = np.asarray(surf, dtype=np.float64)
    if kind == "barrel":
        stype = np.zeros(n * L, np.uint8)
        sval = np.tile(surf, n)
    else:
        stype = np.ones(n * L, np.uint8)
        sval = (disk_sign(np.asarray(par)[:, 5])[:, None] * surf[None, :]).reshape(-1)
    return fit(par, cov, q, offsets, stype, sval, np.reshape(hits, (-1, 3)), np.reshape(hitcov, (-1, 6)), **kw)


def fit_event(ev: dict, kind: str, **kw):
    return fit_layers(ev["par"], ev["cov"], ev["q"], ev["hits"], ev["hitcov"], ev["surf"], kind, **kw)


def fit_ragged(ev: dict, **kw):
    return fit(ev["par"], ev["cov"], ev["q"], ev["offsets"], ev["surf_type"], ev["surf_val"],
               ev["hits"], ev["hitcov"], **kw)
