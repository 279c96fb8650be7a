"""ctypes binding of libp2r.so; same names and arguments as include/p2r.h."""
from __future__ import annotations

import ctypes as C
import os
import re

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libp2r.so")
_HEADER = os.path.join(os.path.dirname(_HERE), "include", "p2r.h")

P2R_OK, P2R_EINVAL, P2R_ELAYOUT, P2R_EHIP, P2R_ENOTUNED, P2R_ENOSPACE = 0, -1, -2, -3, -4, -5
ST_NO_CROSSING = 1 << 0
ST_NEWTON_FAIL = 1 << 1
ST_FP64_FALLBACK = 1 << 2
ST_S_NOT_PD = 1 << 3
ST_BAD_INPUT = 1 << 4
ST_ML_REJECTED = 1 << 5
ST_HIT_MISSING = 1 << 6
ST_CHI2_CUT = 1 << 7
ST_DONE = 1 << 31


def _header_define(name: str) -> int:
    """Integer value of a #define in include/p2r.h (one source for the limits)."""
    m = re.search(rf"^#define {name} \(?(-?\d+)", open(_HEADER).read(), flags=re.M)
    if not m:
        raise RuntimeError(f"{name} is not defined in {_HEADER}")
    return int(m.group(1))


P2R_MAX_HITS = _header_define("P2R_MAX_HITS")
P2R_NOALLOC_MAX_TRACKS = _header_define("P2R_NOALLOC_MAX_TRACKS")


class P2RError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libp2r error {code}: {msg}")
        self.code = code


class Opts(C.Structure):
    _fields_ = [("bz_tesla", C.c_float), ("newton_tol_cm", C.c_float), ("newton_max_iter", C.c_int32),
                ("chi2_cut", C.c_float), ("fp64_fallback", C.c_int32), ("width", C.c_int32),
                ("mlp", C.c_void_p), ("use_graph", C.c_int32), ("helix_evals", C.c_void_p),
                ("cyl_start", C.c_int32), ("fp64", C.c_int32), ("update_2d", C.c_int32)]


_lib = None
vp = C.c_void_p


def library_path() -> str:
    return _SO


def library():
    """Load libp2r.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            raise RuntimeError(f"{_SO} is missing: build it with python paper_2401_14221_amd/build.py")
        L = C.CDLL(_SO)
        i32, i64 = C.c_int32, C.c_int64
        L.p2r_opts_default.argtypes = [C.POINTER(Opts)]
        L.p2r_opts_default.restype = None
        L.p2r_last_error.restype = C.c_char_p
        L.p2r_version.restype = C.c_char_p
        L.p2r_ctx_create.argtypes = [C.POINTER(vp), C.c_int, C.c_char_p]
        L.p2r_ctx_destroy.argtypes = [vp]
        L.p2r_ctx_destroy.restype = None
        L.p2r_layout_width.argtypes = [vp, C.c_int, C.POINTER(i32)]
        L.p2r_variant_name.argtypes = [vp, C.c_int]
        L.p2r_variant_name.restype = C.c_char_p
        for f in (L.p2r_propagate_update, L.p2z_propagate_update):
            f.argtypes = [vp, C.POINTER(Opts), i32, i32, vp, vp, vp, vp, vp, vp, vp]
        L.p2r_autotune.argtypes = [vp, C.c_int, i32, i32, vp]
        for f in (L.p2r_propagate_update_host, L.p2z_propagate_update_host):
            f.argtypes = [vp, C.POINTER(Opts), i32, i32, vp, vp, vp, vp, vp, vp, i32, vp]
        L.p2r_set_variant.argtypes = [vp, C.c_int, C.c_char_p]
        L.p2r_variant_at.argtypes = [C.c_int, C.c_int]
        L.p2r_variant_at.restype = C.c_char_p
        L.fit_tracks_batched.argtypes = [vp, C.POINTER(Opts), i32, i64, i32] + [vp] * 13
        L.fit_tracks_batched_noalloc.argtypes = [vp, C.POINTER(Opts), i32, i64, i32] + [vp] * 13
        L.p2r_ctx_reserve.argtypes = [vp, i32, i32]
        L.p2r_device_allocations.restype = C.c_ulonglong
        L.p2r_ctx_reserve_host.argtypes = [vp, i32, i32]
        L.p2r_mlp_create.argtypes = [vp, C.POINTER(vp), C.c_uint64]
        L.p2r_mlp_reserve.argtypes = [vp, i32]
        L.p2r_mlp_destroy.argtypes = [vp]
        L.p2r_mlp_destroy.restype = None
        L.p2r_mlp_n_params.restype = C.c_int
        L.p2r_mlp_set_params.argtypes = [vp, vp]
        L.p2r_mlp_get_params.argtypes = [vp, vp]
        L.p2r_mlp_features.argtypes = [vp, C.POINTER(Opts), i32] + [vp] * 7 + [vp]
        L.p2r_mlp_forward.argtypes = [vp, vp, vp, i32, vp]
        L.p2r_mlp_grads.argtypes = [vp, vp, vp, i32, vp, vp, vp]
        L.p2r_mlp_train_step.argtypes = [vp, vp, vp, i32, C.c_float, vp, vp]
        L.p2r_mlp_save.argtypes = [vp, C.c_char_p]
        L.p2r_mlp_load.argtypes = [vp, C.c_char_p]
        _lib = L
    return _lib


def device_allocations() -> int:
    """Device allocations the library has made in this process."""
    return int(library().p2r_device_allocations())


def exported_symbols():
    """Names of the functions include/p2r.h declares."""
    txt = open(_HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[\w\s\*]+?\b(\w+)\s*\(", txt, flags=re.M)) - {"defined"})


def variant_names(which: int) -> list:
    """Names of the compiled plain variants for which (0 p2r, 1 p2z, 2 ragged)."""
    out, i = [], 0
    while True:
        nm = library().p2r_variant_at(which, i)
        if nm is None:
            return out
        out.append(nm.decode())
        i += 1


def _check(rc):
    if rc != 0:
        raise P2RError(rc, library().p2r_last_error().decode())


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def default_opts(**kw) -> Opts:
    o = Opts()
    library().p2r_opts_default(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


class Context:
    """A libp2r context on one device (tuned variants, workspace, graphs)."""

    def __init__(self, device: int = 0, tune_cache: str | None = None):
        if not torch.cuda.is_available():
            raise RuntimeError("libp2r needs a HIP GPU; none is visible")
        self.device = device
        self._ragged_cap = (0, -1)          # (tracks, surfaces per track) reserved
        self._h = vp()
        _check(library().p2r_ctx_create(C.byref(self._h), device,
                                        tune_cache.encode() if tune_cache else None))

    def close(self):
        if self._h:
            library().p2r_ctx_destroy(self._h)
            self._h = vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # --------------------------------------------------------------- info
    def layout_width(self, which: int = 0) -> int:
        w = C.c_int32()
        _check(library().p2r_layout_width(self._h, which, C.byref(w)))
        return w.value

    def variant_name(self, which: int = 0) -> str:
        return library().p2r_variant_name(self._h, which).decode()

    def set_variant(self, which: int, name: str):
        _check(library().p2r_set_variant(self._h, which, name.encode()))

    def autotune(self, which: int, n_tracks: int, n_layers: int, stream=None):
        _check(library().p2r_autotune(self._h, which, n_tracks, n_layers, _stream(stream)))
        if which == 2:                      # the ragged tuner reserves the workspace for its shape
            self._ragged_cap = (max(self._ragged_cap[0], n_tracks), max(self._ragged_cap[1], n_layers))

    def reserve(self, max_tracks: int, max_surfaces: int):
        """Size the ragged workspace (p2r_ctx_reserve); grow-only."""
        _check(library().p2r_ctx_reserve(self._h, int(max_tracks), int(max_surfaces)))
        self._ragged_cap = (max(self._ragged_cap[0], int(max_tracks)), max(self._ragged_cap[1], int(max_surfaces)))

    def reserve_host(self, max_layers: int, chunk_tracks: int = 0):
        """Size the host pipeline's staging (p2r_ctx_reserve_host); grow-only."""
        _check(library().p2r_ctx_reserve_host(self._h, int(max_layers), int(chunk_tracks)))

    # --------------------------------------------------------------- fits
    def _outputs(self, trk_in, n):
        dev = trk_in.device
        return (torch.empty_like(trk_in), torch.empty(n, dtype=torch.float32, device=dev),
                torch.empty(n, dtype=torch.int32, device=dev))

    def p2r_propagate_update(self, n_tracks, layer_r, trk_in, hits, out=None, opts=None, stream=None, **kw):
        """p2r fit of AoSoA tracks; returns (trk_out, chi2, status) device tensors."""
        opts = opts or default_opts(**kw)
        trk_out, chi2, status = out if out is not None else self._outputs(trk_in, n_tracks)
        _check(library().p2r_propagate_update(self._h, C.byref(opts), n_tracks, layer_r.numel(), _ptr(layer_r),
                                              _ptr(trk_in), _ptr(hits), _ptr(trk_out), _ptr(chi2),
                                              _ptr(status), _stream(stream)))
        return trk_out, chi2, status

    def p2z_propagate_update(self, n_tracks, layer_z, trk_in, hits, out=None, opts=None, stream=None, **kw):
        opts = opts or default_opts(**kw)
        trk_out, chi2, status = out if out is not None else self._outputs(trk_in, n_tracks)
        _check(library().p2z_propagate_update(self._h, C.byref(opts), n_tracks, layer_z.numel(), _ptr(layer_z),
                                              _ptr(trk_in), _ptr(hits), _ptr(trk_out), _ptr(chi2),
                                              _ptr(status), _stream(stream)))
        return trk_out, chi2, status

    def propagate_update_host(self, which, n_tracks, layer, trk_in, hits, out=None, opts=None, stream=None,
                              chunk_tracks=0, **kw):
        """Transfer-inclusive fit of host tensors (which 0 p2r, 1 p2z); returns host (trk_out, chi2, status).

        Pass pinned tensors (pin_memory()) for the copies to overlap; the
        results are complete once `stream` (torch's current by default) has
        reached the end of the call."""
        opts = opts or default_opts(**kw)
        for t in (layer, trk_in, hits):
            if t.is_cuda:
                raise ValueError("the host pipeline takes host tensors")
        if out is None:
            out = (torch.empty_like(trk_in).pin_memory(), torch.empty(n_tracks, dtype=torch.float32).pin_memory(),
                   torch.empty(n_tracks, dtype=torch.int32).pin_memory())
        trk_out, chi2, status = out
        if chunk_tracks >= 0 and 0 <= layer.numel() <= 4096:
            # sizing happens here, before the C call, which itself never allocates
            self.reserve_host(layer.numel(), chunk_tracks)
        fn = library().p2r_propagate_update_host if which == 0 else library().p2z_propagate_update_host
        _check(fn(self._h, C.byref(opts), n_tracks, layer.numel(), _ptr(layer), _ptr(trk_in), _ptr(hits),
                  _ptr(trk_out), _ptr(chi2), _ptr(status), int(chunk_tracks), _stream(stream)))
        return trk_out, chi2, status

    def fit_tracks_batched(self, offsets, surf_type, surf_val, hit_pos, hit_cov, par_in, cov_in, q,
                           n_hits, max_surfaces, out=None, opts=None, stream=None, **kw):
        """Ragged CSR fit; returns (par_out, cov_out, chi2, status)."""
        opts = opts or default_opts(**kw)
        n = par_in.shape[0]
        dev = par_in.device
        if out is None:
            out = (torch.empty((n, 6), dtype=torch.float32, device=dev),
                   torch.empty((n, 21), dtype=torch.float32, device=dev),
                   torch.empty(n, dtype=torch.float32, device=dev),
                   torch.empty(n, dtype=torch.int32, device=dev))
        par_out, cov_out, chi2, status = out
        if n > self._ragged_cap[0] or max_surfaces > self._ragged_cap[1]:
            # sizing happens here, before the C call, which itself never allocates
            if 0 <= max_surfaces <= 255:
                self.reserve(max(n, self._ragged_cap[0]), max(max_surfaces, self._ragged_cap[1]))
        _check(library().fit_tracks_batched(self._h, C.byref(opts), n, int(n_hits), int(max_surfaces),
                                            _ptr(offsets), _ptr(surf_type),
                                            _ptr(surf_val), _ptr(hit_pos), _ptr(hit_cov), _ptr(par_in),
                                            _ptr(cov_in), _ptr(q), _ptr(par_out), _ptr(cov_out), _ptr(chi2),
                                            _ptr(status), _stream(stream)))
        return par_out, cov_out, chi2, status


    def fit_tracks_batched_noalloc(self, offsets, surf_type, surf_val, hit_pos, hit_cov, par_in, cov_in, q,
                                   n_hits, max_surfaces, out, opts=None, stream=None, **kw):
        """The ragged fit without any allocation (library-held scratch, no graph):
        `out` = (par_out, cov_out, chi2, status) must be given; returns it."""
        opts = opts or default_opts(**kw)
        par_out, cov_out, chi2, status = out
        _check(library().fit_tracks_batched_noalloc(self._h, C.byref(opts), par_in.shape[0], int(n_hits),
                                                    int(max_surfaces), _ptr(offsets), _ptr(surf_type),
                                                    _ptr(surf_val), _ptr(hit_pos), _ptr(hit_cov), _ptr(par_in),
                                                    _ptr(cov_in), _ptr(q), _ptr(par_out), _ptr(cov_out), _ptr(chi2),
                                                    _ptr(status), _stream(stream)))
        return out


class Mlp:
    """Path-length MLP on the GPU (weights, Adam state and kernels in libp2r)."""

    def __init__(self, ctx: Context, params=None, seed: int = 0):
        self.ctx = ctx
        self._h = vp()
        self._batch_cap = 0
        _check(library().p2r_mlp_create(ctx._h, C.byref(self._h), int(seed) & (2**64 - 1)))
        self.n_params = library().p2r_mlp_n_params()
        if params is not None:
            self.set_params(params)

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h:
            library().p2r_mlp_destroy(self._h)
            self._h = vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, flat):
        import numpy as np
        a = np.ascontiguousarray(flat, dtype=np.float32)
        assert a.size == self.n_params
        _check(library().p2r_mlp_set_params(self._h, a.ctypes.data_as(C.c_void_p)))

    def get_params(self):
        import numpy as np
        a = np.zeros(self.n_params, dtype=np.float32)
        _check(library().p2r_mlp_get_params(self._h, a.ctypes.data_as(C.c_void_p)))
        return a

    def features(self, par, q, R, s_label=None, stream=None, **kw):
        """Device tensors par (n,6), q (n,), R (n,) [, s_label (n,)] -> x (n,7), t (n,) or None, s_line (n,)."""
        n = par.shape[0]
        dev = par.device
        x = torch.empty((n, 7), dtype=torch.float32, device=dev)
        sl = torch.empty(n, dtype=torch.float32, device=dev)
        t = torch.empty(n, dtype=torch.float32, device=dev) if s_label is not None else None
        o = default_opts(**kw)
        _check(library().p2r_mlp_features(self._h, C.byref(o), n, _ptr(par), _ptr(q), _ptr(R), _ptr(s_label),
                                          _ptr(x), _ptr(t), _ptr(sl), _stream(stream)))
        return x, t, sl

    def forward(self, x, stream=None):
        y = torch.empty(x.shape[0], dtype=torch.float32, device=x.device)
        _check(library().p2r_mlp_forward(self._h, _ptr(x), _ptr(y), x.shape[0], _stream(stream)))
        return y

    def reserve(self, max_batch: int):
        """Size the gradient partials (p2r_mlp_reserve); grow-only."""
        _check(library().p2r_mlp_reserve(self._h, int(max_batch)))
        self._batch_cap = max(self._batch_cap, int(max_batch))

    def _ensure(self, B: int):
        # sizing happens here, before the C call, which itself never allocates
        if 0 < B and B > self._batch_cap:
            self.reserve(B)

    def grads(self, x, t, stream=None):
        self._ensure(x.shape[0])
        g = torch.empty(self.n_params, dtype=torch.float32, device=x.device)
        loss = torch.empty(1, dtype=torch.float32, device=x.device)
        _check(library().p2r_mlp_grads(self._h, _ptr(x), _ptr(t), x.shape[0], _ptr(g), _ptr(loss), _stream(stream)))
        return g, loss

    def train_step(self, x, t, lr, loss_out=None, stream=None):
        self._ensure(x.shape[0])
        _check(library().p2r_mlp_train_step(self._h, _ptr(x), _ptr(t), x.shape[0], float(lr), _ptr(loss_out),
                                            _stream(stream)))

    def save(self, path):
        _check(library().p2r_mlp_save(self._h, path.encode()))

    def load(self, path):
        _check(library().p2r_mlp_load(self._h, path.encode()))
