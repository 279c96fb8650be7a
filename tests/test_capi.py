"""Host-side checks of the C ABI: the library loads, exports what the
header declares, and rejects bad arguments before touching a GPU."""
import ctypes as C

import pytest

import paper_2401_14221_amd as p2r
from paper_2401_14221_amd import _lib


def test_library_exports_every_declared_symbol():
    lib = p2r.library()
    names = _lib.exported_symbols()
    for must in ("p2r_propagate_update", "p2z_propagate_update", "fit_tracks_batched", "p2r_ctx_create",
                 "p2r_autotune", "p2r_last_error"):
        assert must in names
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_opts_default_and_version():
    o = _lib.default_opts()
    assert o.bz_tesla == pytest.approx(3.8)
    assert o.newton_tol_cm == pytest.approx(1e-6)
    assert o.newton_max_iter == 8 and o.fp64_fallback == 3 and o.width == 0 and not o.mlp
    assert p2r.library().p2r_version().startswith(b"p2r-mi355x")


@pytest.mark.parametrize("fn", ["p2r_propagate_update", "p2z_propagate_update"])
def test_null_context_rejected_without_launch(fn):
    lib = p2r.library()
    o = _lib.default_opts()
    rc = getattr(lib, fn)(None, C.byref(o), 10, 5, None, None, None, None, None, None, None)
    assert rc == p2r.P2R_EINVAL
    assert b"ctx" in lib.p2r_last_error()


def test_null_context_other_calls():
    lib = p2r.library()
    w = C.c_int32()
    assert lib.p2r_layout_width(None, 0, C.byref(w)) == p2r.P2R_EINVAL
    assert lib.p2r_autotune(None, 0, 10, 10, None) == p2r.P2R_EINVAL
    assert lib.p2r_ctx_create(None, 0, None) == p2r.P2R_EINVAL
    lib.p2r_ctx_destroy(None)          # no-op


def test_set_variant_argument_errors():
    lib = p2r.library()
    assert lib.p2r_set_variant(None, 0, b"p2r_w64_e0_u1") == p2r.P2R_EINVAL
    assert b"ctx" in lib.p2r_last_error()


def test_variant_listing_is_host_only():
    names = p2r.variant_names(0)
    assert "p2r_w64_e0_u1" in names and all(n.startswith("p2r_w") for n in names)
    assert p2r.variant_names(1) and all(n.startswith("p2z_") for n in p2r.variant_names(1))
    assert p2r.variant_names(2) and p2r.variant_names(7) == []


def test_sizing_and_noalloc_calls_reject_null_handles():
    """The sizing calls and the allocation-free fit check their handles on
    the host, before any HIP call."""
    lib = p2r.library()
    assert lib.p2r_ctx_reserve(None, 10, 5) == p2r.P2R_EINVAL
    assert lib.p2r_ctx_reserve_host(None, 20, 0) == p2r.P2R_EINVAL
    assert lib.p2r_mlp_reserve(None, 64) == p2r.P2R_EINVAL
    out = C.c_void_p()
    assert lib.p2r_mlp_create(None, C.byref(out), 7) == p2r.P2R_EINVAL
    o = _lib.default_opts()
    rc = lib.fit_tracks_batched_noalloc(None, C.byref(o), 10, 100, 25, *([None] * 13))
    assert rc == p2r.P2R_EINVAL
    assert p2r.device_allocations() == 0
