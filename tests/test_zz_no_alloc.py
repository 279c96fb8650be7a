"""fit_tracks_batched_noalloc, called through the C ABI: the same results as
fit_tracks_batched on the same inputs (bit for bit: the same kernels), with
no device allocation, on two calls in a row (the second smaller, so stale
scratch from the first must not leak into it), and a clear refusal above its
size limit.  Collected last (the file name), as its scratch is shared by
every call on the GPU."""
import ctypes as C

import numpy as np
import pytest
import torch

import paper_2401_14221_amd as p2r
from paper_2401_14221_amd import _lib
from synth import events as ev

pytestmark = pytest.mark.gpu

CUT = 30.0


def _upload(d):
    f = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float32, device="cuda")  # noqa: E731
    return [torch.as_tensor(d["offsets"], dtype=torch.int64, device="cuda"),
            torch.as_tensor(d["surf_type"], dtype=torch.uint8, device="cuda"), f(d["surf_val"]), f(d["hits"]),
            f(d["hitcov"]), f(d["par"]), f(d["cov"]), torch.as_tensor(d["q"], dtype=torch.int8, device="cuda")]


def _outputs(n):
    return [torch.full((n, 6), np.nan, device="cuda"), torch.full((n, 21), np.nan, device="cuda"),
            torch.full((n,), np.nan, device="cuda"), torch.zeros(n, dtype=torch.int32, device="cuda")]


def _call(fn, ctx, d, ins, outs, stream, max_surfaces=25):
    o = _lib.default_opts(chi2_cut=CUT, use_graph=0)
    ptr = lambda t: C.c_void_p(t.data_ptr())  # noqa: E731
    return fn(ctx._h, C.byref(o), d["par"].shape[0], int(d["offsets"][-1]), max_surfaces, *[ptr(t) for t in ins],
              *[ptr(t) for t in outs], C.c_void_p(stream.cuda_stream))


def _host(outs):
    return dict(par=outs[0].cpu().numpy(), cov=outs[1].cpu().numpy(), chi2=outs[2].cpu().numpy(),
                status=outs[3].cpu().numpy().view(np.uint32))


def test_noalloc_matches_fit_tracks_batched():
    lib = _lib.library()
    ctx = p2r.Context(0)
    s = torch.cuda.Stream()
    try:
        for n, seed in ((6000, 41), (2500, 42)):              # the second call is smaller
            d = ev.make_ragged_event(ev.RAGGED.with_(seed=seed), n_tracks=n)
            ins = _upload(d)
            ref_out = _outputs(n)
            ctx.reserve(n, 25)
            assert _call(lib.fit_tracks_batched, ctx, d, ins, ref_out, s) == 0
            torch.cuda.synchronize()
            na_out = _outputs(n)
            before = p2r.device_allocations()
            print(f"noalloc call n={n} seed={seed}", flush=True)
            assert _call(lib.fit_tracks_batched_noalloc, ctx, d, ins, na_out, s) == 0, lib.p2r_last_error()
            torch.cuda.synchronize()
            assert p2r.device_allocations() == before
            g, ref = _host(na_out), _host(ref_out)
            # the same kernels on the same inputs: identical results (the
            # ragged parity tests compare those with the oracle)
            for k in ("par", "cov", "chi2", "status"):
                assert np.array_equal(g[k], ref[k], equal_nan=True), (n, k)
            assert np.all(g["status"] & p2r.ST_DONE)
    finally:
        ctx.close()


def test_noalloc_refuses_more_tracks_than_its_scratch_holds():
    lib = _lib.library()
    ctx = p2r.Context(0)
    try:
        n = int(p2r.P2R_NOALLOC_MAX_TRACKS) + 1
        o = _lib.default_opts(use_graph=0)
        dummy = torch.zeros(8, dtype=torch.int64, device="cuda")
        p = C.c_void_p(dummy.data_ptr())
        rc = lib.fit_tracks_batched_noalloc(ctx._h, C.byref(o), n, 0, 25, p, None, None, None, None, p, p, p, p, p,
                                            p, p, None)
        assert rc == p2r.P2R_ENOSPACE
        assert b"at most" in lib.p2r_last_error()
    finally:
        ctx.close()


def test_noalloc_at_its_limits():
    """P2R_NOALLOC_MAX_TRACKS tracks with max_surfaces = 255 (the largest
    sort-key histogram): every region of the scratch array at its full size,
    with the same results as fit_tracks_batched."""
    lib = _lib.library()
    ctx = p2r.Context(0)
    s = torch.cuda.Stream()
    try:
        n = int(p2r.P2R_NOALLOC_MAX_TRACKS)
        d = ev.make_ragged_event(ev.RAGGED.with_(seed=43), n_tracks=n)
        ins = _upload(d)
        ref_out = _outputs(n)
        ctx.reserve(n, 255)
        assert _call(lib.fit_tracks_batched, ctx, d, ins, ref_out, s, max_surfaces=255) == 0
        torch.cuda.synchronize()
        na_out = _outputs(n)
        before = p2r.device_allocations()
        print(f"noalloc call n={n} max_surfaces=255", flush=True)
        assert _call(lib.fit_tracks_batched_noalloc, ctx, d, ins, na_out, s, max_surfaces=255) == 0, \
            lib.p2r_last_error()
        torch.cuda.synchronize()
        assert p2r.device_allocations() == before
        g, ref = _host(na_out), _host(ref_out)
        for k in ("par", "cov", "chi2", "status"):
            assert np.array_equal(g[k], ref[k], equal_nan=True), k
        assert np.all(g["status"] & p2r.ST_DONE)
    finally:
        ctx.close()
