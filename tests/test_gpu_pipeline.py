"""Transfer-inclusive host pipeline (chunks on three streams) against the
FP64 oracle, and against the device-resident fit: the same kernels on the
same data, so those results are bit-for-bit identical whatever the
chunking."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
import paper_2401_14221_amd as p2r
from synth import events as ev

from .parity import compare

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = p2r.Context(0)
    yield c
    c.close()


def _device(ctx, which, d, W):
    if which == 0:
        trk = p2r.pack_tracks(d["par"], d["cov"], d["q"], W, device="cuda")
        hits = p2r.pack_hits_p2r(d["hits"], d["hitcov"], W, device="cuda")
        surf = torch.as_tensor(d["surf"], dtype=torch.float32, device="cuda")
        r = ctx.p2r_propagate_update(d["par"].shape[0], surf, trk, hits, width=W)
    else:
        trk = p2r.pack_tracks(d["par"], d["cov"], d["q"], 64, device="cuda")
        hits = p2r.pack_hits_p2z(d["hits"], d["hitcov"], device="cuda")
        surf = torch.as_tensor(d["surf"], dtype=torch.float32, device="cuda")
        r = ctx.p2z_propagate_update(d["par"].shape[0], surf, trk, hits)
    torch.cuda.synchronize()
    return [t.cpu() for t in r]


def _host(ctx, which, d, W, chunk):
    if which == 0:
        trk = p2r.pack_tracks(d["par"], d["cov"], d["q"], W).pin_memory()
        hits = p2r.pack_hits_p2r(d["hits"], d["hitcov"], W).pin_memory()
    else:
        trk = p2r.pack_tracks(d["par"], d["cov"], d["q"], 64).pin_memory()
        hits = p2r.pack_hits_p2z(d["hits"], d["hitcov"]).pin_memory()
    surf = torch.as_tensor(d["surf"], dtype=torch.float32)
    s = torch.cuda.Stream()
    r = ctx.propagate_update_host(which, d["par"].shape[0], surf, trk, hits, chunk_tracks=chunk, stream=s,
                                  width=W if which == 0 else 0)
    s.synchronize()
    return [t.clone() for t in r]


@pytest.mark.parametrize("which,W,n,chunk", [(1, 64, 5000, 1000), (1, 64, 4097, 0), (1, 64, 64, 64),
                                             (0, 64, 5000, 1000), (0, 128, 3001, 700), (0, 256, 2000, 256)])
def test_host_pipeline_equals_device_fit(ctx, which, W, n, chunk):
    if which == 0:
        d = ev.make_barrel_event(ev.P2R_THROUGHPUT.with_(seed=81), n_tracks=n)
    else:
        d = ev.make_disk_event(ev.P2Z_THROUGHPUT.with_(seed=82), n_tracks=n)
    a = _device(ctx, which, d, W)
    b = _host(ctx, which, d, W, chunk)
    nb = (n + W - 1) // W
    # whole blocks of the record array (tail lanes are never written by either path)
    pa, ca, qa = p2r.unpack_tracks(a[0], n)
    pb, cb, qb = p2r.unpack_tracks(b[0], n)
    assert torch.equal(pa, pb) and torch.equal(ca, cb) and torch.equal(qa, qb)
    assert torch.equal(a[1], b[1])
    assert torch.equal(a[2], b[2])
    assert b[0].shape[0] == nb
    # and the pipeline's results against the oracle
    g = dict(par=pb.numpy(), cov=cb.numpy(), chi2=b[1].numpy(), status=b[2].numpy().view(np.uint32))
    r = oracle.fit_event(d, "barrel" if which == 0 else "disk")
    print(f"pipeline which={which} W={W} n={n}",
          compare(g, r, ctx=f"host pipeline which={which}", final_surface="cylinder" if which == 0 else "plane"),
          flush=True)


def test_host_pipeline_edge_cases(ctx):
    d = ev.make_disk_event(ev.P2Z_THROUGHPUT.with_(seed=83), n_tracks=100)
    trk = p2r.pack_tracks(d["par"], d["cov"], d["q"], 64).pin_memory()
    hits = p2r.pack_hits_p2z(d["hits"], d["hitcov"]).pin_memory()
    surf = torch.as_tensor(d["surf"], dtype=torch.float32)
    # no tracks: nothing to do
    ctx.propagate_update_host(1, 0, surf, trk, hits)
    with pytest.raises(ValueError):
        ctx.propagate_update_host(1, 100, surf.cuda(), trk, hits)
    with pytest.raises(p2r.P2RError):
        ctx.propagate_update_host(1, 100, surf, trk, hits, chunk_tracks=-5)
    m = p2r.Mlp(ctx)
    with pytest.raises(p2r.P2RError):
        ctx.propagate_update_host(0, 100, surf, trk, hits, mlp=m.handle.value)
    # the sizing call's argument checks
    for bad in ((-1, 0), (5000, 0), (20, -3)):
        with pytest.raises(p2r.P2RError) as e:
            ctx.reserve_host(*bad)
        assert e.value.code == p2r.P2R_EINVAL
    with pytest.raises(p2r.P2RError) as e:
        m.reserve(0)
    assert e.value.code == p2r.P2R_EINVAL
    # pageable host memory works too (copies serialise)
    r = ctx.propagate_update_host(1, 100, surf, trk.clone(), hits.clone(), chunk_tracks=64)
    torch.cuda.synchronize()
    a = _device(ctx, 1, d, 64)
    assert torch.equal(a[1], r[1])


def test_host_pipeline_no_allocation_after_reserve(ctx):
    """The pipeline calls allocate nothing once p2r_ctx_reserve_host has sized
    the staging; more layers or larger chunks than reserved are refused
    before anything is copied or launched."""
    c = p2r.Context(0)
    try:
        d = ev.make_disk_event(ev.P2Z_THROUGHPUT.with_(seed=84), n_tracks=3000)
        trk = p2r.pack_tracks(d["par"], d["cov"], d["q"], 64).pin_memory()
        hits = p2r.pack_hits_p2z(d["hits"], d["hitcov"]).pin_memory()
        surf = torch.as_tensor(d["surf"], dtype=torch.float32)
        L = surf.numel()
        c.reserve_host(L, 1024)
        torch.cuda.synchronize()
        n0 = p2r.device_allocations()
        s = torch.cuda.Stream()
        r1 = c.propagate_update_host(1, 3000, surf, trk, hits, chunk_tracks=1024, stream=s)
        s.synchronize()
        r2 = c.propagate_update_host(1, 3000, surf, trk, hits, chunk_tracks=512, stream=s)
        s.synchronize()
        assert p2r.device_allocations() == n0
        assert torch.equal(r1[1], r2[1]) and torch.equal(r1[2], r2[2])
        # the raw C call (no binding-side sizing) with chunks above the reservation
        lib = p2r._lib.library()
        o = p2r._lib.default_opts()
        out = [torch.empty_like(trk).pin_memory(), torch.empty(3000).pin_memory(),
               torch.empty(3000, dtype=torch.int32).pin_memory()]
        rc = lib.p2z_propagate_update_host(c._h, ctypes.byref(o), 3000, L, surf.data_ptr(), trk.data_ptr(),
                                           hits.data_ptr(), out[0].data_ptr(), out[1].data_ptr(), out[2].data_ptr(),
                                           2048, None)
        assert rc == p2r.P2R_ENOSPACE
        assert p2r.device_allocations() == n0
    finally:
        c.close()
