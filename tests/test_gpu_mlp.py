"""GPU parity of the path-length MLP kernels against the NumPy FP64 reference,
and the learned start of the p2r fit."""
import os

import numpy as np
import pytest
import torch

import oracle
from oracle import mlp as omlp
import paper_2401_14221_amd as p2r
from paper_2401_14221_amd import learned
from synth import events as ev

from .parity import compare

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = p2r.Context(0)
    yield c
    c.close()


def _params(seed, noise=0.05):
    p = {k: v.astype(np.float64) for k, v in ev.make_mlp_init(seed).items()}
    g = np.random.default_rng(seed)
    for k in p:
        p[k] = (p[k] + noise * g.normal(size=p[k].shape)).astype(np.float32).astype(np.float64)
    return p


def _pairs(n_tracks=600, seed=31):
    d = ev.make_mlp_pairs(n_tracks, seed=seed)
    x, sl = omlp.features(d["par"], d["q"], d["R"])
    return d, x.astype(np.float32).astype(np.float64), sl


def test_features_match_reference(ctx):
    d, x_ref, sl_ref = _pairs()
    m = p2r.Mlp(ctx)
    f = lambda a: torch.as_tensor(a, dtype=torch.float32, device="cuda")  # noqa: E731
    x, t, sl = m.features(f(d["par"]), f(d["q"]), f(d["R"]), s_label=f(d["s"]))
    x = x.cpu().numpy()
    assert np.allclose(x, x_ref, rtol=2e-5, atol=2e-6)
    assert np.allclose(sl.cpu().numpy(), sl_ref, rtol=2e-6)
    t_ref = omlp.target(d["s"].astype(np.float32), sl_ref)
    assert np.allclose(t.cpu().numpy(), t_ref, rtol=1e-3, atol=2e-3)


@pytest.mark.parametrize("B", [64, 1000, 4097])
def test_forward_matches_bf16_reference(ctx, B):
    d, x, _ = _pairs()
    x = x[:B]
    p = _params(5)
    m = p2r.Mlp(ctx, learned.flat_params(p))
    y = m.forward(torch.as_tensor(x, dtype=torch.float32, device="cuda")).cpu().numpy()
    y_ref, _ = omlp.forward(p, x, bf16=True)
    y_fp64, _ = omlp.forward(p, x, bf16=False)
    scale = np.abs(y_ref).max()
    err = np.abs(y - y_ref).max() / scale
    print(f"B={B}: max |y - y_bf16ref| / max|y| = {err:.2e}; BF16 quantisation vs FP64 "
          f"{np.abs(y_ref - y_fp64).max() / scale:.2e}", flush=True)
    assert err < 1e-4


def _grad_term_bounds(p, x, t):
    """Per gradient element, the sum and the largest of |per-sample term| (the
    condition of each batch sum), from the BF16-operand reference's
    intermediates."""
    y, c = omlp.forward(p, x, bf16=True)
    B = y.shape[0]
    W2, W3 = np.asarray(p["W2"], np.float64), np.asarray(p["W3"], np.float64)
    dy = np.abs(2.0 * (y - t) / B)
    dz2 = dy[:, None] * np.abs(W3[0])[None, :] * (c["z2"] > 0)
    dz1 = (np.abs(omlp.bf16_round(dz2)) @ np.abs(omlp.bf16_round(W2))) * (c["z1"] > 0)
    h1, h2, xx = np.abs(c["h1"]), np.abs(c["h2"]), np.abs(c["x"])
    # the weight gradients' operands go through the matrix cores in BF16
    r = omlp.bf16_round
    dz2r, h1r, dz1r, xr = np.abs(r(dz2)), np.abs(r(h1)), np.abs(r(dz1)), np.abs(r(xx))
    S = dict(W3=(dy @ h2)[None, :], b3=np.array([dy.sum()]), W2=dz2r.T @ h1r, b2=dz2.sum(0),
             W1=dz1r.T @ xr, b1=dz1.sum(0))
    M = dict(W3=(dy[:, None] * h2).max(0)[None, :], b3=np.array([dy.max()]),
             W2=(dz2r[:, :, None] * h1r[:, None, :]).max(0), b2=dz2.max(0),
             W1=(dz1r[:, :, None] * xr[:, None, :]).max(0), b1=dz1.max(0))
    return S, M


def test_grads_match_bf16_reference(ctx):
    d, x, _ = _pairs()
    B = 2048
    x = x[:B]
    t = np.random.default_rng(2).normal(size=B) * 0.5
    p = _params(6)
    m = p2r.Mlp(ctx, learned.flat_params(p))
    g, loss = m.grads(torch.as_tensor(x, dtype=torch.float32, device="cuda"),
                      torch.as_tensor(t, dtype=torch.float32, device="cuda"))
    g = learned.split_params(g.cpu().numpy())
    l_ref, g_ref = omlp.loss_and_grads(p, x, t, bf16=True)
    assert float(loss.item()) == pytest.approx(l_ref, rel=1e-4)
    S, M = _grad_term_bounds(p, x, t)
    for k in g_ref:
        a, b = g[k].astype(np.float64), g_ref[k]
        # element-wise: FP32 accumulation over the batch, |err| <= ~B eps32 sum_b |term_b|
        # (1e-5 covers B = 2048 summed in blocks), plus the rare BF16 operand that an FP32
        # intermediate rounds the other way (h1 or dz2 of one sample: at most 2^-8 of that
        # sample's term, allowed three times)
        bound = 1e-5 * S[k] + 3 * 2.0 ** -8 * M[k] + 1e-30
        r = np.abs(a - b) / bound
        print(f"grad {k}: max |err| / bound {r.max():.3f}; rel L2 "
              f"{np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30):.2e}", flush=True)
        assert (r <= 1.0).all(), (k, np.unravel_index(np.argmax(r), r.shape), r.max())


def test_adam_step_and_checkpoint(ctx, tmp_path):
    d, x, _ = _pairs()
    B = 1024
    x = torch.as_tensor(x[:B], dtype=torch.float32, device="cuda")
    t = torch.as_tensor(np.random.default_rng(3).normal(size=B) * 0.5, dtype=torch.float32, device="cuda")
    p0 = learned.flat_params(_params(7))
    m = p2r.Mlp(ctx, p0)
    g, _ = m.grads(x, t)
    m.train_step(x, t, 1e-3)
    p1 = m.get_params()
    exp, _ = omlp.adam_step({"w": p0.astype(np.float64)}, {"w": g.cpu().numpy().astype(np.float64)}, {}, lr=1e-3)
    assert np.allclose(p1, exp["w"], rtol=1e-6, atol=1e-8)
    # checkpoint: save after one step, continue twice; reload and continue twice -> identical
    ck = str(tmp_path / "m.ckpt")
    m.save(ck)
    for _ in range(2):
        m.train_step(x, t, 1e-3)
    a = m.get_params()
    m2 = p2r.Mlp(ctx)
    m2.load(ck)
    assert np.array_equal(m2.get_params(), p1)
    for _ in range(2):
        m2.train_step(x, t, 1e-3)
    assert np.array_equal(m2.get_params(), a)


def test_create_seed_initialises_weights(ctx):
    """p2r_mlp_create's seed: reproducible, seed-dependent, fan-in-scaled
    uniform weights and zero biases."""
    a = learned.split_params(p2r.Mlp(ctx, seed=5).get_params())
    b = learned.split_params(p2r.Mlp(ctx, seed=5).get_params())
    c = learned.split_params(p2r.Mlp(ctx, seed=6).get_params())
    for k in a:
        assert np.array_equal(a[k], b[k]), k
    for k, fan, scale in (("W1", 7, 1.0), ("W2", 64, 1.0), ("W3", 64, 0.1)):
        lim = np.sqrt(6.0 / fan) * scale
        w = a[k].astype(np.float64)
        assert np.abs(w).max() <= lim and not np.array_equal(a[k], c[k]), k
        assert abs(w.mean()) < 0.1 * lim, k
        assert w.std() == pytest.approx(lim / np.sqrt(3), rel=0.2), k
    for k in ("b1", "b2", "b3"):
        assert not a[k].any(), k


def test_training_from_seed_reduces_loss(ctx):
    """A short training run from a fixed seed, always (not the committed
    network): the loss falls and the proposal beats the straight line."""
    m, hist = learned.train(ctx, n_tracks=40_000, epochs=4, batch=4096, seed=1234)
    print("loss per epoch", " ".join(f"{h:.4e}" for h in hist), flush=True)
    assert all(np.isfinite(hist)) and hist[-1] < 0.5 * hist[0]
    q = learned.proposal_quality(m, n_tracks=5000, seed=98)
    print("proposal quality after the short run", q, flush=True)
    assert q["median_err_mlp"] < q["median_err_line"]


def test_no_device_allocation_after_reserve(ctx):
    """Gradient and training calls allocate nothing once p2r_mlp_reserve has
    sized the batch; a larger batch is refused before anything runs."""
    d, x, _ = _pairs()
    m = p2r.Mlp(ctx, seed=3)
    m.reserve(512)
    xt = torch.as_tensor(x[:512], dtype=torch.float32, device="cuda")
    tt = torch.zeros(512, dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    n0 = p2r.device_allocations()
    for B in (512, 100, 512):
        m.grads(xt[:B], tt[:B])
        m.train_step(xt[:B], tt[:B], 1e-3)
    torch.cuda.synchronize()
    assert p2r.device_allocations() == n0
    big = torch.zeros((600, 7), dtype=torch.float32, device="cuda")
    lib = p2r._lib.library()
    rc = lib.p2r_mlp_grads(m.handle, big.data_ptr(), tt.data_ptr(), 600, None, None, None)
    assert rc == p2r.P2R_ENOSPACE
    rc = lib.p2r_mlp_train_step(m.handle, big.data_ptr(), tt.data_ptr(), 600, 1e-3, None, None)
    assert rc == p2r.P2R_ENOSPACE
    assert p2r.device_allocations() == n0


@pytest.fixture(scope="module")
def trained(ctx):
    """The committed network if present, else a short training run."""
    m = p2r.Mlp(ctx)
    if os.path.exists(learned.DEFAULT_CKPT):
        m.load(learned.DEFAULT_CKPT)
        return m
    m, hist = learned.train(ctx, n_tracks=40_000, epochs=4)
    assert hist[-1] < hist[0]
    return m


def test_trained_proposal_beats_straight_line(ctx, trained):
    q = learned.proposal_quality(trained, n_tracks=5000, seed=99)
    print("proposal quality", q, flush=True)
    assert q["median_err_mlp"] < q["median_err_line"]
    assert q["p99_err_mlp"] < 0.2 * q["p99_err_line"]


def _fit(ctx, d, mlp=None, W=64):
    n = d["par"].shape[0]
    trk = p2r.pack_tracks(d["par"], d["cov"], d["q"], W, device="cuda")
    hits = p2r.pack_hits_p2r(d["hits"], d["hitcov"], W, device="cuda")
    radii = torch.as_tensor(d["surf"], dtype=torch.float32, device="cuda")
    ev_ = torch.zeros(1, dtype=torch.int64, device="cuda")
    o = p2r._lib.default_opts(width=W)
    o.helix_evals = ev_.data_ptr()
    if mlp is not None:
        o.mlp = mlp.handle.value
    out, chi2, st = ctx.p2r_propagate_update(n, radii, trk, hits, opts=o)
    torch.cuda.synchronize()
    par, cov, _ = p2r.unpack_tracks(out, n)
    return dict(par=par.cpu().numpy(), cov=cov.cpu().numpy(), chi2=chi2.cpu().numpy(),
                status=st.cpu().numpy().view(np.uint32)), int(ev_.item())


@pytest.mark.parametrize("W", [32, 64, 128, 256])
def test_learned_fit_matches_oracle(ctx, trained, W):
    d = ev.make_barrel_event(ev.LEARNED_EVAL, n_tracks=4099)
    r = oracle.fit_event(d, "barrel")
    g, ev_l = _fit(ctx, d, trained, W)
    g["status"] = g["status"] & ~np.uint32(p2r.ST_ML_REJECTED)
    rep = compare(g, r, ctx=f"learned W={W}")
    gp, ev_p = _fit(ctx, d, None, W)
    tl = 4099 * len(d["surf"])
    print(f"W={W}: helix evaluations per track-layer: learned {ev_l / tl:.3f}, plain {ev_p / tl:.3f}; {rep}",
          flush=True)
    assert ev_l < ev_p



@pytest.mark.parametrize("case", ["low pT", "high pT", "B = 0"])
def test_learned_fit_outside_the_training_range(ctx, trained, case):
    """The network was trained on 0.5..10 GeV tracks in 3.8 T; on loopers
    (0.2..0.6 GeV: many proposals for layers out of reach), on 0.5..5 TeV
    tracks (curvature features ~0) and with no field (omega = 0: the
    straight line is exact) its proposals are rejected or refined, and the
    learned fit still equals the oracle's."""
    pt = (0.2, 0.6) if case == "low pT" else ((500.0, 5000.0) if case == "high pT" else ev.LEARNED_EVAL.pt)
    bz = 0.0 if case == "B = 0" else 3.8
    d = ev.make_barrel_event(ev.LEARNED_EVAL.with_(pt=pt, seed=131 + len(case)), n_tracks=2048)
    r = oracle.fit_event(d, "barrel", bz=bz)
    n = d["par"].shape[0]
    W = 64
    trk = p2r.pack_tracks(d["par"], d["cov"], d["q"], W, device="cuda")
    hits = p2r.pack_hits_p2r(d["hits"], d["hitcov"], W, device="cuda")
    radii = torch.as_tensor(d["surf"], dtype=torch.float32, device="cuda")
    o = p2r._lib.default_opts(width=W, bz_tesla=bz)
    o.mlp = trained.handle.value
    out, chi2, st = ctx.p2r_propagate_update(n, radii, trk, hits, opts=o)
    torch.cuda.synchronize()
    par, cov, _ = p2r.unpack_tracks(out, n)
    g = dict(par=par.cpu().numpy(), cov=cov.cpu().numpy(), chi2=chi2.cpu().numpy(),
             status=st.cpu().numpy().view(np.uint32) & ~np.uint32(p2r.ST_ML_REJECTED))
    # near-straight tracks: 1/pT ill-conditioned against its relative bound (see the plain test)
    kw = {"sens_cap": 1e5} if case == "high pT" else {}
    print(case, compare(g, r, ctx=f"learned, {case}", **kw), flush=True)