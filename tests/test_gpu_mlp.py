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
    for k in g_ref:
        a, b = g[k].reshape(-1).astype(np.float64), g_ref[k].reshape(-1)
        rel = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)
        cos = a @ b / max(np.linalg.norm(a) * np.linalg.norm(b), 1e-30)
        print(f"grad {k}: rel L2 {rel:.2e}, cosine {cos:.8f}", flush=True)
        assert rel < 1e-3 and cos > 0.9999, k


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
