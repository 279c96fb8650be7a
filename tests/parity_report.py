"""Full-size parity report: every track of the p2r, p2z, ragged,
learned-start and hit-frame-update benchmark workloads, and of p2r with the
closed-form crossing start and with every step in FP64, fitted on the GPU
and by the FP64 oracle, compared element by element.  Prints, per workload, the
largest error of every output, how many covariance elements pass under each
branch of the rule in tests/parity.py, how many tracks had a bound widened
by the oracle's measured FP32 sensitivity, and how many end at a shallow
incidence.

Needs a GPU and the built libraries:
  python -m tests.parity_report [p2r p2z ragged learned p2r_2d p2r_cf p2r_f64] [--dump DIR]
(workload names select some of them, default all; --dump writes the GPU and
oracle outputs of the tracks that fail a check to DIR/parity_fail_<name>.npz.)
"""
from __future__ import annotations

import sys
import time

import numpy as np


def _gpu_p2r(p2r, ctx, d, W, mlp=None, update_2d=0, cyl_start=0, fp64=0):
    import torch
    n = d["par"].shape[0]
    trk = p2r.pack_tracks(d["par"], d["cov"], d["q"], W, device="cuda")
    hits = p2r.pack_hits_p2r(d["hits"], d["hitcov"], W, device="cuda")
    radii = torch.as_tensor(d["surf"], dtype=torch.float32, device="cuda")
    opts = p2r._lib.default_opts(width=W, update_2d=update_2d, cyl_start=cyl_start, fp64=fp64)
    if mlp is not None:
        opts.mlp = mlp.handle.value
    out, chi2, st = ctx.p2r_propagate_update(n, radii, trk, hits, opts=opts)
    torch.cuda.synchronize()
    par, cov, _ = p2r.unpack_tracks(out, n)
    st = st.cpu().numpy().view(np.uint32)
    if mlp is not None:
        st = st & ~np.uint32(p2r.ST_ML_REJECTED)      # a GPU-only bit: the proposal was not used
    return dict(par=par.cpu().numpy(), cov=cov.cpu().numpy(), chi2=chi2.cpu().numpy(), status=st)


def _gpu_p2z(p2r, ctx, d):
    import torch
    n = d["par"].shape[0]
    trk = p2r.pack_tracks(d["par"], d["cov"], d["q"], 64, device="cuda")
    hits = p2r.pack_hits_p2z(d["hits"], d["hitcov"], device="cuda")
    zs = torch.as_tensor(d["surf"], dtype=torch.float32, device="cuda")
    out, chi2, st = ctx.p2z_propagate_update(n, zs, trk, hits)
    torch.cuda.synchronize()
    par, cov, _ = p2r.unpack_tracks(out, n)
    return dict(par=par.cpu().numpy(), cov=cov.cpu().numpy(), chi2=chi2.cpu().numpy(),
                status=st.cpu().numpy().view(np.uint32))


def _gpu_ragged(p2r, ctx, d, cut):
    import torch
    f = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float32, device="cuda")  # noqa: E731
    po, co, c2, st = ctx.fit_tracks_batched(
        torch.as_tensor(d["offsets"], dtype=torch.int64, device="cuda"),
        torch.as_tensor(d["surf_type"], dtype=torch.uint8, device="cuda"), f(d["surf_val"]), f(d["hits"]),
        f(d["hitcov"]), f(d["par"]), f(d["cov"]), torch.as_tensor(d["q"], dtype=torch.int8, device="cuda"),
        int(d["offsets"][-1]), 25, stream=torch.cuda.Stream(), chi2_cut=cut)
    torch.cuda.synchronize()
    return dict(par=po.cpu().numpy(), cov=co.cpu().numpy(), chi2=c2.cpu().numpy(),
                status=st.cpu().numpy().view(np.uint32))


def report(name, g, r, final_surface, dump=None):
    from tests.parity import NORM_TOL, compare, failures, incidence_condition
    f = failures(g, r)
    n = len(g["chi2"])
    print(f"== {name}: {n} tracks, {len(f['excluded'])} excluded", flush=True)
    bad = {k: f[k] for k in ("status", "par", "chi2", "cov")}
    print("  tracks failing: " + ", ".join(f"{k} {len(v)}" for k, v in bad.items()))
    keep = np.ones(n, bool)
    keep[f["excluded"]] = False
    for k in ("par", "chi2", "cov"):
        rr, raw, w = f[k + "_ratio"], f[k + "_raw"], np.where(keep, f["widen_" + k], 1.0)
        print(f"  {k}: largest error / bound {rr.max():.3f}; 99.99% {np.quantile(rr, 0.9999):.3f}; "
              f"99.9% {np.quantile(rr, 0.999):.3f}; error / base bound above 1 in {int((raw > 1).sum())} tracks; "
              f"bound widened in {int((w > 1).sum())} tracks (widest x{w.max():.3g})")
    if dump is not None:
        idx = np.unique(np.concatenate([v for v in bad.values()] + [np.zeros(0, np.int64)])).astype(np.int64)
        extra = {}
        if "f32" in r:
            extra = {f"s_{k}": np.asarray(r["f32"][k])[idx] for k in ("par", "cov", "chi2", "status")}
        np.savez(dump, idx=idx, **{f"g_{k}": np.asarray(g[k])[idx] for k in ("par", "cov", "chi2", "status")},
                 **{f"r_{k}": np.asarray(r[k])[idx] for k in ("par", "cov", "chi2", "status", "nused")}, **extra)
    if any(len(v) for v in bad.values()):
        return None
    rep = compare(g, r, ctx=name, final_surface=final_surface)
    print("  max rel error, parameters (x y z 1/pT phi theta):",
          " ".join(f"{v:.2e}" for v in rep["max_rel_par"]))
    print(f"  max rel error, chi2: {rep['max_rel_chi2']:.2e}")
    print(f"  covariance, error / sqrt(C_ii C_jj): max {rep['cov_norm_err_max']:.2e}, "
          f"99.9% {rep['cov_norm_err_p999']:.2e} (bound {NORM_TOL:g})")
    print(f"  covariance elements: {rep['cov_rel_pass']} pass the relative bound, "
          f"{rep['cov_norm_only']} only the normalised one, {rep['cov_widened_only']} only the widened one; "
          f"{rep['tracks_widened']} tracks had a bound widened; {rep['fp64_fallbacks']} tracks took the FP64 update")
    kap = incidence_condition(r["par"], final_surface)
    print("  tracks whose final surface has 1/cos(incidence) above 2, 5, 10, 20, 50: "
          + ", ".join(str(int((kap > t).sum())) for t in (2, 5, 10, 20, 50)))
    return rep


def _dump(name):
    """Where the failing tracks' outputs go (a --dump DIR argument), or None."""
    if "--dump" not in sys.argv:
        return None
    import os
    d = sys.argv[sys.argv.index("--dump") + 1]
    os.makedirs(d, exist_ok=True)
    return os.path.join(d, f"parity_fail_{name}.npz")


def main():
    import torch  # noqa: F401

    import oracle
    import paper_2401_14221_amd as p2r
    from paper_2401_14221_amd import learned
    from synth import events as ev
    from tests.parity import final_surface_of

    names = ("p2r", "p2z", "ragged", "learned", "p2r_2d", "p2r_cf", "p2r_f64")
    args = [a for a in sys.argv[1:] if not a.startswith("--")]
    if "--dump" in sys.argv:
        args.remove(sys.argv[sys.argv.index("--dump") + 1])
    chosen = [a for a in args if a in names] or list(names)
    ctx = p2r.Context(0)
    W = 256
    exact = {}
    for name in chosen:
        t = time.time()
        if name == "p2z":
            d = ev.make_disk_event(ev.P2Z_THROUGHPUT)
            g = _gpu_p2z(p2r, ctx, d)
            r = oracle.fit_event(d, "disk", nthreads=16)
            report(f"p2z {ev.P2Z_THROUGHPUT.name}", g, r, "plane", dump=_dump(name))
        elif name == "ragged":
            d = ev.make_ragged_event(ev.RAGGED)
            cut = 30.0
            g = _gpu_ragged(p2r, ctx, d, cut)
            r = oracle.fit_ragged(d, chi2_cut=cut, nthreads=16)
            fs = final_surface_of(r["par"], d["offsets"], d["surf_type"], d["surf_val"])
            report(f"ragged {ev.RAGGED.name} (chi2 cut {cut:g})", g, r, fs, dump=_dump(name))
        elif name == "learned":
            mlp = p2r.Mlp(ctx)
            mlp.load(learned.DEFAULT_CKPT)
            d = ev.make_barrel_event(ev.LEARNED_EVAL)
            g = _gpu_p2r(p2r, ctx, d, W, mlp=mlp)
            r = oracle.fit_event(d, "barrel", nthreads=16)
            report(f"p2r learned start {ev.LEARNED_EVAL.name} (W={W})", g, r, "cylinder", dump=_dump(name))
        else:
            u2d = name == "p2r_2d"
            d = ev.make_barrel_event(ev.P2R_THROUGHPUT)
            g = _gpu_p2r(p2r, ctx, d, W, update_2d=int(u2d), cyl_start=int(name == "p2r_cf"),
                         fp64=int(name == "p2r_f64"))
            if u2d not in exact:      # the oracle has no start choice and no precision switch
                exact[u2d] = oracle.fit_event(d, "barrel", nthreads=16, update_2d=u2d)
            r = exact[u2d]
            what = {"p2r_2d": "p2r update in the hit frame", "p2r_cf": "p2r closed-form crossing start",
                    "p2r_f64": "p2r every step in FP64"}.get(name, "p2r")
            report(f"{what} {ev.P2R_THROUGHPUT.name} (W={W})", g, r, "cylinder", dump=_dump(name))
        print(f"  ({time.time() - t:.0f} s)", flush=True)
        del d, g, r
    ctx.close()


if __name__ == "__main__":
    sys.exit(main())
