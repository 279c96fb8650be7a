"""Benchmark of the fused propagate + Kalman-update fit on one MI355X.

Default workload: p2r, 100 events x 9,600 tracks x 20 barrel layers at
r = 2.5..110 cm (19.2 M track-layers per step), FP32 on the GPU, inputs
resident in HBM.  A step is one launch of the fused fit over the whole
workload.  Protocol (paper, Section 4): untimed warm-up steps (back to back
for --settle-ms, so that the GPU's clock has settled after the idle time of
input generation, then W more), then K timed steps bracketed by device
synchronisation; the kernel's own time is taken with HIP events on the
stream it is launched on.

Prints ONE JSON line.  Besides the headline p2r figure it carries the
roofline of the fit kernel, the FP64 CPU oracle timed on a bounded sample
of the same workload (cpu_baseline), and secondary measurements (p2z with
and without host transfers, the ragged batched fit, the learned start).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

METRIC = "track-layer updates/sec at 1 GPU and % HBM roofline; learned vs plain at 1e-4 rel"
UNIT = "track-layers/s"
HBM_PEAK_GBPS = 8000.0
# FP32 vector peak of MI355X (published; counts an FMA as 2 flops): one wave64
# FP32 instruction per 2 cycles per SIMD at 2.4 GHz, which plain (non-packed)
# FP32 instructions reach when a SIMD holds enough waves
FP32_PEAK_TFLOPS = 157.3
# dense BF16 matrix-core peak of MI355X, and the path-length network's work per
# evaluation (7 -> 64 -> 64 -> 1: 4,608 multiply-adds, 2 flops each)
BF16_PEAK_TFLOPS = 2500.0
MLP_FLOP_PER_EVAL = 2 * (7 * 64 + 64 * 64 + 64)
# algorithmic work per track-layer of the textbook method (3x3 update, Joseph
# covariance, J C J^T with J's structural zeros, two helix evaluations per
# cylinder crossing; FMA = 2 flops): the rate is quoted in these flops whatever
# cheaper form of the same arithmetic the kernel uses
P2R_FLOP_PER_TL = 1261.0
P2Z_FLOP_PER_TL = 930.0
TRACK_BYTES = 28 * 4 * 2 + 4 + 4      # record in + record out + chi2 + status
HIT_BYTES = 9 * 4


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=20, help="untimed steps before the timed ones")
    ap.add_argument("--settle-ms", type=float, default=200.0,
                    help="before the warm-up steps, run the step back to back for this long, untimed: after an "
                         "idle period the GPU's clock needs some tens of milliseconds of sustained work to "
                         "settle, and a p2r step is 0.3 ms")
    ap.add_argument("--no-extra", action="store_true", help="headline p2r figure only")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--variant", default=None,
                    help="time this p2r kernel variant (as reported in config.variant) without autotuning")
    ap.add_argument("--tune-cache", default=None,
                    help="autotuner cache file: a run that finds its workload there times the same variant "
                         "without re-tuning (profiled runs use the variant the timed run chose)")
    ap.add_argument("--sweep-variants", action="store_true",
                    help="run every compiled p2r variant twice on the workload (for per-variant counters)")
    ap.add_argument("--rag-variant", default=None,
                    help="time this ragged kernel variant (as reported in the ragged record) without autotuning")
    ap.add_argument("--only", choices=["p2z", "ragged", "learned"], default=None,
                    help="run just this secondary leg and print its record (for profiling)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run one plain 1 GiB device copy (counter calibration under rocprofv3)")
    return ap.parse_args()


def kernel_source_hash() -> str:
    """Hash of the sources the p2r/p2z kernels are compiled from (kernels.hip
    and the headers it includes); profiles carry it so that counter data taken
    from other kernels is not reported."""
    import hashlib
    d = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2401_14221_amd", "csrc")
    h = hashlib.sha256()
    for f in ("kernels.hip", "launch.h", "mlp.h", "mlp_dev.h", "track_math.h"):
        h.update(f.encode())
        h.update(open(os.path.join(d, f), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(variant: str):
    """HBM bytes per launch of the timed p2r kernel from the committed counter profile.

    None unless the profile was taken from the same kernel sources; the
    record holds every compiled variant (FETCH_SIZE and WRITE_SIZE per
    dispatch, each scaled by its reading for a plain device copy of known
    size)."""
    p = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles", "p2r_fit_traffic.json")
    if not os.path.exists(p):
        return None
    rec = json.load(open(p))
    if rec.get("kernel_source_hash") != kernel_source_hash():
        return None
    v = rec.get("variants", {}).get(variant)
    return None if v is None else v.get("hbm_bytes_per_launch")


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


SETTLE_S = 0.2          # set from --settle-ms
LAST_SETTLE_STEPS = 0   # untimed settle steps of the last timed() call (profiles locate the timed launches)


def settle(fn):
    """Run `fn` back to back, untimed, for SETTLE_S seconds of wall time (in
    rounds of 8 steps, each waited for, so that the host does not queue far
    ahead of the GPU).  Returns the number of steps run."""
    import torch
    t0 = time.perf_counter()
    n = 0
    while time.perf_counter() - t0 < SETTLE_S:
        for _ in range(8):
            fn()
        n += 8
        torch.cuda.synchronize()
    return n


def timed(fn, steps, warmup, stream):
    """Mean device time of one step over `steps` steps (HIP events on `stream`
    around them, after SETTLE_S seconds of untimed steps, `warmup` more and a
    synchronisation), the host wall time per step, and the standard deviation
    of the per-step times (events recorded between the steps)."""
    import torch
    global LAST_SETTLE_STEPS
    LAST_SETTLE_STEPS = settle(fn)
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    t0 = time.perf_counter()
    ev[0].record(stream)
    for i in range(steps):
        fn()
        ev[i + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per = np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(steps)])
    return ev[0].elapsed_time(ev[steps]) / steps, wall / steps * 1e3, float(per.std())


def copy_bandwidth(dev, stream):
    """GB/s of a plain 1 GiB device-to-device copy (bytes read + written): the
    bandwidth a streaming kernel can reach, next to the published peak."""
    import torch
    src = torch.empty(1 << 28, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)

    def cp():
        with torch.cuda.stream(stream):
            dst.copy_(src)

    ms, _, _ = timed(cp, 5, 2, stream)
    del src, dst
    return 2 * (1 << 30) / (ms * 1e-3) / 1e9


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1 (the fit needs no "
                                   "cross-GPU exchange: shard tracks by event, one process per GPU)"}))
        sys.exit(2)
    global SETTLE_S
    SETTLE_S = max(0.0, args.settle_ms) * 1e-3
    import torch
    import paper_2401_14221_amd as p2r
    from synth import events as ev

    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(device=dev)
    ctx = p2r.Context(0, tune_cache=args.tune_cache)
    if args.calib_copy:
        # one plain device copy of 1 GiB: the counters' reading for known bytes
        src = torch.empty(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.only:
        leg = {"p2z": p2z_leg, "ragged": ragged_leg, "learned": learned_leg}[args.only]
        print(json.dumps({"leg": args.only, "result": leg(ctx, args, stream, ev, p2r, dev)}))
        return
    cfg = ev.P2R_THROUGHPUT
    L = len(cfg.surfaces)
    n = cfg.n_total
    if args.variant:
        ctx.set_variant(0, args.variant)
    elif not args.no_autotune:
        with torch.cuda.stream(stream):
            ctx.autotune(0, n, L, stream=stream)
    W = ctx.layout_width(0)
    log(f"p2r variant {ctx.variant_name(0)} (W={W}); generating {cfg.name}")
    t = time.time()
    d = ev.make_barrel_event(cfg)
    log(f"generated in {time.time() - t:.1f}s")
    trk = p2r.pack_tracks(d["par"], d["cov"], d["q"], W, device=dev)
    hits = p2r.pack_hits_p2r(d["hits"], d["hitcov"], W, device=dev)
    radii = torch.as_tensor(d["surf"], dtype=torch.float32, device=dev)
    out = (torch.empty_like(trk), torch.empty(n, dtype=torch.float32, device=dev),
           torch.empty(n, dtype=torch.int32, device=dev))
    opts = p2r._lib.default_opts(width=W)
    torch.cuda.synchronize()

    def step():
        ctx.p2r_propagate_update(n, radii, trk, hits, out=out, opts=opts, stream=stream)

    if args.sweep_variants:
        rec = {}
        for name in p2r.variant_names(0):
            ctx.set_variant(0, name)
            Wv = ctx.layout_width(0)
            tv = p2r.pack_tracks(d["par"], d["cov"], d["q"], Wv, device=dev)
            hv = p2r.pack_hits_p2r(d["hits"], d["hitcov"], Wv, device=dev)
            ov = (torch.empty_like(tv), out[1], out[2])
            o_v = p2r._lib.default_opts(width=Wv)
            torch.cuda.synchronize()          # the packing ran on the current stream

            def step_v():
                ctx.p2r_propagate_update(n, radii, tv, hv, out=ov, opts=o_v, stream=stream)

            rec[name] = timed(step_v, 2, 1, stream)[0]
            del tv, hv, ov
            log(f"sweep {name}: {rec[name]:.3f} ms")
        print(json.dumps({"sweep": rec, "kernel_source_hash": kernel_source_hash()}))
        return

    ms, wall_ms, ms_std = timed(step, args.steps, args.warmup, stream)
    copy_gbps = copy_bandwidth(dev, stream)
    tl = n * L
    value = tl / (ms * 1e-3)
    st = out[2].cpu().numpy().view(np.uint32)
    nused = ((st >> 8) & 0xFF).astype(np.int64)
    alg_bytes = n * TRACK_BYTES + tl * HIT_BYTES
    gbps = alg_bytes / (ms * 1e-3) / 1e9
    tflops = tl * P2R_FLOP_PER_TL / (ms * 1e-3) / 1e12
    log(f"p2r: {ms:.3f} ms/step, {value:.3e} track-layers/s, {gbps:.0f} GB/s algorithmic, {tflops:.1f} TFLOP/s")
    res = {
        "metric": METRIC, "value": value, "unit": UNIT, "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "settle_ms": args.settle_ms, "settle_steps": LAST_SETTLE_STEPS,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded RK4 truth simulation, smeared hits)",
        "config": {"workload": cfg.name, "events": cfg.n_events, "tracks_per_event": cfg.n_tracks,
                   "layers": L, "track_layers": tl, "width": W, "variant": ctx.variant_name(0),
                   "parallelism": "one lane per track, one GPU"},
        "roofline": {"bound": "alu", "achieved": tflops, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": tflops / FP32_PEAK_TFLOPS, "traffic": measured_traffic(ctx.variant_name(0)),
                     "kernel": ctx.variant_name(0), "flop_per_track_layer": P2R_FLOP_PER_TL},
        "hbm": {"achieved": gbps, "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": gbps / HBM_PEAK_GBPS,
                "bytes_per_launch": alg_bytes, "copy_measured": copy_gbps, "frac_of_copy": gbps / copy_gbps},
        "fit": {"updates_applied": int(nused.sum()), "track_layers": tl,
                "fp64_fallbacks": int(((st & p2r.ST_FP64_FALLBACK) != 0).sum()),
                "no_crossing_tracks": int(((st & p2r.ST_NO_CROSSING) != 0).sum()),
                "newton_fail_tracks": int(((st & p2r.ST_NEWTON_FAIL) != 0).sum()),
                "wall_ms_per_step": wall_ms, "ms_per_step_std": ms_std},
    }
    res["config"]["kernel_source_hash"] = kernel_source_hash()
    if not args.no_extra:
        # the same workload from the closed-form FP32 crossing as Newton's start
        # (one helix evaluation per layer instead of two)
        opts_cf = p2r._lib.default_opts(width=W, cyl_start=1)

        def step_cf():
            ctx.p2r_propagate_update(n, radii, trk, hits, out=out, opts=opts_cf, stream=stream)

        ms_cf, _, _ = timed(step_cf, args.steps, args.warmup, stream)
        res["closed_form_start"] = {"ms_per_step": ms_cf, "value": tl / (ms_cf * 1e-3), "unit": UNIT}
        log(f"p2r closed-form start: {ms_cf:.3f} ms/step")
        # the update in the hit's (r-phi, z) frame (two measured coordinates)
        opts_2d = p2r._lib.default_opts(width=W, update_2d=1)

        def step_2d():
            ctx.p2r_propagate_update(n, radii, trk, hits, out=out, opts=opts_2d, stream=stream)

        ms_2d, _, _ = timed(step_2d, args.steps, args.warmup, stream)
        res["update_2d"] = {"ms_per_step": ms_2d, "value": tl / (ms_2d * 1e-3), "unit": UNIT,
                            "note": "Kalman update in the hit's (r-phi, z) frame, chi2 with 2 dof"}
        log(f"p2r hit-frame update: {ms_2d:.3f} ms/step")
        # every step in FP64 (same inputs, results rounded to FP32)
        opts_64 = p2r._lib.default_opts(width=W, fp64=1)

        def step_64():
            ctx.p2r_propagate_update(n, radii, trk, hits, out=out, opts=opts_64, stream=stream)

        ms_64, _, _ = timed(step_64, max(3, args.steps // 2), args.warmup, stream)
        res["fp64"] = {"ms_per_step": ms_64, "value": tl / (ms_64 * 1e-3), "unit": UNIT,
                       "note": "every step in FP64 on the same FP32 inputs; results rounded to FP32"}
        log(f"p2r FP64: {ms_64:.3f} ms/step")
    del trk, hits, out
    if not args.no_extra:
        res["extra"] = extra_legs(ctx, args, stream, ev, p2r, dev)
    if not args.no_cpu:
        res["cpu_baseline"] = cpu_baseline(d, ev)
    print(json.dumps(res))


def extra_legs(ctx, args, stream, ev, p2r, dev):
    out = {"p2z": p2z_leg(ctx, args, stream, ev, p2r, dev),
           "ragged": ragged_leg(ctx, args, stream, ev, p2r, dev)}
    out["learned"] = learned_leg(ctx, args, stream, ev, p2r, dev)
    return out


def p2z_leg(ctx, args, stream, ev, p2r, dev):
    """p2z, 100 x 8192 x 20 disks; also the rate with host->device and device->host copies included."""
    import torch
    cfg = ev.P2Z_THROUGHPUT
    L = len(cfg.surfaces)
    n = cfg.n_total
    if not args.no_autotune:
        with torch.cuda.stream(stream):
            ctx.autotune(1, n, L, stream=stream)
    log(f"p2z variant {ctx.variant_name(1)}; generating {cfg.name}")
    d = ev.make_disk_event(cfg)
    trk_h = p2r.pack_tracks(d["par"], d["cov"], d["q"], 64).pin_memory()
    hits_h = p2r.pack_hits_p2z(d["hits"], d["hitcov"]).pin_memory()
    trk = trk_h.to(dev)
    hits = hits_h.to(dev)
    zs = torch.as_tensor(d["surf"], dtype=torch.float32, device=dev)
    o = (torch.empty_like(trk), torch.empty(n, dtype=torch.float32, device=dev),
         torch.empty(n, dtype=torch.int32, device=dev))
    opts = p2r._lib.default_opts()

    def step():
        ctx.p2z_propagate_update(n, zs, trk, hits, out=o, opts=opts, stream=stream)

    ms, _, _ = timed(step, args.steps, args.warmup, stream)
    settle_steps = LAST_SETTLE_STEPS
    opts_64 = p2r._lib.default_opts(fp64=1)

    def step_64():
        ctx.p2z_propagate_update(n, zs, trk, hits, out=o, opts=opts_64, stream=stream)

    ms_64, _, _ = timed(step_64, max(3, args.steps // 2), args.warmup, stream)
    out_h = torch.empty_like(trk_h).pin_memory()
    c2_h = torch.empty(n, dtype=torch.float32).pin_memory()
    st_h = torch.empty(n, dtype=torch.int32).pin_memory()

    def step_xfer():
        with torch.cuda.stream(stream):
            trk.copy_(trk_h, non_blocking=True)
            hits.copy_(hits_h, non_blocking=True)
            ctx.p2z_propagate_update(n, zs, trk, hits, out=o, opts=opts, stream=stream)
            out_h.copy_(o[0], non_blocking=True)
            c2_h.copy_(o[1], non_blocking=True)
            st_h.copy_(o[2], non_blocking=True)

    ms_x, _, _ = timed(step_xfer, max(3, args.steps // 2), args.warmup, stream)
    zs_h = torch.as_tensor(d["surf"], dtype=torch.float32)

    def step_pipe():
        ctx.propagate_update_host(1, n, zs_h, trk_h, hits_h, out=(out_h, c2_h, st_h), opts=opts, stream=stream)

    ms_p, _, _ = timed(step_pipe, max(3, args.steps // 2), args.warmup, stream)
    tl = n * L
    alg = n * TRACK_BYTES + tl * HIT_BYTES
    out = {"workload": cfg.name, "variant": ctx.variant_name(1),
           "ms_per_step": ms, "value": tl / (ms * 1e-3), "unit": UNIT, "settle_steps": settle_steps,
           "hbm_frac": alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBPS,
           "tflops": tl * P2Z_FLOP_PER_TL / (ms * 1e-3) / 1e12,
           "with_transfers": {"ms_per_step": ms_x, "value": tl / (ms_x * 1e-3),
                              "note": "pinned host buffers, H2D + fit + D2H on one stream"},
           "pipelined": {"ms_per_step": ms_p, "value": tl / (ms_p * 1e-3),
                         "h2d_bytes": int(trk_h.numel() * 4 + hits_h.numel() * 4),
                         "d2h_bytes": int(trk_h.numel() * 4 + n * 8),
                         "note": "p2z_propagate_update_host: pinned host buffers, chunks of 131072 tracks "
                                 "on three streams (copies overlap the fit)"},
           "fp64": {"ms_per_step": ms_64, "value": tl / (ms_64 * 1e-3)}}
    log(f"p2z: {ms:.3f} ms/step; FP64 {ms_64:.3f} ms; with transfers {ms_x:.3f} ms, pipelined {ms_p:.3f} ms")
    return out


def ragged_leg(ctx, args, stream, ev, p2r, dev):
    """Ragged batched fit, 1,000,000 tracks with 5..25 mixed surfaces, one graph launch per step."""
    import torch
    cfg = ev.RAGGED
    log(f"generating {cfg.name}")
    d = ev.make_ragged_event(cfg)
    f = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float32, device=dev)  # noqa: E731
    off = torch.as_tensor(d["offsets"], dtype=torch.int64, device=dev)
    stype = torch.as_tensor(d["surf_type"], dtype=torch.uint8, device=dev)
    sval, hpos, hcov = f(d["surf_val"]), f(d["hits"]), f(d["hitcov"])
    par, cov = f(d["par"]), f(d["cov"])
    q = torch.as_tensor(d["q"], dtype=torch.int8, device=dev)
    n = par.shape[0]
    H = int(d["offsets"][-1])
    ro = (torch.empty((n, 6), device=dev), torch.empty((n, 21), device=dev), torch.empty(n, device=dev),
          torch.empty(n, dtype=torch.int32, device=dev))
    ropts = p2r._lib.default_opts(chi2_cut=30.0)      # outliers up to ~100 sigma: per-hit chi2 cut
    lmax = cfg.extra["lmax"]
    if args.rag_variant:
        ctx.set_variant(2, args.rag_variant)
    elif not args.no_autotune:
        with torch.cuda.stream(stream):
            ctx.autotune(2, n, lmax, stream=stream)
    ctx.reserve(n, lmax)                               # sizing, outside the timed steps
    log(f"ragged variant {ctx.variant_name(2)}")

    def rstep():
        ctx.fit_tracks_batched(off, stype, sval, hpos, hcov, par, cov, q, H, lmax, out=ro, opts=ropts,
                               stream=stream)

    ms_r, _, _ = timed(rstep, args.steps, args.warmup, stream)
    alg_r = n * (TRACK_BYTES + 8) + H * (HIT_BYTES + 5)
    out = {"workload": cfg.name, "ms_per_step": ms_r, "value": H / (ms_r * 1e-3), "unit": UNIT,
           "settle_steps": LAST_SETTLE_STEPS, "track_layers": H, "hbm_frac": alg_r / (ms_r * 1e-3) / 1e9 / HBM_PEAK_GBPS,
           "variant": ctx.variant_name(2),
           "note": "one HIP graph per step: counting sort of the tracks, then the fit with the hits staged "
                   "through LDS"}
    log(f"ragged: {ms_r:.3f} ms/step, {H / (ms_r * 1e-3):.3e} track-layers/s")
    return out


def learned_leg(ctx, args, stream, ev, p2r, dev):
    """Learned vs plain start on the 100 x 9600 x 20 evaluation workload (same GPU, same tolerance)."""
    import torch
    from paper_2401_14221_amd import learned
    if not os.path.exists(learned.DEFAULT_CKPT):
        return {"skipped": "no trained network (paper_2401_14221_amd/data/mlp_p2r.ckpt)"}
    mlp = p2r.Mlp(ctx)
    mlp.load(learned.DEFAULT_CKPT)
    cfg = ev.LEARNED_EVAL
    L = len(cfg.surfaces)
    n = cfg.n_total
    W = ctx.layout_width(0)
    log(f"generating {cfg.name}")
    d = ev.make_barrel_event(cfg)
    trk = p2r.pack_tracks(d["par"], d["cov"], d["q"], W, device=dev)
    hits = p2r.pack_hits_p2r(d["hits"], d["hitcov"], W, device=dev)
    radii = torch.as_tensor(d["surf"], dtype=torch.float32, device=dev)
    torch.cuda.synchronize()                  # the packing ran on the current stream
    res = {"workload": cfg.name}
    outs = {}
    # the three starts of the helix-to-cylinder solve on the same workload:
    # straight line, closed-form FP32 crossing, learned proposal
    for name, m, cyl_start in (("plain", None, 0), ("closed_form", None, 1), ("learned", mlp, 0)):
        o = (torch.empty_like(trk), torch.empty(n, dtype=torch.float32, device=dev),
             torch.empty(n, dtype=torch.int32, device=dev))
        opts = p2r._lib.default_opts(width=W, cyl_start=cyl_start)
        if m is not None:
            opts.mlp = m.handle.value

        def step():
            ctx.p2r_propagate_update(n, radii, trk, hits, out=o, opts=opts, stream=stream)

        ms, _, _ = timed(step, args.steps, args.warmup, stream)
        cnt = torch.zeros(1, dtype=torch.int64, device=dev)
        opts.helix_evals = cnt.data_ptr()
        step()
        torch.cuda.synchronize()
        st = o[2].cpu().numpy().view(np.uint32)
        res[name] = {"ms_per_step": ms, "value": n * L / (ms * 1e-3), "unit": UNIT,
                     "helix_evals_per_track_layer": float(cnt.item()) / (n * L),
                     "ml_rejected_tracks": int(((st & p2r.ST_ML_REJECTED) != 0).sum())}
        outs[name] = o
    par_p, _, _ = p2r.unpack_tracks(outs["plain"][0], n)
    par_l, _, _ = p2r.unpack_tracks(outs["learned"][0], n)
    dphi = torch.remainder(par_l[:, 4] - par_p[:, 4] + np.pi, 2 * np.pi) - np.pi
    dpar = (par_l - par_p).abs()
    dpar[:, 4] = dphi.abs()
    scale = torch.maximum(par_p.abs(), torch.tensor([1, 1, 1, 0, 1, 0], dtype=torch.float32, device=dev))
    res["max_rel_diff_learned_vs_plain"] = float((dpar / scale.clamp_min(1e-30)).max())
    res["speed_ratio_learned_over_plain"] = res["plain"]["ms_per_step"] / res["learned"]["ms_per_step"]
    res["speed_ratio_closed_form_over_plain"] = res["plain"]["ms_per_step"] / res["closed_form"]["ms_per_step"]
    # the network's matrix-core work alone, at the dense BF16 peak: a floor on
    # the learned start's added time, however its kernel is written
    res["mlp_mfma_floor_ms"] = n * L * MLP_FLOP_PER_EVAL / (BF16_PEAK_TFLOPS * 1e12) * 1e3
    log(f"learned: {res['learned']['ms_per_step']:.3f} ms vs plain {res['plain']['ms_per_step']:.3f} ms vs "
        f"closed-form start {res['closed_form']['ms_per_step']:.3f} ms; evals/track-layer "
        f"{res['learned']['helix_evals_per_track_layer']:.3f} vs {res['plain']['helix_evals_per_track_layer']:.3f} "
        f"vs {res['closed_form']['helix_evals_per_track_layer']:.3f}; MLP matrix-core floor "
        f"{res['mlp_mfma_floor_ms']:.3f} ms")
    return res


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _time_oracle(oracle, d, nthreads, warmup=2, runs=10):
    for _ in range(warmup):
        oracle.fit_event(d, "barrel", nthreads=nthreads, sensitivity=False)
    times = []
    for _ in range(runs):
        t = time.perf_counter()
        oracle.fit_event(d, "barrel", nthreads=nthreads, sensitivity=False)
        times.append(time.perf_counter() - t)
    return float(np.mean(times)), float(np.std(times))


def cpu_baseline(d, ev):
    """FP64 oracle timed on the host: all cores of this process's CPU set (at
    most 16 threads) on the whole workload, and one core on the first 1/16 of
    its tracks; 2 warm-ups, then the mean of 10 runs, each.

    About 1.2 s per all-core run and 1.2 s per single-core run on 16-core
    hosts (~30 s in total)."""
    import oracle
    host_cpus = len(os.sched_getaffinity(0))
    nthreads = min(host_cpus, 16)
    n, L = d["par"].shape[0], d["hits"].shape[1]
    m, s = _time_oracle(oracle, d, nthreads)
    v = n * L / m
    n1 = max(1, n // 16)
    d1 = {k: (v_[:n1] if k in ("par", "cov", "q", "hits", "hitcov") else v_) for k, v_ in d.items()}
    m1, s1 = _time_oracle(oracle, d1, 1)
    v1 = n1 * L / m1
    model = _cpu_model()
    log(f"cpu oracle ({model}): {v:.3e} track-layers/s on {nthreads} threads ({m:.2f} +- {s:.2f} s per run); "
        f"{v1:.3e} on 1 thread ({m1:.2f} +- {s1:.2f} s per run of {n1} tracks)")
    return {"value": v, "unit": UNIT, "cores": nthreads, "kind": "oracle",
            "cpu_model": model, "host_cpus": host_cpus,
            "single_core": {"value": v1, "unit": UNIT, "cores": 1,
                            "sample": f"the first {n1} tracks x {L} layers"},
            "sample": f"the whole workload, {n} tracks x {L} layers, FP64 oracle (dual-number Jacobian, "
                      f"full 6x6 algebra), mean of 10 runs after 2 warm-ups (s.d. {s:.3f} s)"}


if __name__ == "__main__":
    main()
