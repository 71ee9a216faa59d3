#!/usr/bin/env python3
"""Throughput of the HIP rasterizer + AdpSplit path on one MI355X.

Workload (the metric's configuration): 1,000,000 clustered Gaussians, SH
degree 3, FP32, one 1256x828 view.  One step = forward render with the fused
L1 error map, the error-region statistics of the view (5% of the Gaussians
are split candidates), and the backward pass for a fixed synthetic upstream
gradient.  All inputs are seeded, synthetic and resident in HBM before the
timed region.  The error statistics and the backward pass both read only
the render's outputs: the timed step runs the statistics on a second stream
beside the reverse pass (--no-overlap: everything on one stream; both times
are reported).  Also reported: the densification step (500,000 Gaussians, 16
views, top-5% candidates, adaptive split) and the CPU oracle on a bounded
sample of the same workload.

Prints one JSON line.  Options: --steps K --warmup W --gpus N (1 only),
--no-cpu-baseline, --no-densify, --no-training, --no-batched, --no-serve,
--no-overlap, --tuning (replay a tuning without the autotuner).
"""
import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X published peaks
PEAK_HBM_GBS = 8000.0
# VALU: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 39.3 T lane-ops/s (one
# non-packed FP32 op per lane per clock; transcendentals at a quarter rate)
PEAK_VALU_TOPS = 256 * 64 * 2.4e9 / 1e12

# Algorithmic VALU lane-ops, counted from the formulas of Eq. (rendering)
# (add/sub/mul/fma/min/compare/select = 1, exp = 4 at quarter rate).  Every
# algorithmic pair (a pixel inside a Gaussian's compact box, in depth order
# up to the pixel's stop point) evaluates alpha and tests it:
#   offset 2, exponent 9, exp 4, alpha 2, alpha test 1                  -> 18
# and only a contributor (alpha >= 1/255) composites or takes gradients:
#   forward: transmittance 2, stop test 1, weight 1, colour 3,
#            dominant test + select 3                                   -> 10
#   reverse: restore T 5 (reciprocal 4 + mul), colour grads 3,
#            accumulators 9, dL/dalpha 7, background term 3,
#            opacity / exponent grads 2, mean grads 6, conic grads 6    -> 41
# The pair and contributor counts are the oracle's (tests/golden).
OPS_ALPHA_PER_PAIR = 18
OPS_FWD_PER_CONTRIB = 10
OPS_BWD_PER_CONTRIB = 41


def blend_ops(pairs, contributors):
    """Algorithmic lane-ops of the forward and of the reverse blend."""
    return (pairs * OPS_ALPHA_PER_PAIR + contributors * OPS_FWD_PER_CONTRIB,
            pairs * OPS_ALPHA_PER_PAIR + contributors * OPS_BWD_PER_CONTRIB)


def _args():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-densify", action="store_true")
    ap.add_argument("--no-training", action="store_true", help="skip the end-to-end densification training leg")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched multi-view leg")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving leg")
    ap.add_argument("--serve-seconds", type=float, default=30.0, help="Poisson arrivals of the serving leg (seconds)")
    ap.add_argument("--json", default="", help="also write the JSON line to this file")
    ap.add_argument("--no-tune", action="store_true", help="skip the autotuner (default tuning)")
    ap.add_argument("--no-overlap", action="store_true",
                    help="time the step with every stage on one stream (the value; by default the error statistics "
                         "run on a second stream beside the reverse pass)")
    ap.add_argument("--tuning", default="",
                    help="skip the autotuner and set this tuning, e.g. lds_batch=256,longest_first=1,bin_tile=32 "
                         "(fields of api.set_tuning; the profiles replay the bench's choice with it)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="run one plain 1 GiB device copy first (calibrates rocprofv3 FETCH_SIZE / WRITE_SIZE)")
    return ap.parse_args()


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def sh3_bytes():
    return 4 * (3 + 3 + 4 + 1 + 48)


def training_step_bench(args):
    import numpy as np
    import torch

    from paper_2605_06876_amd import api, synth

    api.lib()   # raises if the HIP library is missing: no fallback
    torch.cuda.set_device(0)
    log("bench: generating the 1M-Gaussian workload")
    scene, cam, gt = synth.c2_inputs()
    n, W, H = scene.n, cam.width, cam.height
    ctx = api.Context(0, max_pixels=W * H)   # the error statistics' scratch, reserved at set-up
    g = api.Gaussians.from_scene(scene)
    gtt = torch.from_numpy(gt).cuda()
    G = torch.from_numpy(np.random.default_rng(7).normal(0.0, 1.0 / (3 * W * H), (3, H, W)).astype(np.float32)).cuda()
    rng = np.random.default_rng(8)
    is_cand = torch.from_numpy((rng.uniform(size=n) < 0.05).astype(np.uint8)).cuda()
    params = api.SplitParams()
    regions = api.RegionBuffer(W * H // params.m_min + 1)
    attr = torch.zeros(n, dtype=torch.int32, device="cuda")
    g2d = torch.zeros(n, dtype=torch.float32, device="cuda")
    vis = torch.zeros(n, dtype=torch.int32, device="cuda")
    # capacity fixed up front (16 pairs per Gaussian): the frame never reads the
    # pair count back to grow, so a step never waits on the host; the count is
    # checked against the capacity after the timed loop
    key_cap = 16 * n
    frame = api.Frame(ctx, n, W, H, key_cap=key_cap, auto_grow=False)
    image = torch.empty(3, H, W, dtype=torch.float32, device="cuda")
    grads = api.Gaussians.empty(n, scene.sh_degree)
    dm = frame.device_maps()
    from paper_2605_06876_amd import autotune
    if args.tuning:
        kv = dict(item.split("=") for item in args.tuning.split(",") if item)
        api.set_tuning(ctx, **{k: int(v) for k, v in kv.items()})
        best, tune_ms = api.get_tuning(ctx), {}
    elif args.no_tune:
        best, tune_ms = api.get_tuning(ctx), {}
    else:
        log("bench: autotuning the blend launch (untimed)")
        # ten steps per candidate and round: the dispatch candidates differ by
        # about 1%, within the spread of three
        best, tune_ms = autotune.autotune(ctx, g, cam, frame, gt=gtt, dL=G, reps=10, use_cache=False, cache_path=None)

    # The error statistics and the reverse pass both only read the render's
    # outputs, so the statistics run on a second stream (default priority)
    # forked after the render and joined before the step ends.
    main = torch.cuda.current_stream()
    side = torch.cuda.Stream()
    ev_fork, ev_join = torch.cuda.Event(), torch.cuda.Event()

    def step_overlapped():
        api.render(ctx, g, cam, frame, gt=gtt, image=image)
        ev_fork.record(main)
        side.wait_event(ev_fork)
        with torch.cuda.stream(side):
            regions.count.zero_()
            api.accumulate_error_stats(ctx, W, H, dm["err"], dm["err_minmax"], dm["dom"], gtt, 0, is_cand, params,
                                       regions, attr)
            ev_join.record(side)
        api.render_backward(ctx, g, cam, frame, G, grads=grads, g2d_norm=g2d, vis_count=vis)
        main.wait_event(ev_join)

    def step_sequential():
        regions.count.zero_()
        api.render(ctx, g, cam, frame, gt=gtt, image=image)
        api.accumulate_error_stats(ctx, W, H, dm["err"], dm["err_minmax"], dm["dom"], gtt, 0, is_cand, params,
                                   regions, attr)
        api.render_backward(ctx, g, cam, frame, G, grads=grads, g2d_norm=g2d, vis_count=vis)

    def timed(step):
        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / args.steps

    log("bench: timing %d steps (statistics on a second stream, then all on one)" % args.steps)
    ms_seq = timed(step_sequential)
    ms_ovl = timed(step_overlapped)
    ms = ms_seq if args.no_overlap else ms_ovl
    # stage times come from one-stream steps: each stage's events then time
    # that stage alone, not its share of a device it splits with another
    step = step_sequential
    # per-stage times in separate steps: the stage events add a gap at every
    # stage boundary, so they stay out of the timed loop above
    stage_steps = max(1, min(args.steps, 10))
    api.timing_enable(ctx, True)
    api.timing_read(ctx)
    for _ in range(stage_steps):
        step()
    torch.cuda.synchronize()
    stages = api.timing_read(ctx)
    api.timing_enable(ctx, False)
    K = frame.n_keys()
    if K > key_cap:
        raise RuntimeError("bench: %d pairs exceed the frame's capacity of %d" % (K, key_cap))
    n_regions = int(regions.count.item())
    return dict(ms=ms, ms_sequential=ms_seq, ms_overlapped=ms_ovl, stages=stages, K=K, n=n, W=W, H=H,
                n_regions=n_regions, steps=args.steps,
                stage_steps=stage_steps, ctx=ctx,
                tuning=best, tuning_ms={k: round(v, 4) for k, v in tune_ms.items()})


def densify_bench(ctx):
    """500,000 Gaussians, 16 views of 1256x828, candidates = top 5% by the
    view-averaged screen-space gradient norm (the split rule of Sec. 3 with
    the gradient threshold set by rank), then AdpSplit."""
    import numpy as np
    import torch

    from paper_2605_06876_amd import api, synth

    n, W, H, V = 500_000, 1256, 828, 16
    scene = synth.scene_clusters(n, 1003, 3)
    views = synth.sphere_cameras(V, 4.0, [(W, H)], seed=1003)
    gts = [torch.from_numpy(synth.smooth_image(H, W, 2000 + v)).cuda() for v in range(V)]
    g = api.Gaussians.from_scene(scene)
    frame = api.Frame(ctx, n, W, H, key_cap=16 * n)
    image = torch.empty(3, H, W, dtype=torch.float32, device="cuda")
    g2d = torch.zeros(n, dtype=torch.float32, device="cuda")
    vis = torch.zeros(n, dtype=torch.int32, device="cuda")
    grads = api.Gaussians.empty(n, 3)
    # ADC statistic from 16 backward passes of the L1 loss (untimed set-up)
    for cam, gt in zip(views, gts):
        api.render(ctx, g, cam, frame, gt=gt, image=image)
        dL = torch.sign(image - gt) / (3 * W * H)
        api.render_backward(ctx, g, cam, frame, dL.contiguous(), grads=grads, g2d_norm=g2d, vis_count=vis)
    gi = (g2d / vis.clamp(min=1)).cpu().numpy()
    order = np.lexsort((np.arange(n), -gi))
    cand = np.sort(order[: n // 20]).astype(np.int32)
    is_cand = torch.zeros(n, dtype=torch.uint8, device="cuda")
    is_cand[torch.from_numpy(cand.astype(np.int64)).cuda()] = 1
    cand_t = torch.from_numpy(cand).cuda()
    noise = torch.from_numpy(synth.vanilla_noise(len(cand), 5)).cuda()
    params = api.SplitParams()
    regions = api.RegionBuffer(V * W * H // params.m_min // 4)
    attr = torch.zeros(n, dtype=torch.int32, device="cuda")
    out = api.Gaussians.empty(n + len(cand) * api.split_rows_per_candidate(params), 3)
    dm = frame.device_maps()
    ctx.reserve(max_pixels=W * H, max_gaussians=n, max_candidates=len(cand), max_regions=regions.capacity,
                max_views=V)

    def densify():
        regions.count.zero_()
        attr.zero_()
        for v, (cam, gt) in enumerate(zip(views, gts)):
            api.render(ctx, g, cam, frame, gt=gt, image=image)
            api.accumulate_error_stats(ctx, W, H, dm["err"], dm["err_minmax"], dm["dom"], gt, v, is_cand, params,
                                       regions, attr)
        return api.adaptive_split(ctx, g, cand_t, regions, views, attr, params, noise, out=out)

    # the same step with the V sampled views rendered by one batched launch
    bframe = api.BatchFrame.for_views(ctx, n, views, key_cap=16 * n * V)
    bimages = [torch.empty(3, H, W, dtype=torch.float32, device="cuda") for _ in views]

    def densify_batched():
        regions.count.zero_()
        attr.zero_()
        api.render_batch(ctx, g, views, bframe, gts=gts, images=bimages)
        for v in range(V):
            m = bmaps[v]
            api.accumulate_error_stats(ctx, W, H, m["err"], m["err_minmax"], m["dom"], gts[v], v, is_cand, params,
                                       regions, attr)
        return api.adaptive_split(ctx, g, cand_t, regions, views, attr, params, noise, out=out)

    densify()
    torch.cuda.synchronize()
    api.timing_enable(ctx, True)
    api.timing_read(ctx)
    reps = 3
    t0 = time.perf_counter()
    for _ in range(reps):
        res = densify()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st = api.timing_read(ctx)
    api.timing_enable(ctx, False)
    loop_rows, loop_n = int(res[2].sum().item()), int(res[4].item())
    api.render_batch(ctx, g, views, bframe, gts=gts, images=bimages)   # sizes the batch frame
    bmaps = [bframe.device_maps(v) for v in range(V)]
    rb = densify_batched()
    torch.cuda.synchronize()
    tb = time.perf_counter()
    for _ in range(reps):
        rb = densify_batched()
    torch.cuda.synchronize()
    batched_ms = (time.perf_counter() - tb) * 1e3 / reps
    if int(rb[2].sum().item()) != loop_rows or int(rb[4].item()) != loop_n:
        raise RuntimeError("bench: batched densification differs from the per-view loop")
    bframe.close()
    mode = res[1].cpu().numpy()
    # the split step of each method on the same regions (Table 2's ablation
    # steps, the fixed-N random split with N = 2 as in 3DGS and N = 5)
    variants = {}
    for name, kw in (("adpsplit", {}), ("fixed_n2", dict(variant=api.VARIANT_FIXED_N, fixed_n=2)),
                     ("fixed_n5", dict(variant=api.VARIANT_FIXED_N, fixed_n=5, noise_n=5)),
                     ("adaptive_n", dict(variant=api.VARIANT_ADAPTIVE_N, noise_n=params.n_max)),
                     ("child_init", dict(variant=api.VARIANT_CHILD_INIT))):
        vp = api.SplitParams(**kw)
        nz = noise if vp.noise_n <= 2 else torch.from_numpy(
            np.random.default_rng(5).standard_normal((len(cand), vp.noise_n, 3)).astype(np.float32)).cuda()
        vout = api.Gaussians.empty(n + len(cand) * api.split_rows_per_candidate(vp), 3)
        r = api.adaptive_split(ctx, g, cand_t, regions, views, attr, vp, nz, out=vout)
        torch.cuda.synchronize()
        tv = time.perf_counter()
        for _ in range(reps):
            r = api.adaptive_split(ctx, g, cand_t, regions, views, attr, vp, nz, out=vout)
        torch.cuda.synchronize()
        variants[name] = dict(split_ms=round((time.perf_counter() - tv) * 1e3 / reps, 3),
                              new_rows=int(r[2].sum().item()), n_out=int(r[4].item()))
    # the full density-control step (select, the 16 views' renders and error
    # statistics, clone, split, row map, prune, moment gather) with every count
    # on the device, run eagerly and replayed as one HIP graph; selection by
    # rank: the gradient threshold is the n/20-th largest view-averaged
    # gradient, and every selected Gaussian is a split candidate
    from paper_2605_06876_amd import densify as dens
    a64 = (g2d.double() / vis.clamp(min=1).double()).cpu().numpy()
    thr = float(np.sort(a64)[::-1][n // 20 - 1])
    m0, v0 = api.Gaussians.empty(n, 3), api.Gaussians.empty(n, 3)
    step = dens.DensifyStep(ctx, n, 3, "adpsplit", params, views, gts, regions, cand_cap=n // 20 + 1024,
                            key_cap_per_entry=16)
    step.noise.copy_(torch.from_numpy(synth.vanilla_noise(step.cc, 5, step.noise_n)).view_as(step.noise))
    sargs = (g, m0, v0, g2d, vis, thr, 0.0, 0.005, 0.0)
    step.run(*sargs)
    torch.cuda.synchronize()
    ts = time.perf_counter()
    for _ in range(reps):
        step.run(*sargs)
    torch.cuda.synchronize()
    step_eager_ms = (time.perf_counter() - ts) * 1e3 / reps
    eager_n = int(step.n_out.item())
    gs = torch.cuda.Stream()
    graph = step.capture(gs, *sargs)
    graph.launch(gs)
    gs.synchronize()
    tg = time.perf_counter()
    for _ in range(reps):
        graph.launch(gs)
    gs.synchronize()
    step_graph_ms = (time.perf_counter() - tg) * 1e3 / reps
    if int(step.n_out.item()) != eager_n:
        raise RuntimeError("bench: graph replay of the density-control step differs from the eager step")
    full_step = dict(ms_eager=round(step_eager_ms, 3), ms_graph=round(step_graph_ms, 3),
                     candidates=int(step.sel[3].item()), n_out=eager_n,
                     note="select + 16 batched renders with error statistics + clone + split + row map + prune + "
                          "moment gather, counts on the device")
    graph.close()
    step.close()
    return dict(ms=(t1 - t0) * 1e3 / reps, ms_batched_views=round(batched_ms, 3), n=n, views=V, candidates=len(cand),
                full_step=full_step,
                regions=int(regions.count.item()),
                new_rows=int(res[2].sum().item()), n_out=int(res[4].item()),
                modes=dict(vanilla=int((mode == 0).sum()), reset=int((mode == 1).sum()), adaptive=int((mode == 2).sum())),
                stage_ms={k: round(v[0] / reps, 4) for k, v in st.items() if v[1]}, split_variants=variants)


def training_bench(ctx):
    """Synthetic end-to-end densification training (3DGS's loop with adaptive
    density control): a 200,000-Gaussian teacher rendered from 48 training and
    8 held-out cameras at 640x480; a student initialised from 20,000 noisy
    teacher centres; densification every 100 iterations from 300.  The arms
    of Table 1 and Fig. 2 (train.compare_arms): the vanilla N = 2 split on the
    full schedule (3750 iterations, densification until 3500), and on the
    shortened one (3000, until 2100) the vanilla split, five random children,
    the vanilla split with its threshold lowered to AdpSplit's final count,
    and AdpSplit (20 sampled views).  Held-out PSNR against training time
    (evaluation excluded) and the number of Gaussians, every 250 iterations."""
    from paper_2605_06876_amd import train

    pb = train.Problem(ctx, n_teacher=200_000, n_train=48, n_eval=8, size=(640, 480), seed=7)
    res = train.compare_arms(ctx, pb, iters=3000, densify_until=2100, seed=0, n_init=20_000)
    out = dict(teacher=200_000, size="640x480", train_views=48, eval_views=8, init=20_000,
               schedules=res.pop("schedules"))
    for arm, r in res.items():
        out[arm] = {k: v for k, v in r.items() if k != "history"}
        out[arm]["curve"] = [[h["it"], h["train_s"], h["psnr"], h["n"]] for h in r["history"]]
    out["curve_columns"] = ["iteration", "train_s", "psnr_db", "gaussians"]
    return out


C4_SIZES = [(640, 480), (800, 600), (960, 640), (1024, 768), (1256, 828), (1280, 720), (1440, 960), (1600, 1064)]


def batched_bench(reps=10):
    """8 cameras of uneven resolution (640x480 up to 1600x1064) on a radius-4
    sphere over 1,500,000 clustered Gaussians (SH 3): forward + backward of
    all views as (a) the plain per-view loop (one render and one backward
    call per view), (b) one batched render + one batched backward, (c) the
    batched step replayed from a HIP graph.  Same tuning for all three (tuned
    on the batched step)."""
    import numpy as np
    import torch

    from paper_2605_06876_amd import api, autotune, synth

    n = 1_500_000
    scene = synth.scene_clusters(n, 1004, 3)
    cams = synth.sphere_cameras(len(C4_SIZES), 4.0, C4_SIZES, seed=1004)
    g = api.Gaussians.from_scene(scene)
    del scene
    rng = np.random.default_rng(1004)
    dLs = [torch.from_numpy(rng.normal(0.0, 1.0 / (3 * c.width * c.height), (3, c.height, c.width))
                            .astype(np.float32)).cuda() for c in cams]
    images = [torch.empty(3, c.height, c.width, device="cuda") for c in cams]
    grads = api.Gaussians.empty(n, 3)
    px = sum(c.width * c.height for c in cams)
    ctx = api.Context(0)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        probe = api.BatchFrame.for_views(ctx, n, cams, key_cap=64 * n)
        api.render_batch(ctx, g, cams, probe, images=images)
        s.synchronize()
        K = probe.n_keys()
        probe.close()
        frame = api.BatchFrame.for_views(ctx, n, cams, key_cap=K + K // 4 + 4096, auto_grow=False)
        frames = [api.Frame(ctx, n, c.width, c.height, key_cap=K) for c in cams]

        def batched():
            api.render_batch(ctx, g, cams, frame, images=images)
            api.render_backward_batch(ctx, g, frame, dLs, grads=grads)

        def loop():
            for c, f, im, dl in zip(cams, frames, images, dLs):
                api.render(ctx, g, c, f, image=im)
                api.render_backward(ctx, g, c, f, dl, grads=grads)

        key = autotune.workload_key(px // len(cams), 1, n, 3, views=len(cams))
        best, tune_ms = autotune.autotune_step(ctx, batched, key, reps=2, cache_path=None, use_cache=False)
        batched()
        s.synchronize()
        graph = api.Graph.capture(ctx, batched, s)

    def timed(fn):
        with torch.cuda.stream(s):
            fn()
            s.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                fn()
            s.synchronize()
        return (time.perf_counter() - t0) * 1e3 / reps

    ms_loop = timed(loop)
    ms_batch = timed(batched)
    ms_graph = timed(lambda: graph.launch(s))
    graph.close()
    return dict(views=len(cams), sizes=["%dx%d" % wh for wh in C4_SIZES], gaussians=n, pixels=px, pairs_tile=K,
                tuning=best, ms_per_view_loop=round(ms_loop, 4), ms_batched=round(ms_batch, 4),
                ms_batched_graph=round(ms_graph, 4),
                mpix_s_per_view_loop=round(px / ms_loop / 1e3, 2), mpix_s_batched=round(px / ms_batch / 1e3, 2),
                mpix_s_batched_graph=round(px / ms_graph / 1e3, 2),
                speedup_batched_graph_vs_loop=round(ms_loop / ms_graph, 3))


def serving_bench(seconds=30.0, rate=200.0, sweep_rates=(400.0, 1000.0, 1600.0, 2200.0, 3000.0), sweep_seconds=3.0,
                  tight_gib=8, tight_rate=2200.0, burst=400):
    """Four resident scenes (300k, 600k, 1.2M, 2M clustered Gaussians, SH 3);
    render requests with random poses on a radius-4 sphere and resolutions
    drawn from {640x480, 1280x720, 1920x1080} (mean 1.10 Mpx).  Continuous
    batching over 3 slots of up to 8 views vs the plain sequential loop, on
    the same request lists:
      poisson  Poisson arrivals at `rate`/s for `seconds`, slots sized from
               the free HBM after the scenes less 10% (each slot capped at
               serve.MAX_SLOT_PAIRS pairs);
      sweep    `sweep_seconds` of arrivals at each rate of `sweep_rates`, up
               to past the sequential loop's saturation;
      tight    a `tight_gib` GiB budget over the 3 slots (admission binds: the
               estimated pairs close batches early), at `tight_rate`/s;
      burst    `burst` requests arriving at once.
    Latency = completion event minus arrival; Mpix/s = pixels served over
    the wall time from the first arrival to the last completion."""
    import torch

    from paper_2605_06876_amd import api, serve, synth

    sizes = [(640, 480), (1280, 720), (1920, 1080)]
    ns = [300_000, 600_000, 1_200_000, 2_000_000]
    scenes = [api.Gaussians.from_scene(synth.scene_clusters(n, 2001 + k, 3)) for k, n in enumerate(ns)]
    ctx = api.Context(0)
    n_slots, max_views = 3, 8
    torch.cuda.synchronize()
    budget = int(0.9 * torch.cuda.mem_get_info()[0])
    cam_fn = lambda rng, w, h: synth.random_pose_camera(rng, 4.0, w, h)

    def fresh(reqs):
        return [serve.Request(r.rid, r.scene, r.cam, r.arrival) for r in reqs]

    def both(ex, spec, reqs):
        sched = serve.Scheduler(ex, spec, ns, keep_images=False)
        wall = serve.serve_open_loop(sched, reqs)
        res = dict(batched=serve.latency_stats(sched.completed, wall), batches=sched.batches,
                   mean_batch=round(len(reqs) / max(sched.batches, 1), 2), pair_bound=sched.pair_bound)
        seq = fresh(reqs)
        wall = serve.serve_sequential(ex, seq, keep_images=False)
        res["sequential"] = serve.latency_stats(seq, wall)
        return res

    def executor(budget_bytes):
        spec = serve.default_spec(ns, sizes, max_views, budget_bytes, n_slots)
        ex = serve.GpuExecutor(ctx, scenes, spec, n_slots)
        warm = serve.poisson_requests(24, 0.0, len(ns), sizes, cam_fn, seed=1)
        serve.serve_open_loop(serve.Scheduler(ex, spec, ns, keep_images=False), warm)
        serve.serve_sequential(ex, fresh(warm), keep_images=False)
        torch.cuda.synchronize()
        return spec, ex

    spec, ex = executor(budget)
    out = dict(scenes=ns, sizes=["%dx%d" % s for s in sizes], slots=n_slots, max_views=max_views,
               budget_bytes=budget, hbm=serve.hbm_footprint(scenes, spec, n_slots), slot_pairs=spec.pairs)
    reqs = serve.poisson_requests(int(seconds * rate), rate, len(ns), sizes, cam_fn, seed=2005)
    ov = ex.overflows
    out["poisson"] = dict(rate_per_s=rate, seconds=seconds, **both(ex, spec, reqs), overflows=ex.overflows - ov)
    out["sweep"] = []
    for k, rt in enumerate(sweep_rates):
        reqs = serve.poisson_requests(int(sweep_seconds * rt), rt, len(ns), sizes, cam_fn, seed=2100 + k)
        ov = ex.overflows
        out["sweep"].append(dict(rate_per_s=rt, seconds=sweep_seconds, **both(ex, spec, reqs),
                                 overflows=ex.overflows - ov))
    reqs = serve.poisson_requests(burst, 0.0, len(ns), sizes, cam_fn, seed=2006)
    out["burst"] = dict(requests=burst, **both(ex, spec, reqs))
    ex.close()
    del ex
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    spec_t, ex_t = executor(tight_gib << 30)
    reqs = serve.poisson_requests(int(sweep_seconds * tight_rate), tight_rate, len(ns), sizes, cam_fn, seed=2200)
    ov, so = ex_t.overflows, ex_t.single_overflows
    out["tight"] = dict(budget_gib=tight_gib, slot_pairs=spec_t.pairs, rate_per_s=tight_rate, seconds=sweep_seconds,
                        hbm=serve.hbm_footprint(scenes, spec_t, n_slots), **both(ex_t, spec_t, reqs),
                        overflows=ex_t.overflows - ov, single_overflows=ex_t.single_overflows - so)
    ex_t.close()
    return out


def cpu_baseline():
    """The CPU oracle on the same training step: projection of all 1M
    Gaussians, forward + backward compositing of every pixel of the 1256x828
    view, reverse projection, and the error statistics of the oracle's own
    render with the same 5% candidate mask.  Nothing is scaled."""
    import numpy as np

    import oracle
    from paper_2605_06876_amd import synth

    scene, cam, gt = synth.c2_inputs()
    W, H, n = cam.width, cam.height, scene.n
    G = np.random.default_rng(7).normal(0.0, 1.0 / (3 * W * H), (3, H, W)).astype(np.float32)
    is_cand = (np.random.default_rng(8).uniform(size=n) < 0.05).astype(np.uint8)
    t0 = time.perf_counter()
    pr = oracle.project(scene, cam)
    r = oracle.render_rows(pr, dL_dcolor=G.transpose(1, 2, 0).reshape(-1, 3).astype(np.float64))
    oracle.project_backward(scene, cam, r["grad"])
    img = r["color"].reshape(H, W, 3).transpose(2, 0, 1).astype(np.float32)
    dom = r["dom"].reshape(H, W).astype(np.int32)
    oracle.error_stats(img, gt, dom, is_cand, 0, oracle.SplitParams(), np.zeros(n, np.int32))
    t1 = time.perf_counter()
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
    return dict(value=round(W * H / (t1 - t0) / 1e6, 5), unit="Mpix/s", cores=threads, kind="oracle",
                sample="the whole step: 1,000,000 Gaussians, all 1,039,968 pixels of the 1256x828 view, forward + "
                       "backward + error statistics (%.1f s)" % (t1 - t0),
                seconds=round(t1 - t0, 2), pairs_per_px=round(float(r["pairs"].mean()), 2))


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.machine()


def load_workload_constants():
    path = os.path.join(ROOT, "tests", "golden", "c2_workload.json")
    with open(path) as f:
        return json.load(f)


KERNEL_SOURCES = {
    "project": "project.hip", "scan": "binning.hip", "emit": "binning.hip", "sort": "radix.hip",
    "ranges": "binning.hip", "blend_fwd": "blend.hip", "blend_bwd": "blend.hip", "project_bwd": "project_bwd.hip",
    "error_stats": "errstats.hip",
}


def source_hash(stage):
    import hashlib
    path = os.path.join(ROOT, "paper_2605_06876_amd", "csrc", KERNEL_SOURCES[stage])
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic(stage):
    """HBM bytes per launch from the committed rocprofv3 --pmc summary
    (FETCH_SIZE and WRITE_SIZE scaled by a plain copy's counters), or None
    when there is none or the kernel's source changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        tr = json.load(f).get(stage)
    if not tr or tr.get("source_sha256_16") != source_hash(stage):
        return None
    return tr.get("bytes_per_launch")


def main():
    args = _args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library runs on a single device and has no multi-GPU path. "
              "Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)
    import torch

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.copy_probe:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    res = training_step_bench(args)
    consts = load_workload_constants()
    P_alg, C_alg = consts["pairs"], consts["contributors"]
    ops_fwd, ops_bwd = blend_ops(P_alg, C_alg)
    n, W, H, K = res["n"], res["W"], res["H"], res["K"]
    # stage time per step (a stage may record more than one segment per step)
    per_step = {k: v[0] / res["stage_steps"] for k, v in res["stages"].items() if v[1]}
    # algorithmic work per launch of each stage
    work = {
        "project": ("hbm", n * (sh3_bytes() + 64) / 1e9, "GB"),
        "scan": ("hbm", n * 8 / 1e9, "GB"),
        "emit": ("hbm", (n * 16 + K * 12) / 1e9, "GB"),
        "sort": ("hbm", K * 24 / 1e9, "GB"),
        "ranges": ("hbm", (K * 8 + 8 * ((W + 15) // 16) * ((H + 15) // 16)) / 1e9, "GB"),
        "blend_fwd": ("alu", ops_fwd / 1e12, "TOP"),
        "blend_bwd": ("alu", ops_bwd / 1e12, "TOP"),
        "project_bwd": ("hbm", n * (2 * sh3_bytes() + 36 + 4 + 16) / 1e9, "GB"),
        "error_stats": ("hbm", W * H * 30 / 1e9, "GB"),
    }
    dom_stage = max((k for k in per_step if k in work), key=lambda k: per_step[k])
    bound, amount, u = work[dom_stage]
    t = per_step[dom_stage] / 1e3
    if bound == "hbm":
        roof = dict(bound="hbm", achieved=round(amount / t, 1), peak=PEAK_HBM_GBS, unit="GB/s")
    else:
        roof = dict(bound="alu", achieved=round(amount / t, 3), peak=round(PEAK_VALU_TOPS, 2), unit="TOP/s")
    roof["frac"] = round(roof["achieved"] / roof["peak"], 4)
    roof["kernel"] = dom_stage
    roof["avg_ms"] = round(per_step[dom_stage], 4)
    roof["traffic"] = measured_traffic(dom_stage)
    all_roofs = {}
    for k, (b, amt, unit) in work.items():
        if k in per_step and per_step[k] > 0:
            ach = amt / (per_step[k] / 1e3)
            pk = PEAK_HBM_GBS if b == "hbm" else PEAK_VALU_TOPS
            all_roofs[k] = dict(ms=round(per_step[k], 4), achieved=round(ach, 2),
                                unit="GB/s" if b == "hbm" else "TOP/s", frac=round(ach / pk, 4))
    # both blends against the VALU roofline together (the forward stage
    # includes the single-block post-forward kernel)
    blend_roof = None
    if per_step.get("blend_fwd", 0) > 0 and per_step.get("blend_bwd", 0) > 0:
        t_fb = (per_step["blend_fwd"] + per_step["blend_bwd"]) / 1e3
        ach = (ops_fwd + ops_bwd) / 1e12 / t_fb
        blend_roof = dict(bound="alu", achieved=round(ach, 3), peak=round(PEAK_VALU_TOPS, 2), unit="TOP/s",
                          frac=round(ach / PEAK_VALU_TOPS, 4), stages=["blend_fwd", "blend_bwd"],
                          ms=round(t_fb * 1e3, 4))
    mpix = W * H / 1e6
    value = mpix / (res["ms"] / 1e3)
    fb_ms = sum(per_step.get(k, 0.0) for k in ("project", "scan", "emit", "sort", "ranges", "blend_fwd", "blend_bwd",
                                                "project_bwd"))
    out = {
        "metric": "fwd+bwd Mpix/s @1M Gaussians 1256x828",
        "value": round(value, 2),
        "unit": "Mpix/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(res["ms"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded clustered scene, smooth synthetic target; the paper's datasets are unavailable)",
        "config": {"workload": "training step: render + L1 error statistics (5% candidates) + backward, "
                               "1,000,000 Gaussians SH3, one 1256x828 view",
                   "gaussians": n, "width": W, "height": H, "sh_degree": 3, "pairs_tile": K, "pairs_alg": P_alg,
                   "contributors_alg": C_alg,
                   "regions": res["n_regions"], "tuning": res["tuning"]},
        "tuning_candidates_ms": res["tuning_ms"],
        "roofline": roof,
        "stage_ms": {k: round(v, 4) for k, v in per_step.items()},
        "stage_roofline": all_roofs,
        "blend_roofline": blend_roof,
        "fwd_bwd_kernels_ms": round(fb_ms, 4),
        "step_streams": {"ms_statistics_beside_reverse_pass": round(res["ms_overlapped"], 4),
                         "ms_one_stream": round(res["ms_sequential"], 4),
                         "value_from": "one stream" if args.no_overlap else "statistics beside the reverse pass"},
    }
    if not args.no_densify:
        log("bench: densification step (500k Gaussians, 16 views)")
        out["densify"] = densify_bench(res["ctx"])
    if not args.no_training:
        log("bench: end-to-end densification training (full-schedule, shortened, five-child, equal-count and AdpSplit arms)")
        out["training"] = training_bench(res["ctx"])
    if not args.no_batched:
        log("bench: batched training render (8 uneven views, 1.5M Gaussians)")
        out["batched"] = batched_bench()
    if not args.no_serve:
        log("bench: serving (4 resident scenes, Poisson arrivals)")
        out["serving"] = serving_bench(args.serve_seconds)
    if not args.no_cpu_baseline:
        log("bench: CPU oracle baseline")
        out["cpu_baseline"] = cpu_baseline()
        out["cpu_baseline"]["cpu_model"] = cpu_model()
    line = json.dumps(out)
    print(line, flush=True)
    if args.json:
        with open(args.json, "w") as f:
            f.write(line + "\n")


if __name__ == "__main__":
    main()
