"""Sensitivity of one AdpSplit densification step to its knobs (the paper's
sensitivity study varies r_erode, L, N_max, m_min and the number of sampled
views V, Sec. 5 and the appendix tables), on a synthetic densification
workload: Gaussians, views and targets as the densification leg of bench.py
(clustered Gaussians, views on a sphere, smooth synthetic targets), split
candidates = the top 5% by view-averaged screen-space gradient.

One knob varies at a time from the defaults (tau_l1 0.1, r_erode 2, m_min 5,
L 3, N_max 19, V 16 here: the workload has 16 views).  Reported per setting:
the time of the step (error statistics of V views + the split; renders
included), regions, new rows (children and parent copies), the output count,
and the device memory in use after the step (hipMemGetInfo, relative to the
start of the sweep; the library's scratch only grows, so this tracks the
peak).

    python -m paper_2605_06876_amd.sweep --out profiles/knob_sweep_densify.md
"""
import argparse
import json
import time

import numpy as np
import torch

from . import api, synth

DEFAULTS = dict(r_erode=2, L=3, n_max=19, m_min=5, V=16)
GRID = dict(r_erode=[0, 1, 2, 4, 8], L=[1, 2, 3, 5, 8], n_max=[2, 5, 9, 19, 39], m_min=[1, 5, 20, 80],
            V=[2, 4, 8, 16])


class DensifyWorkload:
    def __init__(self, ctx, n=300_000, size=(960, 640), n_views=16, seed=1003):
        self.ctx, self.n = ctx, n
        self.W, self.H = size
        scene = synth.scene_clusters(n, seed, 3)
        self.views = synth.sphere_cameras(n_views, 4.0, [size], seed=seed)
        self.gts = [torch.from_numpy(synth.smooth_image(self.H, self.W, 2000 + v)).cuda() for v in range(n_views)]
        self.g = api.Gaussians.from_scene(scene)
        self.frame = api.Frame(ctx, n, self.W, self.H, key_cap=16 * n)
        self.image = torch.empty(3, self.H, self.W, dtype=torch.float32, device="cuda")
        g2d = torch.zeros(n, dtype=torch.float32, device="cuda")
        vis = torch.zeros(n, dtype=torch.int32, device="cuda")
        grads = api.Gaussians.empty(n, 3)
        for cam, gt in zip(self.views, self.gts):
            api.render(ctx, self.g, cam, self.frame, gt=gt, image=self.image)
            dL, _ = api.l1_loss(ctx, self.image, gt)
            api.render_backward(ctx, self.g, cam, self.frame, dL, grads=grads, g2d_norm=g2d, vis_count=vis)
        gi = (g2d / vis.clamp(min=1)).cpu().numpy()
        order = np.lexsort((np.arange(n), -gi))
        self.cand = np.sort(order[: n // 20]).astype(np.int32)
        self.is_cand = torch.zeros(n, dtype=torch.uint8, device="cuda")
        self.is_cand[torch.from_numpy(self.cand.astype(np.int64)).cuda()] = 1
        self.cand_t = torch.from_numpy(self.cand).cuda()
        self.dm = self.frame.device_maps()

    def step(self, params, V, reps=3):
        ctx, W, H = self.ctx, self.W, self.H
        nc = len(self.cand)
        noise = torch.from_numpy(synth.vanilla_noise(nc, 5)).cuda()
        regions = api.RegionBuffer(V * W * H // max(params.m_min, 1) // 4 + 1024)
        attr = torch.zeros(self.n, dtype=torch.int32, device="cuda")
        out = api.Gaussians.empty(self.n + nc * max(2, params.n_max + 1), 3)
        ctx.reserve(max_pixels=W * H, max_gaussians=self.n, max_candidates=nc, max_regions=regions.capacity,
                    max_views=V)

        def once():
            regions.count.zero_()
            attr.zero_()
            for v in range(V):
                api.render(ctx, self.g, self.views[v], self.frame, gt=self.gts[v], image=self.image)
                api.accumulate_error_stats(ctx, W, H, self.dm["err"], self.dm["err_minmax"], self.dm["dom"],
                                           self.gts[v], v, self.is_cand, params, regions, attr)
            return api.adaptive_split(ctx, self.g, self.cand_t, regions, self.views[:V], attr, params, noise, out=out)

        once()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            r = once()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / reps
        mode = r[1].cpu().numpy()
        res = dict(ms=round(ms, 3), regions=int(regions.count.item()), new_rows=int(r[2].sum().item()),
                   n_out=int(r[4].item()), adaptive=int((mode == 2).sum()), vanilla=int((mode == 0).sum()),
                   reset=int((mode == 1).sum()))
        del regions, attr, out, r
        return res


def run(ctx, out_md=None, log=print):
    wl = DensifyWorkload(ctx)
    torch.cuda.synchronize()
    free0, total = torch.cuda.mem_get_info()
    rows = []
    for knob, values in GRID.items():
        for val in values:
            s = dict(DEFAULTS)
            s[knob] = val
            p = api.SplitParams(r_erode=s["r_erode"], L=s["L"], n_max=s["n_max"], m_min=s["m_min"])
            r = wl.step(p, s["V"])
            torch.cuda.synchronize()
            free, _ = torch.cuda.mem_get_info()
            r["mem_gib"] = round((free0 - free) / 2 ** 30, 3)
            r.update(knob=knob, value=val)
            rows.append(r)
            log(json.dumps(r))
    if out_md:
        write_md(out_md, rows, wl)
    return rows


def write_md(path, rows, wl):
    lines = ["# Knob sweep of one AdpSplit densification step", "",
             "Command (repository root, on the GPU host): "
             "`python -m paper_2605_06876_amd.sweep --out profiles/knob_sweep_densify.md`", "",
             "Workload: %d clustered Gaussians (SH 3), 16 views of %dx%d on a radius-4 sphere, smooth synthetic "
             "targets, %d split candidates (top 5%% by view-averaged screen-space gradient).  One knob varies from "
             "the defaults (r_erode 2, L 3, N_max 19, m_min 5, V 16).  Time = error statistics of V views (renders "
             "included) + the split, mean of 3.  Memory = device memory in use after the step relative to the start "
             "(the library's scratch only grows, so it tracks the peak)." % (wl.n, wl.W, wl.H, len(wl.cand)), "",
             "| Knob | Value | Step (ms) | Regions | New rows | Adaptive / vanilla / reset | Gaussians after | "
             "Memory (GiB) |", "|---|---:|---:|---:|---:|---|---:|---:|"]
    for r in rows:
        lines.append("| %s | %s | %.2f | %d | %d | %d / %d / %d | %d | %.3f |" % (
            r["knob"], r["value"], r["ms"], r["regions"], r["new_rows"], r["adaptive"], r["vanilla"], r["reset"],
            r["n_out"], r["mem_gib"]))
    open(path, "w").write("\n".join(lines) + "\n")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default="")
    args = ap.parse_args()
    ctx = api.Context(0)
    run(ctx, args.out or None, log=lambda m: print(m, flush=True))


if __name__ == "__main__":
    main()
