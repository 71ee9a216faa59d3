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
and the step's own peak device memory.  Each setting runs on a fresh context
with its own frame, region buffer and outputs, after torch's cache is
emptied, so no setting inherits another's allocations: the peak is the
library's memory for the setting (context reservation + frame, from the
library's size queries, which walk the same tables as its allocations) plus
the peak of the step's tensors (regions, attribution counts, noise, split
outputs; torch's peak counter, reset per setting).  The scene, views and
targets the settings share are reported once.  (hipMemGetInfo across the
creation is also recorded; the runtime reuses memory freed by the previous
setting's context, so it can read below the allocation.)

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
        """The step for one setting on a fresh context; returns its figures."""
        W, H, n = self.W, self.H, self.n
        nc = len(self.cand)
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        torch.cuda.reset_peak_memory_stats()
        alloc0 = torch.cuda.memory_allocated()
        free0 = torch.cuda.mem_get_info()[0]
        cap = V * W * H // max(params.m_min, 1) // 4 + 1024
        reserve = dict(max_pixels=W * H, max_gaussians=n, max_candidates=nc, max_regions=cap, max_views=V)
        ctx = api.Context(0, **reserve)
        frame = api.Frame(ctx, n, W, H, key_cap=16 * n, auto_grow=False, forward_only=True)
        torch.cuda.synchronize()
        lib_bytes = free0 - torch.cuda.mem_get_info()[0]
        lib_query = api.reserve_bytes(**reserve) + api.frame_bytes(1, n, W * H, ((W + 15) // 16) * ((H + 15) // 16),
                                                                   16 * n, forward_only=True)
        dm = frame.device_maps()
        image = torch.empty(3, H, W, dtype=torch.float32, device="cuda")
        noise = torch.from_numpy(synth.vanilla_noise(nc, 5)).cuda()
        regions = api.RegionBuffer(cap)
        attr = torch.zeros(n, dtype=torch.int32, device="cuda")
        out = api.Gaussians.empty(n + nc * api.split_rows_per_candidate(params), 3)

        def once():
            regions.count.zero_()
            attr.zero_()
            for v in range(V):
                api.render(ctx, self.g, self.views[v], frame, gt=self.gts[v], image=image)
                api.accumulate_error_stats(ctx, W, H, dm["err"], dm["err_minmax"], dm["dom"], self.gts[v], v,
                                           self.is_cand, params, regions, attr)
            return api.adaptive_split(ctx, self.g, self.cand_t, regions, self.views[:V], attr, params, noise,
                                      out=out)

        once()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            r = once()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / reps
        n_reg = int(regions.count.item())
        assert n_reg <= cap, "region buffer too small for this setting"
        mode = r[1].cpu().numpy()
        tensors_peak = torch.cuda.max_memory_allocated() - alloc0
        res = dict(ms=round(ms, 3), regions=n_reg, new_rows=int(r[2].sum().item()), n_out=int(r[4].item()),
                   adaptive=int((mode == 2).sum()), vanilla=int((mode == 0).sum()), reset=int((mode == 1).sum()),
                   lib_gib=round(lib_bytes / 2 ** 30, 3), lib_query_gib=round(lib_query / 2 ** 30, 3),
                   tensors_gib=round(tensors_peak / 2 ** 30, 3),
                   peak_gib=round((lib_query + tensors_peak) / 2 ** 30, 3))
        del regions, attr, out, r, noise, image, dm
        frame.close()
        ctx.close()
        return res

    def base_gib(self):
        """Device memory of what every setting shares: scene, targets, candidates."""
        b = sum(t.numel() * t.element_size() for t in self.g.tensors())
        b += sum(t.numel() * t.element_size() for t in self.gts)
        b += self.is_cand.numel() + self.cand_t.numel() * 4
        return round(b / 2 ** 30, 3)


def run(ctx, out_md=None, log=print):
    wl = DensifyWorkload(ctx)
    wl.frame.close()
    rows = []
    for knob, values in GRID.items():
        for val in values:
            s = dict(DEFAULTS)
            s[knob] = val
            p = api.SplitParams(r_erode=s["r_erode"], L=s["L"], n_max=s["n_max"], m_min=s["m_min"])
            r = wl.step(p, s["V"])
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
             "included) + the split, mean of 3.  Each setting runs on a fresh context after torch's cache is "
             "emptied.  Library = context reservation + frame, from the library's size queries "
             "(as_ctx_reserve_bytes + as_frame_bytes); tensors = peak of the step's own tensors (region buffer "
             "sized V W H / (4 m_min) + 1024 records, attribution counts, noise, split outputs; torch's peak "
             "counter); peak = their sum.  Shared by every setting and not included: scene, targets and "
             "candidates, %.3f GiB." % (wl.n, wl.W, wl.H, len(wl.cand), wl.base_gib()), "",
             "| Knob | Value | Step (ms) | Regions | New rows | Adaptive / vanilla / reset | Gaussians after | "
             "Library (GiB) | Tensors (GiB) | Peak (GiB) |", "|---|---:|---:|---:|---:|---|---:|---:|---:|---:|"]
    for r in rows:
        lines.append("| %s | %s | %.2f | %d | %d | %d / %d / %d | %d | %.3f | %.3f | %.3f |" % (
            r["knob"], r["value"], r["ms"], r["regions"], r["new_rows"], r["adaptive"], r["vanilla"], r["reset"],
            r["n_out"], r["lib_query_gib"], r["tensors_gib"], r["peak_gib"]))
    open(path, "w").write("\n".join(lines) + "\n")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default="")
    args = ap.parse_args()
    ctx = api.Context(0)
    run(ctx, args.out or None, log=lambda m: print(m, flush=True))


if __name__ == "__main__":
    main()
