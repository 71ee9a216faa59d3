"""Synthetic end-to-end densification training: 3DGS's optimisation loop with
adaptive density control (Sec. 3), where the split of large high-gradient
Gaussians is either AdpSplit (Sec. 4, the method) or the vanilla fixed-N = 2
random split it replaces (Eq. (vanilla_split_sample)).

A teacher scene (synthetic clustered Gaussians) is rendered from training and
held-out cameras with the library; a student initialised from a sparse noisy
subsample of the teacher's centres is trained against the training renders.
Every step runs in the library's kernels: render, L1 loss and gradient,
reverse pass, Adam, and at each densification interval selection, clone,
split (for AdpSplit: V renders with error statistics, then the adaptive
split), prune and the carry-over of the Adam moments through the row maps.
Host code only orders the calls, reads back counts and allocates.

The schedule is 3DGS's, shortened (defaults below): densify every 100
iterations inside a window, opacity reset inside the window, the learning
rate of the means decayed log-linearly, the gradient threshold 2e-4 of 3DGS
(stated for NDC coordinates) converted to pixel units.  Differences from the
reference loop, all stated in the design notes: L1 loss only (no D-SSIM), the
full SH degree from the start, no screen-space size prune.
"""
import math
import time

import numpy as np
import torch

from . import api, densify, synth


class TrainConfig:
    def __init__(self, method="adpsplit", iters=3000, densify_from=300, densify_until=2100, densify_every=100,
                 opacity_reset_every=1200, grad_threshold_ndc=2e-4, percent_dense=0.01, min_opacity=0.005,
                 max_world_scale=0.1, views_per_split=20, split_params=None, eval_every=250, max_gaussians=2_000_000,
                 lr_means_final=0.01, seed=0, vanilla_n=2):
        assert method in ("adpsplit", "vanilla")
        self.vanilla_n = vanilla_n   # children of the random split (3DGS: 2; Fig. 2's pilot: 5)
        self.method, self.iters = method, iters
        self.densify_from, self.densify_until, self.densify_every = densify_from, densify_until, densify_every
        self.opacity_reset_every, self.grad_threshold_ndc = opacity_reset_every, grad_threshold_ndc
        self.percent_dense, self.min_opacity, self.max_world_scale = percent_dense, min_opacity, max_world_scale
        self.views_per_split = views_per_split
        self.split_params = split_params if split_params is not None else api.SplitParams()
        self.eval_every, self.max_gaussians, self.lr_means_final, self.seed = eval_every, max_gaussians, lr_means_final, seed


class Problem:
    """Teacher, cameras and target images (rendered once with the library)."""

    def __init__(self, ctx, n_teacher=100_000, n_train=48, n_eval=8, size=(480, 360), radius=3.0, seed=7,
                 sh_degree=3):
        self.ctx, self.W, self.H, self.sh_degree = ctx, size[0], size[1], sh_degree
        self.teacher = synth.scene_clusters(n_teacher, seed, sh_degree, log_scale_mu=-4.0, log_scale_sd=0.6)
        self.train_cams = synth.sphere_cameras(n_train, radius, [size], seed=seed)
        self.eval_cams = synth.sphere_cameras(n_eval, radius * 1.05, [size], seed=seed + 1000)
        # 3DGS's scene extent: 1.1 times the largest camera distance from the cameras' centre
        centres = np.stack([-np.asarray(c.R, np.float64).T @ np.asarray(c.t, np.float64) for c in self.train_cams])
        self.extent = 1.1 * float(np.linalg.norm(centres - centres.mean(0), axis=1).max())
        g = api.Gaussians.from_scene(self.teacher)
        frame = api.Frame(ctx, g.n, self.W, self.H, key_cap=32 * g.n)
        self.train_gt = [api.render(ctx, g, c, frame).clone() for c in self.train_cams]
        self.eval_gt = [api.render(ctx, g, c, frame).clone() for c in self.eval_cams]
        torch.cuda.synchronize()
        frame.close()


def init_student(teacher, n0, seed, noise=0.01):
    """3DGS-style initialisation from a sparse point cloud: a random subset of
    the teacher's centres with positional noise, colours from the teacher's DC
    term, isotropic scales from the mean squared distance to the three nearest
    neighbours, identity rotations, opacity 0.1, higher SH zero."""
    from scipy.spatial import cKDTree
    rng = np.random.default_rng(seed)
    idx = np.sort(rng.choice(teacher.n, n0, replace=False))
    pts = teacher.means[:, idx].T.astype(np.float64) + rng.normal(0, noise, (n0, 3))
    d, _ = cKDTree(pts).query(pts, k=4)
    d2 = np.maximum((d[:, 1:] ** 2).mean(1), 1e-7)
    nk = (teacher.sh_degree + 1) ** 2
    sh = np.zeros((nk, 3, n0), np.float32)
    sh[0] = teacher.sh[0][:, idx] + rng.normal(0, 0.05, (3, n0))
    f = np.float32
    return synth.Scene(pts.T.astype(f), np.repeat(np.log(np.sqrt(d2))[None], 3, 0).astype(f),
                       np.tile(np.array([[1], [0], [0], [0]], f), (1, n0)),
                       np.full(n0, math.log(0.1 / 0.9), f), sh, teacher.sh_degree)


class Trainer:
    def __init__(self, ctx, problem, cfg, n_init=10_000):
        self.ctx, self.pb, self.cfg = ctx, problem, cfg
        self.rng = np.random.default_rng(cfg.seed)
        self.g = api.Gaussians.from_scene(init_student(problem.teacher, n_init, cfg.seed))
        self.deg = self.g.sh_degree
        self.hp = api.AdamParams()
        W, H = problem.W, problem.H
        # 3DGS's threshold is on the NDC-space gradient, d/d(ndc) = (W/2, H/2) d/d(pixel)
        self.thr = cfg.grad_threshold_ndc / (0.25 * (W + H))
        self.image = torch.empty(3, H, W, dtype=torch.float32, device="cuda")
        self.frame = None
        self._reset_state(self.g.n, fresh_moments=True)
        self.regions = api.RegionBuffer(cfg.views_per_split * W * H // cfg.split_params.m_min // 4 + 1024)
        self.history, self.densify_ms, self.split_counts = [], [], []
        self.dstep = None
        self.train_s, self.reset_done = 0.0, False

    def _reset_state(self, n, fresh_moments=False):
        if fresh_moments:
            self.m = api.Gaussians.empty(n, self.deg)
            self.v = api.Gaussians.empty(n, self.deg)
        self.grads = api.Gaussians.empty(n, self.deg)
        self.accum = torch.zeros(n, dtype=torch.float32, device="cuda")
        self.vis = torch.zeros(n, dtype=torch.int32, device="cuda")
        self._ensure_frame(n)

    def _ensure_frame(self, n):
        if self.frame is None or self.frame.n_cap < n:
            if self.frame is not None:
                self.frame.close()
            self.frame = api.Frame(self.ctx, max(2 * n, 1), self.pb.W, self.pb.H, key_cap=32 * max(2 * n, 1))
            self.dm = self.frame.device_maps()

    def lr_means(self, it):
        t = min(max(it / self.cfg.iters, 0.0), 1.0)
        a = 1.6e-4 * self.pb.extent
        return math.exp(math.log(a) * (1 - t) + math.log(a * self.cfg.lr_means_final) * t)

    def step(self, it):
        pb, ctx = self.pb, self.ctx
        k = int(self.rng.integers(len(pb.train_cams)))
        api.render(ctx, self.g, pb.train_cams[k], self.frame, image=self.image)
        dL, _ = api.l1_loss(ctx, self.image, pb.train_gt[k])
        api.render_backward(ctx, self.g, pb.train_cams[k], self.frame, dL, grads=self.grads, g2d_norm=self.accum,
                            vis_count=self.vis)
        self.hp.lr_means = self.lr_means(it)
        api.adam_step(ctx, self.g, self.grads, self.m, self.v, self.hp, it)

    def densify(self, it):
        """One density-control step (densify.DensifyStep: every count stays on
        the device until the step ends), then the new set's row count is read."""
        cfg, pb, ctx = self.cfg, self.pb, self.ctx
        g, n = self.g, self.g.n
        step = self.dstep
        if step is None or step.n < n:   # buffers for twice the rows, kept for later steps
            if step is not None:
                step.close()
            if cfg.method == "adpsplit":
                k = min(cfg.views_per_split, len(pb.train_cams))
                step = densify.DensifyStep(ctx, 2 * n, self.deg, "adpsplit", cfg.split_params, pb.train_cams[:k],
                                           pb.train_gt[:k], self.regions)
            else:
                step = densify.DensifyStep(ctx, 2 * n, self.deg, "vanilla",
                                           api.SplitParams(variant=api.VARIANT_FIXED_N, fixed_n=cfg.vanilla_n))
            self.dstep = step
        if cfg.method == "adpsplit":
            vi = self.rng.choice(len(pb.train_cams), len(step.views), replace=False)
            step.set_views([pb.train_cams[k] for k in vi], [pb.train_gt[k] for k in vi])
        step.noise.copy_(torch.from_numpy(synth.vanilla_noise(step.cc, int(self.rng.integers(1 << 30)),
                                                              step.noise_n)).view_as(step.noise))
        # the world-size prune from the first opacity reset on
        max_scale = cfg.max_world_scale * pb.extent if self.reset_done else 0.0
        step.run(g, self.m, self.v, self.accum, self.vis, self.thr, cfg.percent_dense * pb.extent, cfg.min_opacity,
                 max_scale)
        self.g, self.m, self.v, self.last_state_map = step.result()
        n_cand, n_after = int(step.sel[3].item()), self.g.n
        clones = int(step.sel[0][:n].sum().item())
        self.split_counts.append(int(step.count[:n_cand].sum().item()) if n_cand else 0)
        self._reset_state(n_after)
        return dict(it=it, n_before=n, clones=clones, candidates=n_cand, n_after=n_after)

    def evaluate(self):
        pb, ctx = self.pb, self.ctx
        psnr = []
        for cam, gt in zip(pb.eval_cams, pb.eval_gt):
            api.render(ctx, self.g, cam, self.frame, image=self.image)
            _, sums = api.l1_loss(ctx, self.image, gt, want_grad=False)
            mse = float(sums[1].item()) / (3 * pb.W * pb.H)
            psnr.append(-10.0 * math.log10(max(mse, 1e-12)))
        return float(np.mean(psnr))

    def run(self, log=None):
        cfg = self.cfg
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        self.history.append(dict(it=0, train_s=0.0, psnr=self.evaluate(), n=self.g.n))
        t0 = time.perf_counter()
        for it in range(1, cfg.iters + 1):
            self.step(it)
            if cfg.densify_from <= it <= cfg.densify_until and it % cfg.densify_every == 0 and \
                    self.g.n < cfg.max_gaussians:
                td = time.perf_counter()
                info = self.densify(it)
                torch.cuda.synchronize()
                self.densify_ms.append((time.perf_counter() - td) * 1e3)
                if log:
                    log("  it %d: %s" % (it, info))
            if it % cfg.opacity_reset_every == 0 and it < cfg.densify_until:
                api.reset_opacity(self.ctx, self.g, 0.01, self.m.opacity_logits, self.v.opacity_logits)
                self.reset_done = True
            if it % cfg.eval_every == 0 or it == cfg.iters:
                torch.cuda.synchronize()
                self.train_s += time.perf_counter() - t0
                self.history.append(dict(it=it, train_s=round(self.train_s, 4), psnr=round(self.evaluate(), 4),
                                         n=self.g.n))
                torch.cuda.synchronize()
                t0 = time.perf_counter()
        return dict(method=cfg.method, final_psnr=self.history[-1]["psnr"], final_n=self.g.n,
                    train_s=round(self.train_s, 4), densify_ms_mean=round(float(np.mean(self.densify_ms)), 3)
                    if self.densify_ms else 0.0, densify_calls=len(self.densify_ms),
                    split_rows=int(sum(self.split_counts)), history=self.history)


def train_one(ctx, pb, cfg, n_init, log=None):
    tr = Trainer(ctx, pb, cfg, n_init=n_init)
    try:
        return tr.run(log=log)
    finally:
        tr.frame.close()
        if tr.dstep is not None:
            tr.dstep.close()


def compare(ctx, problem=None, iters=3000, seed=0, n_init=10_000, log=None, **kw):
    """Vanilla split vs AdpSplit on the same problem and initialisation."""
    pb = problem if problem is not None else Problem(ctx)
    return {m: train_one(ctx, pb, TrainConfig(method=m, iters=iters, seed=seed, **kw), n_init, log)
            for m in ("vanilla", "adpsplit")}


def compare_arms(ctx, pb, iters=3000, densify_until=2100, seed=0, n_init=10_000, full_scale=1.25,
                 full_densify_scale=5.0 / 3.0, match_tries=5, log=None):
    """The arms of Table 1 and Fig. 2 on one problem and initialisation.

    Table 1 trains each baseline with its full schedule, with a shortened
    densification schedule (-S: densification stops at 9k instead of 15k
    iterations, training at 24k instead of 30k) and with AdpSplit on the
    shortened schedule.  Here the shortened schedule is (iters,
    densify_until) and the full one stretches both by the paper's ratios
    (15k/9k for densification, 30k/24k for training).  Arms:
      vanilla_full   3DGS's N = 2 split, full schedule
      vanilla        N = 2 split, shortened schedule (-S)
      vanilla_n5     five random children per split, shortened (Fig. 2's pilot)
      vanilla_equal  N = 2 split, shortened, with the gradient threshold
                     lowered until the final Gaussian count is that of the
                     AdpSplit arm (a control for the count: Fig. 2 shows that
                     more Gaussians alone do not give better reconstructions)
      adpsplit       AdpSplit, shortened schedule."""
    kw = dict(seed=seed)
    short = dict(iters=iters, densify_until=densify_until)
    full = dict(iters=int(round(iters * full_scale)), densify_until=int(round(densify_until * full_densify_scale)))
    out = dict(schedules=dict(short=short, full=full))
    out["vanilla_full"] = train_one(ctx, pb, TrainConfig(method="vanilla", **full, **kw), n_init, log)
    out["vanilla"] = train_one(ctx, pb, TrainConfig(method="vanilla", **short, **kw), n_init, log)
    out["vanilla_n5"] = train_one(ctx, pb, TrainConfig(method="vanilla", vanilla_n=5, **short, **kw), n_init, log)
    out["adpsplit"] = train_one(ctx, pb, TrainConfig(method="adpsplit", **short, **kw), n_init, log)
    # equal count: bisect the threshold's scale in log space towards AdpSplit's final count
    target = out["adpsplit"]["final_n"]
    thr0 = TrainConfig().grad_threshold_ndc
    lo, hi = math.log(0.05), 0.0       # the final count falls as the threshold grows
    best = None
    for _ in range(match_tries):
        mid = 0.5 * (lo + hi)
        r = train_one(ctx, pb, TrainConfig(method="vanilla", grad_threshold_ndc=thr0 * math.exp(mid), **short, **kw),
                      n_init, log)
        r["threshold_scale"] = round(math.exp(mid), 4)
        if best is None or abs(r["final_n"] - target) < abs(best["final_n"] - target):
            best = r
        if r["final_n"] > target:
            lo = mid
        else:
            hi = mid
    out["vanilla_equal"] = best
    return out
