"""One step of adaptive density control with every count on the device.

3DGS's density control (Sec. 3) clones small and splits large Gaussians whose
view-averaged screen-space gradient is high and prunes transparent ones;
AdpSplit (Sec. 4, Sec. 5 "Implementation") replaces the split and keeps the
rest.  This module runs one such step as a fixed sequence of library calls on
one stream:

  select -> [AdpSplit: render the sampled views, error statistics] -> clone
  -> adaptive (or fixed-N) split -> row map -> prune -> gather the optimiser
  moments,

where every intermediate count (candidates, rows after the clone, after the
split, after the prune) stays in device memory and every buffer is sized for
the worst case up front.  Nothing in the step reads a count back, so the
sequence can be recorded once as a HIP graph and replayed (`capture`,
`launch`), or run eagerly (`run`); both give the same rows bit for bit.  The
caller reads the final row count after the step.

The error statistics are gathered from renders of the set as it stands when
the step starts, before this step's clones are appended: the split candidates
and their ids are those of that set, and clones (appended after it) are never
candidates.  Buffers are capacity-sized: 2n rows after the clone, then the
split's bound 2n + c (N_max + 1) rows, for n input rows and a candidate
capacity c (n unless the caller bounds it: candidates past it, in id order,
are left unsplit).
"""
import torch

from . import api


class DensifyStep:
    """Buffers and the call sequence of a densification of up to n rows (the
    buffers are kept for later steps on sets of at most n rows).

    ctx      : context (reserved here for the step's sizes)
    n, deg   : largest input row count and the SH degree
    method   : "adpsplit" or "vanilla" (3DGS's random split)
    params   : api.SplitParams of the split (a fixed-N variant for "vanilla";
               None gives the defaults: AdpSplit's, or N = 2)
    views    : cameras of the sampled views (AdpSplit), gts their targets
    regions  : api.RegionBuffer for the sampled views' regions
    cand_cap : candidates the split takes at most (default n)
    key_cap_per_entry : pair capacity of the renders per (view, Gaussian); a
               render over it drops the deepest pairs, so it is generous
    """

    def __init__(self, ctx, n, deg, method="adpsplit", params=None, views=(), gts=(), regions=None, cand_cap=None,
                 key_cap_per_entry=32):
        assert method in ("adpsplit", "vanilla")
        self.ctx, self.n, self.deg, self.method = ctx, n, deg, method
        if method == "adpsplit":
            self.params = params if params is not None else api.SplitParams()
            self.views, self.gts = list(views), list(gts)
            assert self.views and regions is not None
        else:   # 3DGS's random split (N = 2 unless the params say otherwise)
            self.params = params if params is not None else api.SplitParams(variant=api.VARIANT_FIXED_N, fixed_n=2)
            assert self.params.variant == api.VARIANT_FIXED_N
            self.views, self.gts = [], []
        # the fixed-N split reads no region: an empty one-record buffer
        self.regions = regions if regions is not None else api.RegionBuffer(1)
        p = self.params
        per = api.split_rows_per_candidate(p)
        self.noise_n = max(2, p.n_max if p.variant == api.VARIANT_ADAPTIVE_N else 0,
                           p.fixed_n if p.variant == api.VARIANT_FIXED_N else 0)
        if p.noise_n < self.noise_n:   # the noise input holds noise_n normals per candidate
            self.params = p = api.SplitParams(p.tau_l1, p.r_erode, p.m_min, p.L, p.n_max, p.gamma_d, p.gamma_c, p.eps,
                                              p.eta, p.variant, p.flags, p.fixed_n, self.noise_n)
        self.cc = n if cand_cap is None else max(1, min(int(cand_cap), n))
        self.cap1 = 2 * n
        self.cap2 = self.cap1 + self.cc * per
        dev = dict(device="cuda")
        self.sel = (torch.zeros(max(n, 1), dtype=torch.uint8, **dev), torch.zeros(max(n, 1), dtype=torch.uint8, **dev),
                    torch.zeros(max(n, 1), dtype=torch.int32, **dev), torch.zeros(1, dtype=torch.int64, **dev))
        self.attr = torch.zeros(max(self.cap1, 1), dtype=torch.int32, **dev)
        self.noise = torch.zeros(self.cc, self.noise_n, 3, dtype=torch.float32, **dev)
        self.g1 = api.Gaussians.empty(max(self.cap1, 1), deg)
        self.st1 = torch.empty(max(self.cap1, 1), dtype=torch.int32, **dev)
        self.n1 = torch.zeros(1, dtype=torch.int64, **dev)
        self.g2 = api.Gaussians.empty(max(self.cap2, 1), deg)
        self.mode = torch.zeros(self.cc, dtype=torch.uint8, **dev)
        self.count = torch.zeros(self.cc, dtype=torch.int32, **dev)
        self.offset = torch.zeros(self.cc, dtype=torch.int64, **dev)
        self.n2 = torch.zeros(1, dtype=torch.int64, **dev)
        self.st2 = torch.empty(max(self.cap2, 1), dtype=torch.int32, **dev)
        self.out = api.Gaussians.empty(max(self.cap2, 1), deg)
        self.st3 = torch.empty(max(self.cap2, 1), dtype=torch.int32, **dev)
        self.n_out = torch.zeros(1, dtype=torch.int64, **dev)
        self.m_out = api.Gaussians.empty(max(self.cap2, 1), deg)
        self.v_out = api.Gaussians.empty(max(self.cap2, 1), deg)
        self.frame = None
        if method != "adpsplit":   # the split's camera table needs one entry; no region refers to it
            from . import synth
            self._cam0 = synth.look_at((0.0, 0.0, -4.0), (0.0, 0.0, 0.0), 16, 16, 60.0)
        if method == "adpsplit":
            W, H = self.views[0].width, self.views[0].height
            k = min(len(self.views), api.MAX_VIEWS)
            self.frame = api.BatchFrame.for_views(ctx, n, self.views[:k], key_cap=key_cap_per_entry * n * k,
                                                  auto_grow=False, forward_only=True)
            self.images = [torch.empty(3, H, W, dtype=torch.float32, **dev) for _ in range(k)]
        # set-up: the context scratch of every call of the step (none allocates)
        ctx.reserve(max_gaussians=max(self.cap2, 1), max_candidates=self.cc,
                    max_pixels=max([v.width * v.height for v in self.views] + [1]),
                    max_regions=self.regions.capacity, max_views=max(len(self.views), 1))

    def set_views(self, views, gts):
        """Other sampled views (as many as at construction, the same size)."""
        assert self.method == "adpsplit" and len(views) == len(self.views) and len(gts) == len(views)
        self.views, self.gts = list(views), list(gts)

    def run(self, g, m, v, accum, vis, grad_threshold, size_threshold, min_opacity, max_scale):
        """Enqueue the step on the current stream (inputs: g, m, v with n' <= n
        rows, accum, vis [n']); the result is out, m_out, v_out with n_out rows."""
        ctx = self.ctx
        n = g.n
        assert n <= self.n
        sel = tuple(t[:n] for t in self.sel[:3]) + (self.sel[3],)
        clone, is_cand, cand, n_cand = api.densify_select(ctx, g, accum, vis, grad_threshold, size_threshold,
                                                          out=sel)
        self.attr.zero_()
        if self.method == "adpsplit":
            self.regions.count.zero_()
            W, H = self.views[0].width, self.views[0].height
            for c0 in range(0, len(self.views), api.MAX_VIEWS):
                views = self.views[c0:c0 + api.MAX_VIEWS]
                gts = self.gts[c0:c0 + api.MAX_VIEWS]
                api.render_batch(ctx, g, views, self.frame, gts=gts, images=self.images[:len(views)])
                for j in range(len(views)):
                    mp = self.frame.device_maps(j)
                    api.accumulate_error_stats(ctx, W, H, mp["err"], mp["err_minmax"], mp["dom"], gts[j], c0 + j,
                                               is_cand, self.params, self.regions, self.attr[:n])
        # 1. clones appended after the originals: candidate ids stay valid
        api.clone_prune(ctx, g, clone, None, 0.0, 0.0, out=self.g1, state_src=self.st1, n_out=self.n1)
        # 2. the split of the candidates, on the clone output's rows in use
        g1 = self.g1.counted(self.n1)
        cand = self.sel[2][:self.cc]
        api.adaptive_split(ctx, g1, cand, self.regions, self.views if self.views else [self._cam0], self.attr,
                           self.params, self.noise,
                           out=self.g2, mode=self.mode, count=self.count, offset=self.offset, n_out=self.n2,
                           n_cand_dev=n_cand)
        api.split_row_map(ctx, self.cap1, cand, self.mode, self.cap2, state_in=self.st1, n_dev=self.n1,
                          n_cand_dev=n_cand, row_src=self.st2)
        # 3. prune
        api.clone_prune(ctx, self.g2.counted(self.n2), None, self.st2, min_opacity, max_scale, out=self.out,
                        state_src=self.st3, n_out=self.n_out)
        # 4. the Adam moments follow their rows; new rows start from zero
        api.gather_rows(ctx, m, self.st3, self.cap2, dst=self.m_out, n_rows_dev=self.n_out)
        api.gather_rows(ctx, v, self.st3, self.cap2, dst=self.v_out, n_rows_dev=self.n_out)

    def capture(self, stream, *args, **kw):
        """Record run(*args) on `stream` as a HIP graph (api.Graph)."""
        return api.Graph.capture(self.ctx, lambda: self.run(*args, **kw), stream)

    def result(self):
        """(Gaussians, m, v, row map) of the rows in use (reads the row count)."""
        k = int(self.n_out.item())
        return self.out.rows(k), self.m_out.rows(k), self.v_out.rows(k), self.st3[:k].clone()

    def close(self):
        if self.frame is not None:
            self.frame.close()
            self.frame = None
