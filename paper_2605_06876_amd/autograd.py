"""torch.autograd wrapper of as_render / as_render_backward.

The forward keeps no per-Gaussian intermediates in torch: the frame holds the
per-pixel final transmittance and last-contributor index, and the backward
recomputes the blend per tile from them (the reverse pass of Eq. (rendering)).
A frame serves one forward/backward pair at a time: render into it again only
after the backward of the previous render has run.
"""
import torch

from . import api


class RenderFunction(torch.autograd.Function):
    @staticmethod
    def forward(fctx, means, log_scales, quats, opacity_logits, sh, state):
        ctx, frame, cam, gt, sh_degree, stats = state
        g = api.Gaussians(means.contiguous(), log_scales.contiguous(), quats.contiguous(),
                          opacity_logits.contiguous(), sh.contiguous(), sh_degree)
        image = api.render(ctx, g, cam, frame, gt=gt)
        fctx.state = state
        fctx.g = g
        return image

    @staticmethod
    def backward(fctx, dL_dimage):
        ctx, frame, cam, gt, sh_degree, stats = fctx.state
        g2d, vis = (stats if stats is not None else (None, None))
        grads = api.render_backward(ctx, fctx.g, cam, frame, dL_dimage.contiguous(), g2d_norm=g2d, vis_count=vis)
        return grads.means, grads.log_scales, grads.quats, grads.opacity_logits, grads.sh, None


class Rasterizer:
    """Differentiable renderer of one view size.

    >>> r = Rasterizer(n_cap, width, height)
    >>> img = r(means, log_scales, quats, opacity_logits, sh, sh_degree, cam)
    >>> loss = (img - target).abs().mean(); loss.backward()

    When ``track_stats`` is set, every backward adds |dL/d mean2d| and a
    visibility count per Gaussian (the ADC statistic) into ``g2d_norm`` and
    ``vis_count``."""

    def __init__(self, n_cap, width, height, device=0, track_stats=False):
        self.ctx = api.Context(device)
        self.frame = api.Frame(self.ctx, n_cap, width, height)
        self.n_cap = n_cap
        self.g2d_norm = torch.zeros(n_cap, dtype=torch.float32, device="cuda") if track_stats else None
        self.vis_count = torch.zeros(n_cap, dtype=torch.int32, device="cuda") if track_stats else None

    def __call__(self, means, log_scales, quats, opacity_logits, sh, sh_degree, cam, gt=None):
        n = means.shape[1]
        stats = None
        if self.g2d_norm is not None:
            if n > self.n_cap:
                raise ValueError("more Gaussians than the rasterizer was made for")
            stats = (self.g2d_norm[:n], self.vis_count[:n])
        return RenderFunction.apply(means, log_scales, quats, opacity_logits, sh,
                                    (self.ctx, self.frame, cam, gt, sh_degree, stats))

    def error_maps(self):
        """Device addresses of the last render's error map, its min/max and the dominant map."""
        return self.frame.device_maps()
