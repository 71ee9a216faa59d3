"""CPU FP64 oracle of the optimisation loop around the path.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg use it; the product path never does.  It shares no code with
the HIP path.

Each function is the plain definition, written out with numpy in FP64:
  adam_step       Adam with bias correction (Kingma and Ba, Alg. 1), one
                  learning rate per parameter group as in 3DGS
  l1_loss         mean absolute error of an image and its gradient
                  sign(d) / (3 H W), plus the sums behind the PSNR
  densify_select  3DGS's adaptive density control (Sec. 3): view-averaged
                  screen-space gradient against a threshold, clone when the
                  largest scale is small, split candidate otherwise
  split_row_map   which input row each row of the split's output copies
  clone_prune     keep = opacity and size tests, kept rows then their clones
  gather_rows     row gather with zero rows for -1
  reset_opacity   opacity <- min(opacity, cap) with the opacity moments zeroed

Parity status (tests/test_oracle_train.py): adam_step pinned against
torch.optim.Adam in FP64 (an independent implementation) and the first-step
closed form; the others pinned by hand-built cases with known answers and by
the split oracle's own output layout (split_row_map).

A Gaussian set is a dict with "means" [3,n], "log_scales" [3,n], "quats"
[4,n], "opacity_logits" [n], "sh" [(d+1)^2,3,n].
"""
import numpy as np

FIELDS = ("means", "log_scales", "quats", "opacity_logits", "sh")


def _as64(g):
    return {k: np.asarray(g[k], np.float64) for k in FIELDS}


def adam_step(params, grads, m, v, hp, step):
    """One bias-corrected Adam step; returns (params, m, v) in FP64.

    hp: dict with lr_means, lr_log_scales, lr_quats, lr_opacity, lr_sh_dc,
    lr_sh_rest, beta1, beta2, eps.  SH coefficient 0 takes lr_sh_dc."""
    p, g, mm, vv = _as64(params), _as64(grads), _as64(m), _as64(v)
    b1, b2, eps = float(hp["beta1"]), float(hp["beta2"]), float(hp["eps"])
    bc1 = 1.0 - b1 ** step
    bc2 = 1.0 - b2 ** step
    lr = {"means": hp["lr_means"], "log_scales": hp["lr_log_scales"], "quats": hp["lr_quats"],
          "opacity_logits": hp["lr_opacity"]}
    out_p, out_m, out_v = {}, {}, {}
    for k in FIELDS:
        mk = b1 * mm[k] + (1.0 - b1) * g[k]
        vk = b2 * vv[k] + (1.0 - b2) * g[k] * g[k]
        if k == "sh":
            rate = np.full(p[k].shape, float(hp["lr_sh_rest"]))
            rate[0] = float(hp["lr_sh_dc"])
        else:
            rate = float(lr[k])
        out_p[k] = p[k] - rate * (mk / bc1) / (np.sqrt(vk / bc2) + eps)
        out_m[k], out_v[k] = mk, vk
    return out_p, out_m, out_v


def l1_loss(image, gt):
    """(dL/dimage, (sum |d|, sum d^2)) with d = image - gt over [3,H,W]."""
    d = np.asarray(image, np.float64) - np.asarray(gt, np.float64)
    n3 = d.size
    return np.sign(d) / n3, (float(np.abs(d).sum()), float((d * d).sum()))


def densify_select(g, g2d_accum, vis_count, grad_threshold, size_threshold):
    """(clone mask, candidate mask, candidate ids ascending)."""
    a = np.asarray(g2d_accum, np.float64) / np.maximum(np.asarray(vis_count, np.int64), 1)
    selected = a >= grad_threshold
    largest = np.exp(np.asarray(g["log_scales"], np.float64).max(axis=0))
    big = largest > size_threshold
    clone = selected & ~big
    cand = selected & big
    return clone, cand, np.nonzero(cand)[0].astype(np.int32)


def split_row_map(n, cand, mode, capacity, state_in=None):
    """row_src [capacity]: the surviving input rows in order (through
    state_in when given), -1 after them.  A candidate's parent survives only
    when its mode is RESET (1)."""
    removed = np.zeros(n, bool)
    for c, md in zip(np.asarray(cand), np.asarray(mode)):
        if int(md) != 1:
            removed[int(c)] = True
    surv = np.nonzero(~removed)[0]
    out = np.full(capacity, -1, np.int64)
    out[: len(surv)] = surv if state_in is None else np.asarray(state_in, np.int64)[surv]
    return out


def clone_prune(g, clone_mask, state_in, min_opacity, max_scale):
    """(out set, state_src): kept rows in order, then the clones of kept rows
    in order; state_src is state_in[i] (or i) for kept rows, -1 for clones."""
    n = g["opacity_logits"].shape[0]
    o = 1.0 / (1.0 + np.exp(-np.asarray(g["opacity_logits"], np.float64)))
    keep = o >= min_opacity
    if max_scale > 0:
        keep &= np.exp(np.asarray(g["log_scales"], np.float64).max(axis=0)) <= max_scale
    dup = keep & (np.zeros(n, bool) if clone_mask is None else np.asarray(clone_mask, bool))
    rows = np.concatenate([np.nonzero(keep)[0], np.nonzero(dup)[0]])
    out = {k: np.asarray(g[k])[..., rows] for k in FIELDS}
    base = np.arange(n) if state_in is None else np.asarray(state_in, np.int64)
    state = np.concatenate([base[keep], np.full(int(dup.sum()), -1, np.int64)])
    return out, state


def gather_rows(src, row_map):
    """dst row r = src row map[r], zeros where map[r] = -1."""
    row_map = np.asarray(row_map, np.int64)
    out = {}
    for k in FIELDS:
        a = np.asarray(src[k], np.float64)
        r = np.zeros(a.shape[:-1] + (len(row_map),))
        ok = row_map >= 0
        r[..., ok] = a[..., row_map[ok]]
        out[k] = r
    return out


def reset_opacity(opacity_logits, max_opacity):
    """opacity <- min(opacity, max_opacity), in logit space."""
    cap = np.log(max_opacity / (1.0 - max_opacity))
    return np.minimum(np.asarray(opacity_logits, np.float64), cap)
