"""Parity with the CPU oracle at the benchmark workloads' full sizes, in the
launch configuration the benchmark times.

C2 (1,000,000 Gaussians, SH 3, 1256x828): every pixel of the forward render
and a dense upstream gradient through the reverse pass.  C3 (500,000
Gaussians, 16 views, top-5% candidates): error statistics and the adaptive
split stage-isolated, on the GPU's own renders.  C4 (1,500,000 Gaussians,
8 views of uneven size, 28,380 tiles in one batched launch): every pixel of
every view, forward and backward.

Exclusions: pixels whose FP64 decision (alpha vs 1/255, T(1 - alpha) vs 1e-4,
the dominant weight's lead, o G vs the 0.99 clamp) lies within the measured
FP32 rounding of its threshold are flagged by the oracle.  The forward skips
them; the reverse pass gets a zero upstream gradient there on both sides, so
they contribute nothing and no Gaussian is excluded.  Gaussians whose
culling or box edge lies within transcendental rounding are flagged too (the
oracle's box_flag) and their boxes are excluded from the exact comparison.

Bars: bit-exact decisions (depth keys, boxes, tiles touched, contributor
counts, dominant and last ids, regions, attribution, modes, counts, offsets,
row order); image max-abs <= 1e-4; final transmittance within the relative
bound the oracle's flags assume; every 2D gradient within 1e-3 (m + rms) of
the oracle's, m the summed magnitude of its products; parameter gradients
per tensor ||d||/||ref|| <= 1e-3 and, stage-isolated (the oracle's chain rule
fed the GPU's 2D gradients), every element within 1e-3 (|ref| + rms)."""
import sys

import numpy as np
import pytest

import oracle
from paper_2605_06876_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2605_06876_amd import api  # noqa: E402

# the benchmark's tuned launch on C2 and C4 (LDS depth 256, longest-first /
# work-ordered dispatch, one block per tile, pairs binned by 32 x 32 squares,
# 6-bit pair digits)
TUNING = dict(lds_batch=256, longest_first=True, persistent=False, radix_bits=6, bin_tile=32)
C4_SIZES = [(640, 480), (800, 600), (960, 640), (1024, 768), (1256, 828), (1280, 720), (1440, 960), (1600, 1064)]
GRAD_FIELDS = ("means", "log_scales", "quats", "opacity_logits", "sh")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def tuned_ctx(**reserve):
    c = api.Context(0, **reserve)
    api.set_tuning(c, **TUNING)
    return c


def grad2d_host(frame, view, n):
    v = frame.view(view)
    return frame._dev(v.grad2d, 36 * n).view(np.float32).reshape(n, 9).astype(np.float64)


def oracle_grad2d(g):
    return np.concatenate([g["mean2d"], g["conic"], g["opacity"][:, None], g["rgb"]], 1)


def check_projection_exact(pr, st, label):
    """Culling, depth keys, boxes and tiles touched bit-exact, apart from the
    Gaussians the oracle flags at transcendental rounding distance."""
    valid = pr.valid.astype(bool)
    bf = pr.box_flag.astype(bool)
    gvalid = st["ntiles"] > 0
    np.testing.assert_array_equal(gvalid[~bf], valid[~bf])
    both = valid & gvalid
    np.testing.assert_array_equal(st["depth_key"][both], pr.depth_key[both])
    ok = both & ~bf
    np.testing.assert_array_equal(st["box"][ok].astype(np.int32), pr.box[ok])
    say("%s: %d visible Gaussians, %d box-flagged" % (label, valid.sum(), bf.sum()))


def check_forward(img, st, r, W, H, label):
    """Every unflagged pixel: image max-abs <= 1e-4, contributor counts,
    dominant and last-contributor ids bit-exact.  Returns the flag map."""
    flag = r["flag"].reshape(H, W).astype(bool)
    ok = ~flag
    ref = r["color"].reshape(H, W, 3).transpose(2, 0, 1)
    err = np.abs(img.astype(np.float64) - ref)[:, ok].max()
    nc_o = r["ncontrib"].reshape(H, W)
    dom_o = r["dom"].reshape(H, W)
    last_o = r["last"].reshape(H, W)
    bad_nc = (st["n_contrib"].astype(np.int64) != nc_o)
    bad_dom = (st["dom"].astype(np.int64) != dom_o)
    has = st["n_contrib"] > 0
    last_g = np.full((H, W), -1, np.int64)
    last_g[has] = st["gauss"][st["last"][has]].astype(np.int64)
    bad_last = last_g != last_o
    say("%s: flagged %d of %d pixels; image max-abs %.2e on the rest; mismatches on flagged pixels: "
        "ncontrib %d, dom %d, last %d" % (label, flag.sum(), W * H, err, (bad_nc & flag).sum(),
                                          (bad_dom & flag).sum(), (bad_last & flag).sum()))
    if "margins" in r:
        m = r["margins"].reshape(H, W, 4)
        bad = bad_nc | bad_dom | bad_last
        if bad.any():
            say("%s: largest margins among mismatched pixels (alpha, T, dom, clamp): %s"
                % (label, np.array2string(np.where(np.isinf(m[bad]), 0, m[bad]).max(0), precision=3)))
    assert err <= 1e-4, err
    assert not (bad_nc & ok).any(), (bad_nc & ok).sum()
    assert not (bad_dom & ok).any(), (bad_dom & ok).sum()
    assert not (bad_last & ok).any(), (bad_last & ok).sum()
    T_o = r["T"].reshape(H, W)
    relT = np.abs(st["t_final"].astype(np.float64) - T_o)[ok] / T_o[ok]
    # within the FP32 error bound of T the oracle's flags assume (plus 1e-6)
    tb = r["t_bound"].reshape(H, W)[ok] + 1e-6
    say("%s: final transmittance max relative error %.3g on unflagged pixels, %.3g of its bound"
        % (label, relT.max(), (relT / tb).max()))
    assert (relT <= tb).all(), (relT > tb).sum()
    return flag


def check_grad2d(g_gpu, g_ref, g_abs, label, tol=1e-3, pr=None):
    """Every 2D gradient of every Gaussian within tol (|ref| + rms(ref)) of
    the oracle's, per quantity, with |ref| taken as the summed magnitude of the
    products that form it (its rounding scale where the products cancel).
    Elements beyond tol of their own magnitude are counted and reported: they
    are gradients formed at pixels deep behind nearly opaque contributors,
    whose FP32 transmittance carries a relative error near 1e-3 (within the
    oracle's bound for it)."""
    d = np.abs(g_gpu - g_ref)
    rms = np.sqrt((g_ref ** 2).mean(axis=0))
    bound = tol * (g_abs + rms)
    worst = np.max(d / np.maximum(g_abs, 1e-300), axis=0)
    say("%s: 2D gradients, largest |diff| / magnitude per quantity: %s; beyond %.0e of their own magnitude: "
        "%d of %d" % (label, " ".join("%.3g" % w for w in worst), tol, (d > tol * g_abs).sum(), d.size))
    bad = d > bound
    if bad.any() and pr is not None:
        for i, k in zip(*np.nonzero(bad)):
            a, b, c = pr.conic[i]
            say("  out of bound: Gaussian %d quantity %d: gpu %.6g oracle %.6g magnitude %.6g; "
                "1/(1 - rho^2) = %.3g, opacity %.3g" % (i, k, g_gpu[i, k], g_ref[i, k], g_abs[i, k],
                                                         a * c / (a * c - b * b), pr.opacity[i]))
    assert not bad.any(), "%d of %d 2D gradient elements out of bound" % (bad.sum(), bad.size)


def check_param_grads(grads, gref, gstage, label, tol=1e-3):
    for name in GRAD_FIELDS:
        a = getattr(grads, name).cpu().numpy().astype(np.float64)
        b = gref[name]
        rel = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)
        c = gstage[name]
        rms = np.sqrt((c ** 2).mean())
        elem = np.abs(a - c) <= tol * (np.abs(c) + rms)
        say("%s: %s end-to-end relative %.2e; stage-isolated elements in bound %d of %d"
            % (label, name, rel, elem.sum(), elem.size))
        assert rel <= tol, (name, rel)
        assert elem.all(), (name, (~elem).sum())


# ---- C2: 1,000,000 Gaussians, 1256x828, SH 3 -------------------------------------------

@pytest.fixture(scope="module")
def c2():
    ctx = tuned_ctx()
    scene, cam, gt = synth.c2_inputs()
    n, W, H = scene.n, cam.width, cam.height
    say("c2 full: render on the GPU")
    g = api.Gaussians.from_scene(scene)
    frame = api.Frame(ctx, n, W, H, key_cap=16 * n, auto_grow=False)
    gtt = torch.from_numpy(gt).cuda()
    img = api.render(ctx, g, cam, frame, gt=gtt)
    torch.cuda.synchronize()
    st = frame.host_state(n)
    assert st["n_keys"] <= 16 * n
    say("c2 full: oracle projection and forward over %d pixels" % (W * H))
    pr = oracle.project(scene, cam)
    r = oracle.render_rows(pr, margins=True)
    yield dict(ctx=ctx, scene=scene, cam=cam, gt=gt, g=g, frame=frame, img=img.cpu().numpy(), st=st, pr=pr, r=r)
    frame.close()


def test_c2_full_projection(c2):
    check_projection_exact(c2["pr"], c2["st"], "c2")


def test_c2_full_forward_every_pixel(c2):
    cam = c2["cam"]
    check_forward(c2["img"], c2["st"], c2["r"], cam.width, cam.height, "c2")


def test_c2_alpha_rounding_measured(c2):
    """The blend's FP32 alpha against the oracle's FP64 o G on a million
    (pixel, Gaussian) pairs inside the Gaussians' boxes, weighted toward the
    box edge where alpha meets 1/255: every relative difference must lie
    within the error bound the oracle's near-threshold flags assume for that
    pair (alpha_bound: a multiple of the unit roundoff times the magnitudes of
    the exponent's terms)."""
    pr, st = c2["pr"], c2["st"]
    rng = np.random.default_rng(44)
    vis = np.nonzero((pr.valid == 1) & (st["ntiles"] > 0) & (pr.box_flag == 0))[0]
    ids = rng.choice(vis, 1_000_000)
    b = pr.box[ids].astype(np.int64)
    # half uniform in the box, half on its boundary rows and columns
    u = rng.uniform(size=(len(ids), 2))
    x = b[:, 0] + np.floor(u[:, 0] * (b[:, 2] - b[:, 0] + 1)).astype(np.int64)
    y = b[:, 1] + np.floor(u[:, 1] * (b[:, 3] - b[:, 1] + 1)).astype(np.int64)
    edge = rng.uniform(size=len(ids)) < 0.5
    x = np.where(edge & (u[:, 0] < 0.5), b[:, 0], np.where(edge, b[:, 2], x))
    pix = np.stack([x, y], 1).astype(np.int32)
    a64, bound = oracle.alpha_pairs(pr, pix, ids, with_bound=True)
    a32 = api.debug_blend_alpha(c2["frame"], torch.from_numpy(pix).cuda(),
                                torch.from_numpy(ids.astype(np.int32)).cuda()).cpu().numpy().astype(np.float64)
    # pairs whose alpha is far below 1/255 underflow toward FP32's subnormals;
    # no decision lies there
    use = a64 >= 1e-6
    rel = np.abs(a32 - a64)[use] / a64[use]
    ratio = rel / bound[use]
    near = (np.abs(a64 * 255 - 1) < 0.1)[use]
    say("c2: FP32 alpha over %d pairs: relative error max %.3g (99.99%% %.3g), near 1/255 (%d pairs) max %.3g; "
        "largest error / bound %.3g" % (use.sum(), rel.max(), np.quantile(rel, 0.9999), near.sum(), rel[near].max(),
                                         ratio.max()))
    assert use.sum() > 800_000
    assert ratio.max() <= 1.0


@pytest.fixture(scope="module")
def c2_backward(c2):
    """Dense upstream gradient (the benchmark's), zero at flagged pixels."""
    cam = c2["cam"]
    W, H = cam.width, cam.height
    G = np.random.default_rng(7).normal(0.0, 1.0 / (3 * W * H), (3, H, W)).astype(np.float32)
    flag = c2["r"]["flag"].reshape(H, W).astype(bool)
    G[:, flag] = 0.0
    Gt = torch.from_numpy(G).cuda()
    # as in the benchmark's steady state: the first reverse pass reserves the
    # checkpoints, the next render writes them and the reverse pass walks the
    # long tiles as segments
    api.render_backward(c2["ctx"], c2["g"], cam, c2["frame"], Gt)
    api.render(c2["ctx"], c2["g"], cam, c2["frame"], gt=torch.from_numpy(c2["gt"]).cuda())
    grads = api.render_backward(c2["ctx"], c2["g"], cam, c2["frame"], Gt)
    torch.cuda.synchronize()
    n = c2["g"].n
    g2d = grad2d_host(c2["frame"], 0, n)
    say("c2 full: oracle reverse pass over %d pixels" % (W * H))
    rb = oracle.render_rows(c2["pr"], dL_dcolor=G.transpose(1, 2, 0).reshape(-1, 3).astype(np.float64),
                            grad_abs=True)
    return dict(G=G, grads=grads, g2d=g2d, rb=rb)


def test_c2_full_backward_2d_gradients(c2, c2_backward):
    rb = c2_backward["rb"]
    check_grad2d(c2_backward["g2d"], oracle_grad2d(rb["grad"]), rb["grad"]["abs"], "c2", pr=c2["pr"])


def test_c2_full_backward_parameter_gradients(c2, c2_backward):
    scene, cam = c2["scene"], c2["cam"]
    gref = oracle.project_backward(scene, cam, c2_backward["rb"]["grad"])
    g2 = c2_backward["g2d"]
    gstage = oracle.project_backward(scene, cam, dict(mean2d=g2[:, 0:2], conic=g2[:, 2:5], opacity=g2[:, 5],
                                                      rgb=g2[:, 6:9]))
    check_param_grads(c2_backward["grads"], gref, gstage, "c2")


# ---- C3: 500,000 Gaussians, 16 views, top-5% candidates (stage-isolated) ----------------

def test_c3_error_stats_and_split_stage_isolated():
    """The densification workload: the GPU renders the 16 sampled views in
    one batched launch; its images and dominant maps feed both the GPU's and
    the oracle's error statistics, whose regions and attribution counts must
    be identical, and the GPU's regions then feed both splits, whose modes,
    counts, offsets and output rows must match."""
    n, W, H, V = 500_000, 1256, 828, 16
    ctx = tuned_ctx(max_pixels=W * H, max_gaussians=n, max_candidates=n // 20, max_regions=V * W * H // 5 // 4,
                    max_views=V)
    scene = synth.scene_clusters(n, 1003, 3)
    views = synth.sphere_cameras(V, 4.0, [(W, H)], seed=1003)
    gts_np = [synth.smooth_image(H, W, 2000 + v) for v in range(V)]
    gts = [torch.from_numpy(a).cuda() for a in gts_np]
    g = api.Gaussians.from_scene(scene)
    # candidates: the top 5% by the view-averaged screen-space gradient norm of
    # the L1 loss (as the benchmark selects them)
    frame = api.Frame(ctx, n, W, H, key_cap=16 * n)
    image = torch.empty(3, H, W, dtype=torch.float32, device="cuda")
    g2d = torch.zeros(n, dtype=torch.float32, device="cuda")
    vis = torch.zeros(n, dtype=torch.int32, device="cuda")
    grads = api.Gaussians.empty(n, 3)
    for cam, gt in zip(views, gts):
        api.render(ctx, g, cam, frame, gt=gt, image=image)
        dL = torch.sign(image - gt) / (3 * W * H)
        api.render_backward(ctx, g, cam, frame, dL.contiguous(), grads=grads, g2d_norm=g2d, vis_count=vis)
    gi = (g2d / vis.clamp(min=1)).cpu().numpy()
    frame.close()
    order = np.lexsort((np.arange(n), -gi))
    cand = np.sort(order[: n // 20]).astype(np.int32)
    is_cand = np.zeros(n, np.uint8)
    is_cand[cand] = 1
    say("c3: %d candidates; batched render of %d views" % (len(cand), V))
    bframe = api.BatchFrame.for_views(ctx, n, views, key_cap=16 * n * V)
    images = api.render_batch(ctx, g, views, bframe, gts=gts)
    prm_o = oracle.SplitParams()
    prm = api.SplitParams()
    regions = api.RegionBuffer(V * W * H // prm.m_min // 4)
    attr_g = torch.zeros(n, dtype=torch.int32, device="cuda")
    is_cand_t = torch.from_numpy(is_cand).cuda()
    for v in range(V):
        m = bframe.device_maps(v)
        api.accumulate_error_stats(ctx, W, H, m["err"], m["err_minmax"], m["dom"], gts[v], v, is_cand_t, prm,
                                   regions, attr_g)
    torch.cuda.synchronize()
    got = regions.host()
    attr_o = np.zeros(n, np.int32)
    want = []
    for v in range(V):
        st = bframe.host_state(n, view=v)
        img = images[v].cpu().numpy()
        r, _ = oracle.error_stats(img, gts_np[v], st["dom"], is_cand, v, prm_o, attr_o)
        want.append(r)
    want = np.concatenate(want)
    bframe.close()
    say("c3: %d regions, %d attributed pixels" % (len(want), attr_o.sum()))
    assert len(got) == len(want)
    for f in ("cand", "view", "label", "area", "band", "sx", "sy", "sxx", "sxy", "syy", "cx", "cy", "cov", "e1",
              "sigma1", "sigma2"):
        np.testing.assert_array_equal(got[f], want[f], err_msg=f)
    np.testing.assert_array_equal(got["rgb"].astype(np.float64), want["rgb"])
    np.testing.assert_array_equal(attr_g.cpu().numpy(), attr_o)
    # the split on those regions
    noise = synth.vanilla_noise(len(cand), 5)
    say("c3: adaptive split of %d candidates" % len(cand))
    out = api.Gaussians.empty(n + len(cand) * (prm.n_max + 1), 3)
    res = api.adaptive_split(ctx, g, torch.from_numpy(cand).cuda(), regions, views, attr_g, prm,
                             torch.from_numpy(noise).cuda(), out=out)
    torch.cuda.synchronize()
    ref = oracle.adaptive_split(scene, cand, want, views, attr_o, prm_o, noise)
    mode, count, offset, n_out = res[1].cpu().numpy(), res[2].cpu().numpy(), res[3].cpu().numpy(), int(res[4].item())
    say("c3: modes vanilla %d reset %d adaptive %d; %d output rows"
        % ((ref["mode"] == 0).sum(), (ref["mode"] == 1).sum(), (ref["mode"] == 2).sum(), ref["n_out"]))
    np.testing.assert_array_equal(mode, ref["mode"])
    np.testing.assert_array_equal(count, ref["count"])
    np.testing.assert_array_equal(offset, ref["offset"])
    assert n_out == ref["n_out"]
    # survivors are exact copies; children and parent copies to 1e-5
    n_surv = n_out - int(ref["count"].sum())
    for f in GRAD_FIELDS:
        a = getattr(out, f)[..., :n_surv].cpu().numpy()
        np.testing.assert_array_equal(a, ref[f][..., :n_surv], err_msg=f)
    ch = slice(n_surv, n_out)
    np.testing.assert_allclose(out.means[:, ch].cpu().numpy(), ref["means"][:, ch], rtol=1e-5, atol=1e-6)
    np.testing.assert_allclose(out.opacity_logits[ch].cpu().numpy(), ref["opacity_logits"][ch], rtol=1e-5,
                               atol=1e-6)
    np.testing.assert_allclose(out.sh[:, :, ch].cpu().numpy(), ref["sh"][:, :, ch], rtol=1e-5, atol=1e-6)
    q = out.quats[:, ch].cpu().numpy().astype(np.float64)
    ls = out.log_scales[:, ch].cpu().numpy().astype(np.float64)
    Cg = cov_from(q, ls)
    Co = cov_from(ref["quats"][:, ch].astype(np.float64), ref["log_scales"][:, ch].astype(np.float64))
    scale = np.abs(Co).max(axis=(0, 1)) + 1e-30
    assert (np.abs(Cg - Co).max(axis=(0, 1)) <= 1e-5 * scale).all()


def cov_from(q, ls):
    q = q / np.linalg.norm(q, axis=0, keepdims=True)
    w, x, y, z = q
    R = np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                  [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                  [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])
    s2 = np.exp(2 * ls)
    return np.einsum("ikn,kn,jkn->ijn", R, s2, R)


# ---- C4: 1,500,000 Gaussians, 8 views of uneven size in one batched launch ----------------

@pytest.fixture(scope="module")
def c4():
    ctx = tuned_ctx()
    n = 1_500_000
    scene = synth.scene_clusters(n, 1004, 3)
    cams = synth.sphere_cameras(len(C4_SIZES), 4.0, C4_SIZES, seed=1004)
    g = api.Gaussians.from_scene(scene)
    tiles = sum(((c.width + 15) // 16) * ((c.height + 15) // 16) for c in cams)
    say("c4 full: batched render of %d views, %d tiles" % (len(cams), tiles))
    assert tiles > 16384
    frame = api.BatchFrame.for_views(ctx, n, cams, key_cap=64 * n)
    images = api.render_batch(ctx, g, cams, frame)
    rng = np.random.default_rng(1004)
    dLs = [rng.normal(0.0, 1.0 / (3 * c.width * c.height), (3, c.height, c.width)).astype(np.float32) for c in cams]
    torch.cuda.synchronize()
    yield dict(ctx=ctx, scene=scene, cams=cams, g=g, frame=frame, images=images, dLs=dLs, n=n)
    frame.close()


def test_c4_every_view_forward_and_backward(c4):
    """Each of the 8 views of the batched launch against the oracle's render
    of that view; then the batched reverse pass (upstream gradients zeroed at
    each view's flagged pixels) against the oracle's per-view reverse passes
    summed over the views."""
    ctx, g, frame, cams, n = c4["ctx"], c4["g"], c4["frame"], c4["cams"], c4["n"]
    dLs = [d.copy() for d in c4["dLs"]]
    g2d_ref = []
    prs = []
    for v, cam in enumerate(cams):
        W, H = cam.width, cam.height
        st = frame.host_state(n, view=v)
        pr = oracle.project(c4["scene"], cam)
        prs.append(pr)
        check_projection_exact(pr, st, "c4 view %d" % v)
        r = oracle.render_rows(pr, margins=True)
        flag = check_forward(c4["images"][v].cpu().numpy(), st, r, W, H, "c4 view %d (%dx%d)" % (v, W, H))
        dLs[v][:, flag] = 0.0
    # the first reverse pass reserves the checkpoints; the next render writes
    # them and the second reverse pass walks long tiles as segments
    dLt = [torch.from_numpy(d).cuda() for d in dLs]
    api.render_backward_batch(ctx, g, frame, dLt)
    api.render_batch(ctx, g, cams, frame, images=c4["images"])
    grads = api.render_backward_batch(ctx, g, frame, dLt)
    torch.cuda.synchronize()
    g_sum = None
    gstage = None
    for v, cam in enumerate(cams):
        say("c4: oracle reverse pass of view %d" % v)
        rb = oracle.render_rows(prs[v], dL_dcolor=dLs[v].transpose(1, 2, 0).reshape(-1, 3).astype(np.float64),
                                grad_abs=True)
        gv = grad2d_host(frame, v, n)
        check_grad2d(gv, oracle_grad2d(rb["grad"]), rb["grad"]["abs"], "c4 view %d" % v, pr=prs[v])
        gp = oracle.project_backward(c4["scene"], cam, rb["grad"])
        gs = oracle.project_backward(c4["scene"], cam, dict(mean2d=gv[:, 0:2], conic=gv[:, 2:5], opacity=gv[:, 5],
                                                             rgb=gv[:, 6:9]))
        g_sum = gp if g_sum is None else {k: g_sum[k] + gp[k] for k in gp}
        gstage = gs if gstage is None else {k: gstage[k] + gs[k] for k in gs}
    check_param_grads(grads, g_sum, gstage, "c4")
