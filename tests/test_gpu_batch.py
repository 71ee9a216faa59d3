"""Batched multi-view rendering and graph capture through the C-ABI.

A batched render must give every view exactly what a render of that view
alone gives (the per-pixel operations and their order do not depend on the
other views): images, transmittance, contributor counts and dominant ids
bit-identical; gradients summed over the views equal to the sum of the
single-view gradients up to float-atomic order (relative 1e-5).  The single
view path itself is held to the oracle in test_gpu_render.py; one batched
view is also compared with the oracle here directly.  Graph replays must equal
eager calls on the inputs present at replay time."""
import gc
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

FIELDS = ("means", "log_scales", "quats", "opacity_logits", "sh")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    return api.Context(0)


SIZES = [(64, 48), (100, 75), (33, 47), (128, 96), (17, 130)]


def cams_for(sizes, seed):
    return synth.sphere_cameras(len(sizes), 3.2, sizes, seed=seed)


def single(ctx, g, cam, gt=None):
    frame = api.Frame(ctx, g.n, cam.width, cam.height)
    img = api.render(ctx, g, cam, frame, gt=gt)
    torch.cuda.synchronize()
    return frame, img


def rel(x, y):
    return (torch.linalg.norm(x - y) / torch.linalg.norm(y).clamp_min(1e-30)).item()


@pytest.mark.parametrize("persistent,bin_tile,lpt", [(False, 16, True), (True, 16, True), (False, 32, True),
                                                     (True, 32, True), (False, 32, False)])
def test_batch_equals_single_views(ctx, persistent, bin_tile, lpt):
    """Each view of a batch (uneven sizes, ragged last bins) against a render
    of that view alone with the same tuning, including pairs binned by 32 x 32
    squares with the dispatch order that groups a bin's tiles by XCD."""
    c = api.Context(0)
    api.set_tuning(c, persistent=persistent, bin_tile=bin_tile, longest_first=lpt)
    scene = synth.scene_clusters(6000, seed=71, sh_degree=3, log_scale_mu=-3.8, log_scale_sd=0.5)
    g = api.Gaussians.from_scene(scene)
    cams = cams_for(SIZES, seed=3)
    gts = [torch.from_numpy(synth.smooth_image(cm.height, cm.width, seed=k)).cuda() for k, cm in enumerate(cams)]
    frame = api.BatchFrame.for_views(c, g.n, cams)
    imgs = api.render_batch(c, g, cams, frame, gts=gts)
    dLs = [torch.from_numpy(np.random.default_rng(20 + k).normal(size=(3, cm.height, cm.width)).astype(np.float32)).cuda()
           for k, cm in enumerate(cams)]
    acc_b = torch.zeros(g.n, device="cuda")
    cnt_b = torch.zeros(g.n, dtype=torch.int32, device="cuda")
    gb = api.render_backward_batch(c, g, frame, dLs, g2d_norm=acc_b, vis_count=cnt_b)
    torch.cuda.synchronize()
    sum_g = None
    acc_s = torch.zeros(g.n, device="cuda")
    cnt_s = torch.zeros(g.n, dtype=torch.int32, device="cuda")
    for k, cam in enumerate(cams):
        fr, img = single(c, g, cam, gt=gts[k])
        assert torch.equal(imgs[k], img), "view %d image" % k
        a, b = frame.host_state(g.n, view=k), fr.host_state(g.n)
        for key in ("t_final", "n_contrib", "dom", "err", "err_minmax", "depth_key", "box", "ntiles"):
            np.testing.assert_array_equal(a[key], b[key], err_msg="view %d %s" % (k, key))
        # the view's pairs: same Gaussians in the same order per tile
        for t in range(0, a["ranges"].shape[0], 7):
            s0, e0 = a["ranges"][t]
            s1, e1 = b["ranges"][t]
            np.testing.assert_array_equal(a["gauss"][s0:e0], b["gauss"][s1:e1], err_msg="view %d tile %d" % (k, t))
        gs = api.render_backward(c, g, cam, fr, dLs[k], g2d_norm=acc_s, vis_count=cnt_s)
        if sum_g is None:
            sum_g = [getattr(gs, f).clone() for f in FIELDS]
        else:
            for i, f in enumerate(FIELDS):
                sum_g[i] += getattr(gs, f)
    torch.cuda.synchronize()
    for i, f in enumerate(FIELDS):
        r = rel(getattr(gb, f), sum_g[i])
        say("%s: batch vs sum of views rel %.2e" % (f, r))
        assert r <= 1e-5, f
    assert torch.equal(cnt_b, cnt_s)
    assert rel(acc_b, acc_s) <= 1e-6


def test_batch_of_different_scenes(ctx):
    scenes = [synth.scene_clusters(n, seed=90 + n, sh_degree=3, log_scale_mu=-3.8, log_scale_sd=0.5)
              for n in (3000, 500, 7000)]
    gs = [api.Gaussians.from_scene(s) for s in scenes]
    cams = cams_for([(96, 64), (40, 40), (150, 90)], seed=5)
    frame = api.BatchFrame.for_views(ctx, [g.n for g in gs], cams)
    imgs = api.render_batch(ctx, gs, cams, frame)
    torch.cuda.synchronize()
    for k in range(3):
        fr, img = single(ctx, gs[k], cams[k])
        assert torch.equal(imgs[k], img), k
        a, b = frame.host_state(gs[k].n, view=k), fr.host_state(gs[k].n)
        for key in ("t_final", "n_contrib", "dom"):
            np.testing.assert_array_equal(a[key], b[key], err_msg="view %d %s" % (k, key))
    # a backward over views of different sets is refused
    with pytest.raises(api.AdpSplitError):
        api.render_backward_batch(ctx, gs[0], frame, [torch.zeros(3, c.height, c.width, device="cuda") for c in cams])


def test_batched_view_against_oracle(ctx):
    """The third view of a batch against the FP64 oracle (flagged pixels excluded)."""
    scene = synth.scene_uniform_sh0(1500, seed=44)
    cams = cams_for([(80, 60), (64, 64), (72, 40)], seed=8)
    g = api.Gaussians.from_scene(scene)
    frame = api.BatchFrame.for_views(ctx, g.n, cams)
    imgs = api.render_batch(ctx, g, cams, frame)
    torch.cuda.synchronize()
    cam = cams[2]
    pr = oracle.project(scene, cam)
    ref, maps = oracle.render_image(pr)
    flag = maps["flag"] != 0
    got = imgs[2].cpu().numpy()
    d = np.abs(got - ref).max(axis=0)
    assert d[~flag].max() <= 1e-4
    st = frame.host_state(g.n, view=2)
    np.testing.assert_array_equal(st["n_contrib"][~flag], maps["ncontrib"][~flag])
    np.testing.assert_array_equal(st["dom"][~flag], maps["dom"][~flag])
    say("flagged pixels: %d of %d" % (flag.sum(), flag.size))


def test_batch_capacity_and_argument_checks(ctx):
    g = api.Gaussians.from_scene(synth.scene_uniform_sh0(100, seed=1))
    cams = cams_for([(32, 32), (32, 32)], seed=1)
    frame = api.BatchFrame(ctx, 2, 150, 32 * 32 * 2, 8)
    with pytest.raises(api.AdpSplitError) as e:   # 200 entries > 150
        api.render_batch(ctx, g, cams, frame)
    assert e.value.status == api.AS_ERR_CAPACITY
    frame3 = api.BatchFrame(ctx, 1, 1000, 10000, 100)
    with pytest.raises(api.AdpSplitError) as e:   # two views > max_views 1
        api.render_batch(ctx, g, cams, frame3)
    assert e.value.status == api.AS_ERR_ARG
    single_frame = api.Frame(ctx, 100, 32, 32)
    with pytest.raises(api.AdpSplitError):        # a single-view frame takes one view
        api.render_batch(ctx, g, cams, single_frame)


def _replay_check(ctx, g, cams, frame, gts, dLs, stream):
    """Eager results for the current inputs."""
    with torch.cuda.stream(stream):
        imgs = api.render_batch(ctx, g, cams, frame, gts=gts)
        gr = api.render_backward_batch(ctx, g, frame, dLs)
    stream.synchronize()
    return [i.clone() for i in imgs], [getattr(gr, f).clone() for f in FIELDS]


def test_graph_replay_matches_eager(ctx):
    """Capture render + backward of a 3-view batch, replay it several times
    with eager work in between and inputs changed in place, and compare every
    replay with an eager run on the same inputs."""
    scene = synth.scene_clusters(5000, seed=12, sh_degree=3, log_scale_mu=-3.8, log_scale_sd=0.5)
    g = api.Gaussians.from_scene(scene)
    cams = cams_for([(96, 80), (48, 64), (130, 70)], seed=9)
    gts = [torch.from_numpy(synth.smooth_image(c.height, c.width, seed=k)).cuda() for k, c in enumerate(cams)]
    dLs = [torch.from_numpy(np.random.default_rng(5 + k).normal(size=(3, c.height, c.width)).astype(np.float32)).cuda()
           for k, c in enumerate(cams)]
    s = torch.cuda.Stream()
    frame = api.BatchFrame.for_views(ctx, g.n, cams, key_cap=1 << 20, auto_grow=False)
    out_imgs = [torch.empty(3, c.height, c.width, device="cuda") for c in cams]
    grads = api.Gaussians.empty(g.n, 3)
    with torch.cuda.stream(s):   # sizes every buffer before the capture
        api.render_batch(ctx, g, cams, frame, gts=gts, images=out_imgs)
        api.render_backward_batch(ctx, g, frame, dLs, grads=grads)
    s.synchronize()

    def step():
        api.render_batch(ctx, g, cams, frame, gts=gts, images=out_imgs)
        api.render_backward_batch(ctx, g, frame, dLs, grads=grads)

    graph = api.Graph.capture(ctx, step, s)
    ref_frame = api.BatchFrame.for_views(ctx, g.n, cams)
    for rep in range(4):
        if rep == 2:   # new inputs in place: the replay must see them
            g.means.add_(0.01)
            g.opacity_logits.mul_(0.9)
        _ = torch.randn(1000, 1000, device="cuda") @ torch.randn(1000, 1000, device="cuda")   # eager work between
        torch.cuda.synchronize()
        graph.launch(s)
        s.synchronize()
        got_imgs = [i.clone() for i in out_imgs]
        got_g = [getattr(grads, f).clone() for f in FIELDS]
        want_imgs, want_g = _replay_check(ctx, g, cams, ref_frame, gts, dLs, torch.cuda.current_stream())
        for k in range(len(cams)):
            assert torch.equal(got_imgs[k], want_imgs[k]), "replay %d view %d" % (rep, k)
        for i, f in enumerate(FIELDS):
            assert rel(got_g[i], want_g[i]) <= 1e-5, "replay %d %s" % (rep, f)
    graph.close()


def test_first_backward_inside_a_capture(ctx):
    """A frame holds its checkpoint buffer from creation, so a reverse pass
    first seen inside a graph capture allocates nothing: captured as a
    frame's first backward, render + backward replays like the eager step."""
    scene = synth.scene_clusters(4000, seed=14, sh_degree=1, log_scale_mu=-3.8, log_scale_sd=0.5)
    g = api.Gaussians.from_scene(scene)
    cams = cams_for([(80, 64), (64, 96)], seed=10)
    dLs = [torch.from_numpy(np.random.default_rng(20 + k).normal(size=(3, c.height, c.width)).astype(np.float32)).cuda()
           for k, c in enumerate(cams)]
    s = torch.cuda.Stream()
    frame = api.BatchFrame.for_views(ctx, g.n, cams, key_cap=1 << 20, auto_grow=False)
    out_imgs = [torch.empty(3, c.height, c.width, device="cuda") for c in cams]
    grads = api.Gaussians.empty(g.n, 1)
    with torch.cuda.stream(s):   # a render only: the backward is first seen inside the capture
        api.render_batch(ctx, g, cams, frame, images=out_imgs)
    s.synchronize()

    def step():
        api.render_batch(ctx, g, cams, frame, images=out_imgs)
        api.render_backward_batch(ctx, g, frame, dLs, grads=grads)

    graph = api.Graph.capture(ctx, step, s)
    ref_frame = api.BatchFrame.for_views(ctx, g.n, cams)
    for rep in range(3):
        graph.launch(s)
        s.synchronize()
        got_g = [getattr(grads, f).clone() for f in FIELDS]
        _, want_g = _replay_check(ctx, g, cams, ref_frame, None, dLs, torch.cuda.current_stream())
        for i, f in enumerate(FIELDS):
            assert rel(got_g[i], want_g[i]) <= 1e-5, "replay %d %s" % (rep, f)
    graph.close()


def test_reverse_pass_clears_its_gradient_rows(ctx):
    """The forward of a render clears the per-entry 2D gradient rows that the
    reverse pass adds into.  A second reverse pass of the same render, and a
    reverse pass captured in a graph without its render, clear them
    themselves: repeated passes and replays give the first pass's gradients
    instead of sums of them."""
    scene = synth.scene_clusters(3000, seed=21, sh_degree=1, log_scale_mu=-3.8, log_scale_sd=0.5)
    g = api.Gaussians.from_scene(scene)
    cams = cams_for([(96, 64), (64, 80)], seed=12)
    dLs = [torch.from_numpy(np.random.default_rng(40 + k).normal(size=(3, c.height, c.width)).astype(np.float32)).cuda()
           for k, c in enumerate(cams)]
    s = torch.cuda.Stream()
    frame = api.BatchFrame.for_views(ctx, g.n, cams, key_cap=1 << 20, auto_grow=False)
    grads = api.Gaussians.empty(g.n, 1)
    with torch.cuda.stream(s):
        api.render_batch(ctx, g, cams, frame)
        api.render_backward_batch(ctx, g, frame, dLs, grads=grads)
        first = [getattr(grads, f).clone() for f in FIELDS]
        api.render_backward_batch(ctx, g, frame, dLs, grads=grads)   # no render in between
    s.synchronize()
    for i, f in enumerate(FIELDS):
        assert rel(getattr(grads, f), first[i]) <= 1e-5, "second pass %s" % f
    with torch.cuda.stream(s):
        api.render_batch(ctx, g, cams, frame)   # eager render; the capture holds the reverse pass alone
    s.synchronize()
    graph = api.Graph.capture(ctx, lambda: api.render_backward_batch(ctx, g, frame, dLs, grads=grads), s)
    for rep in range(3):
        _ = torch.randn(500, 500, device="cuda") @ torch.randn(500, 500, device="cuda")   # eager work between
        torch.cuda.synchronize()
        graph.launch(s)
        s.synchronize()
        for i, f in enumerate(FIELDS):
            assert rel(getattr(grads, f), first[i]) <= 1e-5, "replay %d %s" % (rep, f)
    graph.close()
    del graph, grads, first
    gc.collect()


def test_capture_refuses_a_growing_frame(ctx):
    """A frame with auto_grow reads its pair count back after each render (the
    binding's growth policy), which a graph capture cannot hold."""
    g = api.Gaussians.from_scene(synth.scene_uniform_sh0(200, seed=2))
    cam = cams_for([(32, 32)], seed=2)[0]
    frame = api.Frame(ctx, g.n, 32, 32, auto_grow=True)
    s = torch.cuda.Stream()
    with pytest.raises(api.AdpSplitError) as e:
        api.Graph.capture(ctx, lambda: api.render(ctx, g, cam, frame), s)
    assert e.value.status == api.AS_ERR_STATE
    # the stream is usable again afterwards
    with torch.cuda.stream(s):
        img = api.render(ctx, g, cam, frame)
    s.synchronize()
    assert torch.isfinite(img).all()


def test_frame_destroyed_after_its_context():
    """Python's cycle collector finalises objects in no fixed order, so a frame
    can be freed after its context: that must read nothing from the freed
    context and leave no HIP error for the next call to pick up."""
    c = api.Context(0)
    f = api.Frame(c, 100, 32, 32)
    c.close()
    f.close()
    x = torch.arange(16, dtype=torch.float32).cuda() * 2.0
    torch.cuda.synchronize()
    assert x[-1].item() == 30.0
