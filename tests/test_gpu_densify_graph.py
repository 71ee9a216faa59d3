"""The density-control step with device-side counts (densify.DensifyStep):
the calls that take a device row or candidate count give exactly what they
give with the same count passed from the host, and the whole step (select,
renders of the sampled views with error statistics, clone, split, row map,
prune, moment gather) recorded as one HIP graph replays bit for bit like the
eager step, also with other work on the device between the replays."""
import sys

import numpy as np
import pytest

from paper_2605_06876_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2605_06876_amd import api, densify  # noqa: E402

FIELDS = ("means", "log_scales", "quats", "opacity_logits", "sh")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def host(g, k=None):
    return {f: (getattr(g, f)[..., :k] if k is not None else getattr(g, f)).cpu().numpy() for f in FIELDS}


@pytest.fixture(scope="module")
def state():
    """A 20,000-Gaussian SH3 set with Adam moments and gradient statistics
    that select a few percent for cloning and splitting, 6 sampled views."""
    n, W, H = 20_000, 192, 144
    scene = synth.scene_clusters(n, 21, 3, log_scale_mu=-3.5, log_scale_sd=0.6)
    g = api.Gaussians.from_scene(scene)
    rng = np.random.default_rng(21)
    mk = lambda: api.Gaussians.from_scene(synth.Scene(*[rng.normal(0, 1e-3, a.shape).astype(np.float32)
                                                       for a in (scene.means, scene.log_scales, scene.quats,
                                                                 scene.opacity_logits, scene.sh)], 3))
    m, v = mk(), mk()
    accum = torch.from_numpy(rng.exponential(1.0, n).astype(np.float32)).cuda()
    vis = torch.from_numpy(rng.integers(1, 5, n).astype(np.int32)).cuda()
    views = synth.sphere_cameras(6, 4.0, [(W, H)], seed=21)
    gts = [torch.from_numpy(synth.smooth_image(H, W, 400 + k)).cuda() for k in range(6)]
    return dict(n=n, g=g, m=m, v=v, accum=accum, vis=vis, views=views, gts=gts)


def make_step(ctx, st, method):
    if method == "adpsplit":
        regions = api.RegionBuffer(6 * 192 * 144 // 5)
        step = densify.DensifyStep(ctx, st["n"], 3, "adpsplit", api.SplitParams(), st["views"], st["gts"], regions)
    elif method == "vanilla5":   # five random children per candidate (Fig. 2's pilot)
        step = densify.DensifyStep(ctx, st["n"], 3, "vanilla", api.SplitParams(variant=api.VARIANT_FIXED_N, fixed_n=5))
    else:
        step = densify.DensifyStep(ctx, st["n"], 3, "vanilla")
    step.noise.copy_(torch.from_numpy(synth.vanilla_noise(step.cc, 5, step.noise_n)).view_as(step.noise))
    return step


ARGS = (2.5, 0.05, 0.005, 0.5)   # gradient threshold, clone/split size, min opacity, max world scale


def snapshot(step):
    k = int(step.n_out.item())
    return k, host(step.out, k), host(step.m_out, k), host(step.v_out, k), step.st3[:k].cpu().numpy()


@pytest.mark.parametrize("method", ["adpsplit", "vanilla", "vanilla5"])
def test_graph_replays_equal_the_eager_step(state, method):
    ctx = api.Context(0)
    st = state
    step = make_step(ctx, st, method)
    args = (st["g"], st["m"], st["v"], st["accum"], st["vis"]) + ARGS
    say("densify graph (%s): eager step" % method)
    step.run(*args)
    torch.cuda.synchronize()
    want = snapshot(step)
    n_cand = int(step.sel[3].item())
    say("densify graph (%s): %d -> %d rows, %d candidates" % (method, st["n"], want[0], n_cand))
    assert n_cand > 0 and want[0] != st["n"]
    s = torch.cuda.Stream()
    graph = step.capture(s, *args)
    other = api.Frame(ctx, st["n"], 64, 48, auto_grow=False)
    for rep in range(3):
        for t in (step.out.means, step.m_out.sh, step.st3):   # outputs overwritten before each replay
            t.fill_(-7)
        step.n_out.fill_(0)
        torch.cuda.synchronize()
        graph.launch(s)
        s.synchronize()
        got = snapshot(step)
        say("densify graph (%s): replay %d -> %d rows" % (method, rep, got[0]))
        assert got[0] == want[0]
        for a, b in zip(got[1:4], want[1:4]):
            for f in FIELDS:
                np.testing.assert_array_equal(a[f], b[f], err_msg=f)
        np.testing.assert_array_equal(got[4], want[4])
        # other work between the replays
        api.render(ctx, st["g"], synth.sphere_cameras(1, 4.0, [(64, 48)], seed=rep)[0], other)
        torch.cuda.synchronize()
    graph.close()
    other.close()
    step.close()


def test_device_counts_equal_host_counts(state):
    """as_clone_prune, as_adaptive_split (fixed-N and AdpSplit), as_split_row_map
    and as_gather_rows with a device count equal the same calls with that count
    from the host, on a capacity twice the rows in use."""
    ctx = api.Context(0)
    st = state
    n = st["n"]
    ctx.reserve(max_gaussians=24 * n, max_candidates=n, max_pixels=192 * 144, max_regions=6 * 192 * 144 // 5,
                max_views=6)
    g = st["g"]
    # a capacity-sized copy: the first n rows in use
    cap = api.Gaussians.empty(2 * n, 3)
    for f in FIELDS:
        getattr(cap, f)[..., :n] = getattr(g, f)
        getattr(cap, f)[..., n:] = 3.0   # rows past the count must never be read
    n_dev = torch.tensor([n], dtype=torch.int64, device="cuda")
    clone, is_cand, cand, n_cand = api.densify_select(ctx, g, st["accum"], st["vis"], 2.5, 0.05)
    nc = int(n_cand.item())
    assert nc > 0
    # clone + prune
    a = api.clone_prune(ctx, g, None, None, 0.005, 0.5)
    b = api.clone_prune(ctx, cap.counted(n_dev), None, None, 0.005, 0.5)
    ka, kb = int(a[2].item()), int(b[2].item())
    assert ka == kb
    for f in FIELDS:
        np.testing.assert_array_equal(host(a[0], ka)[f], host(b[0], kb)[f], err_msg=f)
    np.testing.assert_array_equal(a[1][:ka].cpu().numpy(), b[1][:kb].cpu().numpy())
    # split, both variants; the capacity path takes cand with n entries and a device count
    noise = torch.from_numpy(synth.vanilla_noise(n, 9, 2)).cuda()
    regions = api.RegionBuffer(6 * 192 * 144 // 5)
    attr = torch.zeros(2 * n, dtype=torch.int32, device="cuda")
    W, H = 192, 144
    frame = api.BatchFrame.for_views(ctx, n, st["views"], key_cap=32 * n * 6)
    api.render_batch(ctx, g, st["views"], frame, gts=st["gts"])
    for j in range(6):
        mp = frame.device_maps(j)
        api.accumulate_error_stats(ctx, W, H, mp["err"], mp["err_minmax"], mp["dom"], st["gts"][j], j, is_cand,
                                   api.SplitParams(), regions, attr[:n])
    frame.close()
    for prm in (api.SplitParams(), api.SplitParams(variant=api.VARIANT_FIXED_N, fixed_n=2)):
        per = max(2, prm.n_max + 1)
        out_h = api.Gaussians.empty(n + nc * per, 3)
        r_h = api.adaptive_split(ctx, g, cand[:nc].contiguous(), regions, st["views"], attr, prm,
                                 noise[:nc].contiguous(), out=out_h)
        out_d = api.Gaussians.empty(2 * n + n * per, 3)
        r_d = api.adaptive_split(ctx, cap.counted(n_dev), cand, regions, st["views"], attr, prm, noise, out=out_d,
                                 n_cand_dev=n_cand)
        k1, k2 = int(r_h[4].item()), int(r_d[4].item())
        say("device counts: split variant %d: %d rows both ways" % (prm.variant, k1))
        assert k1 == k2
        for i in (1, 2, 3):
            np.testing.assert_array_equal(r_h[i][:nc].cpu().numpy(), r_d[i][:nc].cpu().numpy())
        for f in FIELDS:
            np.testing.assert_array_equal(host(r_h[0], k1)[f], host(r_d[0], k2)[f], err_msg=f)
        # row maps
        m_h = api.split_row_map(ctx, n, cand[:nc].contiguous(), r_h[1][:nc].contiguous(), k1)
        m_d = api.split_row_map(ctx, 2 * n, cand, r_d[1], 2 * n + n * per, n_dev=n_dev, n_cand_dev=n_cand)
        np.testing.assert_array_equal(m_h[:k1].cpu().numpy(), m_d[:k2].cpu().numpy())
        # gather with a device row count
        k_dev = torch.tensor([k1], dtype=torch.int64, device="cuda")
        gh = api.gather_rows(ctx, st["m"], m_h, k1)
        gd = api.gather_rows(ctx, st["m"], m_d, 2 * n + n * per, n_rows_dev=k_dev)
        for f in FIELDS:
            np.testing.assert_array_equal(host(gh, k1)[f], host(gd, k1)[f], err_msg=f)
