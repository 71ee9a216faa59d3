"""The boundary's memory contract, on the GPU: frames and the context's
reservation hold every buffer the four calls of the path use, so after
set-up as_render, as_render_backward, as_accumulate_error_stats and
as_adaptive_split allocate nothing (the device's free memory and torch's
allocator are unchanged across each call), and the size queries report what
set-up actually takes."""
import gc
import sys

import numpy as np
import pytest

from paper_2605_06876_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2605_06876_amd import api  # noqa: E402

MiB = 1 << 20


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def free_bytes():
    torch.cuda.synchronize()
    return torch.cuda.mem_get_info(0)[0]


def test_size_queries_match_set_up():
    n, W, H = 200_000, 640, 480
    cam = synth.sphere_cameras(1, 4.0, [(W, H)], seed=5)[0]
    ctx = api.Context(0)
    key_cap = 16 * n
    q_frame = api.workspace_size(ctx, n, [cam], key_cap)
    tiles = ((W + 15) // 16) * ((H + 15) // 16)
    assert q_frame == api.frame_bytes(1, n, W * H, tiles, key_cap)
    # a forward-only frame holds neither the checkpoints nor the per-pair block masks
    assert (api.frame_bytes(1, n, W * H, tiles, key_cap, forward_only=True) ==
            q_frame - (tiles * 3 * 256 * 16 + 256) - (key_cap * 8 + 256))
    f0 = free_bytes()
    frame = api.Frame(ctx, n, W, H, key_cap=key_cap, auto_grow=False)
    f1 = free_bytes()
    res = dict(max_pixels=W * H, max_gaussians=n, max_candidates=n // 20, max_regions=W * H // 5, max_views=8)
    q_res = api.reserve_bytes(**res)
    ctx.reserve(**res)
    f2 = free_bytes()
    say("frame: query %.1f MiB, taken %.1f MiB; reservation: query %.1f MiB, taken %.1f MiB"
        % (q_frame / MiB, (f0 - f1) / MiB, q_res / MiB, (f1 - f2) / MiB))
    assert 0.98 * q_frame <= f0 - f1 <= q_frame + 64 * MiB
    assert 0.98 * q_res <= f1 - f2 <= q_res + 64 * MiB
    assert ctx.reserved() == res
    frame.close()


def test_the_four_calls_allocate_nothing():
    n, W, H, V = 200_000, 640, 480, 2
    scene = synth.scene_clusters(n, 77, 3)
    views = synth.sphere_cameras(V, 4.0, [(W, H)], seed=77)
    gts = [torch.from_numpy(synth.smooth_image(H, W, 300 + v)).cuda() for v in range(V)]
    rng = np.random.default_rng(77)
    cand = np.sort(rng.choice(n, n // 20, replace=False)).astype(np.int32)
    is_cand = np.zeros(n, np.uint8)
    is_cand[cand] = 1
    prm = api.SplitParams()
    # set-up: context reservation, frame, every input and output
    ctx = api.Context(0, max_pixels=W * H, max_gaussians=n, max_candidates=len(cand), max_regions=V * W * H // 5,
                      max_views=V)
    g = api.Gaussians.from_scene(scene)
    frame = api.Frame(ctx, n, W, H, key_cap=16 * n, auto_grow=False)
    image = torch.empty(3, H, W, dtype=torch.float32, device="cuda")
    dL = torch.from_numpy(rng.normal(0, 1e-6, (3, H, W)).astype(np.float32)).cuda()
    grads = api.Gaussians.empty(n, 3)
    g2d = torch.zeros(n, dtype=torch.float32, device="cuda")
    vis = torch.zeros(n, dtype=torch.int32, device="cuda")
    regions = api.RegionBuffer(V * W * H // 5)
    attr = torch.zeros(n, dtype=torch.int32, device="cuda")
    is_cand_t = torch.from_numpy(is_cand).cuda()
    cand_t = torch.from_numpy(cand).cuda()
    noise = torch.from_numpy(synth.vanilla_noise(len(cand), 3)).cuda()
    out = api.Gaussians.empty(n + len(cand) * (prm.n_max + 1), 3)
    nc = len(cand)
    mode = torch.zeros(nc, dtype=torch.uint8, device="cuda")
    count = torch.zeros(nc, dtype=torch.int32, device="cuda")
    offset = torch.zeros(nc, dtype=torch.int64, device="cuda")
    n_out = torch.zeros(1, dtype=torch.int64, device="cuda")
    dm = frame.device_maps()
    # objects of earlier tests held in reference cycles must not be freed
    # between the measurements below
    gc.collect()
    torch.cuda.synchronize()
    before = free_bytes()
    alloc = torch.cuda.memory_allocated()

    def unchanged(what):
        f = free_bytes()
        say("%s: free memory %+d bytes, torch allocated %+d bytes" % (what, f - before,
                                                                       torch.cuda.memory_allocated() - alloc))
        assert f == before, what
        assert torch.cuda.memory_allocated() == alloc, what

    for v, cam in enumerate(views):
        api.render(ctx, g, cam, frame, gt=gts[v], image=image)
        unchanged("as_render view %d" % v)
        api.render_backward(ctx, g, cam, frame, dL, grads=grads, g2d_norm=g2d, vis_count=vis)
        unchanged("as_render_backward view %d" % v)
        api.accumulate_error_stats(ctx, W, H, dm["err"], dm["err_minmax"], dm["dom"], gts[v], v, is_cand_t, prm,
                                   regions, attr)
        unchanged("as_accumulate_error_stats view %d" % v)
    api.adaptive_split(ctx, g, cand_t, regions, views, attr, prm, noise, out=out, mode=mode, count=count,
                       offset=offset, n_out=n_out)
    unchanged("as_adaptive_split")
    assert 0 < int(n_out.item()) <= out.n
    assert frame.n_keys() <= 16 * n


def test_calls_beyond_the_reservation_are_refused():
    """Sizes above the reservation give AS_ERR_CAPACITY naming the field,
    and nothing is launched or allocated."""
    W, H, n = 64, 48, 500
    ctx = api.Context(0, max_pixels=W * H - 1, max_gaussians=n - 1, max_candidates=4, max_regions=16, max_views=1)
    scene = synth.scene_uniform_sh0(n, seed=4)
    g = api.Gaussians.from_scene(scene)
    cam = synth.sphere_cameras(1, 4.0, [(W, H)], seed=4)[0]
    frame = api.Frame(ctx, n, W, H)
    gt = torch.zeros(3, H, W, device="cuda")
    api.render(ctx, g, cam, frame, gt=gt)
    dm = frame.device_maps()
    regions = api.RegionBuffer(16)
    attr = torch.zeros(n, dtype=torch.int32, device="cuda")
    is_cand = torch.zeros(n, dtype=torch.uint8, device="cuda")
    before = free_bytes()
    with pytest.raises(api.AdpSplitError) as e:
        api.accumulate_error_stats(ctx, W, H, dm["err"], dm["err_minmax"], dm["dom"], gt, 0, is_cand,
                                   api.SplitParams(), regions, attr)
    assert e.value.status == api.AS_ERR_CAPACITY and "max_pixels" in str(e.value)
    with pytest.raises(api.AdpSplitError) as e:
        api.adaptive_split(ctx, g, torch.tensor([1], dtype=torch.int32, device="cuda"), regions, [cam], attr,
                           api.SplitParams(), torch.zeros(1, 2, 3, device="cuda"))
    assert e.value.status == api.AS_ERR_CAPACITY and "max_gaussians" in str(e.value)
    with pytest.raises(api.AdpSplitError) as e:
        api.densify_select(ctx, g, torch.zeros(n, device="cuda"), torch.zeros(n, dtype=torch.int32, device="cuda"),
                           1.0, 1.0)
    assert e.value.status == api.AS_ERR_CAPACITY
    ctx.reserve(max_pixels=W * H)
    api.accumulate_error_stats(ctx, W, H, dm["err"], dm["err_minmax"], dm["dom"], gt, 0, is_cand, api.SplitParams(),
                               regions, attr)
    torch.cuda.synchronize()
    assert free_bytes() <= before
