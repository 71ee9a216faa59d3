"""Serving on the GPU: every request's image is the same whether it was
rendered in a batch with others (views of different scenes and sizes, slots
overlapping on separate streams) or alone (bit-identical; the stated image
tolerance is 1e-4), including batches that overflow the slot's pair
capacity and are rendered again one view at a time."""
import sys

import numpy as np
import pytest

from paper_2605_06876_amd import serve, synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2605_06876_amd import api  # noqa: E402


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


SIZES = [(64, 48), (96, 80), (128, 96), (40, 130)]


@pytest.fixture(scope="module")
def scenes():
    out = []
    for k, n in enumerate((3000, 8000, 20000)):
        s = synth.scene_clusters(n, seed=300 + k, sh_degree=3, log_scale_mu=-3.8, log_scale_sd=0.5)
        out.append(api.Gaussians.from_scene(s))
    return out


def alone(ctx, g, cam):
    f = api.Frame(ctx, g.n, cam.width, cam.height)
    img = api.render(ctx, g, cam, f)
    torch.cuda.synchronize()
    f.close()
    return img


@pytest.mark.parametrize("n_slots,pairs", [(2, None), (3, 20000)])
def test_served_images_equal_single_renders(scenes, n_slots, pairs):
    ctx = api.Context(0)
    sizes = [g.n for g in scenes]
    spec = serve.default_spec(sizes, SIZES, 4, 2 << 30, n_slots)
    if pairs is not None:   # small pair capacity: some batches overflow and are rendered again
        spec.pairs = pairs
    ex = serve.GpuExecutor(ctx, scenes, spec, n_slots)
    reqs = serve.poisson_requests(40, 4000.0, len(scenes), SIZES,
                                  lambda rng, w, h: synth.random_pose_camera(rng, 3.5, w, h), seed=11)
    sched = serve.Scheduler(ex, spec, sizes)
    wall = serve.serve_open_loop(sched, reqs)
    torch.cuda.synchronize()
    st = serve.latency_stats(sched.completed, wall)
    say("slots %d: %d batches, %d overflows, p50 %.3f ms p99 %.3f ms" % (n_slots, sched.batches, ex.overflows,
                                                                       st["p50_ms"], st["p99_ms"]))
    assert len(sched.completed) == 40
    assert sched.batches < 40
    if pairs is not None:
        assert ex.overflows > 0
    for r in reqs:
        ref = alone(ctx, scenes[r.scene], r.cam)
        assert r.image.shape == ref.shape
        assert torch.equal(r.image, ref), "request %d (scene %d, %dx%d, batch of %d)" % (
            r.rid, r.scene, r.cam.width, r.cam.height, r.batch_size)
    ex.close()


def test_sequential_loop_matches_too(scenes):
    ctx = api.Context(0)
    sizes = [g.n for g in scenes]
    spec = serve.default_spec(sizes, SIZES, 4, 1 << 30, 1)
    ex = serve.GpuExecutor(ctx, scenes, spec, 1)
    reqs = serve.poisson_requests(10, 0.0, len(scenes), SIZES,
                                  lambda rng, w, h: synth.random_pose_camera(rng, 3.5, w, h), seed=12)
    serve.serve_sequential(ex, reqs)
    for r in reqs:
        assert torch.equal(r.image, alone(ctx, scenes[r.scene], r.cam))
    ex.close()
