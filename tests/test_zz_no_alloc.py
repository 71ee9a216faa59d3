"""The no-allocation error statistics (as_accumulate_error_stats_noalloc,
scratch in the library's static device array) against the context-scratch
call (as_accumulate_error_stats) through the C-ABI: two calls in a row, the
second on a smaller view, region records and attribution counts bit-identical,
no device memory taken by either call, and a view above the static maximum
refused before anything is launched."""
import sys

import numpy as np
import pytest

from paper_2605_06876_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2605_06876_amd import api  # noqa: E402


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def free_bytes():
    torch.cuda.synchronize()
    return torch.cuda.mem_get_info(0)[0]


def test_noalloc_error_stats_match_the_reserved_call():
    # a small warm-up view (the runtime's own first-use set-up happens there),
    # then the benchmark's 1256x828 view (within the static maximum) and a
    # smaller one
    cases = [(64, 64, 40, 30, 1), (828, 1256, 5000, 31, 2), (200, 333, 300, 32, 1)]
    assert 828 * 1256 <= api.NOALLOC_MAX_PIXELS
    inputs = []
    for H, W, n, seed, r in cases:
        img, gt, dom, is_cand = synth.error_map_fixture(H, W, n, seed=seed, n_sites=max(50, H * W // 800),
                                                        n_blobs=max(30, H * W // 2000))
        inputs.append((H, W, n, r, torch.from_numpy(img).cuda(), torch.from_numpy(gt).cuda(),
                       torch.from_numpy(dom).cuda(), torch.from_numpy(is_cand).cuda()))
    # the reserved call's context; the no-allocation call needs no reservation
    ctx_res = api.Context(0, max_pixels=max(H * W for H, W, *_ in cases))
    ctx_na = api.Context(0)
    maps = [api.error_map(ctx_res, it[4], it[5]) for it in inputs]
    n_max = max(it[2] for it in inputs)
    cap = max(H * W for H, W, *_ in cases) // 5
    reg_res, reg_na = api.RegionBuffer(2 * cap), api.RegionBuffer(2 * cap)
    attr_res = torch.zeros(n_max, dtype=torch.int32, device="cuda")
    attr_na = torch.zeros(n_max, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    for v, ((H, W, n, r, img, gt, dom, is_cand), (err, mm)) in enumerate(zip(inputs, maps)):
        say("no-alloc: view %d, %dx%d, %d Gaussians, r_erode %d" % (v, W, H, n, r))
        prm = api.SplitParams(r_erode=r)
        f0 = free_bytes()
        api.accumulate_error_stats(ctx_res, W, H, err, mm, dom, gt, v, is_cand, prm, reg_res, attr_res[:n])
        f1 = free_bytes()
        api.accumulate_error_stats_noalloc(ctx_na, W, H, err, mm, dom, gt, v, is_cand, prm, reg_na, attr_na[:n])
        f2 = free_bytes()
        say("no-alloc: free memory change %+d (reserved call), %+d (no-allocation call)" % (f1 - f0, f2 - f1))
        if v > 0:
            assert f2 == f1 == f0
        a, b = reg_res.host(), reg_na.host()
        say("no-alloc: %d regions after view %d" % (len(a), v))
        assert len(a) == len(b) and len(a) > 0
        assert a.tobytes() == b.tobytes()
        assert torch.equal(attr_res, attr_na)
    # above the static maximum: refused with AS_ERR_CAPACITY, nothing launched
    W, H = 1025, 1024
    assert W * H > api.NOALLOC_MAX_PIXELS
    big = torch.zeros(H * W, dtype=torch.float64, device="cuda")
    with pytest.raises(api.AdpSplitError) as e:
        api.accumulate_error_stats_noalloc(ctx_na, W, H, big, maps[0][1], torch.zeros(H * W, dtype=torch.int32,
                                           device="cuda"), torch.zeros(3, H, W, device="cuda"), 0,
                                           inputs[0][7], api.SplitParams(), reg_na, attr_na)
    assert e.value.status == api.AS_ERR_CAPACITY and "maximum" in str(e.value)
    assert reg_na.host().tobytes() == reg_res.host().tobytes()
