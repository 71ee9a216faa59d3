"""Autotuner for the launch choices of the rasterizer (as_tuning).

The tuning never changes results: the forward image, counts and dominant map
are bit-identical across tunings (each pixel runs the same operations in the
same order, and every radix width gives the same stable order), and the
backward differs only in the order of its float atomics.  For a workload the
tuner times the caller's own step (a render + backward by default) for every
blend configuration (LDS depth x tile order x persistent grid), then for the
binning square (16 or 32 pixels: the tile size of the pair lists; the blend
tiles stay 16 x 16), then for the tile order and persistent grid again with
that binning, then for every radix digit width, then for the sorts'
launch structure (one launch per digit or three, for the depth and the pair
sort), each with the best choices so far, and keeps the fastest
(the better of two interleaved rounds per candidate, after a warm-up).
Results are cached in a JSON file keyed by the workload.
"""
import json
import math
import os

import torch

from . import api

BLEND_CANDIDATES = [dict(lds_batch=b, longest_first=l, persistent=p)
                    for b in (256, 512, 1024) for l in (True, False) for p in (False, True)]
RADIX_CANDIDATES = (5, 6, 7, 8)
DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "adpsplit_tuning.json")


def workload_key(width, height, n, sh_degree, views=1, arch="gfx950"):
    mp_bucket = round(width * height / 250_000) / 4          # quarter-megapixel buckets
    n_bucket = max(0, round(math.log2(max(n, 1))))           # powers of two
    return "%s|%.2fMpx|n2^%d|sh%d|v%d" % (arch, mp_bucket, n_bucket, sh_degree, views)


SORT_CANDIDATES = (0, 1, 2, 3)   # single-pass sorts: neither, depth only, pairs only, both
BIN_CANDIDATES = (16, 32)        # pixels per side of the pair binning squares


def name_of(t):
    return "batch%d_%s_%s_bin%d_r%d_sp%d" % (t["lds_batch"], "lpt" if t["longest_first"] else "grid",
                                             "persistent" if t["persistent"] else "blocks", t.get("bin_tile", 16),
                                             t["radix_bits"], t.get("single_pass_sort", 0))


def time_step(run, reps):
    """Mean milliseconds of run() over reps calls (after one untimed call)."""
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    run()
    torch.cuda.synchronize()
    ev0.record()
    for _ in range(reps):
        run()
    ev1.record()
    torch.cuda.synchronize()
    return ev0.elapsed_time(ev1) / reps


def _load(cache_path):
    if cache_path and os.path.exists(cache_path):
        try:
            with open(cache_path) as f:
                return json.load(f)
        except (OSError, ValueError):
            pass
    return {}


def autotune_step(ctx, run, key, reps=5, cache_path=DEFAULT_CACHE, use_cache=True):
    """Pick and set the fastest tuning for the step run(); returns
    (tuning dict, {candidate name: ms})."""
    cache = _load(cache_path)
    if use_cache and key in cache:
        best = cache[key]["tuning"]
        api.set_tuning(ctx, **best)
        return best, cache[key].get("ms", {})
    times = {}
    # Warm the device first (clocks, the library's first-use allocations), and
    # keep the better of two interleaved rounds per candidate, so the first
    # candidates are not timed cold.
    for _ in range(3):
        run()
    torch.cuda.synchronize()

    def rounds(cands):
        for _ in range(2):
            for t in cands:
                api.set_tuning(ctx, **t)
                ms = time_step(run, reps)
                times[name_of(t)] = min(times.get(name_of(t), float("inf")), ms)
        return min(cands, key=lambda t: times[name_of(t)])

    best = rounds([dict(c, radix_bits=8, single_pass_sort=0, bin_tile=16) for c in BLEND_CANDIDATES])
    best = rounds([dict(best, bin_tile=bt) for bt in BIN_CANDIDATES])
    # the dispatch again, with the chosen binning: with bins of 32 the
    # longest-first order also groups a bin's four tiles on one XCD, which the
    # first round (bins of 16) cannot see
    best = rounds([dict(best, longest_first=l, persistent=p) for l in (True, False) for p in (False, True)])
    best = rounds([dict(best, radix_bits=rb) for rb in RADIX_CANDIDATES])
    best = rounds([dict(best, single_pass_sort=sp) for sp in SORT_CANDIDATES])
    api.set_tuning(ctx, **best)
    if cache_path:
        cache[key] = dict(tuning=best, ms=times)
        try:
            os.makedirs(os.path.dirname(cache_path), exist_ok=True)
            with open(cache_path, "w") as f:
                json.dump(cache, f, indent=1)
        except OSError:
            pass
    return best, times


def autotune(ctx, g, cam, frame, gt=None, dL=None, reps=5, cache_path=DEFAULT_CACHE, use_cache=True):
    """Tune for one view: the step is a render (with the target, if given)
    and its backward."""
    if dL is None:
        dL = torch.full((3, cam.height, cam.width), 1.0 / (3 * cam.width * cam.height), device="cuda")

    def run():
        api.render(ctx, g, cam, frame, gt=gt)
        api.render_backward(ctx, g, cam, frame, dL)

    return autotune_step(ctx, run, workload_key(cam.width, cam.height, g.n, g.sh_degree), reps, cache_path, use_cache)
