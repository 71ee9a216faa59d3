"""Render-request serving with continuous batching over resident scenes.

Scenes (Gaussian sets) stay resident on the device.  Requests (scene, camera,
arrival time) enter a FIFO queue when they arrive.  The server owns a fixed
number of slots; each slot is a stream plus the memory one batched render
needs (a batch frame of fixed entry / pixel / tile / pair capacity; output
images are allocated per request).  Whenever a slot is free, the oldest
waiting requests are
admitted into it for as long as their footprint fits the slot's memory (the
HBM budget is split over the slots up front, so admission is by footprint),
and the slot renders them as one batched launch (views of different scenes
and sizes together).  Requests that arrive while other batches are on the GPU
are admitted as soon as a slot frees up; the slots' streams overlap on the
device.  A request completes when its slot's completion event has fired;
latency is completion minus arrival.

Admission also bounds a batch's pairs: the scheduler keeps, per (scene,
resolution), an estimate of the pairs one render emits, learnt from the pair
counts of completed batches (each batch's count shared over its requests in
proportion to their estimates, or to Gaussians x pixels before any is
known), and admits a request only while the batch's estimated pairs stay
within a margin of the slot's pair capacity.  Under a tight budget this is
the limit that binds.  A batch whose pairs still overflow the slot (known
only after the render) is rendered again one view at a time in the slot's
own frame, on the slot's stream, without blocking the scheduler; a view that
overflows the slot alone (which no slot sized for a batch meets) is rendered
with a frame that grows on demand.  Every request gets the exact image.

The executor is separable: GpuExecutor renders with the library; the
scheduler logic (admission, batching, bookkeeping) runs the same with any
object providing the same methods (tests drive it with a simulated one).
"""
import collections
import math
import time

import numpy as np


class Request:
    __slots__ = ("rid", "scene", "cam", "arrival", "done", "image", "slot", "batch_size", "retried")

    def __init__(self, rid, scene, cam, arrival):
        self.rid, self.scene, self.cam, self.arrival = rid, scene, cam, arrival
        self.done = None
        self.image = None
        self.slot = None
        self.batch_size = 0
        self.retried = False

    @property
    def pixels(self):
        return self.cam.width * self.cam.height

    @property
    def tiles(self):
        return ((self.cam.width + 15) // 16) * ((self.cam.height + 15) // 16)


# Pair capacity of one slot at most: 2^29 pairs (8.8 GB of keys, values and
# sort buffers) hold a batch of eight 1920x1080 views of a 2M-Gaussian scene
# several times over; a larger budget buys no larger batch.
MAX_SLOT_PAIRS = 1 << 29


class SlotSpec:
    """Capacities of one slot (what one batched launch may use)."""

    def __init__(self, max_views, entries, pixels, tiles, pairs):
        self.max_views, self.entries, self.pixels, self.tiles, self.pairs = max_views, entries, pixels, tiles, pairs

    def bytes(self):
        """Device bytes the slot holds: its forward-only batch frame, as the
        library reports it (as_frame_bytes), plus its in-flight images."""
        from . import api
        frame = api.frame_bytes(self.max_views, self.entries, self.pixels, self.tiles, max(self.pairs, 1),
                                forward_only=True)
        return frame + 12 * self.pixels


def plan_slots(budget_bytes, n_slots, max_views, pixels_per_slot, entries_per_slot, tiles_per_slot):
    """Give each slot the largest pair capacity whose footprint (frame +
    images, from the library's size query) fits its share of the budget."""
    spec = SlotSpec(max_views, entries_per_slot, pixels_per_slot, tiles_per_slot, 1)
    share = budget_bytes // n_slots
    base = spec.bytes()
    probe = 1 << 20
    spec.pairs = 1 + probe
    per_pair = (spec.bytes() - base) / probe
    pairs = int((share - base) / per_pair) if share > base else 0
    if pairs <= 65536:
        raise ValueError("budget of %d bytes cannot hold %d slots" % (budget_bytes, n_slots))
    spec.pairs = int(min(pairs, MAX_SLOT_PAIRS))
    while spec.bytes() > share:
        spec.pairs -= 4096
    return spec


class Scheduler:
    """FIFO admission into free slots, by footprint (entries, pixels, tiles,
    and the estimated pairs within pair_margin of the slot's capacity).
    keep_images=False drops each image once its request completes (a server
    hands it over; a long run would otherwise hold every image)."""

    def __init__(self, executor, spec, scene_sizes, pair_margin=0.9, keep_images=True):
        self.ex = executor
        self.spec = spec
        self.scene_sizes = scene_sizes
        self.pair_margin, self.keep_images = pair_margin, keep_images
        self.queue = collections.deque()
        self.free = list(range(executor.n_slots))
        self.busy = {}                     # slot -> list of requests
        self.completed = []
        self.batches = 0
        self.pair_est = {}                 # (scene, width, height) -> pairs of one render
        self.pair_bound = 0                # batches closed by the pair estimate

    def _key(self, r):
        return (r.scene, r.cam.width, r.cam.height)

    def est_pairs(self, r):
        return self.pair_est.get(self._key(r), 0.0)

    def learn(self, batch, pairs):
        """Share a batch's measured pair count over its requests and fold
        each share into its (scene, resolution) estimate."""
        known = all(self._key(r) in self.pair_est for r in batch)
        w = [self.est_pairs(r) if known else float(self.scene_sizes[r.scene]) * r.pixels for r in batch]
        tot = sum(w)
        for r, wi in zip(batch, w):
            share = pairs * wi / tot if tot > 0 else pairs / len(batch)
            k = self._key(r)
            self.pair_est[k] = share if k not in self.pair_est else 0.75 * self.pair_est[k] + 0.25 * share

    def fits(self, batch, r):
        if len(batch) + 1 > self.spec.max_views:
            return False
        ent = sum(self.scene_sizes[q.scene] for q in batch) + self.scene_sizes[r.scene]
        px = sum(q.pixels for q in batch) + r.pixels
        tl = sum(q.tiles for q in batch) + r.tiles
        if not (ent <= self.spec.entries and px <= self.spec.pixels and tl <= self.spec.tiles):
            return False
        if batch and sum(self.est_pairs(q) for q in batch) + self.est_pairs(r) > self.pair_margin * self.spec.pairs:
            self.pair_bound += 1
            return False
        return True

    def admit(self, r):
        if not self.fits([], r):
            raise ValueError("request %d alone exceeds a slot" % r.rid)
        self.queue.append(r)

    def launch_ready(self):
        """Fill every free slot from the head of the queue."""
        while self.free and self.queue:
            slot = self.free.pop(0)
            batch = [self.queue.popleft()]
            while self.queue and self.fits(batch, self.queue[0]):
                batch.append(self.queue.popleft())
            for r in batch:
                r.slot, r.batch_size = slot, len(batch)
            self.ex.launch(slot, batch)
            self.busy[slot] = batch
            self.batches += 1

    def poll(self, now_fn):
        """Retire finished slots; returns the number of requests completed.
        The executor's retire returns (done, pairs): the batch's measured
        pair count (None if unknown), and done = False when it has launched
        the batch again (an overflow) and the slot stays busy."""
        n = 0
        for slot in list(self.busy):
            if self.ex.finished(slot):
                batch = self.busy[slot]
                res = self.ex.retire(slot, batch)
                done, pairs = (True, None) if res is None else res
                if pairs is not None:
                    self.learn(batch, pairs)
                if not done:
                    continue
                del self.busy[slot]
                t = now_fn()
                for r in batch:
                    r.done = t
                    if not self.keep_images:
                        r.image = None
                self.completed.extend(batch)
                self.free.append(slot)
                n += len(batch)
        return n

    def idle(self):
        return not self.queue and not self.busy


def serve_open_loop(sched, requests, clock=time.perf_counter, spin=None):
    """Replay `requests` (sorted by arrival, seconds from the start) against
    the scheduler in real time; returns when all have completed."""
    t0 = clock()
    now = lambda: clock() - t0
    i, n = 0, len(requests)
    while len(sched.completed) < n:
        t = now()
        while i < n and requests[i].arrival <= t:
            sched.admit(requests[i])
            i += 1
        sched.launch_ready()
        sched.poll(now)
        if spin is not None:
            spin()
    return now()


def serve_sequential(ex, requests, clock=time.perf_counter, keep_images=True):
    """The plain loop: one request at a time, in arrival order, each
    rendered alone as soon as it has arrived and the previous one is done."""
    t0 = clock()
    now = lambda: clock() - t0
    for r in requests:
        while now() < r.arrival:
            pass
        ex.render_one(r)
        r.done = now()
        if not keep_images:
            r.image = None
    return now()


def latency_stats(requests, wall_s):
    lat = np.array([r.done - r.arrival for r in requests]) * 1e3
    px = sum(r.pixels for r in requests)
    return dict(requests=len(requests), p50_ms=round(float(np.percentile(lat, 50)), 3),
                p99_ms=round(float(np.percentile(lat, 99)), 3), mean_ms=round(float(lat.mean()), 3),
                max_ms=round(float(lat.max()), 3), wall_s=round(wall_s, 4),
                mpix_s=round(px / wall_s / 1e6, 2), req_s=round(len(requests) / wall_s, 2))


def poisson_requests(n, rate, n_scenes, sizes, cam_fn, seed):
    """n requests with exponential inter-arrival times (rate per second),
    uniform scene and resolution choices; cam_fn(rng, W, H) makes the pose."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, size=n)) if rate else np.zeros(n)
    out = []
    for k in range(n):
        W, H = sizes[rng.integers(len(sizes))]
        out.append(Request(k, int(rng.integers(n_scenes)), cam_fn(rng, W, H), float(t[k])))
    return out


class GpuExecutor:
    """Slots backed by the library: a stream, a batch frame that never
    synchronises and a pair-count mailbox per slot.  Each request's image is
    allocated on its slot's stream when the batch is launched and handed to
    the caller when it completes."""

    def __init__(self, ctx, scenes, spec, n_slots):
        import torch

        from . import api
        self.api, self.torch = api, torch
        self.ctx, self.scenes, self.spec, self.n_slots = ctx, scenes, spec, n_slots
        self.streams = [torch.cuda.Stream() for _ in range(n_slots)]
        self.frames = [api.BatchFrame(ctx, spec.max_views, spec.entries, spec.pixels, spec.tiles, spec.pairs,
                                      auto_grow=False, forward_only=True) for _ in range(n_slots)]
        # one pair count per view: the batch's in [0], each single's after an overflow
        self.count_dev = [torch.zeros(spec.max_views, dtype=torch.int32, device="cuda") for _ in range(n_slots)]
        self.count_host = [torch.zeros(spec.max_views, dtype=torch.int32).pin_memory() for _ in range(n_slots)]
        self.events = [None] * n_slots
        self.retrying = [False] * n_slots
        self.single = {}
        self.overflows = 0          # batches rendered again view by view
        self.single_overflows = 0   # views that overflowed the slot alone

    def _finish_launch(self, slot):
        torch = self.torch
        s = self.streams[slot]
        self.count_host[slot].copy_(self.count_dev[slot], non_blocking=True)
        ev = torch.cuda.Event()
        ev.record(s)
        self.events[slot] = ev

    def launch(self, slot, batch):
        torch, api = self.torch, self.api
        s = self.streams[slot]
        with torch.cuda.stream(s):
            imgs = [torch.empty(3, r.cam.height, r.cam.width, dtype=torch.float32, device="cuda") for r in batch]
            api.render_batch(self.ctx, [self.scenes[r.scene] for r in batch], [r.cam for r in batch],
                             self.frames[slot], images=imgs)
            self.frames[slot].pair_count_async(self.count_dev[slot][0:1])
            for r, im in zip(batch, imgs):
                r.image = im
            self._finish_launch(slot)

    def finished(self, slot):
        return self.events[slot].query()

    def _count(self, slot, k):
        return int(self.count_host[slot][k]) & 0xFFFFFFFF

    def retire(self, slot, batch):
        """(done, pairs).  A batch whose pairs overflowed the slot is launched
        again one view at a time in the slot's frame on the slot's stream
        (done = False: the slot stays busy); when those have finished, a view
        that overflowed alone is rendered with a growing frame."""
        torch, api = self.torch, self.api
        if self.retrying[slot]:
            self.retrying[slot] = False
            for k, r in enumerate(batch):
                if self._count(slot, k) > self.spec.pairs:
                    self.single_overflows += 1
                    self.render_one(r)
            return True, None
        pairs = self._count(slot, 0)
        if pairs <= self.spec.pairs:
            return True, pairs
        self.overflows += 1
        s = self.streams[slot]
        with torch.cuda.stream(s):
            for k, r in enumerate(batch):
                api.render_batch(self.ctx, [self.scenes[r.scene]], [r.cam], self.frames[slot], images=[r.image])
                self.frames[slot].pair_count_async(self.count_dev[slot][k:k + 1])
                r.retried = True
            self._finish_launch(slot)
        self.retrying[slot] = True
        return False, pairs

    def render_one(self, r):
        torch, api = self.torch, self.api
        key = (r.scene, r.cam.width, r.cam.height)
        f = self.single.get(key)
        if f is None:
            f = api.Frame(self.ctx, self.scenes[r.scene].n, r.cam.width, r.cam.height, auto_grow=True,
                          forward_only=True)
            self.single[key] = f
        r.image = api.render(self.ctx, self.scenes[r.scene], r.cam, f)
        torch.cuda.current_stream().synchronize()

    def close(self):
        for f in self.frames + list(self.single.values()):
            f.close()


def hbm_footprint(scenes, spec, n_slots):
    """Device bytes held by the resident scenes and the slots."""
    sc = sum(4 * (g.means.numel() + g.log_scales.numel() + g.quats.numel() + g.opacity_logits.numel() +
                  g.sh.numel()) for g in scenes)
    return dict(scenes_bytes=int(sc), slots_bytes=int(n_slots * spec.bytes()), total_bytes=int(sc + n_slots * spec.bytes()))


def default_spec(scene_sizes, sizes, max_views, budget_bytes, n_slots, fixed_share=0.5):
    """Slot capacities for max_views views of the largest size and scene; if
    that worst case's entry / pixel / tile buffers would take more than
    fixed_share of a slot's share of the budget, they are scaled down (to no
    less than one largest request), so the pair capacity keeps the rest and
    admission by footprint binds on entries and pixels instead."""
    W, H = max(sizes, key=lambda s: s[0] * s[1])
    one_px, one_tiles, one_ent = W * H, math.ceil(W / 16) * math.ceil(H / 16), max(scene_sizes)
    px, tiles, ent = max_views * one_px, max_views * one_tiles, max_views * one_ent
    fixed = SlotSpec(max_views, ent, px, tiles, 1).bytes()
    share = budget_bytes // n_slots
    if fixed > fixed_share * share:
        f = fixed_share * share / fixed
        px, tiles, ent = max(one_px, int(px * f)), max(one_tiles, int(tiles * f)), max(one_ent, int(ent * f))
    return plan_slots(budget_bytes, n_slots, max_views, px, ent, tiles)
