"""Serving scheduler (continuous batching, admission by footprint) driven by
a simulated executor on the CPU.  The GPU executor's results are checked
against single-view renders in test_gpu_serve.py."""
import numpy as np
import pytest

from paper_2605_06876_amd import serve


class Cam:
    def __init__(self, w, h):
        self.width, self.height = w, h


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


class FakeExecutor:
    """Batches take overhead + per-pixel time of a simulated clock; slots run
    concurrently (the device shares nothing in this model)."""

    def __init__(self, clock, n_slots, overhead=2e-3, per_px=1e-9):
        self.clock, self.n_slots, self.overhead, self.per_px = clock, n_slots, overhead, per_px
        self.end = {}
        self.launches = []
        self.in_flight_max = 0

    def launch(self, slot, batch):
        assert slot not in self.end, "slot reused before it finished"
        self.end[slot] = self.clock() + self.overhead + self.per_px * sum(r.pixels for r in batch)
        self.launches.append((self.clock(), slot, [r.rid for r in batch]))
        self.in_flight_max = max(self.in_flight_max, len(self.end))

    def finished(self, slot):
        return self.clock() >= self.end[slot]

    def retire(self, slot, batch):
        del self.end[slot]
        for r in batch:
            r.image = ("image", r.rid)

    def render_one(self, r):
        self.clock.t += self.overhead + self.per_px * r.pixels
        r.image = ("image", r.rid)


SIZES = [(640, 480), (1280, 720), (1920, 1080)]
SCENES = [300_000, 600_000, 1_200_000, 2_000_000]


def make(n, rate, seed=0):
    return serve.poisson_requests(n, rate, len(SCENES), SIZES, lambda rng, w, h: Cam(w, h), seed)


def spec(max_views=8):
    return serve.default_spec(SCENES, SIZES, max_views, 48 << 30, 2)


def run(reqs, n_slots=2, sp=None, step=1e-4):
    clock = FakeClock()
    ex = FakeExecutor(clock, n_slots)
    sp = sp or spec()
    sched = serve.Scheduler(ex, sp, SCENES)

    def spin():
        clock.t += step
    wall = serve.serve_open_loop(sched, reqs, clock=clock, spin=spin)
    return sched, ex, wall


def test_every_request_completes_once_within_slot_capacity():
    reqs = make(400, 2000.0)
    sched, ex, wall = run(reqs)
    assert sorted(r.rid for r in sched.completed) == list(range(400))
    sp = spec()
    for _, slot, rids in ex.launches:
        batch = [reqs[i] for i in rids]
        assert len(batch) <= sp.max_views
        assert sum(SCENES[r.scene] for r in batch) <= sp.entries
        assert sum(r.pixels for r in batch) <= sp.pixels
        assert sum(r.tiles for r in batch) <= sp.tiles
    assert all(r.done >= r.arrival for r in reqs)
    assert ex.in_flight_max <= 2


def test_fifo_admission_order():
    reqs = make(300, 5000.0, seed=3)
    sched, ex, _ = run(reqs)
    order = [i for _, _, rids in ex.launches for i in rids]
    assert order == sorted(order), "requests must be launched in arrival order"


class CheckedScheduler(serve.Scheduler):
    """Asserts the work-conserving invariant after every launch round: no
    slot stays free while requests wait."""

    def launch_ready(self):
        super().launch_ready()
        assert not (self.free and self.queue)


def test_arrivals_during_busy_slots_join_the_next_free_slot():
    # a burst of 20 at t=0, then stragglers while both slots are busy
    reqs = make(20, 0.0)
    late = make(6, 0.0, seed=9)
    for k, r in enumerate(late):
        r.rid, r.arrival = 20 + k, 1e-3 + 1e-4 * k
    clock = FakeClock()
    ex = FakeExecutor(clock, 2)
    sched = CheckedScheduler(ex, spec(), SCENES)

    def spin():
        clock.t += 1e-4
    serve.serve_open_loop(sched, reqs + late, clock=clock, spin=spin)
    assert sorted(r.rid for r in sched.completed) == list(range(26))
    launch_of = {rid: t for t, _, rids in ex.launches for rid in rids}
    # stragglers were admitted while earlier batches were still running
    assert any(launch_of[r.rid] < max(q.done for q in reqs) for r in late)
    assert len(ex.launches) < 26, "requests are batched"


def test_batching_beats_the_sequential_loop_under_load():
    reqs = make(200, 4000.0, seed=5)
    sched, ex, wall = run(reqs)
    st = serve.latency_stats(sched.completed, wall)
    clock = FakeClock()
    seq = [serve.Request(r.rid, r.scene, r.cam, r.arrival) for r in reqs]
    # sequential loop on the simulated clock
    fx = FakeExecutor(clock, 1)
    for r in seq:
        clock.t = max(clock.t, r.arrival)
        fx.render_one(r)
        r.done = clock.t
    st_seq = serve.latency_stats(seq, clock.t)
    assert st["mpix_s"] > st_seq["mpix_s"]
    assert st["p99_ms"] < st_seq["p99_ms"]


def test_admission_by_footprint():
    sp = serve.plan_slots(8 << 30, 2, 4, 4 * 1920 * 1080, 4 * 2_000_000, 4 * 120 * 68)
    assert 2 * sp.bytes() <= 8 << 30
    with pytest.raises(ValueError):
        serve.plan_slots(1 << 28, 2, 4, 4 * 1920 * 1080, 4 * 2_000_000, 4 * 120 * 68)
    tiny = serve.SlotSpec(2, 1_000_000, 1920 * 1080, 8160, 1 << 20)
    sched = serve.Scheduler(FakeExecutor(FakeClock(), 1), tiny, SCENES)
    big = serve.Request(0, 3, Cam(640, 480), 0.0)      # 2M Gaussians > 1M entries
    with pytest.raises(ValueError):
        sched.admit(big)


class PairExecutor(FakeExecutor):
    """Reports each batch's pair count (per request a fixed function of its
    scene and resolution); a batch over the slot's pair capacity is rendered
    again one view at a time (the slot stays busy) before it completes."""

    def __init__(self, clock, n_slots, pairs_of, cap):
        super().__init__(clock, n_slots)
        self.pairs_of, self.cap = pairs_of, cap
        self.again, self.overflows, self.batch_pairs = set(), 0, []

    def retire(self, slot, batch):
        pairs = sum(self.pairs_of(r) for r in batch)
        if slot in self.again:
            self.again.discard(slot)
            del self.end[slot]
            for r in batch:
                r.image = ("image", r.rid)
            return True, None
        self.batch_pairs.append((pairs, [r.rid for r in batch]))
        if pairs > self.cap:
            self.again.add(slot)
            self.overflows += 1
            self.end[slot] = self.clock() + self.overhead * len(batch)
            return False, pairs
        del self.end[slot]
        for r in batch:
            r.image = ("image", r.rid)
        return True, pairs


def test_admission_learns_pairs_and_overflows_retry_on_the_slot():
    reqs = make(600, 3000.0, seed=21)
    pairs_of = lambda r: SCENES[r.scene] * r.pixels // 100_000     # up to 41M pairs per view
    sp = spec()
    sp.pairs = 60_000_000
    clock = FakeClock()
    ex = PairExecutor(clock, 2, pairs_of, sp.pairs)
    sched = serve.Scheduler(ex, sp, SCENES, keep_images=False)

    def spin():
        clock.t += 1e-4
    serve.serve_open_loop(sched, reqs, clock=clock, spin=spin)
    assert sorted(r.rid for r in sched.completed) == list(range(600))
    assert all(r.image is None for r in reqs)
    # estimates are exact once a (scene, resolution) has been seen, since
    # the first shares follow Gaussians x pixels, which the pairs do here
    for (sc, w, h), est in sched.pair_est.items():
        assert est == pytest.approx(SCENES[sc] * w * h // 100_000, rel=1e-6)
    assert sched.pair_bound > 0, "the pair estimate must limit some batches"
    seen = set()
    for pairs, rids in ex.batch_pairs:
        keys = {(reqs[i].scene, reqs[i].cam.width, reqs[i].cam.height) for i in rids}
        if keys <= seen:
            assert pairs <= 0.9 * sp.pairs or len(rids) == 1
        seen |= keys
    assert 0 < ex.overflows <= 12     # only batches holding a resolution/scene not seen before


def test_latency_stats():
    reqs = [serve.Request(k, 0, Cam(100, 100), 0.0) for k in range(100)]
    for k, r in enumerate(reqs):
        r.done = (k + 1) * 1e-3
    st = serve.latency_stats(reqs, 0.1)
    assert st["p50_ms"] == pytest.approx(50.5)
    assert st["max_ms"] == pytest.approx(100.0)
    assert st["mpix_s"] == pytest.approx(100 * 10000 / 0.1 / 1e6)
