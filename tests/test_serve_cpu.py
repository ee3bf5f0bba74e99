"""The serving scheduler with a fake renderer on a simulated clock: budget admission, slot release and
overlap, no starvation, and failures isolated to one request."""
import pytest

from paper_1702_01530_amd.serve import Renderer, Request, Server, latency_stats


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


class FakeRenderer(Renderer):
    """A request's `camera` is its size: it needs that many bytes and that many paths; a batch finishes
    `per_path` seconds per path after launch."""

    def __init__(self, clock, slots=2, per_path=1e-3, fail_rids=(), fail_launch=False):
        self.clock, self.slots, self.per_path = clock, slots, per_path
        self.fail_rids, self.fail_launch = set(fail_rids), fail_launch
        self.launched = []

    def bytes_needed(self, req):
        return req.camera

    def paths(self, req):
        return req.camera

    def validate(self, req):
        return "unknown scene" if req.scene_id == "bad" else None

    def launch(self, slot, reqs):
        if self.fail_launch:
            raise RuntimeError("device lost")
        self.launched.append((slot, [r.rid for r in reqs], self.clock()))
        return (self.clock() + self.per_path * sum(r.camera for r in reqs), reqs)

    def poll(self, h):
        return self.clock() >= h[0]

    def collect(self, h):
        return [(("image", r.rid), "render failed" if r.rid in self.fail_rids else None) for r in h[1]]


def drive(server, clock, dt=1e-3, limit=100000):
    for _ in range(limit):
        server.step()
        assert server.in_use <= server.budget
        if server.idle():
            return
        clock.t += dt
    raise AssertionError("did not drain")


def test_budget_respected_and_everything_completes():
    clock = Clock()
    r = FakeRenderer(clock)
    s = Server(r, hbm_budget=100, max_batch_paths=60, clock=clock)
    for i in range(40):
        s.submit(Request(i, "a", 5 + (i * 7) % 30))
    drive(s, clock)
    assert len(s.completed) == 40 and all(q.error is None for q in s.completed)
    assert s.peak_in_use <= 100 and s.in_use == 0
    assert all(sum(5 + (rid * 7) % 30 for rid in ids) <= 60 for _, ids, _ in r.launched)


def test_requests_arriving_during_a_batch_start_in_another_slot():
    clock = Clock()
    r = FakeRenderer(clock, slots=2, per_path=1e-2)
    s = Server(r, hbm_budget=1000, max_batch_paths=100, clock=clock)
    s.submit(Request(0, "a", 50))
    s.step()
    assert len(s.inflight) == 1
    clock.t += 0.1  # batch 0 still running (finishes at 0.5)
    s.submit(Request(1, "a", 10))
    s.submit(Request(2, "a", 10))
    s.step()
    assert len(s.inflight) == 2  # admitted while the first batch is on the device: the work overlaps
    assert r.launched[1][1] == [1, 2] and r.launched[1][2] < 0.5
    drive(s, clock)
    done = {q.rid: q for q in s.completed}
    assert done[1].done < done[0].done  # the later, smaller batch finished first
    # a slot is reused once its batch completes
    s.submit(Request(3, "a", 10))
    drive(s, clock)
    assert r.launched[-1][1] == [3]


def test_head_of_line_request_does_not_starve():
    clock = Clock()
    r = FakeRenderer(clock, slots=1, per_path=1e-3)
    s = Server(r, hbm_budget=100, max_batch_paths=100, max_bypass=2, clock=clock)
    s.submit(Request(0, "a", 60))
    s.step()  # occupies 60 of 100
    s.submit(Request(1, "a", 70))  # cannot fit until request 0 completes
    for i in range(2, 30):
        s.submit(Request(i, "a", 10))
    rounds = 0
    while not any(q.rid == 1 for q in s.completed):
        s.step()
        clock.t += 1e-3
        s.submit(Request(100 + rounds, "a", 10))  # small requests keep arriving
        rounds += 1
        assert rounds < 5000
    # request 1 was overtaken by at most max_bypass batches
    pos = [i for i, (_, ids, _) in enumerate(r.launched) if 1 in ids][0]
    assert pos <= 1 + 2 + 1


def test_a_failing_request_fails_alone():
    clock = Clock()
    r = FakeRenderer(clock, fail_rids={3})
    s = Server(r, hbm_budget=1000, max_batch_paths=1000, clock=clock)
    for i in range(6):
        s.submit(Request(i, "a", 10))
    s.submit(Request(6, "bad", 10))  # rejected at submission
    s.submit(Request(7, "a", 10 ** 6))  # larger than the whole budget: rejected
    drive(s, clock)
    errs = {q.rid: q.error for q in s.completed}
    assert errs[3] == "render failed" and errs[6] and errs[7]
    assert all(errs[i] is None for i in (0, 1, 2, 4, 5))
    stats = latency_stats(s.completed)
    assert stats["n"] == 5 and stats["errors"] == 3 and stats["p99_ms"] >= stats["p50_ms"]


def test_failed_launch_frees_the_slot_and_budget():
    clock = Clock()
    r = FakeRenderer(clock, fail_launch=True)
    s = Server(r, hbm_budget=100, max_batch_paths=100, clock=clock)
    s.submit(Request(0, "a", 30))
    s.step()
    assert s.completed[0].error.startswith("launch failed") and s.in_use == 0
    assert sorted(s.free_slots) == [0, 1]
    r.fail_launch = False
    s.submit(Request(1, "a", 30))
    drive(s, clock)
    assert s.completed[-1].error is None


def test_run_plays_back_arrivals():
    clock = Clock()
    r = FakeRenderer(clock, per_path=1e-4)

    class Ticking(Clock):
        pass

    t = {"v": 0.0}

    def tick():
        t["v"] += 1e-4
        return t["v"]

    r.clock = tick
    s = Server(r, hbm_budget=500, max_batch_paths=200, clock=tick)
    arrivals = [(0.001 * i, Request(i, "a", 20)) for i in range(50)]
    done = s.run(arrivals)
    assert len(done) == 50 and all(q.latency >= 0 for q in done)


def test_cost_classes_go_out_in_separate_batches():
    """With group_ratio, a batch takes only requests within that factor of its first request's cost; the others
    start in another free slot of the same step."""
    clock = Clock()
    r = FakeRenderer(clock, slots=3, per_path=1e-3)
    s = Server(r, hbm_budget=10_000, max_batch_paths=1000, clock=clock, group_ratio=4.0)
    for rid, size in enumerate((100, 10, 120, 8, 300, 20)):
        s.submit(Request(rid, "a", size))
    s.step()
    batches = [ids for _, ids, _ in r.launched]
    assert batches[0] == [0, 2, 4]          # costs 100, 120, 300: within 4x of the first request
    assert batches[1] == [1, 3, 5]          # costs 10, 8, 20
    drive(s, clock)
    assert [q.error for q in s.completed] == [None] * 6
    # without grouping everything shares one batch
    clock2 = Clock()
    r2 = FakeRenderer(clock2, slots=3)
    s2 = Server(r2, hbm_budget=10_000, max_batch_paths=1000, clock=clock2)
    for rid, size in enumerate((100, 10, 120, 8, 300, 20)):
        s2.submit(Request(rid, "a", size))
    s2.step()
    assert [ids for _, ids, _ in r2.launched] == [[0, 1, 2, 3, 4, 5]]
    with pytest.raises(ValueError):
        Server(r2, hbm_budget=10_000, max_batch_paths=1000, clock=clock2, group_ratio=0.5)


def test_renderer_memory_is_taken_off_the_budget():
    clock = Clock()

    class Reserving(FakeRenderer):
        def reserved_bytes(self):
            return 60

    s = Server(Reserving(clock), hbm_budget=100, max_batch_paths=1000, clock=clock)
    assert s.budget == 40
    s.submit(Request(0, "a", 50))  # fits 100 but not the 40 left
    assert s.completed[0].error and "budget" in s.completed[0].error
    s.submit(Request(1, "a", 30))
    drive(s, clock)
    assert s.completed[1].error is None and s.peak_in_use <= 40
    with pytest.raises(ValueError):
        Server(Reserving(clock), hbm_budget=60, max_batch_paths=1000, clock=clock)
