"""Scheduler of the relighting service on a simulated backend (no GPU): admission by
footprint, LRU eviction of idle maps, FIFO order, slot limit, rejection of requests larger
than the budget, and the real-time serving loop."""
import math

import numpy as np
import pytest

from paper_2608_24109_amd.server import Request, Scheduler, latency_stats, serve


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


class FakeBackend:
    """Maps of `map_b[a]` bytes, requests of res^2 bytes lasting res^2 * 1e-6 s."""

    def __init__(self, map_b, fixed=100, clock=None):
        self.map_b = map_b
        self.fixed = fixed
        self.clock = clock
        self.loaded = set()
        self.log = []

    def fixed_bytes(self):
        return self.fixed

    def map_bytes(self, a):
        return self.map_b[a]

    def request_bytes(self, r):
        return r.res * r.res

    def load_map(self, a, slot):
        assert a not in self.loaded
        self.loaded.add(a)
        self.log.append(("load", a))

    def evict_map(self, a):
        self.loaded.remove(a)
        self.log.append(("evict", a))

    def launch(self, r, slot):
        assert r.asset in self.loaded, "launched without its map"
        self.log.append(("launch", r.rid, slot))
        return self.clock() + r.res * r.res * 1e-6

    def done(self, t_end):
        return self.clock() >= t_end

    def result(self, t_end):
        return t_end


def _req(rid, asset, res=10, arrival=0.0):
    return Request(rid, asset, 0, res, 0.0, False, arrival)


def _check(s):
    assert s.used <= s.budget and s.peak <= s.budget
    assert s.used == s.fixed + sum(s.resident.values()) + sum(nb for _, _, nb in s.inflight.values())
    for a in s.resident:
        assert a in s.b.loaded
    assert len(s.b.loaded) == len(s.resident)


def test_budget_lru_fifo_and_slots():
    clk = FakeClock()
    b = FakeBackend({0: 400, 1: 300, 2: 500, 3: 200}, clock=clk)
    s = Scheduler(b, budget=1300, slots=2)
    reqs = [_req(0, 0), _req(1, 1), _req(2, 0), _req(3, 2), _req(4, 3), _req(5, 1)]
    for r in reqs:
        s.submit(r)
    started = []
    while not s.idle():
        started += [r.rid for r in s.admit(clk)]
        _check(s)
        assert len(s.inflight) <= 2
        clk.t += 1e-5
        s.poll(clk)
        _check(s)
    assert started == [0, 1, 2, 3, 4, 5]  # FIFO
    assert all(r.status == "done" for r in reqs)
    # request 3 needs asset 2 (500 B): 100 fixed + 400 + 300 resident + 500 > 1300 -> the least
    # recently used idle map (asset 1; asset 0 was used again by request 2) goes first
    ev = [a for k, a, *_ in b.log if k == "evict"]
    assert ev[0] == 1
    assert s.evictions == len(ev) and s.loads == sum(1 for e in b.log if e[0] == "load")


def test_pinned_maps_are_not_evicted_and_requests_wait():
    clk = FakeClock()
    b = FakeBackend({0: 500, 1: 500}, clock=clk)
    s = Scheduler(b, budget=1150, slots=4)
    r0, r1 = _req(0, 0, res=10), _req(1, 1, res=10)
    s.submit(r0)
    s.submit(r1)
    s.admit(clk)
    # r1 (100 B + a 500 B map) does not fit while r0 holds asset 0 and its buffers: it waits,
    # nothing is evicted; once r0 is done, asset 0's idle map makes room
    assert r0.status == "running" and r1.status == "queued" and s.evictions == 0
    clk.t = 1.0
    s.poll(clk)
    s.admit(clk)
    assert r1.status == "running" and s.evictions == 1
    _check(s)


def test_oversized_request_is_rejected():
    clk = FakeClock()
    b = FakeBackend({0: 10}, clock=clk)
    s = Scheduler(b, budget=1000, slots=1)
    big, ok = _req(0, 0, res=40), _req(1, 0, res=10)
    s.submit(big)
    s.submit(ok)
    out = s.admit(clk)
    assert big.status == "rejected" and ok.status == "running" and {r.rid for r in out} == {0, 1}


def test_resident_map_is_reused_without_upload():
    clk = FakeClock()
    b = FakeBackend({0: 100}, clock=clk)
    s = Scheduler(b, budget=10_000, slots=1)
    for i in range(3):
        s.submit(_req(i, 0))
    while not s.idle():
        s.admit(clk)
        clk.t += 1.0
        s.poll(clk)
    assert s.loads == 1 and s.evictions == 0


def test_fixed_bytes_over_budget():
    with pytest.raises(ValueError):
        Scheduler(FakeBackend({}, fixed=10), budget=5, slots=1)


def test_serve_realtime_poisson():
    import time
    rng = np.random.default_rng(0)
    clk = time.monotonic
    b = FakeBackend({a: 1000 for a in range(8)}, clock=clk)
    s = Scheduler(b, budget=100 + 4 * 1000 + 3 * 64 * 64, slots=3)
    t, reqs = 0.0, []
    for i in range(150):
        t += rng.exponential(1.0 / 500.0)
        reqs.append(_req(i, int(rng.integers(8)), res=int(rng.choice([16, 32, 64])), arrival=t))
    serve(s, reqs, clock=clk, idle_sleep=1e-4)
    assert all(r.status == "done" for r in reqs)
    assert all(r.t_done >= r.arrival and r.t_admit >= r.arrival - 1e-9 for r in reqs)
    st = latency_stats(reqs)
    assert st["completed"] == 150 and st["p99_ms"] >= st["p50_ms"] > 0
    assert s.evictions > 0 and s.peak <= s.budget
    assert not math.isnan(st["req_per_s"])


class FakeBatchBackend(FakeBackend):
    """Also renders batches: one launch for several requests, retired together."""

    def launch_batch(self, rs, slot):
        for r in rs:
            assert r.asset in self.loaded, "launched without its map"
        self.log.append(("batch", tuple(r.rid for r in rs), slot))
        return ("batch", self.clock() + sum(r.res * r.res for r in rs) * 1e-6, len(rs))

    def done(self, tok):
        return self.clock() >= (tok[1] if isinstance(tok, tuple) else tok)

    def result(self, tok):
        return [tok[1]] * tok[2] if isinstance(tok, tuple) else tok


def test_batches_take_the_queue_head_in_order():
    """Direct-only requests of at most batch_res^2 pixels that stand together at the head of the
    queue share one slot and one launch (at most batch_max of them); an indirect or larger request
    ends the batch; every request is admitted by its own footprint and retired with its batch."""
    clk = FakeClock()
    b = FakeBatchBackend({a: 50 for a in range(4)}, clock=clk)
    s = Scheduler(b, budget=100_000, slots=2, batch_max=3, batch_res=16)
    reqs = [_req(0, 0), _req(1, 1), _req(2, 2), _req(3, 3), _req(4, 0, res=32), _req(5, 1), _req(6, 2)]
    reqs[5].indirect = True
    for r in reqs:
        s.submit(r)
    seen = []
    while not s.idle():
        seen += [r.rid for r in s.admit(clk)]
        _check(s)
        clk.t += 1.0
        s.poll(clk)
        _check(s)
    assert seen == list(range(7))
    batches = [e[1] for e in b.log if e[0] == "batch"]
    singles = [e[1] for e in b.log if e[0] == "launch"]
    # request 3 is batchable but the request behind it is too large, so it runs alone; 5 is
    # indirect and 6 has no batchable follower
    assert batches == [(0, 1, 2)] and singles == [3, 4, 5, 6]
    assert s.batches == 1 and all(r.status == "done" for r in reqs)


def test_batch_waits_for_memory_like_single_requests():
    clk = FakeClock()
    b = FakeBatchBackend({0: 100, 1: 100, 2: 100}, clock=clk)
    # room for the fixed bytes, two maps and two requests of 10^2: the third request waits
    s = Scheduler(b, budget=100 + 200 + 200, slots=4, batch_max=8, batch_res=16)
    rs = [_req(0, 0), _req(1, 1), _req(2, 2)]
    for r in rs:
        s.submit(r)
    s.admit(clk)
    assert [r.status for r in rs] == ["running", "running", "queued"]
    assert len(s.inflight) == 1 and s.batches == 1
    _check(s)
    clk.t = 1.0
    s.poll(clk)
    s.admit(clk)
    assert rs[2].status == "running"
    _check(s)


class FailingBackend(FakeBatchBackend):
    """Raises in the launch of the requests (or batches holding a request) whose rid is in `bad`."""

    def __init__(self, *a, bad=(), **k):
        super().__init__(*a, **k)
        self.bad = set(bad)

    def launch(self, r, slot):
        if r.rid in self.bad:
            raise RuntimeError(f"launch of request {r.rid} failed")
        return super().launch(r, slot)

    def launch_batch(self, rs, slot):
        if any(r.rid in self.bad for r in rs):
            raise RuntimeError("batch launch failed")
        return super().launch_batch(rs, slot)


def test_failed_launch_fails_only_its_requests():
    """A launch that raises retires its request (or its whole batch) as failed with the error and
    returns the slot and the request memory; the requests around it are served as usual, the map
    stays resident and evictable, and the serving loop ends."""
    clk = FakeClock()
    b = FailingBackend({a: 50 for a in range(4)}, clock=clk, bad={2, 5})
    s = Scheduler(b, budget=100 + 4 * 50 + 3 * 100, slots=2, batch_max=2, batch_res=16)
    reqs = [_req(i, i % 4) for i in range(8)]
    for r in (reqs[2], reqs[3], reqs[6]):
        r.indirect = True  # 2 fails alone; 5 fails inside the batch (4, 5)
    for r in reqs:
        s.submit(r)
    while not s.idle():
        s.admit(clk)
        _check(s)
        clk.t += 1.0
        s.poll(clk)
        _check(s)
    failed = [r.rid for r in reqs if r.status == "failed"]
    assert failed == [2, 4, 5] and s.failures == 3
    assert all(isinstance(reqs[i].result, RuntimeError) for i in failed)
    assert all(r.status == "done" for r in reqs if r.rid not in failed)
    assert s.used == s.fixed + sum(s.resident.values()) and sorted(s.free) == [0, 1]
    assert all(s.pins[a] == 0 for a in range(4))
    st = latency_stats(reqs)
    assert st["failed"] == 3 and st["completed"] == 5


def test_serve_ends_with_failed_requests():
    import time
    clk = time.monotonic
    b = FailingBackend({a: 100 for a in range(3)}, clock=clk, bad={0, 7})
    s = Scheduler(b, budget=100 + 3 * 100 + 2 * 32 * 32, slots=2)
    reqs = [_req(i, i % 3, res=32, arrival=0.001 * i) for i in range(12)]
    serve(s, reqs, clock=clk, idle_sleep=1e-4)
    assert [r.rid for r in reqs if r.status == "failed"] == [0, 7]
    assert sum(r.status == "done" for r in reqs) == 10
