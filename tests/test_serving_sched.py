"""Host-side tests of the serving scheduler (no GPU): admission by memory,
FIFO order, concurrency, eviction, capacity-overflow retry."""
import pytest

from paper_2501_12369_amd.serving import Request, Scheduler


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 1e-5)


class FakeSlot:
    def __init__(self, key, nbytes, clock, service, overflow_once, log, max_batch=1):
        self.key, self.nbytes, self.clock, self.service = key, nbytes, clock, service
        self.overflow_once, self.log = overflow_once, log
        self.max_batch = max_batch
        self.t_end = None
        self.reqs = None
        self.freed = False

    def launch(self, reqs):
        assert not self.freed and 1 <= len(reqs) <= self.max_batch
        assert all(r.key == self.key for r in reqs)
        self.reqs = reqs
        self.t_end = self.clock.t + self.service
        for r in reqs:
            self.log.append(("start", r.rid, self.clock.t, self.key))
        self.log.append(("batch", len(reqs), self.clock.t, self.key))

    def poll(self):
        return self.clock.t >= self.t_end

    def finish(self):
        over = [r.rid for r in self.reqs if r.rid in self.overflow_once]
        if over:
            for rid in over:
                self.overflow_once.discard(rid)
            return False, 999
        return True, 10

    def rerun(self, reqs, K):
        self.nbytes += 1
        for r in reqs:
            self.log.append(("rerun", r.rid, self.clock.t, self.key))

    def image_copy(self, i=0):
        return None

    def free(self):
        self.freed = True
        self.log.append(("free", None, self.clock.t, self.key))


def make(budget, max_slots=8, service=0.010, per_key_bytes=None, overflow_once=(), max_inflight=None, max_batch=1):
    clock = FakeClock()
    log = []
    per_key_bytes = per_key_bytes or {}
    ov = set(overflow_once)

    def need(key):
        return per_key_bytes.get(key, 100)

    def factory(key, hint):
        return FakeSlot(key, need(key), clock, service, ov, log, max_batch)

    return (Scheduler(factory, need, budget, max_slots, clock=clock, sleep=clock.sleep, max_inflight=max_inflight),
            clock, log)


def req(i, t, scene=0, w=64, h=64):
    return Request(i, t, scene, dict(width=w, height=h))


def test_all_complete_and_fifo_per_key():
    s, clock, log = make(budget=1000, max_slots=1)
    rs = [req(i, 0.001 * i) for i in range(10)]
    results, st = s.run(rs)
    assert sorted(r.rid for r in results) == list(range(10))
    starts = [e[1] for e in log if e[0] == "start"]
    assert starts == list(range(10))
    assert st.peak_slots == 1 and st.n == 10
    # one at a time: each request waits for the previous one
    for a, b in zip(results, results[1:]):
        assert b.start >= a.end - 1e-9


def test_concurrent_admission_overlaps_work():
    s, clock, log = make(budget=1000, max_slots=4, service=0.010)
    rs = [req(0, 0.0), req(1, 0.002)]
    results, st = s.run(rs)
    r0, r1 = sorted(results, key=lambda r: r.rid)
    assert r1.start < r0.end  # admitted while the first one is on the GPU
    assert st.peak_slots == 2


def test_memory_budget_is_respected_and_queues():
    # each slot needs 400 bytes; budget 1000 -> at most 2 slots
    s, clock, log = make(budget=1000, max_slots=8, per_key_bytes={(0, 64, 64): 400})
    rs = [req(i, 0.0) for i in range(6)]
    results, st = s.run(rs)
    assert st.peak_bytes <= 1000 and st.peak_slots == 2
    assert len(results) == 6


def test_idle_slots_of_other_keys_are_evicted():
    kb = {(0, 64, 64): 600, (1, 64, 64): 600}
    s, clock, log = make(budget=1000, max_slots=8, per_key_bytes=kb)
    rs = [req(0, 0.0, scene=0), req(1, 0.050, scene=1), req(2, 0.100, scene=0)]
    results, st = s.run(rs)
    assert len(results) == 3 and st.evictions >= 2
    # the slot freed before request 1 belongs to scene 0, the one before request 2 to scene 1
    frees = [e[3] for e in log if e[0] == "free"]
    assert frees[:2] == [(0, 64, 64), (1, 64, 64)]
    assert st.peak_bytes <= 1000


def test_request_above_budget_is_rejected():
    s, clock, log = make(budget=100, per_key_bytes={(0, 64, 64): 101})
    with pytest.raises(MemoryError):
        s.run([req(0, 0.0)])


def test_capacity_overflow_is_rerun():
    s, clock, log = make(budget=1000, overflow_once={3})
    results, st = s.run([req(i, 0.001 * i) for i in range(5)])
    assert st.retries == 1
    assert [r.retried for r in sorted(results, key=lambda r: r.rid)] == [False, False, False, True, False]
    assert any(e[0] == "rerun" and e[1] == 3 for e in log)


def test_latency_statistics():
    s, clock, log = make(budget=1000, max_slots=1, service=0.004)
    rs = [req(i, 0.005 * i) for i in range(50)]
    results, st = s.run(rs)
    assert 3.9 <= st.p50_ms <= 5.0 and st.p99_ms >= st.p50_ms
    assert st.req_per_s == pytest.approx(50 / st.wall_s)


def test_inflight_limit_keeps_slots():
    # two keys, room for both slots: one request in flight at a time, no eviction
    s, clock, log = make(budget=1000, max_slots=8, max_inflight=1)
    rs = [req(i, 0.0, scene=i % 2) for i in range(6)]
    results, st = s.run(rs)
    assert st.peak_inflight == 1 and st.evictions == 0 and st.peak_slots == 2
    rs_sorted = sorted(results, key=lambda r: r.start)
    for a, b in zip(rs_sorted, rs_sorted[1:]):
        assert b.start >= a.end - 1e-9
    # a second run reuses the slots: no new slot, statistics of that run only
    results, st2 = s.run([req(10 + i, 0.0, scene=i % 2) for i in range(4)])
    assert st2.n == 4 and st2.evictions == 0 and st2.peak_slots == 2 and st2.retries == 0
    assert sum(1 for e in log if e[0] == "free") == 0


def test_saturation_waits_for_own_key_without_eviction():
    # two keys, room for one slot each: under a burst each key waits for its own
    # slot instead of evicting the other key's idle slot
    kb = {(0, 64, 64): 400, (1, 64, 64): 400}
    s, clock, log = make(budget=1000, max_slots=8, per_key_bytes=kb)
    results, st = s.run([req(i, 0.0, scene=i % 2) for i in range(10)])
    assert len(results) == 10 and st.evictions == 0 and st.peak_slots == 2
    for key in (0, 1):  # per key, requests start in arrival order
        starts = [e[1] for e in log if e[0] == "start" and e[3][0] == key]
        assert starts == sorted(starts) and len(starts) == 5


def test_admission_looks_past_a_waiting_key():
    # key 0's second request waits for key 0's slot; key 1's request behind it starts at once
    kb = {(0, 64, 64): 600, (1, 64, 64): 300}
    s, clock, log = make(budget=1000, max_slots=8, per_key_bytes=kb, service=0.010)
    results, st = s.run([req(0, 0.0, scene=0), req(1, 0.0, scene=0), req(2, 0.0, scene=1)])
    by = {r.rid: r for r in results}
    assert by[2].start < by[0].end <= by[1].start + 1e-9
    assert st.evictions == 0 and st.peak_slots == 2


def test_requests_of_one_key_share_a_launch():
    """Continuous batching: requests of one key waiting together join one launch
    (up to the slot's batch size); requests arriving while it runs are admitted
    to the next launch when the slot frees up, in arrival order."""
    s, clock, log = make(budget=1000, max_slots=1, service=0.010, max_batch=4)
    rs = [req(i, 0.0) for i in range(10)] + [req(10 + i, 0.005) for i in range(3)]
    results, st = s.run(rs)
    assert sorted(r.rid for r in results) == list(range(13))
    batches = [e[1] for e in log if e[0] == "batch"]
    assert batches == [4, 4, 4, 1]
    starts = [e[1] for e in log if e[0] == "start"]
    assert starts == list(range(13))
    assert st.extra["peak_batch"] == 4
    # every request of a launch ends with it
    ends = {}
    for r in results:
        ends.setdefault(r.start, set()).add(r.end)
    assert all(len(v) == 1 for v in ends.values())


def test_batches_keep_to_their_key_and_limit():
    s, clock, log = make(budget=1000, max_slots=2, service=0.010, max_batch=3)
    rs = [req(i, 0.0, scene=i % 2) for i in range(8)]
    results, st = s.run(rs)
    assert len(results) == 8
    assert max(e[1] for e in log if e[0] == "batch") == 3
    s.batch_limit = 1
    rs2 = [req(20 + i, 0.0) for i in range(4)]
    s.run(rs2)
    assert [e[1] for e in log if e[0] == "batch"][-4:] == [1, 1, 1, 1]
