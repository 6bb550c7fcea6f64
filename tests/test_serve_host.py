"""The serving scheduler on the host, driven by fake executors (no GPU).

The fakes answer with the paper's closed form (a pin, not the library) so the
tests can check routing of answers to requests; what is under test is the
scheduling: waves in flight on several slots, admission by memory in arrival
order with eviction, no starvation, failure isolation, cancellation, lanes
and validation.
"""
import threading
import time

import pytest

from closed_form import gamma2_closed_form
from paper_2409_17688_amd import serve

pytestmark = pytest.mark.timeout(60)


class FakeExecutor:
    """Each path order n resident on a slot costs `cost[n]` bytes once a wave
    of that slot ran it; run_wave sleeps `delay` (or `delay_of[n]` for the
    slowest n of the wave) seconds, optionally failing."""

    def __init__(self, budget=1 << 40, delay=0.0, cost=None, fail_waves=(), nslots=1,
                 delay_of=None):
        self.budget = budget
        self.nslots = nslots
        self.delay = delay
        self.delay_of = delay_of or {}
        self.cost = cost or {}
        self.resident = [set() for _ in range(nslots)]
        self.released = []
        self.waves = []
        self.fail_waves = set(fail_waves)
        self.running = threading.Event()
        self.lock = threading.Lock()
        self.in_flight = 0
        self.max_in_flight = 0
        self.lanes = []

    def need_bytes(self, slot, ns, ms):
        return sum(self.cost.get(n, 0) for n in set(ns) if n not in self.resident[slot])

    def resident_bytes(self):
        return sum(self.cost.get(n, 0) for res in self.resident for n in res)

    def release(self, slot, n):
        self.released.append(n)
        self.resident[slot].discard(n)

    def run_wave(self, slot, ns, ms):
        with self.lock:
            self.waves.append(list(zip(ns, ms)))
            k = len(self.waves)
            self.in_flight += 1
            self.max_in_flight = max(self.max_in_flight, self.in_flight)
            # the wave's powers are allocated when it starts
            self.resident[slot].update(ns)
        self.running.set()
        try:
            time.sleep(max([self.delay] + [self.delay_of.get(n, 0) for n in ns]))
            if k in self.fail_waves:
                raise RuntimeError("injected wave failure")
            return [gamma2_closed_form(n, m) for n, m in zip(ns, ms)]
        finally:
            with self.lock:
                self.in_flight -= 1
            self.running.clear()

    def make_lane(self, n):
        lane = FakeLane(n)
        self.lanes.append(lane)
        return lane


class FakeLane:
    """Answers lane queries on its own thread from the closed form."""

    def __init__(self, n):
        self.n = n
        self.stop = False
        self.answered = []

    def submit(self, req):
        if self.stop:
            return False
        self.answered.append(req.m)
        threading.Timer(0.01, lambda: req._finish(gamma2=gamma2_closed_form(req.n, req.m))).start()
        return True

    def close(self):
        self.stop = True


def test_answers_reach_their_requests():
    srv = serve.Server(FakeExecutor(nslots=2), lane_n=())
    try:
        reqs = [srv.submit(n, m) for n in range(1, 13) for m in (3, 7, 50, 499)
                if n * m < 65535]
        for r in reqs:
            assert r.wait(10) == serve.TP_OK
            assert r.gamma2 == gamma2_closed_form(r.n, r.m)
            assert r.latency is not None and r.latency >= 0
    finally:
        srv.close()


def test_arrivals_during_a_wave_join_the_next_wave_with_one_slot():
    ex = FakeExecutor(delay=0.3)
    srv = serve.Server(ex, lane_n=())
    try:
        first = srv.submit(5, 10)
        assert ex.running.wait(5)
        late = [srv.submit(6, m) for m in range(3, 23)]
        for r in [first] + late:
            assert r.wait(10) == serve.TP_OK
        assert ex.waves[0] == [(5, 10)]
        assert ex.waves[1] == [(6, m) for m in range(3, 23)]
        assert srv.wave_sizes == [1, 20]
    finally:
        srv.close()


def test_a_query_arriving_during_a_long_wave_overlaps_it_and_finishes_first():
    """Two slots: while a slow wave of n = 9 runs on one, a query of another
    path order is admitted into the other at once and finishes before the
    slow wave; a query of n = 9 itself waits for its owner's next wave."""
    ex = FakeExecutor(nslots=2, delay_of={9: 1.0})
    srv = serve.Server(ex, lane_n=())
    try:
        slow = srv.submit(9, 100)
        assert ex.running.wait(5)
        quick = srv.submit(5, 17)
        same = srv.submit(9, 101)
        assert quick.wait(10) == serve.TP_OK and quick.gamma2 == gamma2_closed_form(5, 17)
        assert not slow.done.is_set(), "the quick query should not wait for the slow wave"
        assert slow.wait(10) == serve.TP_OK and same.wait(10) == serve.TP_OK
        assert quick.t_done < slow.t_done < same.t_done
        assert srv.max_in_flight == 2 and ex.max_in_flight == 2
        assert [(9, 101)] in ex.waves and ex.waves.index([(9, 101)]) > ex.waves.index([(9, 100)])
    finally:
        srv.close()


def test_admission_by_memory_evicts_one_path_order_at_a_time():
    # room for two path orders at a time
    ex = FakeExecutor(budget=200, cost={4: 100, 5: 100, 6: 100}, delay=0.05)
    srv = serve.Server(ex, lane_n=())
    try:
        a = srv.submit(4, 10)
        assert a.wait(10) == serve.TP_OK
        b = srv.submit(5, 10)
        assert b.wait(10) == serve.TP_OK
        c = srv.submit(6, 10)  # needs one eviction: the least recently used n = 4
        assert c.wait(10) == serve.TP_OK and c.gamma2 == gamma2_closed_form(6, 10)
        assert ex.released == [4]
        for w in ex.waves:
            assert sum(ex.cost[n] for n in {n for n, _ in w}) <= 200
        assert ex.resident_bytes() <= 200
    finally:
        srv.close()


def test_a_deferred_large_query_is_not_starved_by_small_ones():
    """The oldest query that does not fit blocks the ones behind it: a steady
    stream of fitting small queries cannot keep a large one waiting."""
    ex = FakeExecutor(budget=150, cost={3: 20, 4: 20, 9: 120}, delay=0.02, nslots=2)
    srv = serve.Server(ex, lane_n=())
    stop = threading.Event()
    small = []

    def feed():
        m = 3
        while not stop.is_set():
            small.append(srv.submit(3 + (m % 2), m))
            m += 1
            time.sleep(0.002)

    t = threading.Thread(target=feed)
    try:
        t.start()
        time.sleep(0.1)
        big = srv.submit(9, 77)
        assert big.wait(5) == serve.TP_OK, "the large query starved"
        assert big.gamma2 == gamma2_closed_form(9, 77)
    finally:
        stop.set()
        t.join()
        srv.close()
    assert all(r.wait(10) in (serve.TP_OK, serve.TP_ECANCELED) for r in small)


def test_query_larger_than_the_budget_fails_alone():
    ex = FakeExecutor(budget=100, cost={7: 1000, 3: 10})
    srv = serve.Server(ex, lane_n=())
    try:
        big = srv.submit(7, 40)
        small = srv.submit(3, 9)
        assert big.wait(10) == serve.TP_ENOMEM
        assert small.wait(10) == serve.TP_OK and small.gamma2 == gamma2_closed_form(3, 9)
    finally:
        srv.close()


def test_a_failing_wave_fails_only_its_queries():
    ex = FakeExecutor(delay=0.2, fail_waves={2})
    srv = serve.Server(ex, lane_n=())
    try:
        w1 = srv.submit(4, 5)
        assert ex.running.wait(5)
        w2 = [srv.submit(4, m) for m in (6, 7, 8)]
        assert w1.wait(10) == serve.TP_OK
        for r in w2:
            assert r.wait(10) == serve.TP_EHIP and "injected" in r.error
        w3 = srv.submit(4, 9)
        assert w3.wait(10) == serve.TP_OK and w3.gamma2 == gamma2_closed_form(4, 9)
    finally:
        srv.close()


def test_cancel_before_admission_and_close():
    ex = FakeExecutor(delay=0.3)
    srv = serve.Server(ex, lane_n=())
    first = srv.submit(5, 10)
    assert ex.running.wait(5)
    queued = srv.submit(5, 11)
    assert srv.cancel(queued)
    assert queued.status == serve.TP_ECANCELED
    assert first.wait(10) == serve.TP_OK
    assert not srv.cancel(first)
    srv.close()
    after = srv.submit(5, 12)
    assert after.status == serve.TP_ECANCELED
    assert all((5, 11) not in w for w in ex.waves)


def test_lane_orders_go_to_lanes_and_close_refuses_them():
    ex = FakeExecutor(nslots=2)
    srv = serve.Server(ex, lane_n=(10, 12))
    try:
        reqs = [srv.submit(12, m) for m in (3, 50, 499)] + [srv.submit(10, 7), srv.submit(11, 7)]
        for r in reqs:
            assert r.wait(10) == serve.TP_OK and r.gamma2 == gamma2_closed_form(r.n, r.m)
        assert sorted(l.n for l in ex.lanes) == [10, 12]
        assert all(n != 12 and n != 10 for w in ex.waves for n, _ in w)
    finally:
        srv.close()
    # after close: a lane order (existing lane or a new one) is refused, not queued
    for n in (12, 10, 5):
        r = srv.submit(n, 9)
        assert r.wait(1) == serve.TP_ECANCELED, n
    assert len(ex.lanes) == 2


def test_validation_and_overflow_guard():
    srv = serve.Server(FakeExecutor(), lane_n=())
    try:
        assert srv.submit(3, 2).status == serve.TP_EINVAL
        assert srv.submit(0, 5).status == serve.TP_EINVAL
        assert srv.submit(13, 5).status == serve.TP_EINVAL
        assert srv.submit(12, 5462).status == serve.TP_EOVERFLOW
        ok = srv.submit(12, 5461 // 2)
        # without lanes n = 12 runs in a wave
        assert ok.wait(10) == serve.TP_OK
    finally:
        srv.close()


def test_lane_plan_covers_every_m():
    """The resident lane's decomposition of m (no GPU: the planning rule
    alone): babies for m <= 2(c + 2), a baby r in 3..c+2 with the panel of
    A^(jc) beyond, the plain path below 6 and past the lane's reach."""
    lane = serve.ResidentLane.__new__(serve.ResidentLane)
    lane.c, lane.m_cap, lane.broken = 10, 512, ""
    for m in range(3, 700):
        p = lane._plan(m)
        if m < 6 or m > 512:
            assert p == ("plain",)
        elif m <= 24:
            assert p[0] == "babies" and p[1] + p[2] == m and 3 <= p[2] <= p[1] <= 12
        else:
            assert p[0] == "panel" and 3 <= p[1] <= 12 and p[2] >= 1
            assert p[1] + 10 * p[2] == m and p[2] <= (512 - 3) // 10
    lane.broken = "x"
    assert lane._plan(100) == ("plain",)


def test_lane_chain_never_writes_a_kept_panel():
    """The panel chain's ping-pong (no GPU: buffers are plain objects and the
    step records its level into the buffer it writes): after many steps every
    kept panel still holds the level jc it was kept at."""
    class Buf:
        def __init__(self):
            self.level = None

    class FakeTp:
        def tp_compact_shared_step(self, n, x, b, count, y, by, status, stream=None):
            y.level = x.level + 1

    lane = serve.ResidentLane.__new__(serve.ResidentLane)
    lane.tp, lane.stream, lane.n, lane.count, lane.status = FakeTp(), None, 10, 7, None
    lane.c, lane.panels = 10, {}
    lane._u8 = lambda cols: Buf()
    lane._base = lambda: None
    first = Buf()
    first.level = 3
    lane.chain, lane.spare, lane.level = (first, None), (Buf(), None), 3
    for _ in range(3, 257):
        lane._advance()
        assert lane.chain[0].level == lane.level
        for j, (p, _) in lane.panels.items():
            assert p.level == 10 * j, (j, p.level, lane.level)
    assert sorted(lane.panels) == list(range(1, 26))


def test_percentile_nearest_rank():
    assert serve.percentile(list(range(1, 101)), 50) == 50
    assert serve.percentile(list(range(1, 101)), 99) == 99
    assert serve.percentile([7], 99) == 7
