"""The serving scheduler on the host, driven by fake executors (no GPU).

The fakes answer with the paper's closed form (a pin, not the library) so the
tests can check routing of answers to requests; what is under test is the
scheduling: continuous batching, admission by memory with eviction, failure
isolation, cancellation and validation.
"""
import threading
import time

import pytest

from closed_form import gamma2_closed_form
from paper_2409_17688_amd import serve

pytestmark = pytest.mark.timeout(60)


class FakeExecutor:
    """Each path order n resident costs `cost[n]` bytes while any query of n
    has run; run_wave sleeps `delay` seconds, optionally failing."""

    def __init__(self, budget=1 << 40, delay=0.0, cost=None, fail_waves=()):
        self.budget = budget
        self.delay = delay
        self.cost = cost or {}
        self.resident = set()
        self.released = []
        self.waves = []
        self.fail_waves = set(fail_waves)
        self.running = threading.Event()

    def need_bytes(self, ns, ms):
        return sum(self.cost.get(n, 0) for n in set(ns) if n not in self.resident)

    def resident_bytes(self):
        return sum(self.cost.get(n, 0) for n in self.resident)

    def release(self, n):
        self.released.append(n)
        self.resident.discard(n)

    def run_wave(self, ns, ms):
        self.waves.append(list(zip(ns, ms)))
        self.running.set()
        time.sleep(self.delay)
        self.running.clear()
        if len(self.waves) in self.fail_waves:
            raise RuntimeError("injected wave failure")
        self.resident.update(ns)
        return [gamma2_closed_form(n, m) for n, m in zip(ns, ms)]

    def make_lane(self, n):
        raise AssertionError("no lane expected")


def test_answers_reach_their_requests():
    srv = serve.Server(FakeExecutor(), sweep_n=None)
    try:
        reqs = [srv.submit(n, m) for n in range(1, 12) for m in (3, 7, 50, 499)]
        for r in reqs:
            assert r.wait(10) == serve.TP_OK
            assert r.gamma2 == gamma2_closed_form(r.n, r.m)
            assert r.latency is not None and r.latency >= 0
    finally:
        srv.close()


def test_arrivals_during_a_wave_join_the_next_wave():
    ex = FakeExecutor(delay=0.3)
    srv = serve.Server(ex, sweep_n=None)
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


def test_admission_by_memory_and_eviction():
    # room for two path orders at a time
    ex = FakeExecutor(budget=200, cost={4: 100, 5: 100, 6: 100}, delay=0.05)
    srv = serve.Server(ex, sweep_n=None)
    try:
        a = [srv.submit(4, 10), srv.submit(5, 10)]
        for r in a:
            assert r.wait(10) == serve.TP_OK
        b = srv.submit(6, 10)  # needs one eviction (the least recently used n)
        assert b.wait(10) == serve.TP_OK and b.gamma2 == gamma2_closed_form(6, 10)
        assert ex.released and ex.released[0] in (4, 5)
        # a wave never holds more than the budget
        for w in ex.waves:
            assert sum(ex.cost[n] for n in {n for n, _ in w}) <= 200
    finally:
        srv.close()


def test_query_larger_than_the_budget_fails_alone():
    ex = FakeExecutor(budget=100, cost={7: 1000, 3: 10})
    srv = serve.Server(ex, sweep_n=None)
    try:
        big = srv.submit(7, 40)
        small = srv.submit(3, 9)
        assert big.wait(10) == serve.TP_ENOMEM
        assert small.wait(10) == serve.TP_OK and small.gamma2 == gamma2_closed_form(3, 9)
    finally:
        srv.close()


def test_a_failing_wave_fails_only_its_queries():
    ex = FakeExecutor(delay=0.2, fail_waves={2})
    srv = serve.Server(ex, sweep_n=None)
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
    srv = serve.Server(ex, sweep_n=None)
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


def test_validation_and_overflow_guard():
    srv = serve.Server(FakeExecutor(), sweep_n=None)
    try:
        assert srv.submit(3, 2).status == serve.TP_EINVAL
        assert srv.submit(0, 5).status == serve.TP_EINVAL
        assert srv.submit(13, 5).status == serve.TP_EINVAL
        assert srv.submit(12, 5462).status == serve.TP_EOVERFLOW
        ok = srv.submit(12, 5461 // 2)
        # n = 12 goes to a sweep lane only when enabled; here it is a wave
        assert ok.wait(10) == serve.TP_OK
    finally:
        srv.close()


def test_percentile_nearest_rank():
    assert serve.percentile(list(range(1, 101)), 50) == 50
    assert serve.percentile(list(range(1, 101)), 99) == 99
    assert serve.percentile([7], 99) == 7
