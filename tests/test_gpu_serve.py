"""The server on the GPU: a Poisson stream of mixed queries, every answer
checked against the paper's closed form and, for a sample, against the same
query answered alone by the plain per-query path; two waves in flight; the
resident compact lanes of n = 10..12."""
import sys
import time

import numpy as np
import pytest

import synth
from closed_form import gamma2_closed_form

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def tp():
    import torch
    assert torch.cuda.is_available()
    import paper_2409_17688_amd as tp
    return tp


def _replay(srv, stream, speedup=1.0):
    t0 = time.perf_counter()
    reqs = []
    for t, n, m in stream:
        delay = t / speedup - (time.perf_counter() - t0)
        if delay > 0:
            time.sleep(delay)
        reqs.append(srv.submit(n, m))
    for r in reqs:
        r.wait(300)
    return reqs


def test_served_stream_matches_closed_form_and_plain(tp):
    from paper_2409_17688_amd import serve
    say("served stream")
    stream = synth.serve_stream(seed=5, count=300, qps=2000.0, n_hi=11, m_hi=300)
    stream += [(stream[-1][0] + 0.001 * i, 12, m) for i, m in enumerate((3, 4, 7, 9, 12, 13, 40))]
    ex = serve.GpuExecutor(200 << 30)
    srv = serve.Server(ex, max_wave=256)
    try:
        reqs = _replay(srv, stream)
    finally:
        srv.close()
        ex.close()
    for r in reqs:
        assert r.status == serve.TP_OK, (r.n, r.m, r.error)
        assert r.gamma2 == gamma2_closed_form(r.n, r.m), (r.n, r.m)
    assert srv.waves >= 1 and max(srv.wave_sizes) > 1  # queries were batched
    rng = np.random.default_rng(0)
    for i in rng.choice(len(reqs), size=25, replace=False):
        r = reqs[int(i)]
        assert tp.tp_tropical_power_trace(r.n, r.m) == r.gamma2
    lat = [r.latency for r in reqs]
    assert serve.percentile(lat, 50) <= serve.percentile(lat, 99)


def test_memory_admission_on_device(tp):
    """A 3.5 GiB budget (about 24 powers of A(D_10)) and n = 10 in waves:
    queries of several path orders are still all answered (by eviction
    between waves)."""
    from paper_2409_17688_amd import serve
    say("memory admission")
    ex = serve.GpuExecutor(3584 << 20)
    srv = serve.Server(ex, max_wave=64, lane_n=())
    try:
        reqs = [srv.submit(n, m) for n, m in ((10, 40), (9, 70), (10, 41), (8, 90), (9, 71),
                                              (10, 300), (7, 33))]
        for r in reqs:
            assert r.wait(120) == serve.TP_OK, r.error
            assert r.gamma2 == gamma2_closed_form(r.n, r.m)
        assert ex.resident_bytes() <= 3584 << 20
    finally:
        srv.close()
        ex.close()


def test_query_during_a_long_wave_finishes_first(tp):
    """Two waves in flight: a cold wave of n = 10 with m up to 500 (dense
    giant products in one persistent launch) runs on one slot; a query of
    n = 5 submitted while it runs is admitted into the other slot at once,
    finishes before the long wave, and its answer equals the same query
    answered alone (and in the mix, the long wave's answers equal theirs
    alone)."""
    from paper_2409_17688_amd import serve
    say("two waves in flight")
    ex = serve.GpuExecutor(64 << 30, slots=2)
    srv = serve.Server(ex, max_wave=256, lane_n=())
    try:
        # warm both slots' kernels (code objects load once per process)
        for r in [srv.submit(4, 5), srv.submit(3, 4)]:
            assert r.wait(60) == serve.TP_OK
        long_wave = [srv.submit(10, m) for m in range(300, 501, 10)]
        time.sleep(0.02)
        assert not long_wave[-1].done.is_set(), "the long wave ended before the probe"
        quick = srv.submit(5, 17)
        assert quick.wait(60) == serve.TP_OK
        for r in long_wave:
            assert r.wait(120) == serve.TP_OK, r.error
        say("quick", quick.latency, "long wave", max(r.latency for r in long_wave))
        assert quick.t_done < min(r.t_done for r in long_wave)
        assert srv.max_in_flight == 2
    finally:
        srv.close()
        ex.close()
    assert quick.gamma2 == tp.tp_tropical_power_trace(5, 17) == gamma2_closed_form(5, 17)
    for r in long_wave[::5]:
        assert r.gamma2 == tp.tp_tropical_power_trace(10, r.m) == gamma2_closed_form(10, r.m)


@pytest.mark.parametrize("n", [10, 11, 12])
def test_resident_lane_answers(tp, n):
    """The resident compact lane: babies, pruned panels and the plain path
    below m = 6, each answer == the closed form (every m = 3..80 and a spread
    up to the lane's reach, 512) and, for a sample, == the plain path alone;
    a second pass is answered from resident powers only (no chain step)."""
    from paper_2409_17688_amd import serve
    say("lane", n)
    ms = list(range(3, 81)) + [97, 133, 250, 333, 401, 499, 500, 505, 512]
    if n == 12:
        ms = list(range(3, 41)) + [77, 133, 250, 499, 512]
    import torch
    lane = serve.ResidentLane(n, tp, torch)
    try:
        reqs = [serve.Request(n, m, time.perf_counter()) for m in ms]
        for r in reqs:
            assert lane.submit(r)
        for r in reqs:
            assert r.wait(300) == serve.TP_OK, (n, r.m, r.error)
            assert r.gamma2 == gamma2_closed_form(n, r.m), (n, r.m)
        assert not lane.broken
        assert lane.plain_answers == sum(1 for m in ms if m < 6)
        level = lane.level
        again = [serve.Request(n, m, time.perf_counter()) for m in ms[::-1]]
        for r in again:
            assert lane.submit(r)
        for r in again:
            assert r.wait(60) == serve.TP_OK and r.gamma2 == gamma2_closed_form(n, r.m)
        assert lane.level == level
    finally:
        lane.close()
    for m in (6, 25, 26, 99):
        assert tp.tp_tropical_power_trace(n, m) == gamma2_closed_form(n, m)
