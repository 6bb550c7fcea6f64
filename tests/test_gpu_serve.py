"""The server on the GPU: a Poisson stream of mixed queries, every answer
checked against the paper's closed form and, for a sample, against the same
query answered alone by the plain per-query path."""
import time

import numpy as np
import pytest

import synth
from closed_form import gamma2_closed_form

pytestmark = pytest.mark.gpu


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
    stream = synth.serve_stream(seed=5, count=300, qps=2000.0, n_hi=11, m_hi=300)
    stream += [(stream[-1][0] + 0.001 * i, 12, m) for i, m in enumerate((3, 4, 7, 9, 12, 13))]
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
    """A 3.5 GiB budget (about 24 powers of A(D_10)): queries of several path
    orders are still all answered (by eviction between waves)."""
    from paper_2409_17688_amd import serve
    ex = serve.GpuExecutor(3584 << 20)
    srv = serve.Server(ex, max_wave=64)
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
