"""Host logic of the batch engine, on the CPU: which powers a batch needs.

tp_ctx_need_bytes runs the engine's planning on the host only (no device
call with baby steps set on the context, as here; the choice that may
consult the state's cost is tested on the GPU): per path order, the chain
up to the largest baby step an instance
needs and the giants A^(jc) with their closure under j = h + (j - h), h the
largest power of two <= j (j/2 + j/2 when j is a power of two).  The model
below restates those rules independently; the byte counts must agree."""
import numpy as np
import pytest

import paper_2409_17688_amd as tp


def _closure(j, out):
    if j <= 1 or j in out:
        return
    h = 1
    while h * 2 <= j:
        h *= 2
    left, right = (j // 2, j // 2) if h == j else (h, j - h)
    _closure(left, out)
    _closure(right, out)
    out.add(j)


def model_bytes(n, ms, c, compact_from=10, chain_from=10):
    """Bytes of the powers the planning rules call for.  Path orders from
    compact_from on (TP_PARAM_COMPACT_FROM) keep A^1..A^3 in 16 bits and A^3
    on as u8 residuals (rows of ld bytes) with 256 bytes of base words each;
    their baby steps are at least 4 and run to c + 2, and a pair with a
    baby above 3 keeps its baby at 3 or above.  Path orders from chain_from
    on (TP_PARAM_CHAIN_GIANTS_FROM) make each giant by continuing the chain:
    no smaller giants, two step buffers of the chain's form."""
    N = tp.tp_state_dim(n)
    ld = (N + 63) // 64 * 64
    compact = compact_from > 0 and n >= compact_from and n >= 2
    chained = chain_from > 0 and n >= chain_from
    if compact:
        c = max(c, 4)
    babies = c + 2 if compact else c
    lo = 3 if compact else 1
    top, giants = 1, set()
    for m in ms:
        if m <= 2 * babies:
            top = max(top, (m + 1) // 2)
        else:
            top = max(top, babies)
            if chained:
                giants.add((m - lo) // c)
            else:
                _closure((m - lo) // c, giants)
    temps = 2 if chained and giants else 0
    if not compact:
        exps = set(range(1, top + 1)) | {j * c for j in giants}
        return (len(exps) + temps) * N * ld * 2
    wide = set(range(1, min(top, 3) + 1))
    narrow = {j * c for j in giants}
    if top >= 4 or giants:
        narrow |= set(range(3, top + 1))
    return len(wide) * N * ld * 2 + (len(narrow) + temps) * (N * ld + 256)


@pytest.fixture
def ctx():
    h = tp.tp_ctx_create(1 << 40)
    yield h
    tp.tp_ctx_destroy(h)


@pytest.mark.parametrize("c", [2, 3, 5, 8, 16, 48])
def test_need_bytes_matches_the_planning_rules(ctx, c):
    rng = np.random.default_rng(c)
    for n in (1, 3, 5, 7, 9, 11):
        tp.tp_ctx_set_param(ctx, tp.TP_PARAM_BABY_STEPS + n, c)
    for trial in range(20):
        n = int(rng.choice([1, 3, 5, 7, 9, 11]))
        ms = [int(m) for m in rng.integers(3, 400, int(rng.integers(1, 12)))]
        if n * max(ms) >= 65535:
            continue
        got = tp.tp_ctx_need_bytes(ctx, [n] * len(ms), ms)
        assert got == model_bytes(n, ms, c), (n, ms, c)


@pytest.mark.parametrize("compact_from,chain_from", [(0, 0), (3, 0), (7, 5), (0, 3), (10, 10)])
def test_need_bytes_follows_the_compact_rules(ctx, compact_from, chain_from):
    rng = np.random.default_rng(100 + compact_from + 17 * chain_from)
    tp.tp_ctx_set_param(ctx, tp.TP_PARAM_COMPACT_FROM, compact_from)
    tp.tp_ctx_set_param(ctx, tp.TP_PARAM_CHAIN_GIANTS_FROM, chain_from)
    for n in (2, 3, 5, 7, 9, 11):
        tp.tp_ctx_set_param(ctx, tp.TP_PARAM_BABY_STEPS + n, 5)
    for trial in range(30):
        n = int(rng.choice([2, 3, 5, 7, 9, 11]))
        ms = [int(m) for m in rng.integers(3, 400, int(rng.integers(1, 12)))]
        if n * max(ms) >= 65535:
            continue
        got = tp.tp_ctx_need_bytes(ctx, [n] * len(ms), ms)
        assert got == model_bytes(n, ms, 5, compact_from, chain_from), (n, ms, compact_from)


def test_compact_parameter_bounds(ctx):
    for param in (tp.TP_PARAM_COMPACT_FROM, tp.TP_PARAM_CHAIN_GIANTS_FROM):
        for bad in (-1, 14):
            with pytest.raises(tp.TropicalError):
                tp.tp_ctx_set_param(ctx, param, bad)
        tp.tp_ctx_set_param(ctx, param, 0)
        tp.tp_ctx_set_param(ctx, param, 13)


def test_need_bytes_adds_over_path_orders(ctx):
    for n in (4, 6, 8):
        tp.tp_ctx_set_param(ctx, tp.TP_PARAM_BABY_STEPS + n, 10)
    inst = [(4, 7), (6, 100), (8, 33), (4, 90), (8, 201)]
    ns, ms = [a for a, _ in inst], [b for _, b in inst]
    want = sum(model_bytes(n, [m for a, m in inst if a == n], 10) for n in (4, 6, 8))
    assert tp.tp_ctx_need_bytes(ctx, ns, ms) == want


def test_need_bytes_rejects_bad_instances(ctx):
    with pytest.raises(tp.TropicalError):
        tp.tp_ctx_need_bytes(ctx, [13], [5])
    with pytest.raises(tp.TropicalError):
        tp.tp_ctx_need_bytes(ctx, [4], [2])
    assert tp.tp_ctx_need_bytes(ctx, [], []) == 0


def test_baby_steps_parameter_bounds(ctx):
    with pytest.raises(tp.TropicalError):
        tp.tp_ctx_set_param(ctx, tp.TP_PARAM_BABY_STEPS + 4, -1)
    with pytest.raises(tp.TropicalError):
        tp.tp_ctx_set_param(ctx, 999, 1)
    with pytest.raises(tp.TropicalError):
        tp.tp_ctx_set_param(ctx, tp.TP_PARAM_GRID, 3)  # fewer workgroups than queues
