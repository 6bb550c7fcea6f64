"""Batched gamma_2 (one persistent launch per batch) against the oracle and
against the plain per-query path; resident powers reused across batches;
budget and abort handling."""
import sys

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


@pytest.fixture(scope="module")
def oracle_table(oracle_mod):
    """gamma_2(n, m) from one oracle chain per n, m <= 240, n = 1..9."""
    return {n: oracle_mod.gamma2_sweep(n, 240) for n in range(1, 10)}


def _run(tp, ctx, inst):
    import torch
    ns = [n for n, _ in inst]
    ms = [m for _, m in inst]
    out = tp.tp_batch_power_trace(ctx, ns, ms)
    tp.tp_ctx_check(ctx)
    torch.cuda.synchronize()
    return out.cpu().numpy().tolist()


def test_mixed_batch_of_64(tp, oracle_table):
    inst = synth.batch_instances(seed=0)
    ctx = tp.tp_ctx_create(64 << 30)
    try:
        say("batch of 64")
        got = _run(tp, ctx, inst)
        ref = [int(oracle_table[n][m - 1]) for n, m in inst]
        assert got == ref
        # alone (plain path) == in the batch
        for (n, m), g in zip(inst, got):
            assert tp.tp_tropical_power_trace(n, m) == g, (n, m)
    finally:
        tp.tp_ctx_destroy(ctx)


def test_batches_reuse_resident_powers(tp, oracle_table):
    ctx = tp.tp_ctx_create(64 << 30)
    try:
        rng = np.random.default_rng(7)
        for rep in range(4):
            count = int(rng.integers(1, 40))
            inst = [(int(rng.integers(1, 10)), int(rng.integers(3, 120 + 30 * rep)))
                    for _ in range(count)]
            say("reuse batch", rep, count)
            before = tp.tp_ctx_resident_bytes(ctx)
            got = _run(tp, ctx, inst)
            assert got == [int(oracle_table[n][m - 1]) for n, m in inst], rep
            assert tp.tp_ctx_resident_bytes(ctx) >= before
    finally:
        tp.tp_ctx_destroy(ctx)


def test_order_and_duplicates_do_not_matter(tp, oracle_table):
    inst = synth.batch_instances(seed=3, count=48)
    inst = inst + inst[:5]
    ctx = tp.tp_ctx_create(64 << 30)
    try:
        got = dict()
        for seed in (0, 1):
            perm = np.random.default_rng(seed).permutation(len(inst))
            shuffled = [inst[i] for i in perm]
            res = _run(tp, ctx, shuffled)
            for (n, m), g in zip(shuffled, res):
                assert got.setdefault((n, m), g) == g
                assert g == int(oracle_table[n][m - 1])
    finally:
        tp.tp_ctx_destroy(ctx)


def test_large_n_in_batch_closed_form(tp):
    inst = [(10, 3), (10, 40), (11, 5), (11, 24), (12, 3), (12, 5), (12, 8), (9, 100), (4, 7)]
    ctx = tp.tp_ctx_create(200 << 30)
    try:
        got = _run(tp, ctx, inst)
        assert got == [gamma2_closed_form(n, m) for n, m in inst]
    finally:
        tp.tp_ctx_destroy(ctx)


def test_fused_mode_large_n_closed_form(tp):
    # chain levels of large N inside the one launch (level items of n = 10,
    # 11 and 12 next to small ones)
    inst = [(10, 3), (10, 40), (11, 5), (11, 24), (12, 5), (9, 100), (4, 7)]
    ctx = tp.tp_ctx_create(120 << 30)
    try:
        tp.tp_ctx_set_param(ctx, tp.TP_PARAM_FUSED_CHAIN, 1)
        got = _run(tp, ctx, inst)
        assert got == [gamma2_closed_form(n, m) for n, m in inst]
    finally:
        tp.tp_ctx_destroy(ctx)


def test_budget_exceeded(tp):
    ctx = tp.tp_ctx_create(1 << 20)
    try:
        with pytest.raises(tp.TropicalError) as e:
            tp.tp_batch_power_trace(ctx, [9], [50])
        assert e.value.status == tp.TP_ENOMEM
    finally:
        tp.tp_ctx_destroy(ctx)


def test_abort_path_forced_from_host(tp, oracle_table):
    """A zero wait limit makes the first task that must wait abort the batch;
    the kernel drains and exits, tp_ctx_check reports it, and the next batch
    recomputes the dropped levels correctly."""
    ctx = tp.tp_ctx_create(64 << 30)
    try:
        tp.tp_ctx_set_param(ctx, tp.TP_PARAM_WAIT_LIMIT_US, 0)
        # few baby steps, so that these instances need giants built from
        # giants (tasks that wait), whatever the tuning table says
        for n in (6, 8, 9):
            tp.tp_ctx_set_param(ctx, tp.TP_PARAM_BABY_STEPS + n, 4)
        inst = [(9, 60), (8, 41), (6, 30)]
        tp.tp_batch_power_trace(ctx, [n for n, _ in inst], [m for _, m in inst])
        with pytest.raises(tp.TropicalError) as e:
            tp.tp_ctx_check(ctx)
        assert e.value.status == tp.TP_ECANCELED
        tp.tp_ctx_set_param(ctx, tp.TP_PARAM_WAIT_LIMIT_US, 20_000_000)
        got = _run(tp, ctx, inst)
        assert got == [int(oracle_table[n][m - 1]) for n, m in inst]
    finally:
        tp.tp_ctx_destroy(ctx)


def test_fused_mode_any_grid(tp, oracle_table):
    # chain levels inside the one persistent launch, on grids from the
    # minimum to the whole chip (and beyond: clamped to what is resident),
    # and the abort path in that mode
    inst = synth.batch_instances(seed=12, count=24)
    want = [int(oracle_table[n][m - 1]) for n, m in inst]
    for grid in (37, 0, 8, 1 << 20):
        ctx = tp.tp_ctx_create(64 << 30)
        try:
            tp.tp_ctx_set_param(ctx, tp.TP_PARAM_FUSED_CHAIN, 1)
            tp.tp_ctx_set_param(ctx, tp.TP_PARAM_GRID, grid)
            say("fused grid", grid)
            assert _run(tp, ctx, inst) == want, grid
            # a second batch on the same context: everything resident
            assert _run(tp, ctx, inst) == want, (grid, "warm")
        finally:
            tp.tp_ctx_destroy(ctx)
    ctx = tp.tp_ctx_create(64 << 30)
    try:
        tp.tp_ctx_set_param(ctx, tp.TP_PARAM_FUSED_CHAIN, 1)
        tp.tp_ctx_set_param(ctx, tp.TP_PARAM_WAIT_LIMIT_US, 0)
        for n in (6, 8, 9):
            tp.tp_ctx_set_param(ctx, tp.TP_PARAM_BABY_STEPS + n, 4)
        few = [(9, 60), (8, 41), (6, 30)]
        tp.tp_batch_power_trace(ctx, [n for n, _ in few], [m for _, m in few])
        with pytest.raises(tp.TropicalError) as e:
            tp.tp_ctx_check(ctx)
        assert e.value.status == tp.TP_ECANCELED
        tp.tp_ctx_set_param(ctx, tp.TP_PARAM_WAIT_LIMIT_US, 20_000_000)
        assert _run(tp, ctx, few) == [int(oracle_table[n][m - 1]) for n, m in few]
    finally:
        tp.tp_ctx_destroy(ctx)


def test_fused_and_split_modes_share_resident_powers(tp, oracle_table):
    # powers computed in one mode answer the next batch in the other
    inst = synth.batch_instances(seed=13, count=16)
    want = [int(oracle_table[n][m - 1]) for n, m in inst]
    ctx = tp.tp_ctx_create(64 << 30)
    try:
        tp.tp_ctx_set_param(ctx, tp.TP_PARAM_FUSED_CHAIN, 1)
        assert _run(tp, ctx, inst[:8]) == want[:8]
        tp.tp_ctx_set_param(ctx, tp.TP_PARAM_FUSED_CHAIN, 0)
        assert _run(tp, ctx, inst) == want
        tp.tp_ctx_set_param(ctx, tp.TP_PARAM_FUSED_CHAIN, 1)
        assert _run(tp, ctx, inst[::-1]) == want[::-1]
    finally:
        tp.tp_ctx_destroy(ctx)


def test_grid_and_step_form_do_not_change_results(tp, oracle_table):
    # persistent grids from the minimum (one workgroup per queue) to the
    # whole chip, and both forms of the chain's sparse step
    inst = synth.batch_instances(seed=11, count=20)
    want = [int(oracle_table[n][m - 1]) for n, m in inst]
    try:
        for grid, form in ((8, tp.TP_STEP_CSR), (37, tp.TP_STEP_BLOCKED), (0, tp.TP_STEP_AUTO)):
            for n in range(4, 10):
                tp.tp_tune_step(n, form)
            ctx = tp.tp_ctx_create(64 << 30)
            try:
                tp.tp_ctx_set_param(ctx, tp.TP_PARAM_GRID, grid)
                got = _run(tp, ctx, inst)
                assert got == want, (grid, form)
            finally:
                tp.tp_ctx_destroy(ctx)
    finally:
        for n in range(4, 10):
            tp.tp_tune_step(n, tp.TP_STEP_AUTO)
        tp.apply_tuning()


@pytest.fixture(scope="module")
def oracle_table_500(oracle_mod):
    """gamma_2(n, m) for m <= 500, n = 1..8 (one oracle chain per n)."""
    return {n: oracle_mod.gamma2_sweep(n, 500) for n in range(1, 9)}


def test_giants_for_long_cycles(tp, oracle_table_500):
    """m up to 500: answers come from chain powers and dense giant products."""
    rng = np.random.default_rng(21)
    inst = [(int(rng.integers(2, 9)), int(rng.integers(3, 501))) for _ in range(60)]
    inst += [(8, 500), (8, 33), (8, 32), (8, 31), (7, 64), (7, 65), (6, 97)]
    ctx = tp.tp_ctx_create(64 << 30)
    try:
        say("giants batch")
        got = _run(tp, ctx, inst)
        assert got == [int(oracle_table_500[n][m - 1]) for n, m in inst]
        # a second batch reuses the resident giants and adds new ones
        inst2 = [(8, m) for m in (499, 400, 257, 129, 3)] + [(5, 450), (5, 449)]
        got2 = _run(tp, ctx, inst2)
        assert got2 == [int(oracle_table_500[n][m - 1]) for n, m in inst2]
    finally:
        tp.tp_ctx_destroy(ctx)


@pytest.mark.parametrize("fused", [0, 1])
@pytest.mark.parametrize("c", [2, 3, 7, 16, 40])
def test_baby_step_length_does_not_change_results(tp, oracle_table_500, c, fused):
    inst = [(n, m) for n in (3, 6, 8) for m in (3, 4, 5, 2 * c, 2 * c + 1, 3 * c + 2, 199, 350)]
    ctx = tp.tp_ctx_create(64 << 30)
    try:
        tp.tp_ctx_set_param(ctx, tp.TP_PARAM_FUSED_CHAIN, fused)
        for n in (3, 6, 8):
            tp.tp_ctx_set_param(ctx, tp.TP_PARAM_BABY_STEPS + n, c)
        need = tp.tp_ctx_need_bytes(ctx, [n for n, _ in inst], [m for _, m in inst])
        got = _run(tp, ctx, inst)
        assert got == [int(oracle_table_500[n][m - 1]) for n, m in inst], c
        assert tp.tp_ctx_resident_bytes(ctx) == need
        assert tp.tp_ctx_need_bytes(ctx, [n for n, _ in inst], [m for _, m in inst]) == 0
    finally:
        tp.tp_ctx_destroy(ctx)


def test_giants_at_large_n_closed_form(tp):
    inst = [(9, 500), (9, 347), (10, 300), (10, 37), (11, 120), (11, 97)]
    ctx = tp.tp_ctx_create(200 << 30)
    try:
        got = _run(tp, ctx, inst)
        assert got == [gamma2_closed_form(n, m) for n, m in inst]
    finally:
        tp.tp_ctx_destroy(ctx)


def test_fused_batches_of_two_contexts_on_two_streams(tp, oracle_table):
    # launches with level barriers are ordered one after another on the
    # device, so two cold fused batches on two streams both complete
    import torch
    inst = synth.batch_instances(seed=14, count=20)
    ns, ms = [n for n, _ in inst], [m for _, m in inst]
    want = [int(oracle_table[n][m - 1]) for n, m in inst]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    ctxs = [tp.tp_ctx_create(32 << 30) for _ in streams]
    try:
        outs = []
        for c, s in zip(ctxs, streams):
            tp.tp_ctx_set_param(c, tp.TP_PARAM_FUSED_CHAIN, 1)
            tp.tp_ctx_set_param(c, tp.TP_PARAM_WAIT_LIMIT_US, 5_000_000)
            outs.append(tp.tp_batch_power_trace(c, ns, ms, stream=s))
        for c, s, o in zip(ctxs, streams, outs):
            tp.tp_ctx_check(c, stream=s)
            s.synchronize()
            assert o.cpu().numpy().tolist() == want
    finally:
        for c in ctxs:
            tp.tp_ctx_destroy(c)


def test_last_work_counts_what_the_batch_computes(tp):
    """tp_ctx_last_work: a cold batch of one instance (n = 4, m = 5, baby
    steps 16, so A^3 x A^2 closes it: levels 2 and 3 of the chain, no
    product, one trace) counts 2 nnz N + N^2 operations and 2 N^2 + 2 * 4 N^2
    + 4 N^2 bytes; the same batch again computes only its trace; a giant
    adds N^3."""
    say("last work")
    N, nnz = tp.tp_state_dim(4), tp.tp_state_nnz(4)
    ctx = tp.tp_ctx_create(1 << 30)
    try:
        tp.tp_ctx_set_param(ctx, tp.TP_PARAM_BABY_STEPS + 4, 16)
        _run(tp, ctx, [(4, 5)])
        w = tp.tp_ctx_last_work(ctx)
        assert w["chain_ops"] == 2 * nnz * N and w["product_ops"] == 0
        assert w["trace_ops"] == N * N
        assert w["bytes"] == 2 * N * N + 2 * 4 * N * N + 4 * N * N
        _run(tp, ctx, [(4, 5)])
        w = tp.tp_ctx_last_work(ctx)
        assert w["chain_ops"] == 0 and w["product_ops"] == 0 and w["trace_ops"] == N * N
        # m = 40 > 2c: the pair (32, 8), giant 2 = A^16 x A^16 and the rest
        # of the chain to A^16
        _run(tp, ctx, [(4, 40)])
        w = tp.tp_ctx_last_work(ctx)
        assert w["product_ops"] == N ** 3 and w["chain_ops"] == 13 * nnz * N
    finally:
        tp.tp_ctx_destroy(ctx)


@pytest.mark.parametrize("fused", [0, 1])
def test_chain_powers_equal_the_oracle(tp, oracle_mod, fused):
    # every resident chain power A^1 .. A^c, entry by entry, against the
    # oracle's chain A^k = A x A^(k-1); in the fused mode levels k >= 2 run
    # on row-block parts (blocks above the part bound are cut by rows at
    # n = 8 and 9)
    import torch
    cs = {5: 9, 8: 7, 9: 4}
    ctx = tp.tp_ctx_create(64 << 30)
    try:
        tp.tp_ctx_set_param(ctx, tp.TP_PARAM_FUSED_CHAIN, fused)
        for n, c in cs.items():
            tp.tp_ctx_set_param(ctx, tp.TP_PARAM_BABY_STEPS + n, c)
        inst = [(n, 2 * c) for n, c in cs.items()]
        say("chain powers, fused", fused)
        got = _run(tp, ctx, inst)
        for n, c in cs.items():
            A = oracle_mod.state_matrix(n)
            P = A
            for k in range(1, c + 1):
                if k > 1:
                    P = oracle_mod.minplus(A, P)
                G = tp.tp_ctx_copy_power(ctx, n, k)
                torch.cuda.synchronize()
                g = G.view(torch.int16).cpu().numpy().view(np.uint16).astype(np.int32)
                bad = np.argwhere(g != P)
                assert bad.size == 0, (n, k, bad[:5].tolist())
            assert got[list(cs).index(n)] == oracle_mod.trace_min(oracle_mod.minplus(P, P))
        with pytest.raises(tp.TropicalError):
            tp.tp_ctx_copy_power(ctx, 8, 99)
    finally:
        tp.tp_ctx_destroy(ctx)


@pytest.mark.parametrize("fused", [0, 1])
def test_compact_sets_equal_the_oracle(tp, oracle_table_500, fused):
    # path orders from 3 on keep A^3 and above as shared-base compact powers:
    # pairs of compact babies, giants as products of compact powers (bases
    # added) and traces adding the two bases, against the oracle; m = 3..6
    # are answered by the 16-bit A^1..A^3, m >= 7 by compact pairs
    rng = np.random.default_rng(31)
    inst = [(int(rng.integers(2, 9)), int(rng.integers(3, 501))) for _ in range(60)]
    inst += [(n, m) for n in (3, 6, 8) for m in (3, 4, 5, 6, 7, 8, 13, 14, 15, 16, 17, 40, 41)]
    ctx = tp.tp_ctx_create(64 << 30)
    try:
        tp.tp_ctx_set_param(ctx, tp.TP_PARAM_FUSED_CHAIN, fused)
        tp.tp_ctx_set_param(ctx, tp.TP_PARAM_COMPACT_FROM, 3)
        for n in range(2, 9):
            tp.tp_ctx_set_param(ctx, tp.TP_PARAM_BABY_STEPS + n, 5)
        say("compact batch, fused", fused)
        need = tp.tp_ctx_need_bytes(ctx, [n for n, _ in inst], [m for _, m in inst])
        got = _run(tp, ctx, inst)
        assert got == [int(oracle_table_500[n][m - 1]) for n, m in inst]
        assert tp.tp_ctx_resident_bytes(ctx) == need
        # resident compact powers answer the next batch, which adds giants
        inst2 = [(8, m) for m in (499, 400, 257, 129, 9)] + [(5, 450), (3, 7), (7, 333)]
        got2 = _run(tp, ctx, inst2)
        assert got2 == [int(oracle_table_500[n][m - 1]) for n, m in inst2]
        with pytest.raises(tp.TropicalError):
            tp.tp_ctx_set_param(ctx, tp.TP_PARAM_COMPACT_FROM, 0)
    finally:
        tp.tp_ctx_destroy(ctx)


def test_compact_powers_equal_the_oracle(tp, oracle_mod):
    # compact babies and giants, expanded to 16 bits by tp_ctx_copy_power,
    # entry by entry against the oracle's chain A^k = A x A^(k-1)
    import torch
    ctx = tp.tp_ctx_create(64 << 30)
    try:
        tp.tp_ctx_set_param(ctx, tp.TP_PARAM_COMPACT_FROM, 3)
        for n in (5, 8):
            tp.tp_ctx_set_param(ctx, tp.TP_PARAM_BABY_STEPS + n, 4)
        inst = [(5, 12), (8, 12), (5, 40), (8, 40)]
        got = _run(tp, ctx, inst)
        for n in (5, 8):
            A = oracle_mod.state_matrix(n)
            P = A
            want = {}
            for k in range(1, 37):
                if k > 1:
                    P = oracle_mod.minplus(A, P)
                if k in (1, 2, 3, 4, 5, 6, 8, 16, 32, 36):
                    want[k] = P
            for k, W in want.items():
                G = tp.tp_ctx_copy_power(ctx, n, k)
                torch.cuda.synchronize()
                g = G.view(torch.int16).cpu().numpy().view(np.uint16).astype(np.int32)
                bad = np.argwhere(g != W)
                assert bad.size == 0, (n, k, bad[:5].tolist())
            assert got[[i for i, (a, _) in enumerate(inst) if a == n][0]] == \
                oracle_mod.trace_min(oracle_mod.minplus(want[6], want[6]))
    finally:
        tp.tp_ctx_destroy(ctx)


@pytest.mark.parametrize("compact", [0, 3])
@pytest.mark.parametrize("fused", [0, 1])
def test_chained_giants_equal_the_oracle(tp, oracle_table_500, oracle_mod, compact, fused):
    # giants made by continuing the chain (TP_PARAM_CHAIN_GIANTS_FROM), in 16
    # bits and in compact form, against the oracle; a second batch seeds its
    # chain from a resident giant; a chained giant entry by entry
    import torch
    rng = np.random.default_rng(41 + compact + fused)
    inst = [(int(rng.integers(2, 9)), int(rng.integers(3, 501))) for _ in range(40)]
    inst += [(5, 40), (5, 41), (8, 333), (8, 13)]
    ctx = tp.tp_ctx_create(64 << 30)
    try:
        tp.tp_ctx_set_param(ctx, tp.TP_PARAM_FUSED_CHAIN, fused)
        tp.tp_ctx_set_param(ctx, tp.TP_PARAM_COMPACT_FROM, compact)
        tp.tp_ctx_set_param(ctx, tp.TP_PARAM_CHAIN_GIANTS_FROM, 3)
        for n in range(2, 9):
            tp.tp_ctx_set_param(ctx, tp.TP_PARAM_BABY_STEPS + n, 5)
        say("chained giants, compact", compact, "fused", fused)
        need = tp.tp_ctx_need_bytes(ctx, [n for n, _ in inst], [m for _, m in inst])
        got = _run(tp, ctx, inst)
        assert got == [int(oracle_table_500[n][m - 1]) for n, m in inst]
        assert tp.tp_ctx_resident_bytes(ctx) == need
        inst2 = [(8, m) for m in (499, 400, 257, 129, 9)] + [(5, 450), (3, 7), (7, 333)]
        got2 = _run(tp, ctx, inst2)
        assert got2 == [int(oracle_table_500[n][m - 1]) for n, m in inst2]
        # (5, 40): a giant of exponent 35 (40 = 35 + 5 in 16 bits; 37 + 3 is
        # not a pair, so compact c = 5 gives 35 + 5 as well)
        A = oracle_mod.state_matrix(5)
        P = A
        for _ in range(34):
            P = oracle_mod.minplus(A, P)
        G = tp.tp_ctx_copy_power(ctx, 5, 35)
        torch.cuda.synchronize()
        g = G.view(torch.int16).cpu().numpy().view(np.uint16).astype(np.int32)
        assert np.array_equal(g, P)
    finally:
        tp.tp_ctx_destroy(ctx)


def test_new_sets_may_chain_to_half_the_longest_cycle(tp, oracle_table):
    # baby steps from the library defaults (c0 = 16): cycle orders up to 50
    # need the giants A^32 and A^48, or, with c1 = 25, none; the planner's
    # rates decide (dense products made slow, then cheap)
    n, ms = 6, [3, 10, 40, 47, 50]
    N = tp.tp_state_dim(n)
    per = N * ((N + 63) // 64 * 64) * 2
    try:
        for gemm_rate, fused, powers in ((1e3, 0, 25), (1e18, 0, 18), (1e3, 1, 25)):
            say("planner gemm rate", gemm_rate, "fused", fused)
            tp.tp_tune_batch(n, 16, 16)
            tp.tp_tune_planner(n, 1e12, gemm_rate)
            ctx = tp.tp_ctx_create(1 << 34)
            try:
                tp.tp_ctx_set_param(ctx, tp.TP_PARAM_FUSED_CHAIN, fused)
                need = tp.tp_ctx_need_bytes(ctx, [n] * len(ms), ms)
                assert need == powers * per
                got = _run(tp, ctx, [(n, m) for m in ms])
                assert got == [int(oracle_table[n][m - 1]) for m in ms]
                assert tp.tp_ctx_resident_bytes(ctx) == need
                # the set keeps its baby steps: a longer cycle adds giants
                more = tp.tp_ctx_need_bytes(ctx, [n], [120])
                assert more > 0
                assert _run(tp, ctx, [(n, 120)]) == [int(oracle_table[n][119])]
            finally:
                tp.tp_ctx_destroy(ctx)
        # baby steps set on the context are kept as they are
        tp.tp_tune_planner(n, 1e12, 1e3)
        ctx = tp.tp_ctx_create(1 << 34)
        try:
            tp.tp_ctx_set_param(ctx, tp.TP_PARAM_BABY_STEPS + n, 16)
            assert tp.tp_ctx_need_bytes(ctx, [n] * len(ms), ms) == 18 * per
        finally:
            tp.tp_ctx_destroy(ctx)
    finally:
        tp.tp_tune_batch(n, 0, 0)
        tp.tp_tune_planner(n, 0.0, 0.0)
        tp.apply_tuning()


def test_fused_sets_chain_within_the_batch_deepest_chain(tp, oracle_table):
    # fused mode: n = 7 (baby steps set to 30 on the context) runs 30 levels;
    # n = 6 (library default c0 = 8) would make giants for cycles up to 50,
    # and chains to 25 instead, within those levels; split mode keeps c0
    # when dense products look cheap
    inst = [(7, 3), (7, 60), (6, 5), (6, 33), (6, 50)]
    ns, ms = [a for a, _ in inst], [b for _, b in inst]
    per = {n: tp.tp_state_dim(n) * ((tp.tp_state_dim(n) + 63) // 64 * 64) * 2 for n in (6, 7)}
    try:
        tp.tp_tune_batch(6, 8, 8)
        tp.tp_tune_planner(6, 1e12, 1e18)
        for fused, n6_powers in ((1, 25), (0, 8 + 3)):
            say("fused", fused)
            ctx = tp.tp_ctx_create(1 << 34)
            try:
                tp.tp_ctx_set_param(ctx, tp.TP_PARAM_FUSED_CHAIN, fused)
                tp.tp_ctx_set_param(ctx, tp.TP_PARAM_BABY_STEPS + 7, 30)
                need = tp.tp_ctx_need_bytes(ctx, ns, ms)
                assert need == 30 * per[7] + n6_powers * per[6]
                assert _run(tp, ctx, inst) == [int(oracle_table[n][m - 1]) for n, m in inst]
                assert tp.tp_ctx_resident_bytes(ctx) == need
            finally:
                tp.tp_ctx_destroy(ctx)
    finally:
        tp.tp_tune_batch(6, 0, 0)
        tp.tp_tune_planner(6, 0.0, 0.0)
        tp.apply_tuning()
