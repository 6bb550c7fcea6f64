"""Split-K products and the tuning tables, through the C ABI.

Split-K products are compared with the CPU oracle element by element (exact
integers) over ragged shapes, both storage types, accumulate on and off and
slice counts from 2 up to more slices than K has 64-column blocks.  The
tuning tables change only which kernel shape runs: a table entry must show in
tp_gemm_choice and every tuned default must reproduce the untuned result.
"""
import json
import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

INF16, INF8 = 65535, 255


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def tp():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2409_17688_amd as tp
    return tp


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _reset_tables(tp):
    # built-in defaults, then the package's own table (if there is one)
    tp.tp_tune_gemm(tp.TP_U16, -1)
    tp.tp_tune_gemm(tp.TP_U8, -1)
    for n in range(1, 13):
        tp.tp_tune_batch(n, 0, 0)
        tp.tp_tune_planner(n, 0.0, 0.0)
        tp.tp_tune_step(n, tp.TP_STEP_AUTO)
    tp.apply_tuning()


SPLIT_SHAPES = [(70, 45, 1000), (130, 257, 777), (64, 64, 4096), (1, 300, 129), (257, 3, 200),
                (33, 65, 64)]


@pytest.mark.parametrize("dtype", [2, 1])
@pytest.mark.parametrize("shape", SPLIT_SHAPES)
def test_split_k_matches_oracle(tp, oracle_mod, dtype, shape):
    M, N, K = shape
    npdt = np.uint16 if dtype == 2 else np.uint8
    inf = INF16 if dtype == 2 else INF8
    hi = 30000 if dtype == 2 else 200
    for seed, frac in ((11, 0.3), (12, 0.95)):
        A = synth.stress_matrix(M, K, seed, 0, hi, frac, npdt)
        B = synth.stress_matrix(K, N, seed + 1, 0, hi, frac, npdt)
        C0 = synth.stress_matrix(M, N, seed + 2, 0, inf - 5, 0.2, npdt)
        ref = oracle_mod.minplus(A.astype(np.int32), B.astype(np.int32), inf)
        for config in (0, 3):
            for ksplit in (2, 3, 8, 64):
                for accumulate in (False, True):
                    say("split-K", dtype, shape, seed, config, ksplit, accumulate)
                    dC = dev(C0)
                    tp.tp_minplus_gemm(dev(A), dev(B), dC, accumulate=accumulate,
                                       config=config, ksplit=ksplit)
                    want = np.minimum(ref, C0.astype(np.int32)) if accumulate else ref
                    got = host(dC).astype(np.int32)
                    assert np.array_equal(got, want), (dtype, shape, config, ksplit, accumulate)


def test_split_k_on_strided_views(tp, oracle_mod):
    # leading dimensions larger than the columns, C written only inside its view
    M, N, K, pad = 100, 90, 700, 13
    A = synth.stress_matrix(M, K + pad, 3, 0, 500, 0.3, np.uint16)
    B = synth.stress_matrix(K, N + pad, 4, 0, 500, 0.3, np.uint16)
    C0 = synth.stress_matrix(M, N + pad, 5, 0, 60000, 0.0, np.uint16)
    dA, dB, dC = dev(A), dev(B), dev(C0)
    tp.tp_minplus_gemm(dA[:, :K], dB[:, :N], dC[:, :N], config=0, ksplit=4)
    got = host(dC).astype(np.int32)
    ref = oracle_mod.minplus(A[:, :K].astype(np.int32), B[:, :N].astype(np.int32), INF16)
    assert np.array_equal(got[:, :N], ref)
    assert np.array_equal(got[:, N:], C0[:, N:].astype(np.int32)), "wrote outside C"


def test_split_k_rejects_bad_arguments(tp):
    A = dev(np.zeros((4, 4), np.uint16))
    for ks in (0, 65):
        with pytest.raises(tp.TropicalError):
            tp.tp_minplus_gemm(A, A, config=0, ksplit=ks)
    with pytest.raises(tp.TropicalError):
        tp.tp_minplus_gemm(A, A, config=tp.tp_gemm_config_count(), ksplit=1)


def test_split_k_state_matrix_square(tp):
    # real power: A(D_8) squared, every config and split equal to the unsplit product
    n = 8
    A = tp.tp_build_state_matrix(n, tp.TP_U16)
    ref = host(tp.tp_minplus_gemm(A, A, config=0, ksplit=1))
    for config in range(tp.tp_gemm_config_count()):
        for ksplit in (2, 5, 16):
            say("A(D_8)^2 config", config, "ksplit", ksplit)
            got = host(tp.tp_minplus_gemm(A, A, config=config, ksplit=ksplit))
            assert np.array_equal(got, ref), (config, ksplit)


def test_tuning_table_choice_and_clear(tp):
    saved = [tp.tp_gemm_choice(tp.TP_U16, N, N, N) for N in (100, 1000, 5000)]
    try:
        tp.tp_tune_gemm(tp.TP_U16, -1)
        tp.tp_tune_gemm(tp.TP_U16, 500, 3, 4)
        tp.tp_tune_gemm(tp.TP_U16, 2000, 2, 1)
        assert tp.tp_gemm_choice(tp.TP_U16, 100, 100, 100) == (3, 4)
        assert tp.tp_gemm_choice(tp.TP_U16, 300, 500, 10) == (3, 4)
        assert tp.tp_gemm_choice(tp.TP_U16, 501, 10, 10) == (2, 1)
        tp.tp_tune_gemm(tp.TP_U16, 500, 1, 2)  # replaces the entry
        assert tp.tp_gemm_choice(tp.TP_U16, 100, 100, 100) == (1, 2)
        # beyond the table: the built-in rule, the same as an empty table
        beyond = tp.tp_gemm_choice(tp.TP_U16, 5000, 5000, 5000)
        tp.tp_tune_gemm(tp.TP_U16, -1)
        assert tp.tp_gemm_choice(tp.TP_U16, 5000, 5000, 5000) == beyond
        with pytest.raises(tp.TropicalError):
            tp.tp_tune_gemm(tp.TP_U16, 100, 99, 1)
        with pytest.raises(tp.TropicalError):
            tp.tp_tune_planner(4, 0.0, 1.0)
        with pytest.raises(tp.TropicalError):
            tp.tp_tune_batch(13, 8, 8)
    finally:
        tp.tp_tune_gemm(tp.TP_U16, -1)
        tp.apply_tuning()
    assert [tp.tp_gemm_choice(tp.TP_U16, N, N, N) for N in (100, 1000, 5000)] == saved


def test_tuned_defaults_do_not_change_results(tp, oracle_mod):
    # an extreme table (tiny tiles and splits everywhere) against the oracle,
    # for products and for gamma_2 through the planner and the batch engine
    try:
        tp.tp_tune_gemm(tp.TP_U16, -1)
        tp.tp_tune_gemm(tp.TP_U16, 1 << 40, 3, 8)
        for n in range(4, 9):
            tp.tp_tune_planner(n, 1e9, 1e14)  # dense products look cheap: more of them
            tp.tp_tune_batch(n, 5, 3)
            tp.tp_tune_step(n, tp.TP_STEP_BLOCKED if n % 2 else tp.TP_STEP_CSR)
        A = synth.stress_matrix(300, 900, 21, 0, 1000, 0.4, np.uint16)
        B = synth.stress_matrix(900, 200, 22, 0, 1000, 0.4, np.uint16)
        got = host(tp.tp_minplus_gemm(dev(A), dev(B))).astype(np.int32)
        assert np.array_equal(got, oracle_mod.minplus(A.astype(np.int32), B.astype(np.int32),
                                                      INF16))
        cases = [(n, m) for n in (4, 6, 8) for m in (3, 7, 20, 41)]
        sweep = {n: oracle_mod.gamma2_sweep(n, 41) for n in (4, 6, 8)}
        want = [int(sweep[n][m - 1]) for n, m in cases]
        plain = [tp.tp_tropical_power_trace(n, m) for n, m in cases]
        assert plain == want
        ctx = tp.tp_ctx_create(8 << 30)
        try:
            res = tp.tp_batch_power_trace(ctx, [n for n, _ in cases], [m for _, m in cases])
            tp.tp_ctx_check(ctx)
            assert host(res).tolist() == want
        finally:
            tp.tp_ctx_destroy(ctx)
    finally:
        _reset_tables(tp)


def test_autotuner_quick_run_writes_a_loadable_table(tp, tmp_path):
    from paper_2409_17688_amd import autotune
    out = tmp_path / "table.json"
    try:
        assert autotune.main(["--quick", "--out", str(out)]) == 0
        table = json.loads(out.read_text())
        assert table["arch"] == "gfx950"
        for N, cfg, ks, t in table["gemm"]["u16"]:
            assert 0 <= cfg < tp.tp_gemm_config_count() and ks >= 1 and t > 0
        assert set(table["batch"]) == {"4"}
        assert autotune.apply_tuning(str(out))
    finally:
        _reset_tables(tp)


def test_autotuner_only_one_section_keeps_the_others(tp, tmp_path):
    from paper_2409_17688_amd import autotune
    out = tmp_path / "table.json"
    try:
        assert autotune.main(["--quick", "--out", str(out)]) == 0
        first = json.loads(out.read_text())
        # mark the kept sections so that a re-tune would show
        first["gemm"]["u16"][0][3] = 123.0
        first["planner"]["4"] = [1.5e9, 2.5e9]
        out.write_text(json.dumps(first))
        assert autotune.main(["--quick", "--only", "batch", "--out", str(out)]) == 0
        second = json.loads(out.read_text())
        assert second["gemm"] == first["gemm"] and second["planner"] == first["planner"]
        assert second["step"] == first["step"]
        assert set(second["batch"]) == {"4"} and second["batch"]["4"][0] in (8, 16)
        assert autotune.apply_tuning(str(out))
    finally:
        _reset_tables(tp)
