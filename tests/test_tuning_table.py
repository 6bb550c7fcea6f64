"""The committed tuning table: well formed, loadable, and what it loads is
what the library reports (host-side calls only, no GPU needed)."""
import json
import os

import pytest

import paper_2409_17688_amd as tp
from paper_2409_17688_amd import tuning

TABLE = tuning.DEFAULT_TABLE


@pytest.fixture(scope="module")
def table():
    if not os.path.exists(TABLE):
        pytest.skip("no tuning table committed")
    with open(TABLE) as f:
        return json.load(f)


def test_table_is_well_formed(table):
    assert table["arch"] == "gfx950"
    for name in ("u16", "u8"):
        rows = table["gemm"][name]
        dims = [r[0] for r in rows]
        assert dims == sorted(dims) and len(set(dims)) == len(dims)
        for N, cfg, ks, t in rows:
            assert 0 <= cfg < tp.tp_gemm_config_count()
            assert 1 <= ks <= 64 and t > 0
    for n, (spmm, gemm) in table["planner"].items():
        assert 1 <= int(n) <= 12 and spmm > 0 and gemm > 0
    for n, form in table["step"].items():
        assert 1 <= int(n) <= 12 and form in (tp.TP_STEP_CSR, tp.TP_STEP_BLOCKED)
    for n, vals in table["batch"].items():
        assert 1 <= int(n) <= 12 and len(vals) in (2, 4)
        assert vals[0] >= 1 and vals[1] > 0
        if len(vals) == 4:
            assert vals[2] >= 1 and vals[3] > 0


def test_loaded_table_drives_the_default_choice(table):
    try:
        assert tuning.apply_tuning(TABLE)
        rows = table["gemm"]["u16"]
        for i, (N, cfg, ks, _) in enumerate(rows):
            assert tp.tp_gemm_choice(tp.TP_U16, N, N, N) == (cfg, ks)
            if i + 1 < len(rows):
                # one past an entry's size falls to the next entry
                nxt = rows[i + 1]
                assert tp.tp_gemm_choice(tp.TP_U16, N + 1, N + 1, N + 1) == (nxt[1], nxt[2])
        # the last entry covers every larger product
        assert tp.tp_gemm_choice(tp.TP_U16, 60000, 60000, 60000) == tuple(rows[-1][1:3])
    finally:
        tp.tp_tune_gemm(tp.TP_U16, -1)
        tp.tp_tune_gemm(tp.TP_U8, -1)
        for n in range(1, 13):
            tp.tp_tune_batch(n, 0, 0)
            tp.tp_tune_planner(n, 0.0, 0.0)
            tp.tp_tune_step(n, tp.TP_STEP_AUTO)
        tuning.apply_tuning()
