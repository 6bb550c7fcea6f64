"""The C ABI on the host: the library loads, exports every declared symbol,
sizes state matrices like Table 1 and rejects bad arguments before any GPU
work.  No compute call is made here."""
import ctypes
import os
import re

import pytest

from conftest import ROOT, read_table


def _declared_symbols():
    names = set()
    inc = os.path.join(ROOT, "include")
    for fn in os.listdir(inc):
        if fn.endswith(".h"):
            text = open(os.path.join(inc, fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names.update(re.findall(r"\b(tp_[a-z0-9_]+)\s*\(", text))
    return sorted(names)


@pytest.fixture(scope="module")
def tp():
    import paper_2409_17688_amd as tp
    return tp


def test_every_declared_symbol_is_exported(tp):
    declared = _declared_symbols()
    assert len(declared) >= 15
    for name in declared:
        assert hasattr(tp.lib, name), name
        assert name in tp.EXPORTED, f"{name} has no binding"


def test_library_is_hip_for_gfx950(tp):
    # the shared object carries a gfx950 code object
    blob = open(tp.LIB_PATH, "rb").read()
    assert b"gfx950" in blob


def test_state_dim_table1(tp):
    for n, rows, _ in read_table("table1_rows.txt"):
        assert tp.tp_state_dim(int(n)) == int(rows)
    assert tp.tp_state_dim(1) == 3


def test_argument_errors_before_gpu_work(tp):
    lib = tp.lib
    assert lib.tp_state_dim(0) == tp.TP_EINVAL
    assert lib.tp_state_dim(14) == tp.TP_EINVAL
    # bad dtype, negative size, short leading dimension, NULL pointers
    assert lib.tp_minplus_gemm(7, 4, 4, 4, 1, 4, 1, 4, 1, 4, 0, None) == tp.TP_EINVAL
    assert lib.tp_minplus_gemm(2, -1, 4, 4, 1, 4, 1, 4, 1, 4, 0, None) == tp.TP_EINVAL
    assert lib.tp_minplus_gemm(2, 4, 4, 8, 1, 4, 1, 4, 1, 4, 0, None) == tp.TP_EINVAL
    assert lib.tp_minplus_gemm(2, 4, 4, 4, None, 4, 1, 4, 1, 4, 0, None) == tp.TP_EINVAL
    assert "leading dimension" in tp.tp_last_error() or "NULL" in tp.tp_last_error()
    assert lib.tp_minplus_gemm_config(2, 4, 4, 4, 1, 4, 1, 4, 1, 4, 0, 99, None) == tp.TP_EINVAL
    assert lib.tp_minplus_gemv(2, 4, 4, 1, 4, 1, 1, 2, None) == tp.TP_EINVAL
    assert lib.tp_trace_of_product(2, 4, 1, 2, 1, 4, 1, None) == tp.TP_EINVAL
    res = ctypes.c_int32(0)
    assert lib.tp_tropical_power_trace(3, 2, ctypes.byref(res), None) == tp.TP_EINVAL
    assert lib.tp_tropical_power_trace(13, 5, ctypes.byref(res), None) == tp.TP_EINVAL
    assert lib.tp_tropical_power_trace(12, 6000, ctypes.byref(res), None) == tp.TP_EOVERFLOW
    assert "65535" in tp.tp_last_error()


def test_binding_raises(tp):
    with pytest.raises(tp.TropicalError):
        tp.tp_state_dim(0)
