"""Loads a tuning table (written by ``autotune``) into the library.

A table maps problem sizes to kernel shapes (tile configuration and K split
of dense products, the sparse step's form, baby steps of the batch engine) and
records measured kernel rates for the schedule planner.  None of it changes a
result.  The package applies ``tuning_gfx950.json`` on import.
"""
from __future__ import annotations

import json
import os

from . import _lib as tp

DEFAULT_TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning_gfx950.json")


def apply_gemm_rows(dt: int, rows) -> None:
    """rows: [max_dim, config, ksplit, seconds] by increasing max_dim."""
    tp.tp_tune_gemm(dt, -1)
    for i, (N, cfg, ks, _) in enumerate(rows):
        # the largest measured size also covers every larger product
        tp.tp_tune_gemm(dt, N if i + 1 < len(rows) else (1 << 40), cfg, ks)


def apply_tuning(path: str | None = None, table: dict | None = None) -> bool:
    """Loads a tuning table into the library; False when there is none."""
    if table is None:
        path = path or DEFAULT_TABLE
        if not os.path.exists(path):
            return False
        with open(path) as f:
            table = json.load(f)
    for name, rows in table.get("gemm", {}).items():
        apply_gemm_rows(tp.TP_U16 if name == "u16" else tp.TP_U8, rows)
    for n, (spmm, gemm) in table.get("planner", {}).items():
        tp.tp_tune_planner(int(n), float(spmm), float(gemm))
    for n, form in table.get("step", {}).items():
        tp.tp_tune_step(int(n), int(form))
    for n, vals in table.get("batch", {}).items():
        # [baby steps, seconds] or [baby steps, seconds, fused baby steps, seconds]
        tp.tp_tune_batch(int(n), int(vals[0]), int(vals[2]) if len(vals) >= 4 else 0)
    return True
