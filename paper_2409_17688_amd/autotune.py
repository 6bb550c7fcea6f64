"""Autotuner: measures kernel shapes on this GPU and writes the tuning table.

    python -m paper_2409_17688_amd.autotune                 # full sweep
    python -m paper_2409_17688_amd.autotune --quick --out /tmp/t.json
    python -m paper_2409_17688_amd.autotune --only batch   # one section, others kept

What it tunes (none of it changes a result, only which kernel shape runs):
  * dense products: for the state-matrix orders N(n), n = 4..11, and each
    dtype, every tile configuration x K split; the fastest becomes the
    default for products up to that size (``tp_tune_gemm``);
  * the sparse left step: the faster of its two forms per n, CSR gather or
    row blocks (``tp_tune_step``);
  * the schedule planner of ``tp_tropical_power_trace``: measured (min,+)
    rates of that step and of the tuned dense product per n
    (``tp_tune_planner``);
  * the batch engine, n = 4..9: baby steps c for the default mode and for
    the fused mode, on a batch of 32 instances with m uniform in 3..256,
    median of three cold batches per candidate (``tp_tune_batch``).  The
    batch engine adapts these per batch (longer chains instead of giants
    where they pay, and in the fused mode where the batch's deepest chain
    runs anyway).

Every candidate is checked against the reference shape (tile configuration
0 without a split for products, the built-in batch parameters for batches):
results must be identical, element for element, or the tuner stops.  Inputs
are the real state matrices A(D_n), built by the library; the batch
instances come from numpy's default_rng(seed).  Times come from HIP events
on the launch stream (products, sparse steps) or the host clock around a
complete batch (batches).

The table is a JSON file; ``tuning.apply_tuning`` (run by the package on
import) loads the package's ``tuning_gfx950.json``.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np
import torch

from . import _lib as tp
from .tuning import DEFAULT_TABLE, apply_gemm_rows, apply_tuning  # noqa: F401

KSPLITS = (1, 2, 4, 8, 16)
# candidates in this order; a later one must be faster by more than TIE to
# replace the best so far (large tiles first: they win near-ties at large N)
CONFIG_ORDER = (4, 1, 2, 0, 3)
TIE = 0.01
SECTIONS = ("gemm", "planner", "batch")


def _events(fn, min_ms=20.0, max_reps=50):
    """Average seconds per call of fn on the current stream (HIP events)."""
    fn()
    torch.cuda.synchronize()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    fn()
    e.record()
    torch.cuda.synchronize()
    one = max(s.elapsed_time(e), 1e-3)
    reps = int(max(3, min(max_reps, min_ms / one)))
    s.record()
    for _ in range(reps):
        fn()
    e.record()
    torch.cuda.synchronize()
    return s.elapsed_time(e) / reps / 1e3


def _padded(N, dtype):
    ld = (N + 63) // 64 * 64
    return torch.empty((N, ld), dtype=dtype, device="cuda")[:, :N]


def tune_gemm(ns, dtypes, log):
    """{dtype name: [[max_dim, config, ksplit, seconds], ...]} over N(n)."""
    out = {}
    for dt in dtypes:
        tdt = torch.uint16 if dt == tp.TP_U16 else torch.uint8
        rows = []
        for n in ns:
            N = tp.tp_state_dim(n)
            A = _padded(N, tdt)
            tp.tp_build_state_matrix(n, dt, out=A)
            ref = tp.tp_minplus_gemm(A, A, _padded(N, tdt), config=0, ksplit=1).clone()
            best = None
            for cfg in CONFIG_ORDER:
                for ks in KSPLITS:
                    # a split only pays when the output has few tiles
                    if ks > 1 and (N < 128 * ks or N >= 4096):
                        continue
                    C = _padded(N, tdt)
                    tp.tp_minplus_gemm(A, A, C, config=cfg, ksplit=ks)
                    if not torch.equal(C, ref):
                        raise RuntimeError(f"product n={n} config={cfg} ksplit={ks} differs")
                    t = _events(lambda: tp.tp_minplus_gemm(A, A, C, config=cfg, ksplit=ks))
                    if best is None or t < best[3] * (1.0 - TIE):
                        best = [N, cfg, ks, t]
            log(f"gemm dtype={dt} n={n} N={N}: config {best[1]} ksplit {best[2]} "
                f"{best[3] * 1e3:.3f} ms ({N ** 3 / best[3] / 1e12:.2f} T/s)")
            rows.append(best)
            del A, C, ref
        out["u16" if dt == tp.TP_U16 else "u8"] = rows
    return out


def tune_planner(ns, log):
    """({n: [sparse step ops/s, dense product ops/s]}, {n: step form}): the
    faster form of the sparse left step by n, and the rates the planner
    sees (tuned product shapes applied)."""
    out, forms = {}, {}
    last_gemm = None
    for n in ns:
        N = tp.tp_state_dim(n)
        nnz = tp.tp_state_nnz(n)
        X, Y = _padded(N, torch.uint16), _padded(N, torch.uint16)
        tp.tp_build_state_matrix(n, tp.TP_U16, out=X)
        ref = tp.tp_state_left_mul(n, X, _padded(N, torch.uint16), form=tp.TP_STEP_CSR).clone()
        ts = None
        for form in (tp.TP_STEP_CSR, tp.TP_STEP_BLOCKED):
            tp.tp_state_left_mul(n, X, Y, form=form)
            if not torch.equal(Y, ref):
                raise RuntimeError(f"sparse step n={n} form={form} differs")
            t = _events(lambda: tp.tp_state_left_mul(n, X, Y, form=form), min_ms=10.0,
                        max_reps=20)
            if ts is None or t < ts * (1.0 - TIE):
                ts, forms[n] = t, form
        if n <= 11:
            # the shape the planner's own products run (tuned config and K split)
            C = _padded(N, torch.uint16)
            cfg, ks = tp.tp_gemm_choice(tp.TP_U16, N, N, N)
            tg = _events(lambda: tp.tp_minplus_gemm(X, X, C, config=cfg, ksplit=ks), min_ms=10.0,
                         max_reps=20)
            last_gemm = N ** 3 / tg
            del C
        out[n] = [nnz * N / ts, last_gemm]
        log(f"planner n={n}: sparse step {out[n][0] / 1e12:.3f} T/s (form {forms[n]}), "
            f"dense product {out[n][1] / 1e12:.3f} T/s")
        del X, Y, ref
    return out, forms


def _batch_time(ns, ms, params, reps=3):
    """(median seconds of `reps` cold batches on fresh contexts, answers)."""
    times, res = [], None
    for _ in range(reps):
        ctx = tp.tp_ctx_create(64 << 30)
        try:
            for k, v in params.items():
                tp.tp_ctx_set_param(ctx, k, v)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = tp.tp_batch_power_trace(ctx, ns, ms)
            tp.tp_ctx_check(ctx)
            t = time.perf_counter() - t0
            res = r.cpu().numpy().tolist()
        finally:
            tp.tp_ctx_destroy(ctx)
        times.append(t)
    return sorted(times)[len(times) // 2], res


def tune_batch(ns, baby_list, seed, log):
    """{n: [baby steps, seconds, fused baby steps, seconds]}: fastest cold
    batch of 32 instances in each mode (median of three per candidate)."""
    rng = np.random.default_rng(seed)
    out = {}
    # load the batch kernel once so that the first candidate is not charged for it
    _batch_time([4], [5], {}, reps=1)
    for n in ns:
        ms = [int(m) for m in rng.integers(3, 257, 32)]
        nl = [n] * len(ms)
        tp.tp_tropical_power_trace(n, 3)  # state in the cache
        _, ref = _batch_time(nl, ms, {}, reps=1)
        row = []
        for fused in (0, 1):
            best = None
            for c in baby_list:
                t, res = _batch_time(nl, ms, {tp.TP_PARAM_BABY_STEPS + n: c,
                                              tp.TP_PARAM_FUSED_CHAIN: fused})
                if res != ref:
                    raise RuntimeError(f"batch n={n} c={c} fused={fused} differs")
                if best is None or t < best[1] * (1.0 - TIE):
                    best = [c, t]
            log(f"batch n={n} fused={fused}: baby steps {best[0]} {best[1] * 1e3:.2f} ms")
            row += best
        out[n] = row
    return out


def _dump(table, f):
    """JSON with one line per table row group (readable diffs)."""
    items = list(table.items())
    f.write("{\n")
    for i, (k, v) in enumerate(items):
        if isinstance(v, dict):
            f.write(f" {json.dumps(k)}: {{\n")
            sub = list(v.items())
            for j, (k2, v2) in enumerate(sub):
                f.write(f"  {json.dumps(str(k2))}: {json.dumps(v2)}")
                f.write(",\n" if j + 1 < len(sub) else "\n")
            f.write(" }")
        else:
            f.write(f" {json.dumps(k)}: {json.dumps(v)}")
        f.write(",\n" if i + 1 < len(items) else "\n")
    f.write("}\n")


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--out", default=DEFAULT_TABLE)
    ap.add_argument("--quick", action="store_true", help="small sweep (tests)")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--only", action="append", choices=SECTIONS,
                    help="tune only this section (repeatable); the others are kept from the "
                         "table at --out (or the package's table) and loaded before tuning")
    args = ap.parse_args(argv)
    only = set(args.only or SECTIONS)
    base = {}
    if only != set(SECTIONS):
        src = args.out if os.path.exists(args.out) else DEFAULT_TABLE
        with open(src) as f:
            base = json.load(f)

    def log(msg):
        print(msg, flush=True)

    # measure from the built-in defaults
    for dt in (tp.TP_U16, tp.TP_U8):
        tp.tp_tune_gemm(dt, -1)
    for n in range(1, 13):
        tp.tp_tune_batch(n, 0, 0)
        tp.tp_tune_planner(n, 0.0, 0.0)
        tp.tp_tune_step(n, tp.TP_STEP_AUTO)
    if args.quick:
        gemm_ns, planner_ns, batch_ns = (4, 5), (4, 5), (4,)
        baby_list = (8, 16)
    else:
        gemm_ns, planner_ns, batch_ns = tuple(range(4, 12)), tuple(range(1, 13)), tuple(range(4, 10))
        baby_list = (4, 6, 8, 12, 16, 24, 32, 48, 64, 96, 128, 192)
    table = {"arch": torch.cuda.get_device_properties(0).gcnArchName.split(":")[0],
             "device": torch.cuda.get_device_name(0),
             "date": time.strftime("%Y-%m-%d"),
             "note": "written by python -m paper_2409_17688_amd.autotune; changes only kernel "
                     "shapes, never results"}
    if "gemm" in only:
        table["gemm"] = tune_gemm(gemm_ns, (tp.TP_U16,), log)
        table["gemm"].update(tune_gemm(tuple(n for n in gemm_ns if n <= 10), (tp.TP_U8,), log))
    else:
        table["gemm"] = base["gemm"]
    for name, rows in table["gemm"].items():
        apply_gemm_rows(tp.TP_U16 if name == "u16" else tp.TP_U8, rows)
    if "planner" in only:
        table["planner"], table["step"] = tune_planner(planner_ns, log)
    else:
        table["planner"], table["step"] = base["planner"], base["step"]
        apply_tuning(table={"planner": table["planner"], "step": table["step"]})
    table["batch"] = tune_batch(batch_ns, baby_list, args.seed, log) if "batch" in only \
        else base["batch"]
    with open(args.out, "w") as f:
        _dump(table, f)
    log(f"wrote {args.out}")
    return 0


if __name__ == "__main__":
    sys.exit(main())
