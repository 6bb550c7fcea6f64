"""Benchmark: raw (min,+) product throughput on one MI355X.

Workload (one step): C = A x B in the (min,+) semiring for square uint16
matrices of order 8192, entries uniform in 0..24 with 30 % set to INF = 65535,
drawn with numpy.random.default_rng(0), A before B.  Inputs are resident in
HBM before timing starts.  One step = one launch of the dense product kernel;
algorithmic work = N^3 (min,+) operations per step.

Prints one JSON line with the throughput, the kernel's roofline position and
the CPU oracle timed on a bounded sample of the same product.

usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-suite]
       [--no-serve]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X: 256 CUs x 64 lanes x 2.4 GHz; one v_pk_add_u16 plus one v_pk_min_u16
# make two (min,+) operations, i.e. one per lane per clock.
PEAK_MINPLUS = 256 * 64 * 2.4e9
N_DEFAULT = 8192

# HBM bytes per launch of the N = 8192 product from rocprofv3 FETCH_SIZE and
# WRITE_SIZE (KiB per dispatch, each scaled by what the counter reads for a
# plain 256 MiB copy: factors 2.00 and 1.00).  Valid for the kernel named
# below only; set to None when that kernel changes until it is measured again.
MEASURED_TRAFFIC = {"kernel": "minplus_gemm_kernel<128,256,32,8,16,3,u16,vec>",
                    "config": 1, "ksplit": 1,
                    "bytes": (1053160 * 2.00 + 131072 * 1.00) * 1024}
# tile configuration index -> kernel template arguments (BM, BN, BK, TM, TN, MINB)
KERNEL_SHAPES = {0: "128,128,32,8,8,4", 1: "128,256,32,8,16,3", 2: "256,128,32,16,8,3",
                 3: "64,64,32,4,4,4", 4: "256,256,32,16,16,2"}


def note(msg):
    """A progress line on stderr as each leg ends (the JSON line stays alone on stdout)."""
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=N_DEFAULT, help="matrix order")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="target duration of the CPU oracle sample")
    ap.add_argument("--no-suite", action="store_true",
                    help="skip timing gamma_2 queries (plain per-query path vs batched)")
    ap.add_argument("--no-serve", action="store_true",
                    help="skip the serving stream (about two minutes)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one plain 256 MiB device-to-device copy before the product, as "
                         "the reference point for HBM byte counters")
    return ap.parse_args()


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(A, B, target_s):
    """The CPU oracle on a bounded sample of the same product: a block of rows
    of C = A x B (each row is an independent (min,+) vector-matrix product),
    on every host core the oracle's OpenMP loop takes, then on one core."""
    import numpy as np

    import oracle
    Ai = A.astype(np.int32)
    Bi = B.astype(np.int32)
    N = A.shape[0]

    def sample(seconds):
        rows, dt = 16, 0.0
        while dt < 0.2 * seconds and rows < N:
            rows = min(N, rows * 2)
            t0 = time.perf_counter()
            oracle.minplus(Ai[:rows], Bi)
            dt = time.perf_counter() - t0
        rows = int(max(16, min(N, rows * seconds / max(dt, 1e-6))))
        t0 = time.perf_counter()
        oracle.minplus(Ai[:rows], Bi)
        return rows, time.perf_counter() - t0

    cores = oracle.threads()
    rows, dt = sample(target_s)
    oracle.set_threads(1)
    try:
        rows1, dt1 = sample(max(1.0, target_s / 4))
    finally:
        oracle.set_threads(cores)
    inf_a = float((A >= 65535).mean())
    return {"value": float(rows) * N * N / dt / 1e9, "unit": "Gminplus-ops/s", "cores": cores,
            "kind": "oracle", "cpu_model": cpu_model(),
            "sample": f"{rows} of {N} rows of C = A x B (same inputs), {dt:.1f} s",
            "one_core_value": round(float(rows1) * N * N / dt1 / 1e9, 2),
            "one_core_sample": f"{rows1} rows, {dt1:.1f} s",
            "note": (f"credited N^3 per product; the oracle skips k where a_ik = INF "
                     f"({100 * inf_a:.0f} % of A), so it executes about "
                     f"{100 * (1 - inf_a):.0f} % of those operations")}


def oracle_query_baseline(synth, budget_s=12.0):
    """The oracle timed on the mixed 64-instance batch, bounded: per path order
    of the batch, the time of one step of its power chain (Algorithm 2, a dense
    N^3 product) measured on a short chain less the time of building its state
    matrix, times the m - 1 steps each instance needs (the oracle answers
    gamma_2(n, m) by m - 1 steps)."""
    import oracle
    inst = synth.batch_instances(seed=0)
    per_step = {}
    spent = 0.0
    for n in sorted({n for n, _ in inst}):
        t0 = time.perf_counter()
        oracle.gamma2_sweep(n, 1)  # the state matrix and one trace, no product
        base = time.perf_counter() - t0
        k = 2
        while True:
            t0 = time.perf_counter()
            oracle.gamma2_sweep(n, k)
            dt = time.perf_counter() - t0
            if dt > 1.0 or k >= 64 or spent + dt > budget_s:
                break
            k *= 2
        spent += dt + base
        per_step[n] = max(dt - base, 1e-9) / (k - 1)
    est = sum((m - 1) * per_step[n] for n, m in inst)
    return {"value": round(len(inst) / est, 3), "unit": "queries/s", "cores": oracle.threads(),
            "kind": "oracle", "cpu_model": cpu_model(),
            "sample": ("mixed 64 instances: per-n step time of the oracle's power chain "
                       f"(measured on chains of up to 64 powers, {spent:.1f} s) times the "
                       f"m - 1 steps of each instance; estimated {est:.0f} s for the batch")}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); this workload has no "
              "multi-GPU path", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2409_17688_amd as tp
    import synth

    N = args.n
    A, B = synth.raw_gemm_pair(N, seed=0)
    # the tile configuration the default path runs for this product (tuning
    # table or built-in rule); tp_minplus_gemm never splits K
    cfg, _ = tp.tp_gemm_choice(tp.TP_U16, N, N, N)
    ksplit = 1
    kernel = f"minplus_gemm_kernel<{KERNEL_SHAPES[cfg]},u16,vec>"
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    dA = torch.from_numpy(A).to(dev)
    dB = torch.from_numpy(B).to(dev)
    dC = torch.empty((N, N), dtype=torch.uint16, device=dev)
    stream = torch.cuda.current_stream()
    if args.copy_calibration:
        src = torch.ones(256 << 20, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    for _ in range(args.warmup):
        tp.tp_minplus_gemm(dA, dB, dC, stream=stream)
    torch.cuda.synchronize()

    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        starts[i].record(stream)
        tp.tp_minplus_gemm(dA, dB, dC, stream=stream)
        ends[i].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern_ms = [s.elapsed_time(e) for s, e in zip(starts, ends)]
    avg_kernel_s = sum(kern_ms) / len(kern_ms) / 1e3
    ops = float(N) ** 3
    value = ops * args.steps / wall / 1e9
    achieved = ops / avg_kernel_s

    # sanity: a few outputs against a direct evaluation of the definition
    C = dC.cpu().numpy()
    rng = np.random.default_rng(1)
    for _ in range(16):
        i, j = (int(v) for v in rng.integers(0, N, 2))
        ref = int(np.minimum(A[i].astype(np.int64) + B[:, j].astype(np.int64), 65535).min())
        if int(C[i, j]) != ref:
            print(f"MISMATCH at ({i},{j}): {int(C[i, j])} != {ref}", file=sys.stderr)
            sys.exit(1)

    line = {
        "metric": "Gminplus-ops/s (raw minplus_gemm)",
        "value": round(value, 1),
        "unit": "Gminplus-ops/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u16",
        "data": "synthetic",
        "config": {"workload": f"minplus_gemm u16 square N={N}, entries uniform 0..24, "
                               "30% INF=65535, numpy default_rng(0) A then B",
                   "N": N, "global_batch": 1, "parallelism": "single GPU"},
        "roofline": {"bound": "alu", "achieved": round(achieved / 1e12, 3),
                     "peak": round(PEAK_MINPLUS / 1e12, 3), "unit": "Tminplus-ops/s",
                     "frac": round(achieved / PEAK_MINPLUS, 4),
                     "traffic": (round(MEASURED_TRAFFIC["bytes"])
                                 if MEASURED_TRAFFIC and N == N_DEFAULT
                                 and (cfg, ksplit) == (MEASURED_TRAFFIC["config"],
                                                       MEASURED_TRAFFIC["ksplit"])
                                 else None),
                     "kernel": kernel + (f" x{ksplit} K slices" if ksplit > 1 else "")},
        "kernel_ms": round(avg_kernel_s * 1e3, 3),
    }
    note(f"product timed: {avg_kernel_s * 1e3:.3f} ms per launch")
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(A, B, args.cpu_seconds)
        note("cpu baseline done")
    if not args.no_suite or not args.no_serve:
        del dA, dB, dC
        torch.cuda.empty_cache()
    if not args.no_suite:
        line["queries"] = query_suite(tp, synth)
        note("query suite done")
        if not args.no_cpu:
            line["queries"]["mixed64"]["cpu_baseline"] = oracle_query_baseline(synth)
            note("oracle query baseline done")
        line["cyclic_walk"] = cyclic_suite(tp)
        note("cyclic walk suite done")
        line["recurrence"] = recurrence_suite(tp)
        note("recurrence suite done")
    if not args.no_serve:
        line["serving"] = serve_suite(tp, synth)
        note("serving done")
    print(json.dumps(line), flush=True)


# Total running time of the paper's whole pipeline (50 powers, Algorithms 3,
# 4 and 5) in its fastest version, by path order (Table 5), in seconds.
PAPER_TOTAL_S = {8: 0.6, 9: 3.5, 10: 32.5, 11: 6 * 60 + 32, 12: 3600 + 29 * 60 + 58}


def recurrence_suite(tp):
    """The recurrence of the powers (Algorithms 3, 4 and 5 on K = 50 powers)
    by path order: wall time of tp_recurrence with the state already built,
    the recurrence found (Tables 3 and 4), and the paper's total time."""
    import torch
    out = {}
    for n, window in ((8, 0), (9, 0), (10, 0), (11, 6), (12, 4)):
        tp.tp_recurrence(n, 3, 1)  # the state of n in the library's cache
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rec, _ = tp.tp_recurrence(n, 50, window)
        t = time.perf_counter() - t0
        out[str(n)] = {"K": 50, "window": rec.window, "seconds": round(t, 4),
                       "r0": rec.r0, "a": rec.a, "b": rec.b, "n0": rec.n0,
                       "paper_total_seconds": PAPER_TOTAL_S[n]}
    return out


def serve_suite(tp, synth, count=2000):
    """Serving: a Poisson stream of `count` queries, n in 6..12 weighted by
    2^-(n-6), m uniform in 3..500 (seed 0), on one server: two batch contexts
    (two waves in flight) for n <= 9 and resident compact lanes for n = 10..12,
    admission by HBM.

    saturation: every query submitted at once, on a cold server (nothing
    resident), then again warm (the powers the first pass left resident);
    warm replay: the stream at 70 % of the warm saturation rate, p50/p99
    latency over all queries and per n;
    cold replay: a fresh server fed the stream at 70 % of the cold saturation
    rate, so the latencies include building the resident powers as queries
    need them;
    plain: tp_tropical_power_trace one query at a time, estimated as the mean
    time of a stratified sample per n times that n's count in the stream
    (answers of the sample are compared with the served ones); served vs
    plain from the cold and from the warm pass."""
    import gc

    import numpy as np
    import torch

    from paper_2409_17688_amd import serve
    free, _ = torch.cuda.mem_get_info()
    budget = max(8 << 30, free - (48 << 30))
    unit = synth.serve_stream(seed=0, count=count, qps=1.0)
    out = {"queries": count, "budget_bytes": int(budget), "slots": 2,
           "lane_orders": sorted(serve.LANE_ORDERS)}

    def lat_stats(reqs, prefix):
        lat = [r.latency for r in reqs]
        by_n = {}
        for r in reqs:
            by_n.setdefault(r.n, []).append(r.latency)
        return {f"{prefix}_p50_ms": round(serve.percentile(lat, 50) * 1e3, 2),
                f"{prefix}_p99_ms": round(serve.percentile(lat, 99) * 1e3, 2),
                f"{prefix}_p99_ms_by_n": {str(n): round(serve.percentile(v, 99) * 1e3, 1)
                                          for n, v in sorted(by_n.items())}}

    def burst(srv):
        t0 = time.perf_counter()
        reqs = [srv.submit(n, m, t_arrive=t0) for _, n, m in unit]
        for r in reqs:
            r.wait(900)
        return reqs, time.perf_counter() - t0

    def replay(srv, qps):
        t0 = time.perf_counter()
        reqs = []
        for t, n, m in unit:
            delay = t / qps - (time.perf_counter() - t0)
            if delay > 0:
                time.sleep(delay)
            reqs.append(srv.submit(n, m))
        for r in reqs:
            r.wait(900)
        return reqs, time.perf_counter() - t0

    def check(reqs, what):
        if any(r.status != serve.TP_OK or r.gamma2 != served[(r.n, r.m)] for r in reqs):
            print(f"serving: {what} differs from the cold pass", file=sys.stderr)
            sys.exit(1)

    ex = serve.GpuExecutor(budget, slots=2)
    srv = serve.Server(ex, max_wave=1024)
    try:
        reqs, t_cold = burst(srv)
        note(f"serving: cold pass {t_cold:.1f} s")
        served = {(r.n, r.m): r.gamma2 for r in reqs}
        bad = [r for r in reqs if r.status != serve.TP_OK]
        if bad:
            print(f"serving failed: {bad[0].n} {bad[0].m} {bad[0].error}", file=sys.stderr)
            sys.exit(1)
        out.update(lat_stats(reqs, "cold_burst"))
        reqs, t_warm = burst(srv)
        note(f"serving: warm pass {t_warm:.1f} s")
        check(reqs, "warm pass")
        qps = 0.7 * count / t_warm
        reqs, t_replay = replay(srv, qps)
        note(f"serving: warm replay {t_replay:.1f} s")
        check(reqs, "warm replay")
        out.update({"saturation_qps_cold": round(count / t_cold, 1),
                    "saturation_qps_warm": round(count / t_warm, 1),
                    "replay_qps": round(qps, 1),
                    "replay_seconds": round(t_replay, 2)})
        out.update(lat_stats(reqs, "replay"))
        out.update({"waves": srv.waves, "max_waves_in_flight": srv.max_in_flight,
                    "resident_bytes": int(ex.resident_bytes()),
                    "lanes": {str(l.n): {"level": l.level, "panels": len(l.panels),
                                         "trace_answers": l.trace_answers,
                                         "plain_answers": l.plain_answers,
                                         "reserved_bytes": int(l.reserved_bytes)}
                              for l in ex.lanes}})
    finally:
        srv.close()
        ex.close()
    del srv, ex
    gc.collect()
    torch.cuda.empty_cache()
    # a fresh server fed at 70 % of the cold saturation rate
    ex = serve.GpuExecutor(budget, slots=2)
    srv = serve.Server(ex, max_wave=1024)
    try:
        qps_c = 0.7 * count / t_cold
        reqs, t_creplay = replay(srv, qps_c)
        note(f"serving: cold replay {t_creplay:.1f} s")
        check(reqs, "cold replay")
        out.update({"cold_replay_qps": round(qps_c, 1),
                    "cold_replay_seconds": round(t_creplay, 2)})
        out.update(lat_stats(reqs, "cold_replay"))
        out["cold_replay_max_waves_in_flight"] = srv.max_in_flight
    finally:
        srv.close()
        ex.close()
    del srv, ex
    gc.collect()
    torch.cuda.empty_cache()
    # plain path on a stratified sample
    rng = np.random.default_rng(1)
    counts, plain_total = {}, 0.0
    for _, n, m in unit:
        counts[n] = counts.get(n, 0) + 1
    for n, cnt in sorted(counts.items()):
        pool = [(nn, m) for _, nn, m in unit if nn == n]
        k = 2 if n >= 12 else 4
        pick = [pool[int(i)] for i in rng.choice(len(pool), size=min(k, len(pool)), replace=False)]
        tp.tp_tropical_power_trace(n, 3)
        t0 = time.perf_counter()
        for nn, m in pick:
            g = tp.tp_tropical_power_trace(nn, m)
            if g != served[(nn, m)]:
                print(f"MISMATCH served vs plain at ({nn},{m})", file=sys.stderr)
                sys.exit(1)
        plain_total += (time.perf_counter() - t0) / len(pick) * cnt
    out["plain_qps_estimate"] = round(count / plain_total, 2)
    out["served_vs_plain_cold"] = round((count / t_cold) / (count / plain_total), 1)
    out["served_vs_plain_warm"] = round((count / t_warm) / (count / plain_total), 1)
    # recurrence mode, reported apart from the served path: one recurrence of
    # the powers per path order of the stream (K = 50), then every query from
    # Theorem 3's solution on the host
    t0 = time.perf_counter()
    recs = {n: tp.tp_recurrence(n, 50, 4 if n >= 12 else (6 if n == 11 else 0))
            for n in sorted(counts)}
    t_setup = time.perf_counter() - t0
    t0 = time.perf_counter()
    ans = [tp.tp_gamma2_recurrence(*recs[n], m) for _, n, m in unit]
    t_ans = time.perf_counter() - t0
    out["recurrence_mode"] = {
        "setup_s": round(t_setup, 3), "answer_us_per_query": round(t_ans / count * 1e6, 2),
        "qps_including_setup": round(count / (t_setup + t_ans), 1),
        "agrees_with_served": all(a == served[(n, m)] for a, (_, n, m) in zip(ans, unit))}
    return out


def cyclic_suite(tp, nmax=200, ms=range(3, 9)):
    """Small cycle, any path: gamma_2(P_n x C_m) for m = 3..8 and every
    n = 1..nmax.  'plain' answers one query by tp_cyclic_walk_gamma2 (n - 1
    dense vector-matrix products), timed on a sample of n per m and scaled to
    the nmax queries of that m; 'sweep' answers all nmax of one m by a single
    tp_cyclic_walk_sweep (one walk, every level read by the end vector).
    Sampled plain answers are compared with the sweep's."""
    import torch
    total_plain, total_sweep, per_m = 0.0, 0.0, {}
    for m in ms:
        tp.tp_cyclic_walk_sweep(m, 2)  # the digraph of m in the library's cache
        tp.tp_cyclic_walk_gamma2(2, m)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sweep = tp.tp_cyclic_walk_sweep(m, nmax).cpu().numpy()
        t_sweep = time.perf_counter() - t0
        sample = sorted({1, nmax // 3, 2 * nmax // 3, nmax})
        t0 = time.perf_counter()
        for n in sample:
            if tp.tp_cyclic_walk_gamma2(n, m) != int(sweep[n - 1]):
                print(f"MISMATCH cyclic walk at ({n},{m})", file=sys.stderr)
                sys.exit(1)
        t_plain = (time.perf_counter() - t0) / len(sample) * nmax
        total_plain += t_plain
        total_sweep += t_sweep
        per_m[str(m)] = {"N": tp.tp_cyclic_dim(m), "nnz": tp.tp_cyclic_nnz(m),
                         "sweep_ms": round(t_sweep * 1e3, 3),
                         "plain_ms_estimate": round(t_plain * 1e3, 2)}
    q = nmax * len(list(ms))
    return {"queries": q, "plain_qps_estimate": round(q / total_plain, 1),
            "sweep_qps": round(q / total_sweep, 1),
            "sweep_speedup": round(total_plain / total_sweep, 1), "by_m": per_m}


def batch_roofline(work, ms):
    """Aggregate position of a cold batch (chain levels, dense products and
    traces between two events on its stream) against the packed-u16 VALU
    peak and HBM."""
    t = ms / 1e3
    return {"bound": "alu", "achieved": round(work["ops"] / t / 1e12, 3),
            "peak": round(PEAK_MINPLUS / 1e12, 3), "unit": "Tminplus-ops/s",
            "frac": round(work["ops"] / t / PEAK_MINPLUS, 4),
            "GBs_algorithmic": round(work["bytes"] / t / 1e9, 1)}


def query_suite(tp, synth):
    """gamma_2 queries, plain per-query path vs batched (one persistent launch).

    mixed:  64 instances, n uniform in 4..9, m uniform in 3..200 (seed 0)
    sweep:  n = 8, m = 3..256 (254 instances)
    'plain' calls tp_tropical_power_trace once per instance (state matrices
    cached, every chain recomputed); 'batched cold' answers all instances in
    one batch on a fresh context (every power allocated and computed inside
    the batch; median of three fresh contexts); 'fused cold' the same with
    the chain levels inside the one persistent launch (TP_PARAM_FUSED_CHAIN);
    'batched warm' repeats the batch on the same context (powers resident,
    only the traces run); for the sweep also 'sweep chain', one chain of 256
    powers with the diagonal minimum of each.  Every batched answer is
    compared with the plain one."""
    import torch
    out = {}
    for name, inst in (("mixed64", synth.batch_instances(seed=0)),
                       ("sweep_n8", [(8, m) for m in range(3, 257)])):
        ns = [n for n, _ in inst]
        ms = [m for _, m in inst]
        for n in sorted(set(ns)):
            tp.tp_tropical_power_trace(n, 3)  # state matrix and workspace in the cache
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plain = [tp.tp_tropical_power_trace(n, m) for n, m in inst]
        t_plain = time.perf_counter() - t0
        # the batch kernel's code object loads once per process: a throwaway
        # batch on its own context takes that out of the cold figure
        ctx = tp.tp_ctx_create(1 << 30)
        try:
            tp.tp_batch_power_trace(ctx, [4], [5])
            tp.tp_ctx_check(ctx)
        finally:
            tp.tp_ctx_destroy(ctx)
        # cold: a fresh context (every power allocated and computed), median
        # of three; warm: the same batch again on the last context
        t_colds, dev_ms = [], []
        for rep in range(3):
            ctx = tp.tp_ctx_create(64 << 30)
            try:
                torch.cuda.synchronize()
                stream = torch.cuda.current_stream()
                ev0 = torch.cuda.Event(enable_timing=True)
                ev1 = torch.cuda.Event(enable_timing=True)
                t0 = time.perf_counter()
                ev0.record(stream)
                res = tp.tp_batch_power_trace(ctx, ns, ms, stream=stream)
                ev1.record(stream)
                tp.tp_ctx_check(ctx)
                t_colds.append(time.perf_counter() - t0)
                dev_ms.append(ev0.elapsed_time(ev1))
                work = tp.tp_ctx_last_work(ctx)
                cold = res.cpu().numpy().tolist()
                if rep < 2:
                    continue
                t0 = time.perf_counter()
                res = tp.tp_batch_power_trace(ctx, ns, ms)
                tp.tp_ctx_check(ctx)
                t_warm = time.perf_counter() - t0
                warm = res.cpu().numpy().tolist()
            finally:
                tp.tp_ctx_destroy(ctx)
        t_cold = sorted(t_colds)[1]
        # the same, with the chain levels inside the one persistent launch
        t_fused = []
        for rep in range(3):
            ctx = tp.tp_ctx_create(64 << 30)
            try:
                tp.tp_ctx_set_param(ctx, tp.TP_PARAM_FUSED_CHAIN, 1)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                res = tp.tp_batch_power_trace(ctx, ns, ms)
                tp.tp_ctx_check(ctx)
                t_fused.append(time.perf_counter() - t0)
                fused = res.cpu().numpy().tolist()
            finally:
                tp.tp_ctx_destroy(ctx)
        t_fused = sorted(t_fused)[1]
        if not (cold == warm == fused == plain):
            print(f"MISMATCH in {name}: batched and plain answers differ", file=sys.stderr)
            sys.exit(1)
        k = len(inst)
        out[name] = {"instances": k,
                     "plain_qps": round(k / t_plain, 1),
                     "batched_cold_qps": round(k / t_cold, 1),
                     "batched_warm_qps": round(k / t_warm, 1),
                     "fused_cold_qps": round(k / t_fused, 1),
                     "cold_speedup": round(t_plain / t_cold, 2),
                     "cold_batch_device_ms": round(sorted(dev_ms)[1], 3),
                     "cold_batch_work": {k: float(f"{v:.4g}") for k, v in work.items()},
                     "cold_batch_roofline": batch_roofline(work, sorted(dev_ms)[1]),
                     "fused_cold_speedup": round(t_plain / t_fused, 2),
                     "warm_speedup": round(t_plain / t_warm, 2)}
        if name == "sweep_n8":
            # one sweep chain X_k = A x X_(k-1) with the diagonal minimum of
            # every power (tp_recurrence with the smallest window): all 254
            # answers from a single chain of 256 powers
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, diag = tp.tp_recurrence(8, 256, 1)
            t_sweep = time.perf_counter() - t0
            if [int(diag[m - 1]) for m in ms] != plain:
                print("MISMATCH in sweep_n8: sweep chain and plain answers differ",
                      file=sys.stderr)
                sys.exit(1)
            out[name]["sweep_chain_qps"] = round(k / t_sweep, 1)
            out[name]["sweep_chain_speedup"] = round(t_plain / t_sweep, 2)
    return out


if __name__ == "__main__":
    main()
