"""Microbenchmarks of the library's kernels at the shapes of path order n.

    python -m paper_2409_17688_amd.kernel_bench --op spmm --n 12 --reps 5
    python -m paper_2409_17688_amd.kernel_bench --op bstep --n 12 --reps 5
    python -m paper_2409_17688_amd.kernel_bench --op gather --n 9 --reps 5
    python -m paper_2409_17688_amd.kernel_bench --op trace --n 12
    python -m paper_2409_17688_amd.kernel_bench --op gemm --n 10 --config 0
    python -m paper_2409_17688_amd.kernel_bench --op batch --instances mixed64
    python -m paper_2409_17688_amd.kernel_bench --op cdiff --n 12
    python -m paper_2409_17688_amd.kernel_bench --op recurrence --n 12 --window 4
    python -m paper_2409_17688_amd.kernel_bench --op apsp --N 8192
    python -m paper_2409_17688_amd.kernel_bench --op cstep --n 12 --reps 5
    python -m paper_2409_17688_amd.kernel_bench --op gemv --m 12 --trans 1
    python -m paper_2409_17688_amd.kernel_bench --op walk --m 8 --nmax 256 --form 1

Matrices use the library's resident layout (rows padded to 64 entries).
Times come from HIP events on the launch stream; one JSON line per run with
the algorithmic work of one launch:
  spmm   nnz(A) * N (min,+) operations; bytes: X read once, Y written (4 N^2)
  bstep  the same product by the blocked sparse step (tp_state_left_mul)
  gather the same product by the packed per-row gather (tp_state_left_mul)
  trace  2 N^2 entries read (4 N^2 bytes)
  gemm   N^3 (min,+) operations
  batch  one persistent launch answering the instances (cold context;
         --compact-from sets which path orders keep compact powers,
         --chain-giants-from which make their giants by the chain)
  cdiff  constant-difference test of A^2 against A (tp_const_diff): 2 N^2
         entries read (4 N^2 bytes)
  recurrence  tp_recurrence(n, K, window): K powers, each compared with the
         window before it, then Algorithms 3 and 4 (wall time)
  cstep  the same product on compact powers (tp_compact_step: 8-bit residuals,
         one offset per row; --shared: tp_compact_shared_step, one base per
         power), from A^3; the offsets' product is included
  apsp   all-pairs shortest paths on a random digraph of order N (weights
         0..49 on 1 % of the pairs, default_rng(0)): ceil(log2(N-1)) dense
         products of N^3 operations
  gemv   one (min,+) vector-matrix (--trans 1) or matrix-vector product with
         the cyclic column digraph's matrix of cycle order m (16 bits, rows
         padded to 64 entries): 2 N^2 bytes of matrix read per launch
  walk   tp_cyclic_walk_sweep(m, nmax, form): the walk along the path over
         cyclic columns, every level read by the end vector; nnz per level
"""
from __future__ import annotations

import argparse
import json
import sys
import time


def _events(torch, fn, reps):
    fn()
    torch.cuda.synchronize()
    s = torch.cuda.Event(enable_timing=True)
    e = torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(reps):
        fn()
    e.record()
    torch.cuda.synchronize()
    return s.elapsed_time(e) / reps / 1e3


def _padded(torch, N):
    ld = (N + 63) // 64 * 64
    return torch.empty((N, ld), dtype=torch.uint16, device="cuda")[:, :N]


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--op", choices=["spmm", "bstep", "gather", "trace", "gemm", "batch", "cdiff",
                                     "recurrence", "apsp", "cstep", "gemv", "walk"],
                    required=True)
    ap.add_argument("--n", type=int, default=10)
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--config", type=int, default=None, help="dense product tile config")
    ap.add_argument("--instances", default="mixed64", help="batch workload: mixed64 or n:mlist")
    ap.add_argument("--fused", action="store_true",
                    help="batch: chain levels inside the persistent launch too")
    ap.add_argument("--compact-from", type=int, default=None,
                    help="batch: TP_PARAM_COMPACT_FROM (path orders kept as compact powers)")
    ap.add_argument("--chain-giants-from", type=int, default=None,
                    help="batch: TP_PARAM_CHAIN_GIANTS_FROM (path orders whose giants the chain makes)")
    ap.add_argument("--K", type=int, default=50, help="recurrence: powers computed")
    ap.add_argument("--window", type=int, default=0, help="recurrence: comparison window")
    ap.add_argument("--N", type=int, default=8192, help="apsp: order of the digraph")
    ap.add_argument("--unroll", type=int, default=0,
                    help="cstep: gathers per round (4 or 8, | 256 for mask groups; 0: default)")
    ap.add_argument("--shared", action="store_true", help="cstep: one base per power")
    ap.add_argument("--entries", action="store_true",
                    help="bstep: each block entry applied on its own (not by mask group)")
    ap.add_argument("--m", type=int, default=12, help="gemv, walk: cycle order")
    ap.add_argument("--trans", type=int, default=1, help="gemv: 1 = x A, 0 = A x")
    ap.add_argument("--nmax", type=int, default=256, help="walk: path orders swept")
    ap.add_argument("--form", type=int, default=0, help="walk: TP_WALK_* form")
    args = ap.parse_args(argv)

    import torch

    from . import _lib as tp
    n = args.n
    out = {"op": args.op}
    if args.op == "gemv":
        m = args.m
        N = tp.tp_cyclic_dim(m)
        A = _padded(torch, N)
        tp.tp_build_cyclic_matrix(m, tp.TP_U16, out=A)
        x, _ = tp.tp_build_cyclic_boundary(m, tp.TP_U16)
        y = torch.empty_like(x)
        t = _events(torch, lambda: tp.tp_minplus_gemv(A, x, trans=bool(args.trans), y=y),
                    args.reps)
        nbytes = 2.0 * N * N + 4.0 * N
        out.update({"m": m, "N": N, "trans": args.trans, "ms": t * 1e3, "bytes": nbytes,
                    "GBs": nbytes / t / 1e9})
    elif args.op == "walk":
        m = args.m
        out_t = torch.empty(args.nmax, dtype=torch.int32, device="cuda")
        tp.tp_cyclic_walk_sweep(m, args.nmax, out_t, form=args.form)
        times = []
        for _ in range(args.reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            tp.tp_cyclic_walk_sweep(m, args.nmax, out_t, form=args.form)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        t = min(times)
        out.update({"m": m, "N": tp.tp_cyclic_dim(m), "nnz": tp.tp_cyclic_nnz(m),
                    "nmax": args.nmax, "form": args.form, "ms": t * 1e3,
                    "us_per_level": t / max(args.nmax - 1, 1) * 1e6})
    elif args.op == "apsp":
        import numpy as np
        N = args.N
        rng = np.random.default_rng(0)
        W = rng.integers(0, 50, (N, N)).astype(np.uint16)
        W[rng.random((N, N)) > 0.01] = 65535
        Wd = torch.from_numpy(W.view(np.int16)).cuda().view(torch.uint16)
        D, T = torch.empty_like(Wd), torch.empty_like(Wd)
        t = _events(torch, lambda: tp.tp_apsp(Wd, D, T), args.reps)
        sq = max(0, (N - 2).bit_length())
        out.update({"N": N, "squarings": sq, "ms": t * 1e3,
                    "Tminplus_ops": sq * float(N) ** 3 / t / 1e12})
    elif args.op == "recurrence":
        tp.tp_recurrence(n, 3, 1)  # the state of n in the library's cache
        times = []
        for _ in range(args.reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rec, _ = tp.tp_recurrence(n, args.K, args.window)
            times.append(time.perf_counter() - t0)
        out.update({"n": n, "K": args.K, "window": rec.window, "found": rec.found, "r0": rec.r0,
                    "a": rec.a, "b": rec.b, "n0": rec.n0, "s": min(times),
                    "s_all": [round(t, 3) for t in times]})
    elif args.op == "cstep":
        N = tp.tp_state_dim(n)
        nnz = tp.tp_state_nnz(n)
        X, Y = _padded(torch, N), _padded(torch, N)
        tp.tp_build_state_matrix(n, tp.TP_U16, out=X)
        tp.tp_state_left_mul(n, X, Y)
        tp.tp_state_left_mul(n, Y, X)  # A^3
        ld = (N + 63) // 64 * 64
        X8 = torch.empty((N, ld), dtype=torch.uint8, device="cuda")
        Y8 = torch.empty_like(X8)
        st = torch.zeros(1, dtype=torch.int32, device="cuda")
        tp.tp_tune_compact_step(args.unroll)
        if args.shared:
            bx = torch.empty(2, dtype=torch.int32, device="cuda")
            by = torch.empty_like(bx)
            tp.tp_compact_shared_from_u16(X, X8, bx, st)
            del X, Y
            bufs = [(X8, bx), (Y8, by)]

            def step():  # alternate the buffers: each step starts from the last output
                (a, ba), (c, bc) = bufs
                tp.tp_compact_shared_step(n, a, ba, N, c, bc, st)
                bufs.reverse()
            t = _events(torch, step, args.reps)
        else:
            RX = torch.empty(N, dtype=torch.int32, device="cuda")
            RY = torch.empty_like(RX)
            tp.tp_compact_from_u16(X, X8, RX, st)
            del X, Y
            t = _events(torch, lambda: tp.tp_compact_step(n, X8, RX, N, Y8, RY, st), args.reps)
        out.update({"n": n, "N": N, "nnz": nnz, "unroll": args.unroll, "shared": args.shared,
                    "ms": t * 1e3, "Tminplus_ops": nnz * N / t / 1e12, "status": int(st.item())})
    elif args.op in ("spmm", "bstep", "gather", "trace", "gemm", "cdiff"):
        N = tp.tp_state_dim(n)
        X, Y = _padded(torch, N), _padded(torch, N)
        tp.tp_build_state_matrix(n, tp.TP_U16, out=X)
        out.update({"n": n, "N": N})
        if args.op == "spmm":
            nnz = tp.tp_state_nnz(n)
            rowptr, col, z = tp.tp_build_state_csr(n)
            t = _events(torch, lambda: tp.tp_minplus_spmm(rowptr, col, z, X, Y), args.reps)
            out.update({"nnz": nnz, "ms": t * 1e3, "Tminplus_ops": nnz * N / t / 1e12})
        elif args.op in ("bstep", "gather"):
            nnz = tp.tp_state_nnz(n)
            form = tp.TP_STEP_BLOCKED if args.op == "bstep" else tp.TP_STEP_CSR
            if args.op == "bstep" and args.entries:
                form = tp.TP_STEP_BLOCKED_ENTRIES
            t = _events(torch, lambda: tp.tp_state_left_mul(n, X, Y, form=form), args.reps)
            out.update({"nnz": nnz, "ms": t * 1e3, "Tminplus_ops": nnz * N / t / 1e12})
        elif args.op == "cdiff":
            tp.tp_state_left_mul(n, X, Y)
            t = _events(torch, lambda: tp.tp_const_diff(Y, X), args.reps)
            out.update({"ms": t * 1e3, "GBs": 4.0 * N * N / t / 1e9})
        elif args.op == "trace":
            tp.tp_minplus_spmm(*tp.tp_build_state_csr(n), X, Y)
            t = _events(torch, lambda: tp.tp_trace_of_product(X, Y), args.reps)
            out.update({"ms": t * 1e3, "GBs": 4.0 * N * N / t / 1e9})
        else:
            C = _padded(torch, N)
            t = _events(torch, lambda: tp.tp_minplus_gemm(X, X, C, config=args.config),
                        args.reps)
            out.update({"config": args.config, "ms": t * 1e3, "Tminplus_ops": N ** 3 / t / 1e12})
    else:
        import os
        sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
        import synth
        if args.instances == "mixed64":
            inst = synth.batch_instances(seed=0)
        else:
            nn, ms = args.instances.split(":")
            inst = [(int(nn), int(m)) for m in ms.split(",")]
        ns, ms = [a for a, _ in inst], [b for _, b in inst]
        for nn in sorted(set(ns)):
            tp.tp_tropical_power_trace(nn, 3)
        times = []
        for _ in range(args.reps):
            ctx = tp.tp_ctx_create(64 << 30)
            try:
                tp.tp_ctx_set_param(ctx, tp.TP_PARAM_FUSED_CHAIN, int(args.fused))
                if args.compact_from is not None:
                    tp.tp_ctx_set_param(ctx, tp.TP_PARAM_COMPACT_FROM, args.compact_from)
                if args.chain_giants_from is not None:
                    tp.tp_ctx_set_param(ctx, tp.TP_PARAM_CHAIN_GIANTS_FROM,
                                        args.chain_giants_from)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                tp.tp_batch_power_trace(ctx, ns, ms)
                tp.tp_ctx_check(ctx)
                times.append(time.perf_counter() - t0)
                resident = tp.tp_ctx_resident_bytes(ctx)
            finally:
                tp.tp_ctx_destroy(ctx)
        out.update({"instances": len(inst), "fused": args.fused,
                    "compact_from": args.compact_from,
                    "chain_giants_from": args.chain_giants_from, "resident_bytes": resident,
                    "ms": min(times) * 1e3, "ms_all": [round(t * 1e3, 2) for t in times]})
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
