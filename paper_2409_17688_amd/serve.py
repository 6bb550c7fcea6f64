"""Serving gamma_2(P_n x C_m) queries on one GPU with continuous batching.

Queries (n, m) arrive at any time.  They are answered from powers of the
state matrix A(D_n) kept resident in HBM (Theorem 2: gamma_2 is the trace of
A^a x A^b for any a + b = m):

* path orders below ``sweep_n`` go to a batch context (``tp_ctx_*``): the
  scheduler thread collects whatever is pending into a *wave*, admits queries
  in arrival order while the powers they would add fit in the context's HBM
  budget (evicting the resident powers of the least recently used path orders
  when the head of the queue does not fit), and runs the wave as one
  persistent launch.  Queries that arrive while a wave runs join the next
  wave as soon as it ends, so the device goes from one wave to the next
  without idling; inside a wave all admitted queries' work overlaps.
* path orders from ``sweep_n`` on (n = 12 by default: one power is 5.6 GB and
  a dense product takes seconds) go to a *sweep lane*: one shared chain
  A^k = A x A^(k-1) (Algorithm 2) advanced on its own stream with three
  buffers; every query with ceil(m/2) = k is answered by one trace of a
  product when the chain passes level k (floor(m/2) is k or k - 1).  Queries
  for a level the chain has passed wait for the next sweep.  The lane runs
  concurrently with the waves on the device.

A failing wave fails only its own queries; the loop keeps serving.  The
scheduler does not depend on the GPU: any object with the executor methods
used below can drive it (the tests use fakes to force admission limits,
errors and cancellation).
"""
from __future__ import annotations

import collections
import threading
import time
from dataclasses import dataclass, field

TP_OK = 0
TP_EINVAL = -1
TP_ENOMEM = -2
TP_EOVERFLOW = -3
TP_EHIP = -4
TP_ECANCELED = -6


@dataclass
class Request:
    n: int
    m: int
    t_arrive: float
    t_start: float | None = None
    t_done: float | None = None
    gamma2: int | None = None
    status: int = 1  # 1 = pending, 0 = done, < 0 = failed (a TP_E* code)
    error: str = ""
    done: threading.Event = field(default_factory=threading.Event)

    @property
    def latency(self) -> float | None:
        return None if self.t_done is None else self.t_done - self.t_arrive

    def wait(self, timeout: float | None = None) -> int:
        self.done.wait(timeout)
        return self.status

    def _finish(self, gamma2=None, status=TP_OK, error=""):
        self.gamma2 = gamma2
        self.status = status
        self.error = error
        self.t_done = time.perf_counter()
        self.done.set()


def validate(n: int, m: int):
    """(status, message) for a query the library cannot take, else None."""
    if not (1 <= n <= 12):
        return TP_EINVAL, f"n = {n} outside 1..12"
    if m < 3:
        return TP_EINVAL, f"the cycle order m = {m} must be at least 3"
    if n * m >= 65535:
        return TP_EOVERFLOW, f"n * m = {n * m} could reach INF in 16-bit entries"
    return None


class GpuExecutor:
    """Runs waves on a batch context and sweep lanes on their own streams."""

    def __init__(self, hbm_budget_bytes: int, tuning: dict | None = None):
        import torch

        from . import _lib as tp
        self.tp = tp
        self.torch = torch
        self.budget = int(hbm_budget_bytes)
        self.ctx = tp.tp_ctx_create(self.budget)
        self.stream = torch.cuda.Stream()
        for key, val in (tuning or {}).items():
            param, n = key
            tp.tp_ctx_set_param(self.ctx, param + n, val)

    def need_bytes(self, ns, ms) -> int:
        return self.tp.tp_ctx_need_bytes(self.ctx, ns, ms)

    def resident_bytes(self) -> int:
        return self.tp.tp_ctx_resident_bytes(self.ctx)

    def release(self, n: int) -> None:
        self.tp.tp_ctx_release(self.ctx, n, stream=self.stream)

    def run_wave(self, ns, ms):
        with self.torch.cuda.stream(self.stream):
            out = self.tp.tp_batch_power_trace(self.ctx, ns, ms, stream=self.stream)
            self.tp.tp_ctx_check(self.ctx, stream=self.stream)
            return out.cpu().tolist()

    def make_lane(self, n: int) -> "SweepLane":
        return SweepLane(n, self.tp, self.torch)

    def close(self) -> None:
        if self.ctx:
            self.torch.cuda.synchronize()
            self.tp.tp_ctx_destroy(self.ctx)
            self.ctx = None


class SweepLane:
    """One shared power chain for path order n on its own stream."""

    def __init__(self, n: int, tp, torch):
        self.n, self.tp, self.torch = n, tp, torch
        self.N = tp.tp_state_dim(n)
        ld = (self.N + 63) // 64 * 64
        self.stream = torch.cuda.Stream()
        with torch.cuda.stream(self.stream):
            self.bufs = [torch.empty((self.N, ld), dtype=torch.uint16, device="cuda")[:, :self.N]
                         for _ in range(3)]
        tp.tp_state_nnz(n)  # builds (and caches) the state's sparse forms
        self.lock = threading.Condition()
        self.pending = collections.defaultdict(list)  # level a -> requests
        self.stop = False
        self.sweeps = 0
        self.levels = 0
        self.thread = threading.Thread(target=self._run, name=f"sweep-n{n}", daemon=True)
        self.thread.start()

    def submit(self, req: Request) -> None:
        with self.lock:
            self.pending[(req.m + 1) // 2].append(req)
            self.lock.notify()

    def close(self) -> None:
        with self.lock:
            self.stop = True
            self.lock.notify()
        self.thread.join()
        with self.lock:
            for reqs in self.pending.values():
                for r in reqs:
                    r._finish(status=TP_ECANCELED, error="server closed")
            self.pending.clear()

    def _answer(self, k: int, X: dict) -> None:
        with self.lock:
            reqs = self.pending.pop(k, [])
        if not reqs:
            return
        tp, torch = self.tp, self.torch
        outs = []
        with torch.cuda.stream(self.stream):
            for r in reqs:
                r.t_start = r.t_start or time.perf_counter()
                b = r.m - k
                outs.append(tp.tp_trace_of_product(X[k], X[b], stream=self.stream))
            vals = [int(o.item()) for o in outs]
        for r, v in zip(reqs, vals):
            r._finish(gamma2=v)

    def _run(self) -> None:
        tp, torch = self.tp, self.torch
        while True:
            with self.lock:
                while not self.pending and not self.stop:
                    self.lock.wait()
                if self.stop:
                    return
            # one sweep: level 1 upwards while some pending query needs a level ahead
            self.sweeps += 1
            try:
                with torch.cuda.stream(self.stream):
                    X = {1: tp.tp_build_state_matrix(self.n, tp.TP_U16, out=self.bufs[1],
                                                     stream=self.stream)}
                    k = 1
                    while True:
                        self._answer(k, X)
                        with self.lock:
                            ahead = [a for a in self.pending if a > k]
                            if self.stop:
                                return
                        if not ahead:
                            break
                        Y = self.bufs[(k + 1) % 3]
                        tp.tp_state_left_mul(self.n, X[k], Y, stream=self.stream)
                        k += 1
                        self.levels += 1
                        X[k] = Y
                        X.pop(k - 2, None)
            except Exception as e:  # fail what is waiting, keep the lane alive
                with self.lock:
                    failed = [r for reqs in self.pending.values() for r in reqs]
                    self.pending.clear()
                for r in failed:
                    r._finish(status=TP_EHIP, error=str(e))


class Server:
    """Continuous-batching gamma_2 server.

    executor: a GpuExecutor (or any object with need_bytes, resident_bytes,
    release, run_wave, make_lane and a ``budget`` attribute).
    max_wave: most queries admitted into one wave.
    sweep_n: path orders >= sweep_n use a sweep lane (None: never).
    """

    def __init__(self, executor, max_wave: int = 1024, sweep_n: int | None = 12):
        self.ex = executor
        self.max_wave = max_wave
        self.sweep_n = sweep_n
        self.cv = threading.Condition()
        self.pending: collections.deque[Request] = collections.deque()
        self.lanes: dict[int, SweepLane] = {}
        self.last_use: dict[int, float] = {}
        self.waves = 0
        self.wave_sizes: list[int] = []
        self.stop = False
        self.thread = threading.Thread(target=self._loop, name="tropical-scheduler", daemon=True)
        self.thread.start()

    # ---------------------------------------------------------------- API --

    def submit(self, n: int, m: int, t_arrive: float | None = None) -> Request:
        req = Request(int(n), int(m), time.perf_counter() if t_arrive is None else t_arrive)
        bad = validate(req.n, req.m)
        if bad:
            req._finish(status=bad[0], error=bad[1])
            return req
        if self.sweep_n is not None and req.n >= self.sweep_n:
            with self.cv:
                lane = self.lanes.get(req.n)
                if lane is None:
                    lane = self.lanes[req.n] = self.ex.make_lane(req.n)
            lane.submit(req)
            return req
        with self.cv:
            if self.stop:
                req._finish(status=TP_ECANCELED, error="server closed")
                return req
            self.pending.append(req)
            self.cv.notify()
        return req

    def cancel(self, req: Request) -> bool:
        """Withdraws a query that has not been admitted into a wave yet."""
        with self.cv:
            try:
                self.pending.remove(req)
            except ValueError:
                return False
        req._finish(status=TP_ECANCELED, error="cancelled")
        return True

    def close(self) -> None:
        with self.cv:
            self.stop = True
            self.cv.notify()
        self.thread.join()
        for lane in self.lanes.values():
            lane.close()
        with self.cv:
            while self.pending:
                self.pending.popleft()._finish(status=TP_ECANCELED, error="server closed")

    # ---------------------------------------------------------- scheduler --

    def _admit(self, cands):
        """Largest arrival-order prefix-compatible set that fits the budget."""
        admitted, deferred = [], []
        for r in cands:
            trial = admitted + [r]
            need = self.ex.need_bytes([q.n for q in trial], [q.m for q in trial])
            if self.ex.resident_bytes() + need <= self.ex.budget:
                admitted.append(r)
            else:
                deferred.append(r)
        return admitted, deferred

    def _evict_for(self, keep):
        """Releases least recently used path orders not in keep; True if any."""
        victims = sorted((t, n) for n, t in self.last_use.items() if n not in keep)
        for _, n in victims:
            self.ex.release(n)
            del self.last_use[n]
        return bool(victims)

    def _loop(self) -> None:
        while True:
            with self.cv:
                while not self.pending and not self.stop:
                    self.cv.wait()
                if self.stop and not self.pending:
                    return
                if self.stop:
                    return
                cands = [self.pending.popleft()
                         for _ in range(min(self.max_wave, len(self.pending)))]
            admitted, deferred = self._admit(cands)
            if not admitted and self._evict_for({r.n for r in cands}):
                admitted, deferred = self._admit(cands)
            if not admitted and self._evict_for(set()):
                admitted, deferred = self._admit(cands)
            if not admitted:
                # even an empty context cannot hold what the head query needs
                head = deferred.pop(0)
                head._finish(status=TP_ENOMEM,
                             error=f"needs more than the {self.ex.budget}-byte budget")
            with self.cv:
                self.pending.extendleft(reversed(deferred))
            if not admitted:
                continue
            t0 = time.perf_counter()
            for r in admitted:
                r.t_start = t0
                self.last_use[r.n] = t0
            self.waves += 1
            self.wave_sizes.append(len(admitted))
            try:
                vals = self.ex.run_wave([r.n for r in admitted], [r.m for r in admitted])
            except Exception as e:  # this wave fails; the server keeps going
                code = getattr(e, "status", TP_EHIP)
                for r in admitted:
                    r._finish(status=code, error=str(e))
                continue
            for r, v in zip(admitted, vals):
                r._finish(gamma2=int(v))


def percentile(values, q: float) -> float:
    """q-th percentile (0..100) by the nearest-rank rule."""
    v = sorted(values)
    if not v:
        return float("nan")
    k = max(0, min(len(v) - 1, int(-(-q * len(v) // 100)) - 1))
    return v[k]
