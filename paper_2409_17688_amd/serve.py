"""Serving gamma_2(P_n x C_m) queries on one GPU with continuous batching.

Queries (n, m) arrive at any time and are answered from powers of the state
matrix A(D_n) kept resident in HBM (Theorem 2: gamma_2 is the least diagonal
entry of A^m, i.e. the trace of A^a x A^b for any a + b = m).

* Path orders below the lane orders go to batch contexts (``tp_ctx_*``).
  The executor holds ``slots`` contexts, each with its own stream and worker
  thread, so up to ``slots`` waves are in flight on the device at once.  A
  path order's resident powers live in one context (its *owner*); the
  scheduler forms a wave for every idle slot from the pending queries whose
  path order that slot owns or nobody owns yet, in arrival order, while the
  powers they would add fit in the HBM budget (what every context and lane
  holds plus what the waves in flight may still add).  When the oldest
  admissible query does not fit, the least recently used path orders of idle
  slots are released one at a time until it does; if it still does not fit
  the wave stops there, so later queries never overtake it (no starvation);
  a query that cannot fit even then, with nothing else in flight, fails with
  TP_ENOMEM.  A query that arrives while its owner's wave runs joins that
  slot's next wave; one for another path order is admitted into the other
  slot at once and overlaps the running wave on the device.
* The lane orders (n = 10, 11, 12 by default: one power is 0.15 to 5.6 GB in
  16 bits) each get a *resident lane* on its own stream and thread.  It keeps
  shared-base compact powers (8-bit residuals over one base, half the bytes
  of 16 bits): whole powers A^r for r = 3..c+2 (the babies) and, for every
  j >= 1, the columns S of A^(jc) (the giant panels), S the states with at
  most k zeros, chained from the columns S of A by the sparse left step.  A
  query is then one trace of a product: of two babies when m <= 2(c+2), else
  of the rows S of A^r with the panel of A^(jc), m = jc + r, read on the
  diagonal entries of S.  The second is exact whenever the value v found has
  floor(v/m) <= k: every optimal closed walk of length m passes through a
  state with at most floor(gamma_2/m) zeros (its label is the sum of the zero
  counts of the m states it visits, Section 2.2), and rotating the cycle
  starts it there.  Otherwise, and for m outside the lane's reach, the lane
  answers by the plain per-query path.  Panels are computed as queries need
  them; once built they stay, so later queries cost one trace.

A failing wave fails only its own queries; the loop keeps serving.  The
scheduler does not depend on the GPU: any object with the executor methods
used below can drive it (the tests use fakes to force admission limits,
errors, overlap and cancellation).
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

LANE_ORDERS = (10, 11, 12)


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


def _ld(cols: int) -> int:
    return max((cols + 63) // 64 * 64, 64)


class ResidentLane:
    """Resident shared-base compact powers of one path order n on their own
    stream and thread; each query is answered by one trace of a product once
    the powers it needs exist (see the module docstring)."""

    def __init__(self, n: int, tp, torch, c: int = 10, m_cap: int = 512,
                 max_zeros: int | None = None):
        if c < 3:
            raise ValueError("the baby powers start at A^3: c >= 3")
        self.n, self.tp, self.torch = n, tp, torch
        self.c, self.m_cap = c, m_cap
        self.k = (n + 2) // 3 if max_zeros is None else max_zeros
        self.N = tp.tp_state_dim(n)
        self.stream = torch.cuda.Stream()
        with torch.cuda.stream(self.stream):
            self.S = tp.tp_state_select(n, self.k, stream=self.stream)
        self.count = int(self.S.numel())
        self.J = max(0, (m_cap - 3) // c)  # panels j = 1..J serve m <= m_cap
        N, ld, lds = self.N, _ld(self.N), _ld(self.count)
        # steady-state bytes: babies, panels and two chain buffers (the build
        # also holds three 16-bit powers for a moment)
        self.reserved_bytes = c * N * ld + (self.J + 2) * N * lds + 3 * 2 * N * ld
        self.babies: dict[int, tuple] = {}
        self.panels: dict[int, tuple] = {}
        self.level = 0          # highest power whose columns S the chain holds
        self.chain = None       # (x8, base) of that power
        self.spare = None       # (x8, base) buffer the next step writes
        self.broken = ""        # set when a power cannot be held compact
        self.lock = threading.Condition()
        self.pending: list[Request] = []
        self.stop = False
        self.plain_answers = 0
        self.trace_answers = 0
        self.thread = threading.Thread(target=self._run, name=f"lane-n{n}", daemon=True)
        self.thread.start()

    # ------------------------------------------------------------- public --

    def submit(self, req: Request) -> bool:
        with self.lock:
            if self.stop:
                return False
            self.pending.append(req)
            self.lock.notify()
        return True

    def close(self) -> None:
        with self.lock:
            self.stop = True
            self.lock.notify()
        self.thread.join()
        with self.lock:
            for r in self.pending:
                r._finish(status=TP_ECANCELED, error="server closed")
            self.pending.clear()

    # --------------------------------------------------------------- plan --

    def _plan(self, m: int):
        """('babies', a, b) | ('panel', r, j) | ('plain',)."""
        c = self.c
        if self.broken or m < 6 or m > self.m_cap:
            return ("plain",)
        if m <= 2 * (c + 2):
            return ("babies", (m + 1) // 2, m // 2)
        j = (m - 3) // c
        return ("panel", m - j * c, j)

    # -------------------------------------------------------------- build --

    def _u8(self, cols):
        return self.torch.empty((self.N, _ld(cols)), dtype=self.torch.uint8,
                                device="cuda")[:, :cols]

    def _base(self):
        return self.torch.zeros(2, dtype=self.torch.int32, device="cuda")

    def _build_babies(self):
        tp, torch, n, N, s = self.tp, self.torch, self.n, self.N, self.stream
        st = torch.zeros(1, dtype=torch.int32, device="cuda")
        A = torch.empty((N, _ld(N)), dtype=torch.uint16, device="cuda")[:, :N]
        B = torch.empty_like(A)
        tp.tp_build_state_matrix(n, tp.TP_U16, out=A, stream=s)
        tp.tp_state_left_mul(n, A, B, stream=s)          # A^2
        tp.tp_state_left_mul(n, B, A, stream=s)          # A^3
        x, b = self._u8(N), self._base()
        tp.tp_compact_shared_from_u16(A, x, b, st, stream=s)
        del A, B
        self.babies[3] = (x, b)
        for r in range(4, self.c + 3):
            y, by = self._u8(N), self._base()
            tp.tp_compact_shared_step(n, x, b, N, y, by, st, stream=s)
            self.babies[r] = (y, by)
            x, b = y, by
        # the panel chain starts at the columns S of A^3
        P = torch.empty((N, _ld(self.count)), dtype=torch.uint16, device="cuda")[:, :self.count]
        Q = torch.empty_like(P)
        tp.tp_build_state_columns(n, self.S, out=P, stream=s)
        tp.tp_state_left_mul(n, P, Q, stream=s)
        tp.tp_state_left_mul(n, Q, P, stream=s)
        x, b = self._u8(self.count), self._base()
        tp.tp_compact_shared_from_u16(P, x, b, st, stream=s)
        del P, Q
        self.chain, self.spare, self.level = (x, b), (self._u8(self.count), self._base()), 3
        self.status = st
        s.synchronize()
        if int(st.item()) != 0:
            self.broken = "a power of A(D_n) did not fit the compact form"

    def _advance(self):
        """One chain step of the panel; keeps it when the level is jc.  The
        buffer the step read becomes the next step's output unless it holds a
        kept panel (the level before was jc), which is never written again."""
        tp, s = self.tp, self.stream
        (x, b), (y, by) = self.chain, self.spare
        tp.tp_compact_shared_step(self.n, x, b, self.count, y, by, self.status, stream=s)
        self.level += 1
        if self.level % self.c == 0:
            self.panels[self.level // self.c] = (y, by)
        x_kept = any(px is x for px, _ in self.panels.values())
        self.chain = (y, by)
        self.spare = (self._u8(self.count), self._base()) if x_kept else (x, b)

    # ------------------------------------------------------------- answer --

    def _ready(self, plan) -> bool:
        return plan[0] != "panel" or plan[2] in self.panels

    def _answer(self, reqs):
        tp, torch, s = self.tp, self.torch, self.stream
        outs = torch.empty(max(len(reqs), 1), dtype=torch.int32, device="cuda")
        plans = []
        with torch.cuda.stream(s):
            for i, r in enumerate(reqs):
                r.t_start = r.t_start or time.perf_counter()
                p = self._plan(r.m)
                plans.append(p)
                if p[0] == "babies":
                    (xa, ba), (xb, bb) = self.babies[p[1]], self.babies[p[2]]
                    tp.tp_compact_shared_select_trace(xa, ba, xb, bb, None, out=outs[i:i + 1],
                                                      stream=s)
                elif p[0] == "panel":
                    (xr, br), (g, bg) = self.babies[p[1]], self.panels[p[2]]
                    tp.tp_compact_shared_select_trace(xr, br, g, bg, self.S, out=outs[i:i + 1],
                                                      stream=s)
            vals = outs.cpu().tolist()
        for r, p, v in zip(reqs, plans, vals):
            if p[0] == "panel" and v // r.m > self.k:
                p = ("plain",)  # the pruned diagonal cannot vouch for this value
            if p[0] == "plain":
                with torch.cuda.stream(s):
                    v = tp.tp_tropical_power_trace(r.n, r.m, stream=s)
                self.plain_answers += 1
            else:
                self.trace_answers += 1
            r._finish(gamma2=int(v))

    def _run(self) -> None:
        built = False
        while True:
            with self.lock:
                while not self.pending and not self.stop:
                    self.lock.wait()
                if self.stop:
                    return
            try:
                if not built:
                    with self.torch.cuda.stream(self.stream):
                        self._build_babies()
                    built = True
                while True:
                    with self.lock:
                        if self.stop:
                            return
                        ready = [r for r in self.pending if self._ready(self._plan(r.m))]
                        self.pending = [r for r in self.pending if r not in ready]
                        need = [self._plan(r.m)[2] for r in self.pending]
                    if ready:
                        self._answer(ready)
                    if not need:
                        break
                    with self.torch.cuda.stream(self.stream):
                        self._advance()
                        if self.level % self.c == 0:
                            self.stream.synchronize()
                            if int(self.status.item()) != 0:
                                self.broken = "a power of A(D_n) did not fit the compact form"
            except Exception as e:  # fail what is waiting, keep the lane alive
                with self.lock:
                    failed, self.pending = self.pending, []
                for r in failed:
                    r._finish(status=getattr(e, "status", TP_EHIP), error=str(e))


class GpuExecutor:
    """Batch contexts (one stream each) for the waves, resident lanes for the
    lane orders."""

    def __init__(self, hbm_budget_bytes: int, slots: int = 2, tuning: dict | None = None,
                 lane_c: int = 10, lane_m_cap: int = 512):
        import torch

        from . import _lib as tp
        self.tp = tp
        self.torch = torch
        self.budget = int(hbm_budget_bytes)
        self.nslots = int(slots)
        self.ctxs = [tp.tp_ctx_create(self.budget) for _ in range(self.nslots)]
        self.streams = [torch.cuda.Stream() for _ in range(self.nslots)]
        self._resident = [0] * self.nslots  # bytes per context, read after each change
        self.lanes: list[ResidentLane] = []
        self.lane_c, self.lane_m_cap = lane_c, lane_m_cap
        # each context's persistent launch takes at most its share of the
        # chip's workgroup slots (4 per CU at the batch kernel's register
        # budget), so a long wave on one slot leaves room for the other's
        cus = torch.cuda.get_device_properties(torch.cuda.current_device()).multi_processor_count
        share = max(8, cus * 4 // self.nslots) if self.nslots > 1 else 0
        for ctx in self.ctxs:
            tp.tp_ctx_set_param(ctx, tp.TP_PARAM_GRID, share)
            for key, val in (tuning or {}).items():
                param, n = key
                tp.tp_ctx_set_param(ctx, param + n, val)

    def need_bytes(self, slot, ns, ms) -> int:
        return self.tp.tp_ctx_need_bytes(self.ctxs[slot], ns, ms)

    def resident_bytes(self) -> int:
        # cached per context: asking a context whose wave runs would wait for it
        return sum(self._resident) + sum(l.reserved_bytes for l in self.lanes)

    def release(self, slot: int, n: int) -> None:
        self.tp.tp_ctx_release(self.ctxs[slot], n, stream=self.streams[slot])
        self._resident[slot] = self.tp.tp_ctx_resident_bytes(self.ctxs[slot])

    def run_wave(self, slot: int, ns, ms):
        ctx, st = self.ctxs[slot], self.streams[slot]
        try:
            with self.torch.cuda.stream(st):
                out = self.tp.tp_batch_power_trace(ctx, ns, ms, stream=st)
                self.tp.tp_ctx_check(ctx, stream=st)
                return out.cpu().tolist()
        finally:
            self._resident[slot] = self.tp.tp_ctx_resident_bytes(ctx)

    def make_lane(self, n: int) -> ResidentLane:
        lane = ResidentLane(n, self.tp, self.torch, c=self.lane_c, m_cap=self.lane_m_cap)
        self.lanes.append(lane)
        return lane

    def close(self) -> None:
        self.torch.cuda.synchronize()
        for ctx in self.ctxs:
            if ctx:
                self.tp.tp_ctx_destroy(ctx)
        self.ctxs = []
        self.lanes = []


class Server:
    """Continuous-batching gamma_2 server.

    executor: a GpuExecutor, or any object with ``budget``, ``nslots``,
    need_bytes(slot, ns, ms), resident_bytes(), release(slot, n),
    run_wave(slot, ns, ms) and make_lane(n).
    max_wave: most queries admitted into one wave.
    lane_n: path orders served by resident lanes instead of waves.
    """

    def __init__(self, executor, max_wave: int = 1024, lane_n=LANE_ORDERS):
        self.ex = executor
        self.max_wave = max_wave
        self.lane_n = frozenset(lane_n or ())
        self.nslots = int(getattr(executor, "nslots", 1))
        self.cv = threading.Condition()
        self.pending: collections.deque[Request] = collections.deque()
        self.lanes: dict[int, object] = {}
        self.owner: dict[int, int] = {}        # path order -> slot holding its powers
        self.last_use: dict[int, float] = {}   # path order -> last admission
        self.busy = [False] * self.nslots
        self.reserved = [0] * self.nslots      # bytes the wave in flight may add
        self.jobs: list[list[Request] | None] = [None] * self.nslots
        self.waves = 0
        self.wave_sizes: list[int] = []
        self.max_in_flight = 0
        self.stop = False
        self.workers = [threading.Thread(target=self._worker, args=(s,), daemon=True,
                                         name=f"tropical-slot{s}") for s in range(self.nslots)]
        for w in self.workers:
            w.start()
        self.thread = threading.Thread(target=self._loop, name="tropical-scheduler", daemon=True)
        self.thread.start()

    # ---------------------------------------------------------------- API --

    def submit(self, n: int, m: int, t_arrive: float | None = None) -> Request:
        req = Request(int(n), int(m), time.perf_counter() if t_arrive is None else t_arrive)
        bad = validate(req.n, req.m)
        if bad:
            req._finish(status=bad[0], error=bad[1])
            return req
        with self.cv:
            if self.stop:
                req._finish(status=TP_ECANCELED, error="server closed")
                return req
            if req.n in self.lane_n:
                lane = self.lanes.get(req.n)
                if lane is None:
                    try:
                        lane = self.lanes[req.n] = self.ex.make_lane(req.n)
                    except Exception as e:
                        req._finish(status=getattr(e, "status", TP_EHIP), error=str(e))
                        return req
                if not lane.submit(req):
                    req._finish(status=TP_ECANCELED, error="server closed")
                return req
            self.pending.append(req)
            self.cv.notify_all()
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
            self.cv.notify_all()
        self.thread.join()
        for w in self.workers:
            w.join()
        for lane in self.lanes.values():
            lane.close()
        with self.cv:
            while self.pending:
                self.pending.popleft()._finish(status=TP_ECANCELED, error="server closed")

    # ---------------------------------------------------------- scheduler --

    def _free_bytes(self, planned: int) -> int:
        return self.ex.budget - self.ex.resident_bytes() - sum(self.reserved) - planned

    def _evict_one(self, keep) -> bool:
        """Releases the least recently used path order held by an idle slot
        and not in keep; False when there is none."""
        cands = [(t, n) for n, t in self.last_use.items()
                 if n not in keep and n in self.owner and not self.busy[self.owner[n]]]
        if not cands:
            return False
        _, n = min(cands)
        self.ex.release(self.owner[n], n)
        del self.owner[n]
        del self.last_use[n]
        return True

    def _form_waves(self) -> bool:
        """Admits pending queries into waves for the idle slots (caller holds
        cv); True when a wave was handed to a worker."""
        idle = [s for s in range(self.nslots) if not self.busy[s]]
        if not idle or not self.pending:
            return False
        plans = {s: [] for s in idle}
        ms_of = {s: {} for s in idle}      # n -> m values planned on s
        need_of = {s: {} for s in idle}    # n -> bytes those add on s
        slot_of: dict[int, int] = {}       # unowned n -> slot chosen this round
        planned = 0
        admitted = set()
        for r in list(self.pending):
            s = self.owner.get(r.n, slot_of.get(r.n))
            if s is None:
                s = min(idle, key=lambda x: len(plans[x]))
            if self.busy[s]:
                continue  # joins its owner's next wave
            if len(plans[s]) >= self.max_wave:
                continue
            ms = ms_of[s].get(r.n, []) + [r.m]
            delta = self.ex.need_bytes(s, [r.n] * len(ms), ms) - need_of[s].get(r.n, 0)
            keep = {q.n for p in plans.values() for q in p} | {r.n}
            while delta > self._free_bytes(planned) and self._evict_one(keep):
                pass
            if delta > self._free_bytes(planned):
                if not any(plans.values()) and not any(self.busy):
                    # even with everything else released it does not fit
                    self.pending.remove(r)
                    r._finish(status=TP_ENOMEM,
                              error=f"needs more than the {self.ex.budget}-byte budget")
                    continue
                break  # later queries wait behind it
            plans[s].append(r)
            ms_of[s][r.n] = ms
            need_of[s][r.n] = need_of[s].get(r.n, 0) + delta
            slot_of[r.n] = s
            planned += delta
            admitted.add(id(r))
        if not admitted:
            return False
        self.pending = collections.deque(r for r in self.pending if id(r) not in admitted)
        t0 = time.perf_counter()
        for s, plan in plans.items():
            if not plan:
                continue
            for r in plan:
                r.t_start = t0
                self.owner[r.n] = s
                self.last_use[r.n] = t0
            self.busy[s] = True
            self.reserved[s] = sum(need_of[s].values())
            self.jobs[s] = plan
            self.waves += 1
            self.wave_sizes.append(len(plan))
        self.max_in_flight = max(self.max_in_flight, sum(self.busy))
        self.cv.notify_all()
        return True

    def _loop(self) -> None:
        with self.cv:
            while True:
                if self.stop:
                    return
                if not self._form_waves():
                    self.cv.wait()

    def _worker(self, s: int) -> None:
        while True:
            with self.cv:
                while self.jobs[s] is None and not self.stop:
                    self.cv.wait()
                if self.jobs[s] is None:
                    return
                plan = self.jobs[s]
            try:
                vals = self.ex.run_wave(s, [r.n for r in plan], [r.m for r in plan])
            except Exception as e:  # this wave fails; the server keeps going
                code = getattr(e, "status", TP_EHIP)
                for r in plan:
                    r._finish(status=code, error=str(e))
            else:
                for r, v in zip(plan, vals):
                    r._finish(gamma2=int(v))
            with self.cv:
                self.jobs[s] = None
                self.busy[s] = False
                self.reserved[s] = 0
                self.cv.notify_all()


def percentile(values, q: float) -> float:
    """q-th percentile (0..100) by the nearest-rank rule."""
    v = sorted(values)
    if not v:
        return float("nan")
    k = max(0, min(len(v) - 1, int(-(-q * len(v) // 100)) - 1))
    return v[k]
